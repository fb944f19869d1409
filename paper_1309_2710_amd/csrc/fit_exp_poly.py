"""Coefficients of the polynomial in exp_cw (rkc_device.h).

After the reduction x = n ln2 + r, |r| <= ln2/2, exp(r) = 1 + r + r^2 q(r)
with q a degree-9 Chebyshev fit (near minimax) of (exp(r) - 1 - r)/r^2 on
[-ln2/2, ln2/2], computed in 50-digit arithmetic and rounded to double.  The
relative error of 1 + r(1 + r q(r)) with the rounded coefficients is below
1.6e-17 (printed).  Run: python fit_exp_poly.py
"""
import mpmath as mp


def fit(deg=9, dps=50):
    mp.mp.dps = dps
    a = mp.log(2) / 2

    def g(r):
        return mp.mpf(1) / 2 if abs(r) < mp.mpf("1e-30") else (mp.exp(r) - 1 - r) / r ** 2

    poly, _ = mp.chebyfit(g, [-a, a], deg + 1, error=True)
    cs = [float(c) for c in poly]          # highest degree first
    worst = 0
    for i in range(20001):
        x = -a + 2 * a * mp.mpf(i) / 20000
        q = mp.mpf(0)
        for c in cs:
            q = q * x + mp.mpf(c)
        worst = max(worst, abs((1 + x * (1 + x * q)) / mp.exp(x) - 1))
    return cs, worst


if __name__ == "__main__":
    cs, worst = fit()
    for c in cs:
        print(repr(c))
    print("max relative error", mp.nstr(worst, 4))
