"""Coefficients of the polynomial in exp2_core (rkc_device.h).

After the reduction y = n + f, n = round(y), |f| <= 1/2 (exact in double),
2^f = 1 + f (L + f q(f)) with L = ln 2 rounded to double and q a degree-9
Chebyshev fit (near minimax) of (2^f - 1 - f ln 2)/f^2 on [-1/2, 1/2],
computed in 50-digit arithmetic and rounded to double.  The relative error of
1 + f (L + f q(f)) with the rounded L and coefficients is printed (below
3e-17; L's rounding contributes at most |f| |L - ln 2| < 1.2e-17).
Run: python fit_exp_poly.py
"""
import mpmath as mp


def fit(deg=9, dps=50):
    mp.mp.dps = dps
    a = mp.mpf(1) / 2
    L = mp.mpf(float(mp.log(2)))

    def g(f):
        if abs(f) < mp.mpf("1e-30"):
            return mp.log(2) ** 2 / 2
        return (mp.power(2, f) - 1 - mp.log(2) * f) / f ** 2

    poly, _ = mp.chebyfit(g, [-a, a], deg + 1, error=True)
    cs = [float(c) for c in poly]          # highest degree first
    worst = 0
    for i in range(20001):
        x = -a + 2 * a * mp.mpf(i) / 20000
        q = mp.mpf(0)
        for c in cs:
            q = q * x + mp.mpf(c)
        worst = max(worst, abs((1 + x * (L + x * q)) / mp.power(2, x) - 1))
    return cs, float(L), worst


if __name__ == "__main__":
    cs, L, worst = fit()
    for c in cs:
        print(repr(c))
    print("L", repr(L))
    print("max relative error", mp.nstr(worst, 4))
