"""Pins of the oracle's step control (Sec. 2.3 and 2.4): initial step, stage
count, spectral-radius schedule, step-size controllers and the power method,
from the per-attempt trace of orc_cell_trace.

Each pin rests on something other than the oracle's own code:
  - closed forms on A -> B at constant temperature (f is linear, J has the
    single nonzero eigenvalue -k), for the initial step of Sec. 2.4 and for
    the state after every step (the RKC stability polynomial in its cosh form);
  - the order of the local error estimates (h^3 for RKC's, h^5 for the RKCK
    embedded difference): a controller whose exponents match the order drives
    the error of the next step to S^(p+1) on a smooth problem (0.8^3 = 0.512,
    0.9^5 = 0.59049); a wrong exponent or safety factor lands elsewhere;
  - plain power iteration on the explicit Jacobian of linear networks, for
    the estimate and the iteration at which the 1 % test stops it;
  - the rules the paper prints explicitly: growth and shrink limits, the
    rejection factors, every 25 steps or after a rejection, the first RKCK
    trial step equal to the global step.
"""
import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O
from paper_1309_2710_amd.synth import ATM
from tests import mechs

U = 2.0 ** -53


def _R(s, z, dps=50):
    """RKC stability polynomial a_s + b_s T_s(w0 + w1 z) (Sec. 2.4) from the
    closed forms T_j(cosh t) = cosh(j t)."""
    mp.mp.dps = dps
    w0 = 1 + mp.mpf(2) / 13 / (s * s)
    th = mp.acosh(w0)
    sh, ch = mp.sinh(th), mp.cosh(th)
    Ts = mp.cosh(s * th)
    Tp = s * mp.sinh(s * th) / sh
    Tpp = s * (s * mp.cosh(s * th) * sh - mp.sinh(s * th) * ch) / sh ** 3
    w1 = Tp / Tpp
    bs = Tpp / Tp ** 2
    return (1 - bs * Ts) + bs * mp.chebyt(s, w0 + w1 * mp.mpf(z))


# ---------------------------------------------------------------- RKC ----


@pytest.mark.parametrize("k,dt", [(1e5, 1e-3), (1e3, 1e-5), (3e7, 1e-6)])
def test_initial_step_closed_form(k, dt):
    """A -> B: f(y) = (0, -k Y_A, k Y_A), so sigma = 1.2 k (the power method
    starts on the eigenvector f0), Delta_0 = dt0 (f(y0 + dt0 f0) - f0) =
    dt0^2 k^2 Y_A (0, 1, -1) with dt0 = min(1/sigma, dt), and the first
    trial step is 0.1 dt0 / sqrt(||Delta_0||_rms) with weights from y0."""
    rtol, atol = 1e-6, 1e-10
    y0 = np.array([1300.0, 0.6, 0.4])
    M = O.Model(mechs.a_to_b(k=k))
    _, cnt, st = M.trace(y0, ATM, dt, rtol, atol)
    sigma = 1.2 * k
    assert st["sigma"][0] == pytest.approx(sigma, rel=1e-9)
    assert st["new_sigma"][0]
    dt0 = min(1.0 / sigma, dt)
    d = dt0 * dt0 * k * k * y0[1]
    w = atol + rtol * np.abs(y0)
    e0 = np.sqrt(((d / w[1]) ** 2 + (d / w[2]) ** 2) / 3.0)
    h1 = min(max(0.1 * dt0 / np.sqrt(e0), 10 * U * dt), dt)
    assert st["h"][0] == pytest.approx(h1, rel=1e-9)
    assert st["t"][0] == 0.0


@pytest.mark.parametrize("YA,dt", [(0.6, 1e-3), (0.6, 2e-8), (0.05, 1e-3)])
def test_initial_step_closed_form_nonlinear(YA, dt):
    """2 A -> 2 B with equal molar masses and thermo keeps rho and T fixed and
    gives f_A = -a Y_A^2, a = 2 k rho / W: the Jacobian's only nonzero
    eigenvalue is -2 a Y_A (eigenvector f0), and the tentative step enters
    the first step nonlinearly, Delta_0,A = -a dt0^2 f0_A (2 Y_A + dt0 f0_A)."""
    from paper_1309_2710_amd.synth import R_ERG
    k, W, T, rtol, atol = 1e12, 10.0, 1300.0, 1e-6, 1e-10
    M = O.Model(mechs.tiny([W, W], [([0, 0], [1, 1], k, 0.0, 0.0)]))
    y0 = np.array([T, YA, 1.0 - YA])
    _, cnt, st = M.trace(y0, ATM, dt, rtol, atol)
    a = 2.0 * k * (ATM * 10.0 * W / (R_ERG * T)) / W
    # the power method's difference quotients carry the curvature of f over
    # the perturbation sqrt(u) |y| (relative 1e-5 to 1e-4 here)
    assert st["sigma"][0] == pytest.approx(1.2 * 2.0 * a * YA, rel=3e-4)
    sig = st["sigma"][0]
    dt0 = min(1.0 / sig, dt)
    f0 = -a * YA * YA
    dA = dt0 * (-a * (YA + dt0 * f0) ** 2 - f0)
    w = atol + rtol * np.abs(y0)
    e0 = np.sqrt(((dA / w[1]) ** 2 + (dA / w[2]) ** 2) / 3.0)
    h1 = min(max(0.1 * dt0 / np.sqrt(e0), 10 * U * dt), dt)
    assert st["h"][0] == pytest.approx(h1, rel=1e-12)


def test_every_step_multiplies_by_the_stability_polynomial():
    """A -> B with k dt = 1e5: each accepted step maps Y_A to R_s(-k h) Y_A for
    its own (h, s); the run reaches stage counts above 128 (up to 262).  Also
    the whole product while Y_A is representable.  The double recurrences
    of the coefficients and stages lose accuracy like s^2 (measured worst
    relative deviation 2e-9 (s/1000)^2, 1.5e-10 at s = 268); a dropped term,
    a wrong coefficient or a step of the wrong size is off by O(k h)."""
    k, dt, rtol, atol = 1e9, 1e-4, 1e-6, 1e-10
    y0 = np.array([1300.0, 0.6, 0.4])
    M = O.Model(mechs.a_to_b(k=k))
    y, cnt, st = M.trace(y0, ATM, dt, rtol, atol)
    assert cnt["status"] == O.OK
    acc = st["accepted"]
    assert st["s"].max() > 128
    prev = y0[1]
    prod, prod_tol = mp.mpf(y0[1]), 0.0
    n_checked = 0
    for i in np.nonzero(acc)[0]:
        s, h, ya = int(st["s"][i]), st["h"][i], st["y"][i, 1]
        R = _R(s, -k * h)
        tol = 1e-13 + 5e-9 * (s / 1000.0) ** 2
        if abs(prev) > 1e-280:
            assert abs(ya - float(R) * prev) <= tol * abs(prev), (i, s, h, ya, prev)
            prod *= R
            prod_tol += tol * abs(float(prod / R))
            assert abs(ya - float(prod)) <= prod_tol + 1e-300, (i, ya, float(prod))
            n_checked += 1
        prev = ya
    assert n_checked > 50
    # the temperature stays put (identical thermo; the stage combinations of
    # the constant value round by a few ulps), Y_A + Y_B is invariant
    assert np.all(np.abs(st["y"][acc, 0] - 1300.0) <= 1e-12 * 1300.0)
    assert abs(y[1] + y[2] - 1.0) <= 1e-12


@pytest.mark.parametrize("k,dt,rtol,atol", [(1e5, 1e-3, 1e-6, 1e-10), (1e9, 1e-5, 1e-6, 1e-10),
                                            (1e4, 1e-2, 1e-5, 1e-3)])
def test_error_estimate_closed_form(k, dt, rtol, atol):
    """Sec. 2.4, E:rmsE on A -> B, where f = (0, -k Y_A, k Y_A): for every
    accepted step, Delta = 4/5 (y_n - y_{n+1}) + 2/5 h (f_n + f_{n+1}) weighted
    by A + R max(|y_n|, |y_{n+1}|), RMS over the N = 3 components."""
    y0 = np.array([1300.0, 0.6, 0.4])
    M = O.Model(mechs.a_to_b(k=k))
    _, cnt, st = M.trace(y0, ATM, dt, rtol, atol)
    f = lambda y: np.array([0.0, -k * y[1], k * y[1]])
    yn = y0
    n = 0
    for i in np.nonzero(st["accepted"])[0]:
        y1 = st["y"][i]
        h = st["h"][i]
        d = 0.8 * (yn - y1) + 0.4 * h * (f(yn) + f(y1))
        w = atol + rtol * np.maximum(np.abs(yn), np.abs(y1))
        err = np.sqrt(np.mean((d / w) ** 2))
        if err > 1e-3:
            assert st["err"][i] == pytest.approx(err, rel=1e-6), (i, st["err"][i], err)
            n += 1
        yn = y1
    assert n > 20


def test_stage_count_keeps_every_step_stable():
    """Stage count of Sec. 2.4 with the floor reading: s = 1 + floor(sqrt(1 +
    1.54 h sigma)); with sigma = 1.2 k every attempted step is stable on A -> B
    (|R_s(-k h)| <= 1), and a cap s_max takes the largest step it keeps
    stable, ((s_max - 1)^2 - 1) / (1.54 sigma)."""
    k = 1e9
    M = O.Model(mechs.a_to_b(k=k))
    for s_max in (1000, 20):
        _, cnt, st = M.trace([1300.0, 0.6, 0.4], ATM, 1e-5, 1e-6, 1e-10, s_max=s_max)
        assert cnt["status"] == O.OK
        for h, s, sg in zip(st["h"], st["s"], st["sigma"]):
            s = int(s)
            assert 2 <= s <= s_max
            assert abs(float(_R(s, -k * h))) <= 1.0 + 1e-12
            if s < s_max:
                assert s == 1 + int(np.floor(np.sqrt(1.0 + 1.54 * h * sg)))
            else:
                assert h <= ((s_max - 1) ** 2 - 1) / (1.54 * sg) * (1 + 1e-15)
        if s_max == 20:
            capped = st["s"] == 20
            assert capped.sum() > 10
            hc = st["h"][capped]
            assert np.allclose(hc, ((20 - 1) ** 2 - 1) / (1.54 * st["sigma"][capped]),
                               rtol=1e-15, atol=0)


def _smooth_accepted_errors(st, rtol, atol, first=8):
    """Errors of accepted steps in the regime where the error constant is
    smooth: the two previous attempts accepted, no growth clamp, not the last
    step, two stages throughout (s changes the constant) and Y_A large enough
    that rtol |y| dominates the weight."""
    acc, h, err, s, ya = st["accepted"], st["h"], st["err"], st["s"], st["y"][:, 1]
    out = []
    for i in range(first, len(acc) - 1):
        if (acc[i] and acc[i - 1] and acc[i - 2] and h[i] < 9.99 * h[i - 1] and acc[i + 1]
                and s[i] == s[i - 1] == s[i - 2] == 2 and ya[i] > 1e3 * atol / rtol):
            out.append(err[i])
    return np.array(out)


@pytest.mark.parametrize("k,dt,rtol,atol", [(1e5, 1e-3, 1e-6, 1e-10), (2e6, 1e-4, 1e-8, 1e-12),
                                            (1e4, 1e-2, 1e-5, 1e-9)])
def test_rkc_controller_drives_error_to_its_target(k, dt, rtol, atol):
    """The local error estimate of RKC is O(h^3) (second order, Sec. 2.4), so on
    a smooth problem the controller's exponents 1/(p + 1) = 1/3 (and 2/3 in
    the predictive form) with safety factor 0.8 drive the next error to
    0.8^3 = 0.512.  An exponent of 1/2, or a factor of 0.9 (0.729), misses."""
    M = O.Model(mechs.a_to_b(k=k))
    _, cnt, st = M.trace([1300.0, 0.6, 0.4], ATM, dt, rtol, atol)
    e = _smooth_accepted_errors(st, rtol, atol)
    assert len(e) > 20
    # measured: 0.51200 to 0.51335 on these runs
    assert np.all(np.abs(e - 0.512) <= 0.005), (e.min(), e.max())


def test_rkc_growth_limit_and_rejection_rule():
    """Growth limited to 10x and shrink to 0.1x per step (Sec. 2.4); after a
    rejection the step is redone with the factor 0.8 / ||Delta||^(1/(p+1)),
    p = 2, that the paper prints for rejected steps, and the spectral radius
    is re-estimated.  Runs on the autocatalytic A + B -> 2 B (sigmoidal
    growth, which the predictive controller underestimates)."""
    saw_rej = saw_clamp = saw_np = 0
    for (k, yb, dt) in [(1e12, 1e-6, 1e-4), (1e13, 1e-8, 1e-4), (1e11, 1e-4, 1e-3)]:
        m = mechs.tiny([10.0, 10.0], [([0, 1], [1, 1], k, 0.0, 0.0)])
        _, cnt, st = O.Model(m).trace([1300.0, 1.0 - yb, yb], ATM, dt, 1e-6, 1e-10)
        assert cnt["status"] == O.OK
        acc, h, err = st["accepted"], st["h"], st["err"]
        r = h[1:] / h[:-1]
        assert np.all(r <= 10.0 * (1 + 1e-15)) and np.all(r >= 0.1 * (1 - 1e-15))
        saw_clamp += int(np.sum(np.abs(r - 10.0) <= 1e-14 * 10))
        for i in np.nonzero(~acc)[0]:
            saw_rej += 1
            assert i + 1 < len(acc)
            fac = max(0.1, 0.8 * err[i] ** (-1.0 / 3.0))
            assert h[i + 1] == pytest.approx(h[i] * fac, rel=1e-14)
            assert st["t"][i + 1] == st["t"][i]
            assert st["new_sigma"][i + 1]
            # the accepted retry has no error history to extrapolate: its
            # successor uses the same non-predictive factor (clamped)
            j = i + 1
            if acc[j] and j + 1 < len(acc) and st["t"][j + 1] + h[j + 1] != dt:
                fac = min(10.0, max(0.1, 0.8 * err[j] ** (-1.0 / 3.0)))
                assert h[j + 1] == pytest.approx(h[j] * fac, rel=1e-14)
                saw_np += 1
    assert saw_rej >= 5 and saw_clamp >= 3 and saw_np >= 5


@pytest.mark.parametrize("mech,dt", [("a_to_b", 1e-3), ("autocat", 1e-4), ("nonlinear3", 1e-5)])
def test_spectral_radius_every_25_steps_or_after_rejection(mech, dt):
    """Sec. 2.4: the spectral radius is estimated at the start, every 25
    (accepted) steps, and after every rejection."""
    m = {"a_to_b": lambda: mechs.a_to_b(k=1e5),
         "autocat": lambda: mechs.tiny([10.0, 10.0], [([0, 1], [1, 1], 1e12, 0.0, 0.0)]),
         "nonlinear3": mechs.nonlinear3}[mech]()
    N = m["n_species"] + 1
    y0 = np.concatenate([[1300.0], np.full(N - 1, 1.0 / (N - 1))])
    if mech == "autocat":
        y0 = np.array([1300.0, 1 - 1e-6, 1e-6])
    _, cnt, st = O.Model(m).trace(y0, ATM, dt, 1e-6, 1e-10)
    acc, ns = st["accepted"], st["new_sigma"]
    since = 0
    for i in range(len(acc)):
        expect = i == 0 or (not acc[i - 1]) or since >= 25
        assert bool(ns[i]) == expect, (i, since)
        if ns[i]:
            since = 0
        if acc[i]:
            since += 1
    assert cnt["n_sigma"] == int(ns.sum())


# ------------------------------------------------------- power method ----


def _power_iteration(J, v0, maxit=50):
    """Plain power iteration with the 1 % stopping test: returns (1.2 sigma_k,
    k, relative changes)."""
    v = v0 / np.linalg.norm(v0)
    prev, ch = None, []
    for it in range(1, maxit + 1):
        g = J @ v
        sig = np.linalg.norm(g)
        if prev is not None:
            ch.append(abs(sig - prev) / sig)
        if it >= 2 and abs(sig - prev) <= 0.01 * sig:
            return 1.2 * sig, it, ch
        if it == maxit:
            return 1.2 * sig, it, ch
        v = g / sig
        prev = sig


def _chain_J(ks, cycle=False):
    n = len(ks) + (0 if cycle else 1)
    J = np.zeros((n + 1, n + 1))   # row/column 0: temperature
    for j, k in enumerate(ks):
        a, b = 1 + j, 1 + (j + 1) % n
        J[a, a] -= k
        J[b, a] += k
    return J


@pytest.mark.parametrize("ks,cycle", [((1e6, 1e3), False), ((1e6, 5e5), False),
                                      ((1e6, 9e5), False), ((1e6, 1.1e6), False),
                                      ((3e5, 1e6), False), ((1e6, 4e6, 9e6), True),
                                      ((3.751e6, 2.417e5, 4.025e6), True),
                                      ((4.598e6, 1.335e5, 4.477e6), True)])
def test_power_method_is_power_iteration_on_linear_networks(ks, cycle):
    """On a linear network at constant T the difference quotients are J v, so
    the nonlinear power method (Sec. 2.4) is power iteration from f(y0): same
    estimate (times the safety factor 1.2), stopped at the first k >= 2 whose
    estimate changed by at most 1 %, or after 50 iterations (the last two
    cycles never pass the test: changes stay above 1.9 %)."""
    n = len(ks) + (0 if cycle else 1)
    rxn = [([j], [(j + 1) % n], k, 0.0, 0.0) for j, k in enumerate(ks)]
    M = O.Model(mechs.tiny([10.0] * n, rxn))
    y = np.concatenate([[1300.0], np.linspace(0.5, 0.2, n) / np.linspace(0.5, 0.2, n).sum()])
    J = _chain_J(ks, cycle)
    sig_p, it_p, ch = _power_iteration(J, J @ y)
    # the decision at each iteration is far from the 1 % threshold
    assert all(abs(c - 0.01) > 1e-6 for c in ch)
    sig, it = M.sigma(y, ATM)
    assert it == it_p
    assert sig == pytest.approx(sig_p, rel=1e-9)
    if ks in ((3.751e6, 2.417e5, 4.025e6), (4.598e6, 1.335e5, 4.477e6)):
        assert it == 50 and min(ch) > 0.015


@pytest.mark.parametrize("ks", [(1e6, 5e5), (1e6, 9e5), (3e5, 1e6)])
def test_power_method_is_warm_started(ks):
    """Sec. 2.4: the computed eigenvector is kept as the next starting guess.
    On a linear chain J is constant, so every re-estimate starts on the
    dominant direction found before and stops at its second iteration: the
    iterations of a run are those of the first estimate plus two per later
    estimate."""
    M = O.Model(mechs.tiny([10.0] * 3, [([0], [1], ks[0], 0.0, 0.0),
                                        ([1], [2], ks[1], 0.0, 0.0)]))
    y0 = np.array([1300.0, 0.5, 0.3, 0.2])
    _, cnt, st = M.trace(y0, ATM, 2e-4)
    J = _chain_J(ks)
    _, first, _ = _power_iteration(J, J @ y0)
    assert cnt["n_sigma"] > 10
    assert cnt["n_power_iter"] == first + 2 * (cnt["n_sigma"] - 1)


# --------------------------------------------------------------- RKCK ----


def test_rkck_first_trial_step_is_the_global_step_and_rejection_rule():
    """Sec. 2.3: the integration starts with the whole global step (the
    integrator restarts every call), shrinks with S |Delta_0/Delta|^(1/4)
    (S = 0.9) but at most 10x, grows with S |Delta_0/Delta|^(1/5) but at most
    5x (that bound is never reached on these runs: it needs an accepted
    error below 1.9e-4 right after an accepted step)."""
    k = 1e5
    M = O.Model(mechs.a_to_b(k=k))
    for dt in (1e-4, 1e-6):
        _, cnt, st = M.trace([1300.0, 0.6, 0.4], ATM, dt, 1e-10, method=O.RKCK)
        assert cnt["status"] == O.OK
        h, err, acc = st["h"], st["err"], st["accepted"]
        assert h[0] == dt and st["t"][0] == 0.0
        r = h[1:] / h[:-1]
        assert np.all(r <= 5.0 * (1 + 1e-15)) and np.all(r >= 0.1 * (1 - 1e-15))
        for i in np.nonzero(~acc)[0]:
            assert h[i + 1] == pytest.approx(h[i] * max(0.1, 0.9 * err[i] ** -0.25), rel=1e-14)
        assert st["t"][-1] + h[-1] == dt


def _rkck_polys():
    """Linear stability polynomials of the fifth- and fourth-order solutions
    of Table 1 (from the golden file, exact rationals)."""
    from tests.test_oracle_rkc import _stab_coeffs, _table1
    _, _, c, cs = _table1()
    return _stab_coeffs(c), _stab_coeffs(cs)


@pytest.mark.parametrize("k,rtol", [(1e5, 1e-10), (1e7, 1e-8)])
def test_rkck_error_measure_closed_form(k, rtol):
    """Sec. 2.3 on A -> B: Delta = y_{n+1} - y*_{n+1} is Y_A (P5(z) - P4(z))
    (0, 1, -1) with z = -k h and P5, P4 the Table 1 stability polynomials;
    Delta_0 = eps (|y_n| + |h f(y_n)| + 1e-30); the step's measure is the
    largest |Delta_i / Delta_0,i|.  Runs down to Y_A ~ 1e-35, where the
    1e-30 in Delta_0 matters."""
    from fractions import Fraction
    P5, P4 = _rkck_polys()
    D = [float(a - b) for a, b in zip(P5, P4)]
    y0 = np.array([1300.0, 0.6, 0.4])
    M = O.Model(mechs.a_to_b(k=k))
    _, cnt, st = M.trace(y0, ATM, 80.0 / k, rtol, method=O.RKCK)
    yn, n, small = y0, 0, 0
    for i in range(len(st["h"])):
        h = st["h"][i]
        z = -k * h
        dA = yn[1] * sum(d * z ** q for q, d in enumerate(D))
        hf = np.array([0.0, h * k * yn[1], h * k * yn[1]])
        d0 = rtol * (np.abs(yn) + hf + 1e-30)
        e = max(abs(dA / d0[1]), abs(dA / d0[2]))
        assert st["err"][i] == pytest.approx(e, rel=1e-6, abs=1e-12), (i, st["err"][i], e)
        n += 1
        small += yn[1] < 1e-28
        if st["accepted"][i]:
            yn = st["y"][i]
    assert n > 100 and small > 5


@pytest.mark.parametrize("k,rtol", [(1e5, 1e-10), (1e7, 1e-8), (3e3, 1e-12)])
def test_rkck_controller_drives_error_to_its_target(k, rtol):
    """The embedded error estimate is O(h^5) (Table 1: fifth- minus fourth-order
    solution), so the accepted-step rule 0.9 |Delta_0/Delta|^(1/5) drives the
    next error to 0.9^5 = 0.59049 on a smooth problem: here after the start
    transient and while Y_A is far above the delta = 1e-30 of Delta_0."""
    M = O.Model(mechs.a_to_b(k=k))
    _, cnt, st = M.trace([1300.0, 0.6, 0.4], ATM, 200.0 / k, rtol, method=O.RKCK)
    acc, h, err, ya = st["accepted"], st["h"], st["err"], st["y"][:, 1]
    e = np.array([err[i] for i in range(20, len(acc) - 1)
                  if acc[i] and acc[i - 1] and acc[i - 2] and h[i] < 4.99 * h[i - 1]
                  and ya[i] > 1e-25])
    assert len(e) > 100
    assert np.all(np.abs(e - 0.9 ** 5) <= 1e-4), (e.min(), e.max())
