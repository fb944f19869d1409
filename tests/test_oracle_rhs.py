"""Pins of the oracle's source term f(y) (Sec. 2.2, Eqs. E:mass, E:spec-rate,
E:rxn-rate, E:rxn-const, E:energy) against closed forms and exact invariants."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O
from paper_1309_2710_amd import synth
from paper_1309_2710_amd.synth import ATM, R_J, R_ERG
from tests import mechs


def test_first_order_closed_form():
    # A -> B with k = A exactly (beta = 0, Ea = 0): dY_A/dt = -k Y_A, dT/dt = 0.
    m = mechs.a_to_b(k=2.5e6)
    M = O.Model(m)
    f = M.rhs([1234.0], [ATM], [[0.3, 0.7]])[0]
    assert f[0] == 0.0
    assert f[1] == pytest.approx(-2.5e6 * 0.3, rel=1e-15)
    assert f[2] == pytest.approx(+2.5e6 * 0.3, rel=1e-15)


def test_arrhenius_temperature_dependence():
    # k = A T^beta exp(-Ea/(R T)); with Ea = R T ln 2 at T = 1000 the exponential is 1/2,
    # and beta = 1 multiplies by T.
    T = 1000.0
    m = mechs.tiny([10.0, 10.0], [([0], [1], 1e3, 1.0, R_J * T * math.log(2.0))])
    f = O.Model(m).rhs([T], [ATM], [[1.0, 0.0]])[0]
    assert f[1] == pytest.approx(-1e3 * T * 0.5, rel=1e-14)


def test_bimolecular_rate_uses_ideal_gas_density():
    # 2A -> B: Omega = k C_A^2, C_A = rho Y_A / W_A, rho = P W / (R T) for pure A.
    W, T, P, k = 28.0, 1500.0, 2 * ATM, 3e13
    m = mechs.tiny([W, 2 * W], [([0, 0], [1], k, 0.0, 0.0)])
    f = O.Model(m).rhs([T], [P], [[1.0, 0.0]])[0]
    rho = P * 10.0 * W / (R_ERG * T)          # g/cm^3
    C = rho / W                                # mol/cm^3
    Omega = k * C * C
    assert f[1] == pytest.approx(-2.0 * W * Omega / rho, rel=1e-14)
    assert f[2] == pytest.approx(+2.0 * W * Omega / rho, rel=1e-14)


def test_energy_equation_closed_form():
    # A -> B with constant Cp/R = a1 and H/R = a1 T + a6: dT/dt = -(H_B - H_A) Omega / (rho cp)
    W, T, k = 20.0, 1200.0, 1e5
    nA = np.array([3.0, 0, 0, 0, 0, -1000.0, 0])
    nB = np.array([4.0, 0, 0, 0, 0, -9000.0, 0])
    m = mechs.tiny([W, W], [([0], [1], k, 0.0, 0.0)], nasa=[nA, nB])
    Y = np.array([0.4, 0.6])
    f = O.Model(m).rhs([T], [ATM], [Y])[0]
    rho = ATM * 10.0 * W / (R_ERG * T)
    Omega = k * rho * Y[0] / W
    HA = R_J * (3.0 * T - 1000.0)
    HB = R_J * (4.0 * T - 9000.0)
    cp = (Y[0] * 3.0 + Y[1] * 4.0) * R_J / W
    assert f[0] == pytest.approx(-(HB - HA) * Omega / (rho * cp), rel=1e-13)


def test_nasa_range_switch_at_T_mid():
    # high range iff T >= T_mid: give the two ranges different constant Cp and check
    # which one the energy equation used through dT/dt's denominator.
    W, k = 20.0, 1e5
    lo = np.array([3.0, 0, 0, 0, 0, 0.0, 0])
    hi = np.array([5.0, 0, 0, 0, 0, 0.0, 0])
    nB = np.array([3.0, 0, 0, 0, 0, -5000.0, 0])
    m = mechs.tiny([W, W], [([0], [1], k, 0.0, 0.0)], nasa=[(lo, hi), (nB, nB)])
    M = O.Model(m)
    for T, a1A in [(999.999, 3.0), (1000.0, 5.0), (1000.001, 5.0)]:
        f = M.rhs([T], [ATM], [[1.0, 0.0]])[0]
        rho = ATM * 10.0 * W / (R_ERG * T)
        Omega = k * rho / W
        HA = R_J * a1A * T
        HB = R_J * (3.0 * T - 5000.0)
        cp = a1A * R_J / W
        assert f[0] == pytest.approx(-(HB - HA) * Omega / (rho * cp), rel=1e-12)


def _enthalpy_mass(m, T, Y):
    out = 0.0
    for i in range(m["n_species"]):
        a = m["nasa_high"][i] if T >= m["T_mid"][i] else m["nasa_low"][i]
        h = a[0] + a[1] * T / 2 + a[2] * T**2 / 3 + a[3] * T**3 / 4 + a[4] * T**4 / 5 + a[5] / T
        out += Y[i] * R_J * T * h / m["W"][i]
    return out


def _cp_mass(m, T, Y):
    out = 0.0
    for i in range(m["n_species"]):
        a = m["nasa_high"][i] if T >= m["T_mid"][i] else m["nasa_low"][i]
        out += Y[i] * R_J * (a[0] + a[1] * T + a[2] * T**2 + a[3] * T**3 + a[4] * T**4) / m["W"][i]
    return out


@pytest.mark.parametrize("cfg", ["c1", "c2", "c3", "c4", "c3p"])
def test_conservation_invariants(cfg):
    """Mass: sum_i dY_i/dt = 0.  Elements: sum_i n_ei/W_i dY_i/dt = 0.
    Adiabatic constant pressure: sum_i h_i dY_i/dt + cp dT/dt = 0 (exact identity
    from E:mass and E:energy)."""
    m = synth.config_mechanism(cfg)
    M = O.Model(m)
    st = synth.config_states(cfg, 32)
    f = M.rhs(st["T"], st["P"], st["Y"])
    comp = m["comp"].astype(float)
    for c in range(32):
        Ydot = f[c, 1:]
        scale = np.abs(Ydot).sum()
        assert abs(Ydot.sum()) <= 1e-13 * scale
        for e in range(comp.shape[1]):
            terms = comp[:, e] / m["W"] * Ydot
            assert abs(terms.sum()) <= 1e-13 * np.abs(terms).sum() + 1e-300
        T = st["T"][c]
        hs = np.array([_enthalpy_mass({**m, "n_species": 1, "nasa_high": m["nasa_high"][i:i + 1],
                                       "nasa_low": m["nasa_low"][i:i + 1],
                                       "T_mid": m["T_mid"][i:i + 1], "W": m["W"][i:i + 1]},
                                      T, [1.0]) for i in range(m["n_species"])])
        cp = _cp_mass(m, T, st["Y"][c])
        terms = np.concatenate([hs * Ydot, [cp * f[c, 0]]])
        assert abs(terms.sum()) <= 1e-12 * np.abs(terms).sum()


def test_sign_and_index_mistakes_would_be_caught():
    """Guard for the invariant test itself: a plausible bug (dropping one term of
    E:spec-rate) breaks mass conservation by far more than the tolerance."""
    m = synth.config_mechanism("c1")
    M = O.Model(m)
    st = synth.config_states("c1", 8)
    f = M.rhs(st["T"], st["P"], st["Y"])
    bad = f[:, 1:].copy()
    bad[:, 0] *= 0.999
    assert np.any(np.abs(bad.sum(1)) > 1e-10 * np.abs(bad).sum(1))


# --- rounding-level cross-check against a 50-digit evaluation --------------
# (an extra check of accumulated rounding; the pins above are the closed forms
# and invariants)

def _rhs_mp(m, T, P, Y):
    mp.mp.dps = 50
    nS, nR = m["n_species"], m["n_reactions"]
    T = mp.mpf(T); Y = [mp.mpf(float(y)) for y in Y]
    W = [mp.mpf(float(w)) for w in m["W"]]
    R = mp.mpf(R_J); Rerg = mp.mpf(R_ERG)
    rho = mp.mpf(P) * 10 / (Rerg * T * sum(Y[i] / W[i] for i in range(nS)))
    C = [rho * Y[i] / W[i] for i in range(nS)]
    omega = [mp.mpf(0)] * nS
    for j in range(nR):
        k = mp.mpf(float(m["A"][j])) * T ** mp.mpf(float(m["beta"][j])) * mp.exp(
            -mp.mpf(float(m["Ea"][j])) / (R * T))
        Om = k
        for s in m["reac"][j]:
            if s >= 0:
                Om *= C[s]
        for s in m["reac"][j]:
            if s >= 0:
                omega[s] -= Om
        for s in m["prod"][j]:
            if s >= 0:
                omega[s] += Om
    f = [None] * (nS + 1)
    cp = mp.mpf(0); sh = mp.mpf(0)
    for i in range(nS):
        a = m["nasa_high"][i] if float(T) >= m["T_mid"][i] else m["nasa_low"][i]
        a = [mp.mpf(float(x)) for x in a]
        cpR = a[0] + a[1] * T + a[2] * T**2 + a[3] * T**3 + a[4] * T**4
        hRT = a[0] + a[1] * T / 2 + a[2] * T**2 / 3 + a[3] * T**3 / 4 + a[4] * T**4 / 5 + a[5] / T
        cp += Y[i] * R * cpR / W[i]
        sh += R * T * hRT * omega[i]
        f[1 + i] = W[i] * omega[i] / rho
    f[0] = -sh / (rho * cp)
    return f


@pytest.mark.parametrize("cfg,n", [("c1", 4), ("c2", 3)])
def test_rhs_matches_50_digit_evaluation(cfg, n):
    m = synth.config_mechanism(cfg)
    M = O.Model(m)
    st = synth.config_states(cfg, n)
    f = M.rhs(st["T"], st["P"], st["Y"])
    for c in range(n):
        ref = _rhs_mp(m, st["T"][c], st["P"][c], st["Y"][c])
        scale = max(abs(float(x)) for x in ref[1:])
        for i in range(m["n_species"] + 1):
            tol = 1e-12 * (abs(float(ref[0])) if i == 0 else scale) + 1e-300
            assert abs(f[c, i] - float(ref[i])) <= max(tol, 1e-13 * abs(float(ref[i])))
