"""The Appendix A converter (paper_1309_2710_amd.convert): reverse Arrhenius
parameters through k_f / K_c at three temperatures in closed form.

Pins: (i) where k_f / K_c is itself of Arrhenius form (constant heat
capacities: ln K_c is linear in ln T and 1/T) the fit reproduces it exactly,
with beta_r = beta_f - sum(dnu a1) and T_ar = T_af - sum(dnu a6) (and the
ln T and 1/T terms of the concentration-unit factor); (ii) at the three fit
temperatures ln k_r = ln k_f - ln K_c for reactions of a synthetic set; (iii)
the generator's pairs, drawn with the same closed form, are reproduced; (iv)
the oracle's source term of a converted A <=> B vanishes at the equilibrium
composition (detailed balance) at the fit temperatures; (v) structure."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1309_2710_amd import convert, synth
from tests import mechs

R_J = convert.R_J


def _const_cp_pair(dn_products=1):
    """A -> B (+ B when dn_products = 2) with constant-cp NASA-7 thermo."""
    lo = [np.array([3.5, 0, 0, 0, 0, -1200.0, 4.0]), np.array([2.8, 0, 0, 0, 0, 3000.0, 6.5])]
    prods = [1] if dn_products == 1 else [1, 1]
    m = mechs.tiny([20.0, 20.0 / dn_products], [([0], prods, 3.0e9, 0.7, 9.0e4)], nasa=lo)
    return m


@pytest.mark.parametrize("dn", [1, 2])
def test_exact_reverse_when_kf_over_kc_is_arrhenius(dn):
    m = _const_cp_pair(dn)
    Af, bf, Ef = m["A"][0], m["beta"][0], m["Ea"][0]
    a1 = m["nasa_low"][:, 0]
    a6 = m["nasa_low"][:, 5]
    a7 = m["nasa_low"][:, 6]
    d = np.array([-1.0, float(dn)])
    # G/RT = a1 (1 - ln T) + a6/T - a7;  ln K_c = -sum d G/RT + (sum d) ln(P_atm/(R T))
    s = d.sum()
    beta_r = bf - (d @ a1) + s
    Tar = Ef / R_J - (d @ a6)
    lnA_r = math.log(Af) + (d @ a1) - (d @ a7) - s * math.log(synth.ATM * 10.0 / synth.R_ERG)
    A_r, b_r, E_r = convert.reverse_parameters(m, 0, T_fit=(500.0, 1200.0, 3000.0))
    assert b_r == pytest.approx(beta_r, abs=1e-9)
    assert E_r / R_J == pytest.approx(Tar, rel=1e-11, abs=1e-7)
    assert math.log(A_r) == pytest.approx(lnA_r, abs=1e-8)
    # and so k_r = k_f / K_c at any temperature, not only at the fit points
    for T in (400.0, 900.0, 2000.0, 3500.0):
        g = synth.gibbs_RT(m["nasa_low"], m["nasa_high"], m["T_mid"], T)
        lnkf = math.log(Af) + bf * math.log(T) - Ef / (R_J * T)
        lnkr = math.log(A_r) + b_r * math.log(T) - E_r / (R_J * T)
        assert lnkr == pytest.approx(lnkf - synth.ln_kc(d, g, T), abs=1e-8)


def test_fit_points_of_a_synthetic_set():
    m = synth.config_mechanism("c2")
    fwd = {k: v for k, v in m.items()}
    T_fit = (800.0, 1300.0, 2100.0)
    for j in range(0, m["n_reactions"], 2):
        A_r, b_r, E_r = convert.reverse_parameters(fwd, j, T_fit)
        d = np.zeros(m["n_species"])
        for s_ in m["reac"][j]:
            if s_ >= 0:
                d[s_] -= 1
        for s_ in m["prod"][j]:
            if s_ >= 0:
                d[s_] += 1
        for T in T_fit:
            g = synth.gibbs_RT(m["nasa_low"], m["nasa_high"], m["T_mid"], T)
            lnkf = math.log(m["A"][j]) + m["beta"][j] * math.log(T) - m["Ea"][j] / (R_J * T)
            lnkr = math.log(A_r) + b_r * math.log(T) - E_r / (R_J * T)
            assert lnkr == pytest.approx(lnkf - synth.ln_kc(d, g, T), abs=1e-9)


def test_generator_pairs_reproduced():
    """The synthetic sets' reverse reactions were drawn with the same closed
    form at the set's fit temperatures: converting the forward halves gives
    them back."""
    m = synth.config_mechanism("c1")
    nR = m["n_reactions"]
    fwd_idx = np.arange(0, nR, 2)
    half = {k: m[k] for k in ("n_species", "W", "nasa_low", "nasa_high", "T_mid")}
    half.update(n_reactions=len(fwd_idx), reac=m["reac"][fwd_idx], prod=m["prod"][fwd_idx],
                A=m["A"][fwd_idx], beta=m["beta"][fwd_idx], Ea=m["Ea"][fwd_idx])
    conv = convert.to_irreversible(half, np.ones(len(fwd_idx), bool), T_fit=m["T_fit"])
    assert conv["n_reactions"] == nR
    assert np.array_equal(conv["reac"], m["reac"]) and np.array_equal(conv["prod"], m["prod"])
    np.testing.assert_allclose(conv["A"], m["A"], rtol=1e-12)
    np.testing.assert_allclose(conv["beta"], m["beta"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(conv["Ea"], m["Ea"], rtol=1e-12, atol=1e-6)


@pytest.mark.parametrize("T", [700.0, math.sqrt(700.0 * 2500.0), 2500.0])
def test_detailed_balance_at_the_fit_temperatures(T):
    """A <=> B with distinct thermo, converted with the default fit
    temperatures: at the equilibrium composition of T (C_B / C_A = K_c, equal
    molar masses so Y_B / Y_A = K_c) the oracle's dY/dt vanishes to rounding."""
    lo = [np.array([3.2, 1e-4, 0, 0, 0, -1500.0, 5.0]), np.array([3.6, 2e-4, 0, 0, 0, 800.0, 4.2])]
    m = mechs.tiny([25.0, 25.0], [([0], [1], 5.0e8, 0.3, 6.0e4)], nasa=lo)
    conv = convert.to_irreversible(m, [True])
    assert conv["n_reactions"] == 2 and conv["is_reverse"].tolist() == [False, True]
    g = synth.gibbs_RT(m["nasa_low"], m["nasa_high"], m["T_mid"], T)
    K = math.exp(synth.ln_kc(np.array([-1.0, 1.0]), g, T))
    Y = np.array([[1.0 / (1.0 + K), K / (1.0 + K)]])
    f = O.Model(conv).rhs(np.array([T]), np.array([synth.ATM]), Y)[0]
    kf = m["A"][0] * T ** m["beta"][0] * math.exp(-m["Ea"][0] / (R_J * T))
    scale = kf * Y[0, 0]   # one direction's rate of change of Y_A
    assert abs(f[1]) <= 1e-9 * scale and abs(f[2]) <= 1e-9 * scale


def test_structure_and_pressure_dependence():
    from tests.test_oracle_pdep import _pdep
    m = _pdep(mechs.a_b_c(1e6, 3e5), [2, 0], k0=[1e12, 0.0])
    conv = convert.to_irreversible(m, [True, False])
    assert conv["n_reactions"] == 3
    assert conv["source"].tolist() == [0, 0, 1] and conv["is_reverse"].tolist() == [False, True, False]
    assert conv["reac"][1].tolist() == m["prod"][0].tolist()
    assert conv["prod"][1].tolist() == m["reac"][0].tolist()
    assert conv["pdep"].tolist() == [2, 2, 0]
    assert conv["A0"][1] > 0 and conv["A"][2] == m["A"][1]
    with pytest.raises(ValueError):
        convert.to_irreversible(m, [True])
    with pytest.raises(ValueError):
        convert.to_irreversible(m, [True, False], T_fit=(1000.0, 900.0, 2000.0))
