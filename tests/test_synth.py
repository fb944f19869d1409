"""The seeded synthetic workload generator: determinism, exact element
balance, forward/reverse pair structure, the paper's Appendix A three-point
Arrhenius fit, thermodynamic consistency of each pair, and stated ranges."""
import math

import numpy as np
import pytest

from paper_1309_2710_amd import synth


def test_appendix_a_fit_reproduces_three_points_and_matches_linear_solve():
    rng = np.random.default_rng(5)
    for _ in range(20):
        T3 = tuple(sorted(rng.uniform(300, 3000, 3)))
        lnA, b, Ta = rng.uniform(5, 30), rng.uniform(-3, 3), rng.uniform(-5e3, 5e4)
        lnk = [lnA + b * math.log(T) - Ta / T for T in T3]
        fa, fb, fT = synth.fit_three_point(T3, lnk)
        M = np.array([[1.0, math.log(T), -1.0 / T] for T in T3])
        ref = np.linalg.solve(M, np.array(lnk))
        assert np.allclose([fa, fb, fT], ref, rtol=1e-6, atol=1e-6)
        assert np.allclose([fa, fb, fT], [lnA, b, Ta], rtol=1e-6, atol=1e-5)


@pytest.mark.parametrize("cfg", ["c1", "c2", "c3", "c4"])
def test_mechanism_structure(cfg):
    m = synth.config_mechanism(cfg)
    c = synth.CONFIGS[cfg]
    assert m["n_species"] == c["n_species"] and m["n_reactions"] == c["n_reactions"]
    comp = m["comp"]
    for j in range(m["n_reactions"]):
        r = [s for s in m["reac"][j] if s >= 0]
        p = [s for s in m["prod"][j] if s >= 0]
        assert 1 <= len(r) <= 3 and 1 <= len(p) <= 3
        assert (comp[r].sum(0) == comp[p].sum(0)).all()      # exact integer balance
    # reaction 2p+1 is the exact reverse of reaction 2p
    for p in range(m["n_reactions"] // 2):
        assert sorted(m["reac"][2 * p + 1]) == sorted(m["prod"][2 * p])
        assert sorted(m["prod"][2 * p + 1]) == sorted(m["reac"][2 * p])
    # forward draws follow the configured distributions
    lA = np.log10(m["A"][0::2])
    assert lA.min() >= 6.0 and lA.max() <= 14.0
    assert np.abs(m["beta"][0::2]).max() <= 2.0
    assert m["Ea"][0::2].min() >= 0.0 and m["Ea"][0::2].max() <= c["ea_max"]
    assert np.isfinite(m["A"]).all() and (m["A"] > 0).all()
    # molar cp within 20-60 J/(mol K) on 300-3500 K
    for T in np.linspace(300, 3500, 33):
        for i in range(m["n_species"]):
            a = m["nasa_high"][i] if T >= m["T_mid"][i] else m["nasa_low"][i]
            cp = synth.R_J * (a[0] + a[1] * T + a[2] * T**2 + a[3] * T**3 + a[4] * T**4)
            assert 20.0 - 1e-9 <= cp <= 60.0 + 1e-9 or comp[i].sum() == 1


@pytest.mark.parametrize("cfg", ["c1", "c3"])
def test_pairs_obey_equilibrium_at_fit_temperatures(cfg):
    """k_f / k_r = K_c exactly at the three fit temperatures (Appendix A)."""
    m = synth.config_mechanism(cfg)
    nS = m["n_species"]
    for T in m["T_fit"]:
        g = synth.gibbs_RT(m["nasa_low"], m["nasa_high"], m["T_mid"], T)
        for p in range(0, m["n_reactions"] // 2, 7):
            j = 2 * p
            d = np.zeros(nS)
            for s_ in m["reac"][j]:
                if s_ >= 0:
                    d[s_] -= 1
            for s_ in m["prod"][j]:
                if s_ >= 0:
                    d[s_] += 1
            lnkf = math.log(m["A"][j]) + m["beta"][j] * math.log(T) - m["Ea"][j] / (synth.R_J * T)
            lnkr = math.log(m["A"][j + 1]) + m["beta"][j + 1] * math.log(T) \
                - m["Ea"][j + 1] / (synth.R_J * T)
            assert lnkf - lnkr == pytest.approx(synth.ln_kc(d, g, T), abs=1e-6)


def test_stiffness_cap_respected():
    m = synth.config_mechanism("c3")
    c = synth.CONFIGS["c3"]
    T = np.linspace(*c["T_range"], 17)
    ms = (m["reac"] >= 0).sum(1)
    for j in range(m["n_reactions"]):
        lb = synth._ln_rate_bound(math.log(m["A"][j]), m["beta"][j], m["Ea"][j], ms[j], T,
                                  c["P_max"])
        assert lb.max() <= math.log(m["lambda_cap"]) + 1e-9


def test_generation_is_deterministic_and_states_normalised():
    a = synth.make_mechanism(9, 38, ["H", "O", "N"], 77, T_lo=950, T_hi=1600)
    b = synth.make_mechanism(9, 38, ["H", "O", "N"], 77, T_lo=950, T_hi=1600)
    for k in ("A", "beta", "Ea", "reac", "prod", "nasa_low", "nasa_high", "W"):
        assert np.array_equal(a[k], b[k])
    s1 = synth.config_states("c3", 100)
    s2 = synth.config_states("c3", 100)
    assert np.array_equal(s1["Y"], s2["Y"])
    assert np.abs(s1["Y"].sum(1) - 1).max() < 1e-15
    majors = synth.config_mechanism("c3")["major_species"]
    assert (s1["Y"][:, majors].sum(1) >= 0.9 - 1e-12).all()
    s4 = synth.config_states("c4", 2000)
    assert (np.abs(s4["T"] - 800) < 150).sum() + (np.abs(s4["T"] - 2400) < 150).sum() == 2000
    srt = synth.config_states("c2", 50, order="sorted")
    assert (np.diff(srt["T"]) >= 0).all()


def test_served_trace():
    tr = synth.c5_trace(200)
    assert len(tr) == 200
    t = np.array([r["t_arrival"] for r in tr])
    assert (np.diff(t) > 0).all() and 0.5 / 200 < t.mean() / np.arange(1, 201).mean() < 2 / 200
    n = np.array([r["n_cells"] for r in tr])
    assert n.min() >= 1024 and n.max() <= 65536
    assert {r["mech"][0] for r in tr} == {13, 53}
    assert {r["dt"] for r in tr} == {1e-6, 1e-5}
