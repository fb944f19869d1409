"""GPU parity of third-body and falloff reactions (Sec. 2.2, Chemkin forms):
source term and integration on the 53-species set with pressure-dependent
pairs against the oracle, and the closed forms the oracle is pinned to."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1309_2710_amd import synth
from paper_1309_2710_amd.synth import ATM, R_ERG
from tests import mechs
from tests import parity as PT
from tests.test_oracle_pdep import _pdep

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_1309_2710_amd import rkc
    rkc.lib()
    return rkc


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("G", [64, 32])
def test_rhs_parity_pressure_dependent_set(R, G):
    _say("pdep rhs c3p G", G)
    m = synth.config_mechanism("c3p")
    gm = R.Mechanism(m)
    st = synth.config_states("c3p", 257, seed=77)
    fg = R.rhs(gm, st["T"], st["P"], st["Y"], lanes_per_cell=G)
    fo = O.Model(m).rhs(st["T"], st["P"], st["Y"])
    scale = np.abs(fo[:, 1:]).max(axis=1, keepdims=True)
    eY = (np.abs(fg[:, 1:] - fo[:, 1:]) / scale).max()
    eT = (np.abs(fg[:, 0] - fo[:, 0]) / np.abs(fo[:, 0])).max()
    _say("max eY", eY, "eT", eT)
    assert eY <= 1e-12 and eT <= 1e-11


def test_integrate_parity_pressure_dependent_set(R):
    _say("pdep integrate c3p")
    m = synth.config_mechanism("c3p")
    c = synth.CONFIGS["c3p"]
    gm, om = R.Mechanism(m), O.Model(m)
    st = synth.config_states("c3p", 96)
    T, Y = st["T"].copy(), st["Y"].copy()
    out = R.integrate(gm, T, st["P"], Y, c["dt"], c["rtol"], c["atol"], counters=True)
    To, Yo, co = om.integrate(st["T"], st["P"], st["Y"], c["dt"], c["rtol"], c["atol"],
                              threads=16)
    assert (out["status"] == 0).all() and (co["status"] == 0).all()
    rep = PT.check(T, Y, out["counters"], To, Yo, co, c["rtol"], c["atol"], 1)
    _say(rep)


def _gpu_rate_A(R, m, T, P, Y, G=8):
    f = R.rhs(R.Mechanism(m), np.array([T]), np.array([P]), np.array([Y]), lanes_per_cell=G)[0]
    return -f[1] / Y[0]


def test_closed_forms_on_the_gpu(R):
    _say("pdep closed forms")
    W = 10.0
    # third body, unit efficiencies: [M] = P / (R T)
    k, T, P = 3.0e11, 1300.0, 2 * ATM
    m = _pdep(mechs.a_to_b(k, W), [1])
    assert _gpu_rate_A(R, m, T, P, [0.4, 0.6]) == pytest.approx(k * P * 10.0 / (R_ERG * T),
                                                                rel=1e-13)
    # Lindemann closed form
    kinf, k0, T = 2.0e5, 4.0e10, 1000.0
    m = _pdep(mechs.a_to_b(kinf, W), [2], k0=[k0])
    M = ATM * 10.0 / (R_ERG * T)
    Pr = k0 * M / kinf
    assert _gpu_rate_A(R, m, T, ATM, [0.5, 0.5]) == pytest.approx(kinf * Pr / (1 + Pr),
                                                                  rel=1e-13)
    # Troe at the centre of the falloff curve: F = F_cent = 1.25
    Fc = 1.25
    c = -0.4 - 0.67 * math.log10(Fc)
    Pr = 10.0 ** (-c)
    P = Pr * kinf / k0 * R_ERG * T / 10.0
    troe = _pdep(mechs.a_to_b(kinf, W), [3], k0=[k0],
                 troe=[[0.5, 1e300, 1e300, T * math.log(4.0)]])
    lind = _pdep(mechs.a_to_b(kinf, W), [2], k0=[k0])
    ratio = _gpu_rate_A(R, troe, T, P, [0.5, 0.5]) / _gpu_rate_A(R, lind, T, P, [0.5, 0.5])
    assert ratio == pytest.approx(Fc, rel=1e-12)


@pytest.mark.parametrize("troe", [[0.5, 1e-30, 1e30, 0.0], [0.3, 1e-30, 1e3, 1e30],
                                  [0.7, 1e30, 1e-30, 1e-30]])
def test_troe_sentinel_temperatures_against_oracle(R, troe):
    """Troe temperatures used as 'term off' sentinels (1e-30 and 1e30 K): the
    centre value's exponentials have arguments far beyond the exponential's
    int32 exponent range (-T/1e-30 is -1e33), where the result is exactly 0
    or 1; over 800-2400 K the source term must equal the oracle's.  Each case
    keeps one term alive: with all three off F_cent is 0 and its logarithm,
    hence the Troe factor, is undefined (the oracle gives NaN)."""
    _say("troe sentinels", troe)
    kinf, k0 = 2.0e5, 4.0e10
    m = _pdep(mechs.a_to_b(kinf, 10.0), [3], k0=[k0], troe=[troe])
    n = 97
    T = np.linspace(800.0, 2400.0, n)
    P = np.full(n, ATM)
    Y = np.tile([0.45, 0.55], (n, 1))
    fg = R.rhs(R.Mechanism(m), T, P, Y, lanes_per_cell=8)
    fo = O.Model(m).rhs(T, P, Y)
    assert np.isfinite(fo).all()
    assert np.isfinite(fg).all(), fg[~np.isfinite(fg).all(1)][:3]
    e = np.abs(fg[:, 1] - fo[:, 1]) / np.abs(fo[:, 1])
    _say("max rel err", e.max())
    assert e.max() <= 1e-12


def test_arrhenius_argument_below_int32_exponent_range(R):
    """-E/(R T) far below -1.5e9 (T of 1e-8 to 1e-4 K, E/R 2.4e4 K): the rate
    constant is exactly 0, as in the oracle, not a wrapped exponent."""
    _say("arrhenius tiny T")
    m = mechs.tiny([10.0, 10.0], [([0], [1], 1e13, 0.0, 2.0e5)])
    T = np.array([1e-8, 1e-7, 1e-6, 1e-5, 1e-4, 1.0, 1000.0])
    n = len(T)
    P = np.full(n, ATM)
    Y = np.tile([0.5, 0.5], (n, 1))
    fg = R.rhs(R.Mechanism(m), T, P, Y, lanes_per_cell=8)
    fo = O.Model(m).rhs(T, P, Y)
    assert np.isfinite(fg).all()
    assert np.array_equal(fg[:-1], fo[:-1])   # exactly zero rates
    assert fg[-1, 1] == pytest.approx(fo[-1, 1], rel=1e-13)
