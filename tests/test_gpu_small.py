"""GPU parity on hand-built small mechanisms (closed forms and a nonlinear
reversible pair), and forced per-cell failure codes against the oracle's."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1309_2710_amd import synth
from tests import mechs
from tests import parity as PT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_1309_2710_amd import rkc
    rkc.lib()
    return rkc


def _states(nS, n, seed):
    rng = np.random.default_rng(seed)
    return {"T": rng.uniform(900.0, 1500.0, n), "P": np.full(n, synth.ATM),
            "Y": np.ascontiguousarray(rng.dirichlet(np.ones(nS), n))}


SMALL = [("a_to_b", mechs.a_to_b(1e6)), ("a_b_c", mechs.a_b_c(1e6, 3e5)),
         ("nonlinear3", mechs.nonlinear3())]


@pytest.mark.parametrize("name,m", SMALL, ids=[s[0] for s in SMALL])
@pytest.mark.parametrize("G", [8, 16])
def test_small_mechanism_parity(R, name, m, G):
    print("[case] small", name, G, flush=True)
    gm, om = R.Mechanism(m), O.Model(m)
    st = _states(m["n_species"], 200, 11)
    fg = R.rhs(gm, st["T"], st["P"], st["Y"], lanes_per_cell=G)
    fo = om.rhs(st["T"], st["P"], st["Y"])
    scale = np.maximum(np.abs(fo).max(axis=1, keepdims=True), 1e-300)
    assert (np.abs(fg - fo) / scale).max() <= 1e-12
    dt, rtol, atol = 1e-5, 1e-6, 1e-10
    T, Y = st["T"].copy(), st["Y"].copy()
    out = R.integrate(gm, T, st["P"], Y, dt, rtol, atol, lanes_per_cell=G, counters=True)
    To, Yo, co = om.integrate(st["T"], st["P"], st["Y"], dt, rtol, atol)
    assert (out["status"] == 0).all()
    PT.check(T, Y, out["counters"], To, Yo, co, rtol, atol, 2)
    if name == "a_to_b":   # closed form Y_A(dt) = Y_A(0) exp(-k dt), T constant
        ya = st["Y"][:, 0] * np.exp(-1e6 * dt)
        assert np.abs(Y[:, 0] - ya).max() <= 10 * rtol * st["Y"][:, 0].max()
        assert np.array_equal(T, st["T"])


def test_stage_cap_on_stiff_cells_matches_oracle_status(R):
    """s_max = 2 on the stiff 9-species set: the capped step underflows in stiff
    cells; the per-cell codes and the untouched neighbours match the oracle."""
    print("[case] s_max 2 c1", flush=True)
    m = synth.config_mechanism("c1")
    c = synth.CONFIGS["c1"]
    gm, om = R.Mechanism(m), O.Model(m)
    st = synth.config_states("c1", 128)
    T, Y = st["T"].copy(), st["Y"].copy()
    out = R.integrate(gm, T, st["P"], Y, c["dt"], c["rtol"], c["atol"], s_max=2,
                      max_steps=20000, lanes_per_cell=16, counters=True)
    To, Yo, co = om.integrate(st["T"], st["P"], st["Y"], c["dt"], c["rtol"], c["atol"],
                              s_max=2, max_steps=20000)
    sg, so = out["status"], co["status"]
    print("[case] statuses gpu", np.bincount(sg, minlength=5), "oracle",
          np.bincount(so, minlength=5), flush=True)
    assert np.bincount(sg, minlength=5)[1:].sum() > 0      # the cap does bite
    agree = sg == so
    assert agree.mean() >= 0.95
    ok = (sg == 0) & (so == 0)
    assert PT.rel_err(T[ok], Y[ok], To[ok], Yo[ok]).max() <= 1e-6
