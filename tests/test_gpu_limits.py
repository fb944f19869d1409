"""GPU: the largest states the compiled kernels hold.  255 species (N = 256 =
64 lanes x 4 slots) and 31 species on 8 lanes (N = 32 = 8 x 4) match the
oracle in the source term and over a global step; one species more than the
64-lane kernels hold is refused before anything is launched."""
import numpy as np
import pytest

from oracle import oracle as O
from tests import mechs
from tests import parity as PT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_1309_2710_amd import rkc
    rkc.lib()
    return rkc


def _say(*a):
    print("[case]", *a, flush=True)


_mech = mechs.seeded


def _states(m, n, seed):
    return mechs.seeded_states(m, n, seed)


@pytest.mark.parametrize("nS,G", [(255, 64), (31, 8)])
def test_four_slot_source_term(R, nS, G):
    _say("rhs", nS, "species, G", G)
    m = _mech(nS)
    gm, om = R.Mechanism(m), O.Model(m)
    st = _states(m, 77, 7000 + nS)
    fg = R.rhs(gm, st["T"], st["P"], st["Y"], lanes_per_cell=G)
    fo = om.rhs(st["T"], st["P"], st["Y"])
    scale = np.abs(fo[:, 1:]).max(axis=1, keepdims=True)
    eY = (np.abs(fg[:, 1:] - fo[:, 1:]) / scale).max()
    eT = (np.abs(fg[:, 0] - fo[:, 0]) / np.abs(fo[:, 0])).max()
    _say("max eY", eY, "max eT", eT)
    assert eY <= 1e-12 and eT <= 1e-11


@pytest.mark.parametrize("nS,G", [(255, 64), (31, 8)])
def test_four_slot_global_step(R, nS, G):
    _say("integrate", nS, "species, G", G)
    m = _mech(nS)
    gm, om = R.Mechanism(m), O.Model(m)
    n, dt, rtol, atol = 40, 1e-6, 1e-6, 1e-10
    st = _states(m, n, 8000 + nS)
    T, Y = st["T"].copy(), st["Y"].copy()
    out = R.integrate(gm, T, st["P"], Y, dt, rtol, atol, lanes_per_cell=G, counters=True,
                      stats=True)
    To, Yo, co = om.integrate(st["T"], st["P"], st["Y"], dt, rtol, atol)
    assert out["stats"]["lanes_per_cell"] == G
    assert (out["status"] == 0).all() and (co["status"] == 0).all()
    rep = PT.check(T, Y, out["counters"], To, Yo, co, rtol, atol, max(1, n // 100))
    _say(rep)


def test_one_species_more_is_refused(R):
    _say("256 species refused")
    m = dict(_mech(255))
    # one inert species more (no reaction touches it)
    m["n_species"] = 256
    m["W"] = np.append(m["W"], 39.95)
    m["nasa_low"] = np.vstack([m["nasa_low"], m["nasa_low"][-1]])
    m["nasa_high"] = np.vstack([m["nasa_high"], m["nasa_high"][-1]])
    m["T_mid"] = np.append(m["T_mid"], m["T_mid"][-1])
    gm = R.Mechanism(m)
    st = _states(_mech(255), 4, 9000)
    Y = np.ascontiguousarray(np.hstack([st["Y"], np.zeros((4, 1))]))
    with pytest.raises(R.RkcError) as e:
        R.integrate(gm, st["T"].copy(), st["P"], Y, 1e-6)
    assert e.value.code == R.ENOTSUP


def test_cell_count_above_the_limit_is_refused(R):
    """One cell more than RKC_MAX_CELLS is refused before any array is read
    (the arrays passed here are far smaller than the count)."""
    import ctypes as ct
    _say("n_cells above RKC_MAX_CELLS refused")
    gm = R.Mechanism(_mech(31))
    x = np.zeros(64)
    o = R.make_opts()
    big = R.MAX_CELLS + 1
    L = R.lib()
    rc = L.rkc_integrate(gm.handle, big, R._np_ptr(x), R._np_ptr(x), R._np_ptr(x), 1e-6, 1e-6,
                         1e-10, ct.byref(o), None, None)
    assert rc == R.ENOTSUP
    rc = L.rkc_rhs(gm.handle, big, R._np_ptr(x), R._np_ptr(x), R._np_ptr(x), R._np_ptr(x),
                   ct.byref(o))
    assert rc == R.ENOTSUP
