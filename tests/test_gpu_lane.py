"""GPU parity of the one-lane-per-cell kernels (Sec. 3: one thread per ODE):
source term and integration on the 9- and 13-species sets against the
oracle, in both memory layouts, both schedules, RKC and RKCK; stage counts past
the coefficient table; third-body and falloff pairs; failing cells; the
13-species set at its full cell count in the benchmark's launch
configuration, sampled; results that do not depend on the launch."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1309_2710_amd import synth
from tests import mechs
from tests import parity as PT
from tests.test_gpu_paths import check_long_horizon

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)
RKCK_DT, RKCK_TOL = 1e-8, 1e-10


@pytest.fixture(scope="module")
def R():
    from paper_1309_2710_amd import rkc
    rkc.lib()
    return rkc


def _say(*a):
    print("[case]", *a, flush=True)


def _pdep13():
    c = synth.CONFIGS["c2"]
    return synth.add_pressure_dependence(synth.config_mechanism("c2"), 1202, 0.2, 0.2,
                                         T_ref=math.sqrt(c["T_range"][0] * c["T_range"][1]),
                                         P_ref=c["P_max"])


def _species_major(Y):
    return np.ascontiguousarray(Y.T)


@pytest.mark.parametrize("cfg", ["c1", "c2", "c2pd"])
@pytest.mark.parametrize("layout", [0, 1])
def test_rhs_parity_lane(R, cfg, layout):
    _say("lane rhs", cfg, "layout", layout)
    m = _pdep13() if cfg == "c2pd" else synth.config_mechanism(cfg)
    st = synth.config_states("c2" if cfg == "c2pd" else cfg, 333, seed=91)
    gm, om = R.Mechanism(m), O.Model(m)
    Yin = st["Y"] if layout == 0 else _species_major(st["Y"])
    fg = R.rhs(gm, st["T"], st["P"], Yin, lanes_per_cell=1, layout=layout)
    if layout == 1:
        fg = np.ascontiguousarray(fg.T)
    fo = om.rhs(st["T"], st["P"], st["Y"])
    scale = np.abs(fo[:, 1:]).max(axis=1, keepdims=True)
    eY = np.abs(fg[:, 1:] - fo[:, 1:]) / scale
    eT = np.abs(fg[:, 0] - fo[:, 0]) / np.abs(fo[:, 0])
    _say("max eY", eY.max(), "max eT", eT.max())
    assert eY.max() <= 1e-12
    assert eT.max() <= 1e-11


LANE_CASES = [("c1", 1024, O.RKC, 0, 2), ("c1", 1000, O.RKC, 1, 1), ("c1", 1024, O.RKCK, 0, 2),
              ("c2", 777, O.RKC, 1, 2), ("c2", 512, O.RKC, 0, 1), ("c2", 512, O.RKCK, 1, 2)]


@pytest.mark.parametrize("cfg,n,method,layout,sched", LANE_CASES)
def test_integrate_parity_lane(R, cfg, n, method, layout, sched):
    """n not a multiple of the workgroup leaves a ragged last wave."""
    _say("lane integrate", cfg, n, "method", method, "layout", layout, "schedule", sched)
    m = synth.config_mechanism(cfg)
    c = synth.CONFIGS[cfg]
    dt, rtol = (RKCK_DT, RKCK_TOL) if method == O.RKCK else (c["dt"], c["rtol"])
    st = synth.config_states(cfg, n)
    T = st["T"].copy()
    Y = st["Y"].copy() if layout == 0 else _species_major(st["Y"])
    out = R.integrate(R.Mechanism(m), T, st["P"], Y, dt, rtol, c["atol"], method=method,
                      lanes_per_cell=1, layout=layout, schedule=sched, counters=True, stats=True)
    if layout == 1:
        Y = np.ascontiguousarray(Y.T)
    To, Yo, co = O.Model(m).integrate(st["T"], st["P"], st["Y"], dt, rtol, c["atol"],
                                      method=method, threads=THREADS)
    assert out["stats"]["lanes_per_cell"] == 1
    assert (out["status"] == 0).all() and (co["status"] == 0).all()
    assert out["stats"]["n_rhs"] == int(out["counters"][:, 0].sum())
    rep = PT.check(T, Y, out["counters"], To, Yo, co, rtol, c["atol"], PT.max_flips(cfg, n))
    _say(rep, out["stats"])


def test_pressure_dependent_pairs_lane(R):
    _say("lane integrate 13-species with third-body and falloff pairs")
    m = _pdep13()
    c = synth.CONFIGS["c2"]
    st = synth.config_states("c2", 400, seed=93)
    T, Y = st["T"].copy(), st["Y"].copy()
    out = R.integrate(R.Mechanism(m), T, st["P"], Y, c["dt"], c["rtol"], c["atol"],
                      lanes_per_cell=1, counters=True)
    To, Yo, co = O.Model(m).integrate(st["T"], st["P"], st["Y"], c["dt"], c["rtol"], c["atol"],
                                      threads=THREADS)
    assert (out["status"] == 0).all()
    rep = PT.check(T, Y, out["counters"], To, Yo, co, c["rtol"], c["atol"], PT.max_flips("c2", 400))
    _say(rep)


@pytest.mark.parametrize("coefs", [0, 1])
def test_stage_counts_above_the_table_lane(R, coefs):
    """A -> B with k dt = 1e5: steps of 130 to 363 stages, whose coefficients
    the lane kernel recomputes from the recurrences of Sec. 2.4."""
    _say("lane A->B s>128 coefs", coefs)
    k, dt, rtol, atol = 1e9, 1e-4, 1e-6, 1e-10
    m = mechs.a_to_b(k=k)
    rng = np.random.default_rng(5)
    ya = rng.uniform(0.05, 0.95, 96)
    st = {"T": rng.uniform(900.0, 1500.0, 96), "P": np.full(96, synth.ATM),
          "Y": np.ascontiguousarray(np.stack([ya, 1.0 - ya], 1))}
    T, Y = st["T"].copy(), st["Y"].copy()
    out = R.integrate(R.Mechanism(m), T, st["P"], Y, dt, rtol, atol, lanes_per_cell=1,
                      counters=True, stage_coefs=coefs)
    To, Yo, co = O.Model(m).integrate(st["T"], st["P"], st["Y"], dt, rtol, atol, threads=THREADS)
    cg = out["counters"]
    assert (cg[:, 4] > 128).all() and (co["s_max_used"] > 128).all()
    assert (out["status"] == 0).all()
    rep = check_long_horizon(T, Y, cg, To, Yo, co, rtol, atol)
    _say(rep)


def test_binding_stage_cap_lane(R):
    _say("lane c1 s_max 10")
    m = synth.config_mechanism("c1")
    c = synth.CONFIGS["c1"]
    st = synth.config_states("c1", 512)
    T, Y = st["T"].copy(), st["Y"].copy()
    out = R.integrate(R.Mechanism(m), T, st["P"], Y, c["dt"], c["rtol"], c["atol"], s_max=10,
                      lanes_per_cell=1, counters=True)
    To, Yo, co = O.Model(m).integrate(st["T"], st["P"], st["Y"], c["dt"], c["rtol"], c["atol"],
                                      s_max=10, threads=THREADS)
    assert np.array_equal(out["status"], co["status"].astype(np.int32))
    assert np.array_equal(out["counters"][:, 4] == 10, co["s_max_used"] == 10)
    rep = PT.check(T, Y, out["counters"], To, Yo, co, c["rtol"], c["atol"], PT.max_flips("c1", 512))
    _say(rep)


def test_failing_and_bad_cells_lane(R):
    """Cells with bad input are marked and left unchanged; NONFINITE cells of
    the served 13-species pool carry the oracle's status and counters and keep
    their input; every other cell matches the oracle."""
    _say("lane bad input and NONFINITE cells")
    m = synth.c5_mechanism(13, 2)
    c = synth.CONFIGS["c2"]
    pool = synth.make_states(m, 1 << 16, synth.C5_SEED * 10 + 13 * 4 + 2, T_dist=c["T"],
                             P_dist=c["P"], Y_dist=c["Y"])
    idx = np.concatenate([np.arange(44200, 44300), np.arange(45350, 45420)])
    st = {k: np.ascontiguousarray(v[idx]) for k, v in pool.items() if k in ("T", "P", "Y")}
    st["T"][3] = -5.0
    st["P"][7] = 0.0
    st["Y"][11, 2] = np.nan
    dt = 1e-5
    T, Y = st["T"].copy(), st["Y"].copy()
    out = R.integrate(R.Mechanism(m), T, st["P"], Y, dt, c["rtol"], c["atol"], lanes_per_cell=1,
                      counters=True)
    bad = np.zeros(len(idx), bool)
    bad[[3, 7, 11]] = True
    assert (out["status"][bad] == R.CELL_BADINPUT).all()
    good = ~bad
    sg = {k: np.ascontiguousarray(v[good]) for k, v in st.items()}
    To, Yo, co = O.Model(m).integrate(sg["T"], sg["P"], sg["Y"], dt, c["rtol"], c["atol"],
                                      threads=THREADS)
    assert np.array_equal(out["status"][good], co["status"].astype(np.int32))
    fail = np.nonzero(co["status"] != 0)[0]
    assert len(fail) == 2 and (co["status"][fail] == O.NONFINITE).all()
    cg = out["counters"][good]
    for f, col in PT.GPU_COL.items():
        assert np.array_equal(cg[fail, col], co[f][fail]), f
    Tg, Yg = T[good], Y[good]
    assert np.array_equal(Tg[fail], sg["T"][fail]) and np.array_equal(Yg[fail], sg["Y"][fail])
    assert np.array_equal(T[bad], st["T"][bad])
    ok = co["status"] == 0
    rep = PT.check(Tg[ok], Yg[ok], cg[ok], To[ok], Yo[ok], {k: v[ok] for k, v in co.items()},
                   c["rtol"], c["atol"], PT.max_flips("c2", int(ok.sum())))
    _say(rep)


def test_launch_does_not_change_results_lane(R):
    """Plain and persistent schedules, workgroups of 1, 2 and 4 waves, a small
    persistent grid, and both layouts give bitwise the same cells."""
    import torch
    _say("lane launch invariance c2")
    m = synth.config_mechanism("c2")
    c = synth.CONFIGS["c2"]
    st = synth.config_states("c2", 3000)
    dev = torch.device("cuda:0")
    gm = R.Mechanism(m)
    P = torch.from_numpy(st["P"]).to(dev)
    ref = None
    for sched, bg, grid, layout in [(1, 0, 0, 0), (2, 0, 0, 0), (2, 64, 0, 0), (2, 128, 3, 0),
                                    (2, 256, 0, 1), (1, 64, 0, 1)]:
        T = torch.from_numpy(st["T"]).to(dev)
        Y = torch.from_numpy(st["Y"] if layout == 0 else _species_major(st["Y"])).to(dev)
        out = R.integrate(gm, T, P, Y, c["dt"], c["rtol"], c["atol"], lanes_per_cell=1,
                          schedule=sched, block_groups=bg, grid_blocks=grid, layout=layout,
                          counters=True, stats=True)
        torch.cuda.synchronize()
        Yh = Y.cpu().numpy() if layout == 0 else np.ascontiguousarray(Y.cpu().numpy().T)
        res = (T.cpu().numpy(), Yh, out["counters"].cpu().numpy())
        _say(sched, bg, grid, layout, out["stats"]["schedule"], out["stats"]["grid_blocks"],
             out["stats"]["block_threads"])
        if ref is None:
            ref = res
        else:
            for a, b in zip(ref, res):
                assert np.array_equal(a, b)


def test_full_size_c2_sampled_lane(R):
    """The 13-species set at 262144 cells in the benchmark's launch (one lane
    per cell, persistent, species-major state), 256 sampled cells against the
    oracle; every cell finishes and conserves mass."""
    import torch
    _say("lane c2 full size")
    m = synth.config_mechanism("c2")
    c = synth.CONFIGS["c2"]
    st = synth.config_states("c2")
    n = st["T"].shape[0]
    dev = torch.device("cuda:0")
    T = torch.from_numpy(st["T"]).to(dev)
    P = torch.from_numpy(st["P"]).to(dev)
    Y = torch.from_numpy(_species_major(st["Y"])).to(dev)
    out = R.integrate(R.Mechanism(m), T, P, Y, c["dt"], c["rtol"], c["atol"], lanes_per_cell=1,
                      layout=1, counters=True, stats=True)
    torch.cuda.synchronize()
    assert out["stats"]["n_failed"] == 0
    Th = T.cpu().numpy()
    Yh = np.ascontiguousarray(Y.cpu().numpy().T)
    drift = np.abs(Yh.sum(1) - st["Y"].sum(1))
    assert (drift <= PT.mass_drift_bound(out["counters"].cpu().numpy()[:, 0])).all()
    idx = np.random.default_rng(17).choice(n, 256, replace=False)
    To, Yo, co = O.Model(m).integrate(st["T"][idx], st["P"][idx], st["Y"][idx], c["dt"],
                                      c["rtol"], c["atol"], threads=THREADS)
    rep = PT.check(Th[idx], Yh[idx], out["counters"].cpu().numpy()[idx], To, Yo, co, c["rtol"],
                   c["atol"], PT.max_flips("c2", 256))
    _say(rep, out["stats"])


def test_lane_form_limits(R):
    """N above the largest compiled state capacity (32) is refused, as is a
    layout code outside the two defined."""
    _say("lane limits")
    m = mechs.seeded(31)
    st = mechs.seeded_states(m, 8, 3)
    out = R.integrate(R.Mechanism(m), st["T"].copy(), st["P"], st["Y"].copy(), 1e-7,
                      lanes_per_cell=1, check=False)
    assert out["rc"] == R.OK
    big = synth.config_mechanism("c3")
    st = synth.config_states("c3", 4)
    out = R.integrate(R.Mechanism(big), st["T"].copy(), st["P"], st["Y"].copy(), 1e-7,
                      lanes_per_cell=1, check=False)
    assert out["rc"] == R.ENOTSUP
    # a layout code outside the two defined: refused by the C ABI itself
    import ctypes as ct
    gm = R.Mechanism(big)
    T, Y = st["T"].copy(), st["Y"].copy()
    o = R.make_opts(layout=2)
    rc = R.lib().rkc_integrate(gm.handle, 4, R._np_ptr(T), R._np_ptr(st["P"]), R._np_ptr(Y),
                               1e-7, 1e-6, 1e-10, ct.byref(o), None, None)
    assert rc == R.EINVAL
    assert np.array_equal(T, st["T"]) and np.array_equal(Y, st["Y"])
