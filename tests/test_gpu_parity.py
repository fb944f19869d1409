"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs, element by element, plus properties that hold at any size."""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1309_2710_amd import synth
from tests import parity as PT

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    from paper_1309_2710_amd import rkc
    rkc.lib()
    return rkc


_MECHS = {}


def mech(R, cfg):
    if cfg not in _MECHS:
        _MECHS[cfg] = (R.Mechanism(synth.config_mechanism(cfg)), O.Model(synth.config_mechanism(cfg)))
    return _MECHS[cfg]


RHS_CASES = [("c1", 8), ("c1", 16), ("c1", 32), ("c1", 64), ("c2", 8), ("c2", 16), ("c2", 64),
             ("c3", 32), ("c3", 64), ("c4", 64)]


@pytest.mark.parametrize("cfg,G", RHS_CASES)
def test_rhs_parity(R, cfg, G):
    _say("rhs", cfg, "G", G)
    gm, om = mech(R, cfg)
    st = synth.config_states(cfg, 333)
    fg = R.rhs(gm, st["T"], st["P"], st["Y"], lanes_per_cell=G)
    fo = om.rhs(st["T"], st["P"], st["Y"])
    # species rates: relative to the cell's largest species rate (net production
    # sums cancel); temperature rate: relative to itself
    scale = np.abs(fo[:, 1:]).max(axis=1, keepdims=True)
    eY = np.abs(fg[:, 1:] - fo[:, 1:]) / scale
    eT = np.abs(fg[:, 0] - fo[:, 0]) / np.abs(fo[:, 0])
    _say("max eY", eY.max(), "max eT", eT.max())
    assert eY.max() <= 1e-12
    assert eT.max() <= 1e-11


# Temperatures far outside the workloads' range drive the Arrhenius exponents
# (base 2) from deep underflow (about -3000 at 50 K) to near overflow (+800
# for reverse rates with negative activation temperature at 50 K) and past it
# (20 K: the oracle's rates overflow to inf).
EXTREME_T = [50.0, 100.0, 300.0, 5000.0, 2e4, 1e5]


@pytest.mark.parametrize("cfg,G", [("c2", 16), ("c2", 1), ("c3", 64), ("c4p", 0)])
def test_rhs_parity_extreme_temperatures(R, cfg, G):
    _say("rhs extreme T", cfg, "G", G)
    gm, om = mech(R, cfg)
    st = synth.config_states(cfg, 8)
    n = len(st["T"])
    T = np.repeat(np.array(EXTREME_T), n)
    P = np.tile(st["P"], len(EXTREME_T))
    Y = np.tile(st["Y"], (len(EXTREME_T), 1))
    fg = R.rhs(gm, T, P, Y, lanes_per_cell=G)
    fo = om.rhs(T, P, Y)
    assert np.isfinite(fo).all()
    scale = np.abs(fo[:, 1:]).max(axis=1, keepdims=True)
    eY = np.abs(fg[:, 1:] - fo[:, 1:]) / scale
    eT = np.abs(fg[:, 0] - fo[:, 0]) / np.abs(fo[:, 0])
    _say("max eY", eY.max(), "max eT", eT.max(), "scales", scale.min(), scale.max())
    assert eY.max() <= 1e-12
    assert eT.max() <= 1e-11
    # 20 K: rates overflow on both sides, the same cells are non-finite; far
    # below, down to the smallest subnormal, where the kernels bound 1/T in
    # the Arrhenius factors, every cell stays non-finite on both sides (no
    # finite value from a wrapped exponent)
    for Tlow in (20.0, 1e-3, 1e-6, 1e-300, 5e-324):
        Tl = np.full(n, Tlow)
        fgl = R.rhs(gm, Tl, st["P"], st["Y"], lanes_per_cell=G)
        fol = om.rhs(Tl, st["P"], st["Y"])
        assert (np.isfinite(fgl).all(axis=1) == np.isfinite(fol).all(axis=1)).all(), Tlow


def _range_switch_mech(cfg):
    """The set's mechanism with a distinct NASA switch temperature per species
    and a high range that differs from the low one (Cp/R and H/(R T) offset),
    so that choosing the wrong range shows in the source term."""
    m = dict(synth.config_mechanism(cfg))
    nS = m["n_species"]
    m["T_mid"] = 900.0 + 7.0 * np.arange(nS)
    hi = np.array(m["nasa_high"], dtype=np.float64).reshape(nS, 7).copy()
    hi[:, 0] *= 1.05
    hi[:, 5] += 50.0
    m["nasa_high"] = hi
    return m


# c4: the 111-species shape runs the kernels whose species table is read from
# global memory, with the switch temperatures staged in LDS
@pytest.mark.parametrize("cfg,G", [("c2", 16), ("c4", 0)])
def test_rhs_parity_at_range_switch(R, cfg, G):
    _say("rhs at T_mid", cfg, "G", G)
    m = _range_switch_mech(cfg)
    gm, om = R.Mechanism(m), O.Model(m)
    st = synth.config_states(cfg, 8)
    Tm = np.unique(np.asarray(m["T_mid"], dtype=np.float64))
    T = np.concatenate([Tm, np.nextafter(Tm, 0.0)])      # at and one ulp below
    idx = np.arange(len(T)) % len(st["T"])
    P = np.ascontiguousarray(st["P"][idx])
    Y = np.ascontiguousarray(st["Y"][idx])
    fg = R.rhs(gm, T, P, Y, lanes_per_cell=G)
    fo = om.rhs(T, P, Y)
    scale = np.abs(fo[:, 1:]).max(axis=1, keepdims=True)
    eY = np.abs(fg[:, 1:] - fo[:, 1:]) / scale
    eT = np.abs(fg[:, 0] - fo[:, 0]) / np.abs(fo[:, 0])
    _say("max eY", eY.max(), "max eT", eT.max())
    assert eY.max() <= 1e-12
    assert eT.max() <= 1e-11


max_flips = PT.max_flips


# RKCK runs in the paper's nonstiff setting for it (Sec. 3.1: global step
# 1e-8 s, tolerance 1e-10); RKC in each workload's own setting.
RKCK_DT, RKCK_TOL = 1e-8, 1e-10

INTEG_CASES = [("c1", 1024, O.RKC, 16), ("c1", 1024, O.RKC, 8), ("c1", 1024, O.RKC, 64),
               ("c1", 1024, O.RKCK, 16), ("c1", 1024, O.RKCK, 64), ("c2", 512, O.RKC, 16),
               ("c2", 512, O.RKCK, 16), ("c3", 96, O.RKC, 64), ("c3", 96, O.RKC, 32),
               ("c3", 64, O.RKCK, 64), ("c4", 48, O.RKC, 64)]


@pytest.mark.parametrize("cfg,n,method,G", INTEG_CASES)
def test_integrate_parity(R, cfg, n, method, G):
    _say("integrate", cfg, n, "method", method, "G", G)
    gm, om = mech(R, cfg)
    c = synth.CONFIGS[cfg]
    dt, rtol = (RKCK_DT, RKCK_TOL) if method == O.RKCK else (c["dt"], c["rtol"])
    st = synth.config_states(cfg, n)
    Tg, Yg = st["T"].copy(), st["Y"].copy()
    out = R.integrate(gm, Tg, st["P"], Yg, dt, rtol, c["atol"], method=method,
                      lanes_per_cell=G, counters=True, stats=True)
    To, Yo, co = om.integrate(st["T"], st["P"], st["Y"], dt, rtol, c["atol"],
                              method=method, threads=THREADS)
    assert (out["status"] == 0).all() and (co["status"] == 0).all()
    rep = PT.check(Tg, Yg, out["counters"], To, Yo, co, rtol, c["atol"],
                   max_flips(cfg, n), long_set=cfg in PT.LONG_SETS)
    _say(rep, out["stats"])


def test_schedules_and_grain_are_bitwise_invariant(R):
    _say("schedule invariance c2")
    gm, _ = mech(R, "c2")
    c = synth.CONFIGS["c2"]
    st = synth.config_states("c2", 700)
    res = []
    for kw in [dict(schedule=R.SCHED_PLAIN), dict(schedule=R.SCHED_PERSISTENT),
               dict(schedule=R.SCHED_PERSISTENT, grid_blocks=3, block_groups=4),
               dict(schedule=R.SCHED_PLAIN, block_groups=1)]:
        T, Y = st["T"].copy(), st["Y"].copy()
        out = R.integrate(gm, T, st["P"], Y, c["dt"], c["rtol"], c["atol"], lanes_per_cell=16,
                          counters=True, **kw)
        res.append((T, Y, out["counters"]))
    for T, Y, cn in res[1:]:
        assert np.array_equal(T, res[0][0]) and np.array_equal(Y, res[0][1])
        assert np.array_equal(cn, res[0][2])


def test_repeat_runs_bitwise_identical(R):
    _say("repeat c3")
    gm, _ = mech(R, "c3")
    c = synth.CONFIGS["c3"]
    st = synth.config_states("c3", 300)
    outs = []
    for _ in range(2):
        T, Y = st["T"].copy(), st["Y"].copy()
        R.integrate(gm, T, st["P"], Y, c["dt"], c["rtol"], c["atol"])
        outs.append((T, Y))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_edge_cases(R):
    _say("edge cases c1")
    gm, om = mech(R, "c1")
    c = synth.CONFIGS["c1"]
    # empty batch
    e = np.zeros(0)
    out = R.integrate(gm, e.copy(), e.copy(), np.zeros((0, 9)), 1e-6)
    assert out["rc"] == R.OK
    # one cell and a ragged count
    for n in (1, 65):
        st = synth.config_states("c1", n)
        T, Y = st["T"].copy(), st["Y"].copy()
        R.integrate(gm, T, st["P"], Y, c["dt"], c["rtol"], c["atol"], lanes_per_cell=16)
        To, Yo, _ = om.integrate(st["T"], st["P"], st["Y"], c["dt"], c["rtol"], c["atol"])
        assert PT.rel_err(T, Y, To, Yo).max() <= PT.TOL
    # bad inputs are flagged per cell; neighbours unaffected
    st = synth.config_states("c1", 8)
    T, P, Y = st["T"].copy(), st["P"].copy(), st["Y"].copy()
    T[1] = -1.0; P[2] = 0.0; Y[3, 0] = np.nan; T[4] = np.inf
    out = R.integrate(gm, T, P, Y, c["dt"], c["rtol"], c["atol"], lanes_per_cell=16)
    assert out["rc"] == R.ECELLS
    assert list(out["status"][1:5]) == [R.CELL_BADINPUT] * 4
    assert T[1] == -1.0 and np.isinf(T[4])
    To, Yo, co = om.integrate(st["T"][[0, 5, 6, 7]], st["P"][[0, 5, 6, 7]],
                              st["Y"][[0, 5, 6, 7]], c["dt"], c["rtol"], c["atol"])
    assert PT.rel_err(T[[0, 5, 6, 7]], Y[[0, 5, 6, 7]], To, Yo).max() <= PT.TOL
    # step budget exhausted
    st = synth.config_states("c1", 16)
    T, Y = st["T"].copy(), st["Y"].copy()
    out = R.integrate(gm, T, st["P"], Y, c["dt"], c["rtol"], c["atol"], max_steps=1,
                      counters=True)
    _, _, co = om.integrate(st["T"], st["P"], st["Y"], c["dt"], c["rtol"], c["atol"],
                            max_steps=1)
    assert (out["status"] == R.CELL_MAXSTEPS).all() and (co["status"] == O.MAXSTEPS).all()


def _full_size_sampled(R, cfg, n_sample, method=O.RKC, config_step=False):
    """A workload at its full cell count, device-resident, in the launch
    configuration the benchmark uses; the oracle checks a strided sample.
    RKCK runs in its nonstiff setting (global step and tolerance above) unless
    config_step asks for the configuration's own step and tolerance."""
    import torch
    gm, om = mech(R, cfg)
    c = dict(synth.CONFIGS[cfg])
    if method == O.RKCK and not config_step:
        c["dt"], c["rtol"] = RKCK_DT, RKCK_TOL
    st = synth.config_states(cfg)
    n = st["T"].shape[0]
    _say("full", cfg, n, "cells, method", method)
    T = torch.from_numpy(st["T"]).cuda()
    P = torch.from_numpy(st["P"]).cuda()
    Y = torch.from_numpy(st["Y"]).cuda()
    out = R.integrate(gm, T, P, Y, c["dt"], c["rtol"], c["atol"], method=method, counters=True,
                      stats=True)
    torch.cuda.synchronize()
    Tg, Yg = T.cpu().numpy(), Y.cpu().numpy()
    cg = out["counters"].cpu().numpy()
    _say("stats", out["stats"])
    assert (out["status"].cpu().numpy() == 0).all()
    drift = np.abs(Yg.sum(1) - st["Y"].sum(1))
    _say("mass drift max %.3g, largest fraction of its bound %.3f"
         % (drift.max(), (drift / PT.mass_drift_bound(cg[:, 0])).max()))
    assert (drift <= PT.mass_drift_bound(cg[:, 0])).all()
    idx = np.arange(0, n, n // n_sample)[:n_sample]
    To, Yo, co = om.integrate(st["T"][idx], st["P"][idx], st["Y"][idx], c["dt"], c["rtol"],
                              c["atol"], method=method, threads=THREADS)
    rep = PT.check(Tg[idx], Yg[idx], cg[idx], To, Yo, co, c["rtol"], c["atol"],
                   max_flips(cfg, n_sample), long_set=cfg in PT.LONG_SETS)
    _say(rep)


def test_full_size_c3_sampled(R):
    """53sp/634rx at its full 131072 cells (the benchmark's workload)."""
    _full_size_sampled(R, "c3", 64)


def test_full_size_c2_sampled(R):
    """13sp/54rx at its full 262144 cells."""
    _full_size_sampled(R, "c2", 128)


def test_full_size_c4_sampled(R):
    """111sp/1566rx at its full 65536 cells (64 lanes, two state slots per
    lane, 10-term gather segments), 128 cells checked."""
    _full_size_sampled(R, "c4", 128)


def test_full_size_c3p_sampled(R):
    """53sp/634rx with third-body and falloff pairs at its full 131072 cells
    (32-lane groups, the automatic choice for this set)."""
    _full_size_sampled(R, "c3p", 32)


def test_full_size_c4p_sampled(R):
    """111sp/1566rx with third-body and falloff pairs at its full 65536 cells
    (parameters in global memory, the automatic choice for this set)."""
    _full_size_sampled(R, "c4p", 64)


def test_full_size_rkck_c3_config_step_sampled(R):
    """RKCK on 53sp/634rx at its full 131072 cells with the set's own step and
    tolerance (dt 1e-6, epsilon 1e-6: the setting of the paper's comparison of
    the two methods on this mechanism size, Sec. 3.3), where RKCK needs about
    360 evaluations per cell and rejects steps; 32 cells checked."""
    _full_size_sampled(R, "c3", 32, method=O.RKCK, config_step=True)


def test_full_size_rkck_c2_sampled(R):
    """RKCK over the 13-species set's full 262144 cells (persistent schedule)."""
    _full_size_sampled(R, "c2", 64, method=O.RKCK)


def test_ten_consecutive_steps_c3(R):
    """The paper's protocol times ten consecutive global steps (Sec. 3): parity
    after step 1 and after step 10 on a strided sample of the 53-species set,
    each step restarting from the previous result on both sides."""
    _say("ten steps c3")
    gm, om = mech(R, "c3")
    c = synth.CONFIGS["c3"]
    st = synth.config_states("c3")
    idx = np.arange(0, st["T"].shape[0], 4096)[:32]
    Tg, Yg = st["T"][idx].copy(), st["Y"][idx].copy()
    To, Yo = Tg.copy(), Yg.copy()
    P = st["P"][idx].copy()
    same = np.ones(len(idx), bool)
    for k in range(10):
        out = R.integrate(gm, Tg, P, Yg, c["dt"], c["rtol"], c["atol"], counters=True)
        To, Yo, co = om.integrate(To, P, Yo, c["dt"], c["rtol"], c["atol"], threads=THREADS)
        same &= ~PT.counter_mismatch(out["counters"], co)
        if k in (0, 9):
            err = PT.rel_err(Tg, Yg, To, Yo)
            _say("step", k + 1, "max err (same decisions so far)",
                 err[same].max() if same.any() else None, "cells", int(same.sum()))
            assert same.sum() >= len(idx) - max_flips("c3", len(idx))
            assert err[same].max() <= PT.TOL
