"""Comparison helpers for GPU-vs-oracle parity.

Relative error, as fixed for this integrator: |T_g - T_o| / |T_o| for the
temperature and |Y_g - Y_o| / max(|Y_o|, Y_FLOOR) for mass fractions, i.e.
relative for Y >= 1e-6 and absolute 1e-14 below.  The floor is set by what
double precision can reproduce: re-evaluating one rounding in the oracle itself
(Arrhenius in log form, or rho*Y*(1/W) for rho*Y/W) moves species far below
atol by up to 1e-12 absolute in the stiff 9-species workload (s up to ~130),
so a floor at atol = 1e-10 would make 1e-8 unreachable even for the oracle
against itself; with the 1e-6 floor the oracle's self-consistency is 6e-9
(9 species), 8e-11 (13), 4e-11 (53) and 8e-10 (111).  Decision counters (RHS
evaluations, accepted and rejected steps, power-method calls, hash of the
stage-count sequence, status) are compared exactly.

Policy.  Cells whose decision sequences agree must match to TOL.  An adaptive
integrator takes discrete decisions on floating-point thresholds (accept
err <= 1, the 1 % power-method test, the floor in the stage count), so two
correct implementations that differ in rounding can take different decisions
in a few cells; the two results are then both valid solutions.  Such cells
must be rare and must agree within FLIP_WRMS in the integrator's own weighted
RMS norm (atol + rtol max|y|), i.e. within a few local tolerance units.  The
oracle itself shows the effect: re-evaluating its concentrations as
rho*Y*(1/W) instead of rho*Y/W (a one-rounding change) flips decisions in 3 of
48 cells of the 111-species workload, which then differ by at most 0.81 in
that norm.
"""
import numpy as np

TOL = 1e-8
Y_FLOOR = 1e-6
DECISION_FIELDS = ["n_rhs", "n_steps", "n_reject", "n_sigma", "s_hash", "status"]
GPU_COL = {"n_rhs": 0, "n_steps": 1, "n_reject": 2, "n_sigma": 3, "s_max_used": 4, "s_hash": 5,
           "status": 6, "n_power_iter": 7}


def rel_err(Tg, Yg, To, Yo, floor=Y_FLOOR):
    eT = np.abs(Tg - To) / np.abs(To)
    eY = np.abs(Yg - Yo) / np.maximum(np.abs(Yo), floor)
    return np.maximum(eT, eY.max(axis=1))


def counter_mismatch(cg, co):
    """Boolean mask of cells whose decision counters differ (cg: [n][8] GPU)."""
    bad = np.zeros(cg.shape[0], bool)
    for f in DECISION_FIELDS:
        bad |= cg[:, GPU_COL[f]].astype(np.int64) != co[f].astype(np.int64)
    return bad


def report(Tg, Yg, cg, To, Yo, co, atol=1e-10):
    e = rel_err(Tg, Yg, To, Yo)
    mm = counter_mismatch(cg, co)
    same = ~mm
    return {
        "n": len(e),
        "max_rel_err": float(e.max()) if len(e) else 0.0,
        "max_rel_err_matching": float(e[same].max()) if same.any() else 0.0,
        "n_counter_mismatch": int(mm.sum()),
        "max_rel_err_mismatch": float(e[mm].max()) if mm.any() else 0.0,
    }


FLIP_WRMS = 5.0


def wrms(Tg, Yg, To, Yo, rtol=1e-6, atol=1e-10):
    yg = np.concatenate([np.asarray(Tg)[:, None], Yg], 1)
    yo = np.concatenate([np.asarray(To)[:, None], Yo], 1)
    w = atol + rtol * np.maximum(np.abs(yg), np.abs(yo))
    return np.sqrt((((yg - yo) / w) ** 2).mean(1))


def check(Tg, Yg, cg, To, Yo, co, rtol, atol, max_flips):
    """Apply the parity policy; returns the report dict (asserts inside)."""
    rep = report(Tg, Yg, cg, To, Yo, co, atol)
    mm = counter_mismatch(cg, co)
    rep["max_wrms_mismatch"] = float(wrms(Tg[mm], Yg[mm], To[mm], Yo[mm], rtol, atol).max()) \
        if mm.any() else 0.0
    assert rep["max_rel_err_matching"] <= TOL, rep
    assert rep["n_counter_mismatch"] <= max_flips, rep
    assert rep["max_wrms_mismatch"] <= FLIP_WRMS, rep
    return rep
