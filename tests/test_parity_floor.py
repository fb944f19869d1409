"""Where the parity bar comes from: the oracle against itself with one
rounding changed.

Any correct second implementation (the HIP kernels among them) differs from
the oracle in rounding only.  This test rebuilds the oracle from a copy of its
source with one expression rounded differently -- the concentrations as
rho Y (1/W) instead of rho Y / W, or the Arrhenius rate in log form
exp(ln A + beta ln T - E/(R T)) instead of A T^beta exp(-E/(R T)) -- and
compares each copy with the oracle on seeded samples of every workload.  It
asserts that the constants of tests/parity.py sit above what it measures,
with a margin, and that the floor is needed: with the floor at atol the
oracle does not reproduce itself to 1e-8.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import build as oracle_build
from oracle import oracle as O
from paper_1309_2710_amd import synth
from tests import parity as PT

ROUNDINGS = {
    "concentrations as rho Y (1/W)": ("ws->C[i] = rho * Y[i] / m->W[i];",
                                      "ws->C[i] = rho * Y[i] * (1.0 / m->W[i]);"),
    "Arrhenius rate in log form": (
        "double k = m->A[j] * pow(T, m->beta[j]) * exp(-m->Ea[j] / (R_J * T));",
        "double k = exp(log(m->A[j]) + m->beta[j] * log(T) - m->Ea[j] / (R_J * T));"),
}

SAMPLES = [("c1", 1024), ("c2", 2048), ("c3", 256), ("c3p", 128), ("c4", 256)]
THREADS = min(8, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def variants():
    tmp = tempfile.mkdtemp(prefix="orc_round_")
    src = open(oracle_build.SRC).read()
    libs = {}
    for i, (name, (a, b)) in enumerate(ROUNDINGS.items()):
        assert src.count(a) == 1, a
        path = os.path.join(tmp, "r%d.c" % i)
        with open(path, "w") as fh:
            fh.write(src.replace(a, b))
        lib = os.path.join(tmp, "libr%d.so" % i)
        subprocess.run(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
                        "-fPIC", "-shared", "-pthread", "-w", "-o", lib, path, "-lm"], check=True)
        libs[name] = O.load_variant(lib)
    yield libs
    shutil.rmtree(tmp, ignore_errors=True)


def _measure(cfg, n, L):
    c = synth.CONFIGS[cfg]
    m = synth.config_mechanism(cfg)
    st = synth.config_states(cfg, n)
    args = (st["T"], st["P"], st["Y"], c["dt"], c["rtol"], c["atol"])
    To, Yo, co = O.Model(m).integrate(*args, threads=THREADS)
    T1, Y1, c1 = O.Model(m, library=L).integrate(*args, threads=THREADS)
    cg = np.stack([c1[f] for f in O.COUNTER_FIELDS], 1)
    rep = PT.report(T1, Y1, cg, To, Yo, co, c["atol"])
    mm = PT.counter_mismatch(cg, co)
    rep["max_wrms_mismatch"] = float(PT.wrms(T1[mm], Y1[mm], To[mm], Yo[mm], c["rtol"],
                                             c["atol"]).max()) if mm.any() else 0.0
    rep["frac_over_tol"] = rep["n_matching_over_tol"] / max(1, n - rep["n_counter_mismatch"])
    return rep


@pytest.mark.parametrize("cfg,n", SAMPLES)
@pytest.mark.parametrize("rounding", list(ROUNDINGS))
def test_parity_bar_sits_above_the_oracles_own_rounding_noise(variants, cfg, n, rounding):
    rep = _measure(cfg, n, variants[rounding])
    print("[rounding]", cfg, n, rounding, rep, flush=True)
    if cfg in PT.LONG_SETS:
        assert rep["max_rel_err_matching"] <= PT.LONG_TOL / 5
        assert rep["frac_over_tol"] <= PT.LONG_FRAC_OVER / 1.5
        assert rep["n_counter_mismatch"] <= PT.LONG_FLIP_FRAC * n / 1.5
    else:
        assert rep["max_rel_err_matching"] <= PT.TOL / 1.3
        assert rep["n_counter_mismatch"] <= PT.FLIP_FRAC * n / 2
    assert rep["max_wrms_mismatch"] <= PT.FLIP_WRMS / 2


def test_a_floor_at_atol_is_out_of_reach(variants):
    """Why Y_FLOOR is 1e-6 and not atol: trace species of the stiff 9-species
    set move far more than 1e-8 relative to atol under a one-rounding change."""
    worst = max(_measure("c1", 512, L)["max_rel_err_matching_floor_atol"]
                for L in variants.values())
    assert worst > 1e3 * PT.TOL


def test_long_horizon_stiff_case_flips_decisions_between_roundings():
    """The stiff A -> B case of the GPU stage-count tests (k dt = 1e5, about
    700 steps of up to 363 stages per cell): the oracle rebuilt with mu_j of
    Sec. 2.4 formed with the reciprocal of b_{j-1} takes a different step
    sequence in a sizeable fraction of the cells, while every cell still ends
    within 1e-8 of the unchanged oracle.  This is why that case is held to
    the 1e-8 bar in every cell but not to equal decision counters."""
    from tests import mechs
    src = open(oracle_build.SRC).read()
    a = "mu[j] = 2.0 * b[j] * w0 / b[j - 1];"
    assert src.count(a) == 1
    tmp = tempfile.mkdtemp(prefix="orc_mu_")
    try:
        path = os.path.join(tmp, "mu.c")
        with open(path, "w") as fh:
            fh.write(src.replace(a, "mu[j] = 2.0 * b[j] * w0 * (1.0 / b[j - 1]);"))
        lib = os.path.join(tmp, "libmu.so")
        subprocess.run(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
                        "-fPIC", "-shared", "-pthread", "-w", "-o", lib, path, "-lm"], check=True)
        L = O.load_variant(lib)
        m = mechs.a_to_b(k=1e9)
        rng = np.random.default_rng(5)
        ya = rng.uniform(0.05, 0.95, 96)
        st = (rng.uniform(900.0, 1500.0, 96), np.full(96, synth.ATM),
              np.ascontiguousarray(np.stack([ya, 1.0 - ya], 1)))
        args = st + (1e-4, 1e-6, 1e-10)
        To, Yo, co = O.Model(m).integrate(*args, threads=THREADS)
        T1, Y1, c1 = O.Model(m, library=L).integrate(*args, threads=THREADS)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    cg = np.stack([c1[f] for f in O.COUNTER_FIELDS], 1)
    rep = PT.report(T1, Y1, cg, To, Yo, co, 1e-10)
    print("[rounding] A->B k dt 1e5", rep, "steps", co["n_steps"].mean(), flush=True)
    assert co["n_steps"].mean() > 500 and co["s_max_used"].max() > 300
    assert rep["n_counter_mismatch"] >= 10
    assert rep["max_rel_err"] <= PT.TOL / 2
