"""The autotuner: the inputs it times on are left unchanged; schedule, grain
and parameter placement never change results (a run with its choice equals,
bit for bit, a run with the same lanes_per_cell and default launch); the form
it picks is parity-green against the oracle; a repeated call returns the
cached choice without timing; a requested lanes_per_cell is kept."""
import os
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_1309_2710_amd import synth
from tests import parity as PT

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def R():
    from paper_1309_2710_amd import rkc
    rkc.lib()
    return rkc


@pytest.mark.parametrize("cfg,n", [("c2", 3000), ("c3", 1500)])
def test_autotuned_options_keep_results(R, cfg, n):
    print("[case] autotune", cfg, n, flush=True)
    c = synth.CONFIGS[cfg]
    m = synth.config_mechanism(cfg)
    gm = R.Mechanism(m)
    st = synth.config_states(cfg, n)
    T0, Y0 = st["T"].copy(), st["Y"].copy()
    t = time.perf_counter()
    kw, ms = R.autotune(gm, st["T"], st["P"], st["Y"], c["dt"], c["rtol"], c["atol"])
    first_s = time.perf_counter() - t
    print("[case] tuned", kw, ms, "in %.2f s" % first_s, flush=True)
    assert np.array_equal(st["T"], T0) and np.array_equal(st["Y"], Y0)
    assert ms > 0 and kw["schedule"] in (R.SCHED_PLAIN, R.SCHED_PERSISTENT)
    # block_groups 0 is the automatic grain (the first stage times the default)
    assert kw["block_groups"] >= 0 and kw["lanes_per_cell"] in (1, 8, 16, 32, 64)
    # launch options do not change results
    Ta, Ya = st["T"].copy(), st["Y"].copy()
    R.integrate(gm, Ta, st["P"], Ya, c["dt"], c["rtol"], c["atol"],
                lanes_per_cell=kw["lanes_per_cell"])
    Tb, Yb = st["T"].copy(), st["Y"].copy()
    out = R.integrate(gm, Tb, st["P"], Yb, c["dt"], c["rtol"], c["atol"], counters=True, **kw)
    assert np.array_equal(Ta, Tb) and np.array_equal(Ya, Yb)
    # and the chosen form meets the parity bar on a sample
    idx = np.arange(0, n, max(1, n // 200))
    To, Yo, co = O.Model(m).integrate(st["T"][idx], st["P"][idx], st["Y"][idx], c["dt"],
                                      c["rtol"], c["atol"], threads=THREADS)
    PT.check(Tb[idx], Yb[idx], out["counters"][idx], To, Yo, co, c["rtol"], c["atol"],
             PT.max_flips(cfg, len(idx)))
    # cached: the same key returns the same choice without timing
    t = time.perf_counter()
    kw2, ms2 = R.autotune(gm, st["T"], st["P"], st["Y"], c["dt"], c["rtol"], c["atol"])
    again_s = time.perf_counter() - t
    assert kw2 == kw and ms2 == ms
    assert again_s < first_s / 5


def test_requested_lanes_are_kept(R):
    print("[case] autotune with lanes_per_cell = 16", flush=True)
    c = synth.CONFIGS["c2"]
    gm = R.Mechanism(synth.config_mechanism("c2"))
    st = synth.config_states("c2", 2048)
    kw, ms = R.autotune(gm, st["T"], st["P"], st["Y"], c["dt"], c["rtol"], c["atol"],
                        lanes_per_cell=16)
    assert kw["lanes_per_cell"] == 16
    Ta, Ya = st["T"].copy(), st["Y"].copy()
    R.integrate(gm, Ta, st["P"], Ya, c["dt"], c["rtol"], c["atol"], lanes_per_cell=16)
    Tb, Yb = st["T"].copy(), st["Y"].copy()
    R.integrate(gm, Tb, st["P"], Yb, c["dt"], c["rtol"], c["atol"], **kw)
    assert np.array_equal(Ta, Tb) and np.array_equal(Ya, Yb)
