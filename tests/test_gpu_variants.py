"""GPU: every compiled kernel variant (lane-group size, slots per lane,
placement of the reaction parameters) runs a global step that meets the
oracle parity policy, reports the variant that ran, and gives bitwise the
results of the LDS placement at the same group size."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1309_2710_amd import synth
from tests import mechs
from tests import parity as PT

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def R():
    from paper_1309_2710_amd import rkc
    rkc.lib()
    return rkc


def _say(*a):
    print("[case]", *a, flush=True)


# (mechanism, lanes per cell, requested placement, placement that must run);
# placements: 1 registers, 2 LDS, 3 global memory.  The register variants
# hold RU units per lane: c3 (317 units) 5 at 64 lanes, c2 (27) 2 at 16 and
# 4 at 8, c1 (19) 3 at 8.
CASES = [("c3", 64, 1, 1), ("c2", 16, 1, 1), ("c1", 8, 1, 1), ("c2", 8, 1, 1),
         ("c1", 32, 2, 2), ("s31", 16, 2, 2), ("s255", 64, 3, 3), ("c4", 64, 3, 3)]


def _mech_states(cfg, n):
    if cfg.startswith("s"):
        m = mechs.seeded(int(cfg[1:]))
        c = {"dt": 1e-6, "rtol": 1e-6, "atol": 1e-10}
        return m, mechs.seeded_states(m, n, 6100 + n), c
    return synth.config_mechanism(cfg), synth.config_states(cfg, n), synth.CONFIGS[cfg]


@pytest.mark.parametrize("cfg,G,ask,ran", CASES)
def test_variant_global_step(R, cfg, G, ask, ran):
    _say("variant", cfg, "G", G, "placement", ask)
    n = 24 if cfg == "c4" else 48
    m, st, c = _mech_states(cfg, n)
    gm = R.Mechanism(m)
    res = {}
    for pl in sorted({ask, R.PARAMS_LDS}):
        T, Y = st["T"].copy(), st["Y"].copy()
        out = R.integrate(gm, T, st["P"], Y, c["dt"], c["rtol"], c["atol"], lanes_per_cell=G,
                          param_placement=pl, counters=True, stats=True)
        res[pl] = (T, Y, out)
    T, Y, out = res[ask]
    assert out["stats"]["lanes_per_cell"] == G
    assert out["stats"]["param_placement"] == ran
    assert res[R.PARAMS_LDS][2]["stats"]["param_placement"] == R.PARAMS_LDS
    Tl, Yl, ol = res[R.PARAMS_LDS]
    assert np.array_equal(T, Tl) and np.array_equal(Y, Yl)
    assert np.array_equal(out["counters"], ol["counters"])
    To, Yo, co = O.Model(m).integrate(st["T"], st["P"], st["Y"], c["dt"], c["rtol"], c["atol"],
                                      threads=THREADS)
    assert (out["status"] == 0).all() and (co["status"] == 0).all()
    rep = PT.check(T, Y, out["counters"], To, Yo, co, c["rtol"], c["atol"],
                   PT.max_flips(cfg, n), long_set=cfg in PT.LONG_SETS)
    _say(rep)
