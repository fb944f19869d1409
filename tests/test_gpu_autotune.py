"""The autotuner only chooses options that never change results: a run with
its choice equals the default run bit for bit, and the inputs it timed on are
left unchanged."""
import numpy as np
import pytest

from paper_1309_2710_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_1309_2710_amd import rkc
    rkc.lib()
    return rkc


@pytest.mark.parametrize("cfg,n", [("c2", 3000), ("c3", 1500)])
def test_autotuned_options_keep_results(R, cfg, n):
    print("[case] autotune", cfg, n, flush=True)
    c = synth.CONFIGS[cfg]
    gm = R.Mechanism(synth.config_mechanism(cfg))
    st = synth.config_states(cfg, n)
    T0, Y0 = st["T"].copy(), st["Y"].copy()
    kw, ms = R.autotune(gm, st["T"], st["P"], st["Y"], c["dt"], c["rtol"], c["atol"])
    print("[case] tuned", kw, ms, flush=True)
    assert np.array_equal(st["T"], T0) and np.array_equal(st["Y"], Y0)
    assert ms > 0 and kw["schedule"] in (R.SCHED_PLAIN, R.SCHED_PERSISTENT)
    assert kw["block_groups"] >= 1
    Ta, Ya = st["T"].copy(), st["Y"].copy()
    R.integrate(gm, Ta, st["P"], Ya, c["dt"], c["rtol"], c["atol"])
    Tb, Yb = st["T"].copy(), st["Y"].copy()
    R.integrate(gm, Tb, st["P"], Yb, c["dt"], c["rtol"], c["atol"], **kw)
    assert np.array_equal(Ta, Tb) and np.array_equal(Ya, Yb)
