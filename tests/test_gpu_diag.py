"""GPU diagnostics: the divergence measure D (Sec. 3.1) computed by the
library against its plain definition, and the issued-evaluation counter of the
lane-group loop against the per-cell work it must equal."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1309_2710_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_1309_2710_amd import rkc
    rkc.lib()
    return rkc


def _say(*a):
    print("[case]", *a, flush=True)


def _run(R, cfg, n, **kw):
    m = R.Mechanism(synth.config_mechanism(cfg))
    c = synth.CONFIGS[cfg]
    st = synth.config_states(cfg, n)
    T, Y = st["T"].copy(), st["Y"].copy()
    out = R.integrate(m, T, st["P"], Y, c["dt"], c["rtol"], c["atol"], counters=True,
                      stats=True, **kw)
    return out


@pytest.mark.parametrize("width", [32, 64, 7])
def test_divergence_matches_definition(R, width):
    import torch
    _say("divergence c2 700 width", width)
    out = _run(R, "c2", 700, lanes_per_cell=16)
    cn = out["counters"]
    ref = O.divergence(cn[:, R.COUNTER_FIELDS.index("n_rhs")], width)
    Dh = R.divergence(cn, width)                      # host arrays, counters row stride 8
    Dd = R.divergence(torch.from_numpy(cn).cuda(), width).cpu().numpy()
    Ds = R.divergence(np.ascontiguousarray(cn[:, 0]), width)
    assert np.array_equal(Dh, ref) and np.array_equal(Dd, ref) and np.array_equal(Ds, ref)
    _say("mean D", ref.mean())


@pytest.mark.parametrize("G", [64, 16])
def test_issued_slots_equal_per_wave_maximum_work(R, G):
    """Plain schedule: the groups of a wave hold consecutive cells and the wave
    loops until its slowest group is done, so the issued evaluations are
    (groups per wave) x (largest cell work) summed over waves."""
    _say("slots c2 700 G", G)
    out = _run(R, "c2", 700, lanes_per_cell=G, schedule=R.SCHED_PLAIN)
    d = out["counters"][:, 0].astype(np.int64)
    gpw = 64 // G
    want = sum(gpw * int(d[i:i + gpw].max()) for i in range(0, len(d), gpw))
    s = out["stats"]
    _say(s)
    assert s["n_rhs"] == d.sum()
    assert s["n_rhs_slots"] == want
    if G == 64:
        assert s["n_rhs_slots"] == s["n_rhs"]


def test_persistent_slots_bound(R):
    out = _run(R, "c2", 2000, lanes_per_cell=16)
    s = out["stats"]
    _say(s)
    assert s["n_rhs"] <= s["n_rhs_slots"]
