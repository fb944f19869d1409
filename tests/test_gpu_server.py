"""GPU tests of the integration server (include/rkc_server.h): every served
request must equal, bit for bit, a direct rkc_integrate call on the same cells
(a cell's result does not depend on the batch it runs in), whether it is
served alone or in a mix of concurrent requests from several threads; the
direct path itself is checked against the oracle on a sample."""
import threading

import numpy as np
import pytest

from oracle import oracle as O
from paper_1309_2710_amd import synth
from tests import parity as PT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_1309_2710_amd import rkc
    rkc.lib()
    return rkc


def _say(*a):
    print("[case]", *a, flush=True)


MECHS = [("c2", synth.config_mechanism("c2")), ("c3", synth.config_mechanism("c3"))]


def _states(cfg, n, seed):
    c = synth.CONFIGS[cfg]
    return synth.make_states(synth.config_mechanism(cfg), n, seed, T_dist=c["T"], P_dist=c["P"],
                             Y_dist=c["Y"])


def _direct(R, gm, st, dt, c):
    T, Y = st["T"].copy(), st["Y"].copy()
    out = R.integrate(gm, T, st["P"], Y, dt, c["rtol"], c["atol"])
    return T, Y, out["status"]


def test_served_equals_direct_and_oracle(R):
    _say("server c2 + c3 mix")
    srv = R.Server(budget_bytes=256 << 20, n_streams=4)
    ids = [srv.register(m) for _, m in MECHS]
    gms = [R.Mechanism(m) for _, m in MECHS]
    reqs = []
    rng = np.random.default_rng(5)
    for k in range(10):
        which = k % 2
        cfg = MECHS[which][0]
        n = int(rng.integers(1, 700))
        dt = 1e-6 if k % 3 else 2e-6
        st = _states(cfg, n, 900 + k)
        T, Y = st["T"].copy(), st["Y"].copy()
        status = np.full(n, -7, np.int32)
        rid = srv.submit(ids[which], T, st["P"], Y, dt, synth.CONFIGS[cfg]["rtol"],
                         synth.CONFIGS[cfg]["atol"], status=status)
        reqs.append((which, cfg, st, dt, T, Y, status, rid))
    for which, cfg, st, dt, T, Y, status, rid in reqs:
        rc, nf = srv.wait(rid)
        assert rc == R.OK and nf == 0
        Td, Yd, sd = _direct(R, gms[which], st, dt, synth.CONFIGS[cfg])
        assert np.array_equal(T, Td) and np.array_equal(Y, Yd) and np.array_equal(status, sd)
    s = srv.stats()
    _say(s)
    assert s["submitted"] == s["completed"] == 10 and s["failed_requests"] == 0
    assert 1 <= s["launches"] <= 10
    assert s["cells"] == sum(r[2]["T"].shape[0] for r in reqs)
    assert s["n_rhs"] > 0 and 0 < s["p50_ms"] <= s["p99_ms"] <= s["max_ms"]
    assert s["peak_bytes"] <= 256 << 20
    # the direct path against the oracle on one request
    which, cfg, st, dt, T, Y, status, rid = reqs[0]
    om = O.Model(MECHS[which][1])
    c = synth.CONFIGS[cfg]
    To, Yo, co = om.integrate(st["T"], st["P"], st["Y"], dt, c["rtol"], c["atol"], threads=16)
    err = PT.rel_err(T, Y, To, Yo)
    # an adaptive step decision may flip in a few cells (see tests/parity.py)
    assert (err > PT.TOL).sum() <= max(1, len(err) // 100)
    srv.close()


def test_alone_versus_mix_from_threads(R):
    _say("server alone vs mix")
    c = synth.CONFIGS["c3"]
    probe = _states("c3", 300, 4242)
    srv = R.Server(budget_bytes=64 << 20, n_streams=3, max_batch_cells=2000)
    ids = [srv.register(m) for _, m in MECHS]
    T1, Y1 = probe["T"].copy(), probe["Y"].copy()
    rc, _ = srv.wait(srv.submit(ids[1], T1, probe["P"], Y1, c["dt"], c["rtol"], c["atol"]))
    assert rc == R.OK

    T2, Y2 = probe["T"].copy(), probe["Y"].copy()
    errors = []

    def worker(seed):
        try:
            rng = np.random.default_rng(seed)
            mine = []
            for k in range(6):
                which = int(rng.integers(2))
                cfg = MECHS[which][0]
                st = _states(cfg, int(rng.integers(50, 900)), seed * 100 + k)
                T, Y = st["T"].copy(), st["Y"].copy()
                mine.append(srv.submit(ids[which], T, st["P"], Y, synth.CONFIGS[cfg]["dt"],
                                       synth.CONFIGS[cfg]["rtol"], synth.CONFIGS[cfg]["atol"]))
                mine.append((T, Y, st))
            for rid in mine[::2]:
                rc, nf = srv.wait(rid)
                assert rc == R.OK
        except Exception as e:   # surfaced below
            errors.append(e)

    th = [threading.Thread(target=worker, args=(s,)) for s in (1, 2, 3)]
    for t in th:
        t.start()
    rid = srv.submit(ids[1], T2, probe["P"], Y2, c["dt"], c["rtol"], c["atol"])
    for t in th:
        t.join()
    rc, _ = srv.wait(rid)
    assert not errors, errors
    assert rc == R.OK
    assert np.array_equal(T1, T2) and np.array_equal(Y1, Y2)
    s = srv.stats()
    _say(s)
    assert s["completed"] == s["submitted"] == 20
    srv.close()


def test_small_budget_queues_requests(R):
    _say("server small budget")
    c = synth.CONFIGS["c3"]
    srv = R.Server(budget_bytes=1 << 20, n_streams=4)
    mid = srv.register(MECHS[1][1])
    gm = R.Mechanism(MECHS[1][1])
    sts = [_states("c3", 1500, 77 + k) for k in range(4)]   # ~0.7 MB each: one at a time
    outs = []
    for st in sts:
        T, Y = st["T"].copy(), st["Y"].copy()
        outs.append((srv.submit(mid, T, st["P"], Y, c["dt"], c["rtol"], c["atol"]), T, Y, st))
    with pytest.raises(R.RkcError):
        big = _states("c3", 4000, 1)
        srv.submit(mid, big["T"].copy(), big["P"], big["Y"].copy(), c["dt"])
    for rid, T, Y, st in outs:
        assert srv.wait(rid)[0] == R.OK
        Td, Yd, _ = _direct(R, gm, st, c["dt"], c)
        assert np.array_equal(T, Td) and np.array_equal(Y, Yd)
    s = srv.stats()
    _say(s)
    assert s["launches"] == 4 and s["peak_bytes"] <= 1 << 20
    srv.close()
