"""A recorded global step (rkc_graph_create) replayed several times, with
eager work and synchronisations between the replays: every replay must equal,
bit for bit, the eager rkc_integrate call it stands for."""
import numpy as np
import pytest

from paper_1309_2710_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_1309_2710_amd import rkc
    rkc.lib()
    return rkc


@pytest.mark.parametrize("cfg,n,G", [("c1", 1024, 16), ("c3", 600, 64)])
def test_graph_replays_equal_eager_steps(R, cfg, n, G):
    import torch
    print("[case] graph", cfg, n, G, flush=True)
    c = synth.CONFIGS[cfg]
    gm = R.Mechanism(synth.config_mechanism(cfg))
    st = synth.config_states(cfg, n)
    dev = torch.device("cuda:0")
    P = torch.from_numpy(st["P"]).to(dev)
    # eager reference: three consecutive global steps
    Te, Ye = torch.from_numpy(st["T"]).to(dev), torch.from_numpy(st["Y"]).to(dev)
    ref = []
    for _ in range(3):
        R.integrate(gm, Te, P, Ye, c["dt"], c["rtol"], c["atol"], lanes_per_cell=G)
        torch.cuda.synchronize()
        ref.append((Te.cpu().numpy().copy(), Ye.cpu().numpy().copy()))
    # graph over its own buffers
    Tg, Yg = torch.from_numpy(st["T"]).to(dev), torch.from_numpy(st["Y"]).to(dev)
    status = torch.full((n,), -1, dtype=torch.int32, device=dev)
    g = R.Graph(gm, Tg, P, Yg, c["dt"], c["rtol"], c["atol"], lanes_per_cell=G, status=status)
    for k in range(3):
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(Tg.cpu().numpy(), ref[k][0]), k
        assert np.array_equal(Yg.cpu().numpy(), ref[k][1]), k
        assert (status.cpu().numpy() == 0).all()
        _ = (Yg * 2.0).sum().item()   # unrelated eager work between replays
    # restart from the initial state with an eager copy, replay once more
    Tg.copy_(torch.from_numpy(st["T"]).to(dev))
    Yg.copy_(torch.from_numpy(st["Y"]).to(dev))
    g.launch()
    torch.cuda.synchronize()
    assert np.array_equal(Tg.cpu().numpy(), ref[0][0]) and np.array_equal(Yg.cpu().numpy(), ref[0][1])
    g.close()


def test_graph_rejects_host_arrays(R):
    import ctypes as ct
    gm = R.Mechanism(synth.config_mechanism("c1"))
    T = np.full(4, 1200.0)
    o = R.make_opts()
    h = ct.c_void_p()
    rc = R.lib().rkc_graph_create(gm.handle, 4, R._np_ptr(T), R._np_ptr(T), R._np_ptr(T), 1e-6,
                                  1e-6, 1e-10, ct.byref(o), None, ct.byref(h))
    assert rc == R.EINVAL
