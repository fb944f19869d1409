"""Host test of the server's scheduling core with a fake backend (no device):
compiles tests/server_core_test.cpp with g++ against the core header and runs
it.  Also the server ABI's argument checks that need no device."""
import ctypes as ct
import os
import re
import shutil
import subprocess

import pytest

from paper_1309_2710_amd import rkc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_core_with_fake_backend(tmp_path):
    exe = str(tmp_path / "server_core_test")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I" + os.path.join(ROOT, "include"),
                    "-I" + os.path.join(ROOT, "paper_1309_2710_amd", "csrc"),
                    os.path.join(ROOT, "tests", "server_core_test.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout


def test_server_header_matches_binding():
    txt = open(os.path.join(ROOT, "include", "rkc_server.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    declared = sorted(set(re.findall(r"\b(rkc_server_[a-z_]+)\s*\(", txt)))
    assert declared == sorted(rkc.SERVER_EXPORTED)
    L = rkc.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_server_rejects_bad_options_without_a_device():
    L = rkc.lib()
    assert L.rkc_server_opts_default(None) == rkc.EINVAL
    o = rkc.ServerOpts()
    assert L.rkc_server_opts_default(ct.byref(o)) == rkc.OK
    assert (o.budget_bytes, o.n_streams, o.max_batch_cells) == (1 << 30, 4, 1 << 20)
    h = ct.c_void_p()
    for field, bad in [("n_streams", 0), ("n_streams", 17), ("budget_bytes", 1000),
                       ("max_batch_cells", 0), ("lanes_per_cell", 12), ("param_placement", 4)]:
        b = rkc.ServerOpts()
        L.rkc_server_opts_default(ct.byref(b))
        setattr(b, field, bad)
        assert L.rkc_server_create(ct.byref(b), ct.byref(h)) == rkc.EINVAL, field
    assert L.rkc_server_destroy(None) == rkc.OK
    assert L.rkc_server_poll(None, 1, None) == rkc.EINVAL
    assert L.rkc_server_wait(None, 1, None) == rkc.EINVAL
