"""CPU checks of the C ABI library: it loads, exports every function that
include/rkc.h declares, and rejects bad arguments before touching a device."""
import ctypes as ct
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1309_2710_amd import rkc, synth

HDR = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "rkc.h")


def _declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rkc_[a-z_]+)\s*\(", txt)))


def test_header_declares_expected_entry_points():
    assert _declared() == sorted(rkc.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = rkc.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_defaults_and_strings():
    o = rkc.Opts()
    assert rkc.lib().rkc_opts_default(ct.byref(o)) == rkc.OK
    assert (o.method, o.s_max, o.max_steps, o.schedule, o.device_ptrs) == (0, 1000, 1000000, 0, 0)
    assert rkc.lib().rkc_opts_default(None) == rkc.EINVAL
    for code in (0, -1, -2, -3, -4, -5):
        assert rkc.strerror(code) not in ("", "unknown error")
    assert rkc.strerror(-99) == "unknown error"


def _desc_arrays(m):
    keep = {k: np.ascontiguousarray(m[k], np.int32 if k in ("reac", "prod") else np.float64)
            for k in ["W", "nasa_low", "nasa_high", "T_mid", "reac", "prod", "A", "beta", "Ea"]}
    return keep


def _create(m, **over):
    keep = _desc_arrays(m)
    keep.update(over)
    d = rkc.MechDesc(m["n_species"], m["n_reactions"],
                     *[rkc._np_ptr(keep[k]) for k in ["W", "nasa_low", "nasa_high", "T_mid",
                                                       "reac", "prod", "A", "beta", "Ea"]])
    h = ct.c_void_p()
    return rkc.lib().rkc_mech_create(ct.byref(d), ct.byref(h))


def test_mech_create_rejects_bad_descriptions_without_a_device():
    m = synth.config_mechanism("c1")
    L = rkc.lib()
    h = ct.c_void_p()
    assert L.rkc_mech_create(None, ct.byref(h)) == rkc.EINVAL
    bad = np.array(m["reac"], np.int32); bad[0, 0] = 9
    assert _create(m, reac=bad) == rkc.EINVAL
    bad = np.array(m["prod"], np.int32); bad[1, 1] = -2
    assert _create(m, prod=bad) == rkc.EINVAL
    w = np.array(m["W"]); w[0] = 0.0
    assert _create(m, W=w) == rkc.EINVAL
    a = np.array(m["A"]); a[2] = -1.0
    assert _create(m, A=a) == rkc.EINVAL
    e = np.array(m["Ea"]); e[3] = np.nan
    assert _create(m, Ea=e) == rkc.EINVAL
    # temperature exponents beyond 1e5 in magnitude (the kernels bound 1/T in
    # the Arrhenius factors by a value that needs |beta| <= 1e5)
    b = np.array(m["beta"]); b[4] = 2e5
    assert _create(m, beta=b) == rkc.EINVAL
    b = np.array(m["beta"]); b[4] = -np.inf
    assert _create(m, beta=b) == rkc.EINVAL
    d = rkc.MechDesc(1022, 0, *[None] * 9)
    assert L.rkc_mech_create(ct.byref(d), ct.byref(h)) == rkc.ENOTSUP
    d = rkc.MechDesc(0, 0, *[None] * 9)
    assert L.rkc_mech_create(ct.byref(d), ct.byref(h)) == rkc.EINVAL


def test_integrate_rejects_bad_arguments_without_a_device():
    L = rkc.lib()
    x = np.zeros(4)
    assert L.rkc_integrate(None, 4, rkc._np_ptr(x), rkc._np_ptr(x), rkc._np_ptr(x), 1e-6, 1e-6,
                           1e-10, None, None, None) == rkc.EINVAL
    assert L.rkc_rhs(None, 4, None, None, None, None, None) == rkc.EINVAL
    assert L.rkc_mech_destroy(None) == rkc.OK
    assert L.rkc_mech_info(None, None, None, None, None) == rkc.EINVAL


def test_binding_rejects_species_count_mismatch():
    class FakeMech:
        n_species = 9
        handle = None
    T = np.full(4, 1200.0)
    P = np.full(4, 1e5)
    with pytest.raises(ValueError):
        rkc.integrate(FakeMech(), T, P, np.zeros((4, 8)), 1e-6)
    with pytest.raises(ValueError):
        rkc.integrate(FakeMech(), T, np.full(3, 1e5), np.zeros((4, 9)), 1e-6)
    with pytest.raises(ValueError):
        rkc.rhs(FakeMech(), T, P, np.zeros((4, 10)))


def test_mech_create_rejects_bad_pressure_dependence_without_a_device():
    from tests.test_oracle_pdep import _pdep
    from tests import mechs
    L = rkc.lib()
    for kinds, troe in (([7], None), ([3], [[0.5, 0.0, 100.0, 0.0]]), ([3], [[0.5, 100.0, -1.0, 0.0]])):
        m = _pdep(mechs.a_to_b(1e5, 10.0), kinds, k0=[1e10], troe=troe)
        d, keep = rkc._mech_desc(m)
        h = ct.c_void_p()
        assert L.rkc_mech_create(ct.byref(d), ct.byref(h)) == rkc.EINVAL
    m = _pdep(mechs.a_to_b(1e5, 10.0), [1], eff=[[1.0, -0.5]])
    d, keep = rkc._mech_desc(m)
    h = ct.c_void_p()
    assert L.rkc_mech_create(ct.byref(d), ct.byref(h)) == rkc.EINVAL


def test_binding_rejects_arrays_the_abi_cannot_take():
    """Bare pointers carry no type or layout: the binding refuses, before any
    call, what the kernels would misread (wrong dtype, strided, wrong rank)."""
    class FakeMech:
        n_species = 3
        handle = None
    T = np.full(4, 1200.0)
    P = np.full(4, 1e5)
    Y = np.full((4, 3), 1.0 / 3.0)
    with pytest.raises(TypeError):
        rkc.integrate(FakeMech(), T.astype(np.float32), P, Y, 1e-6)
    with pytest.raises(TypeError):
        rkc.integrate(FakeMech(), T, P, np.asfortranarray(np.full((4, 3), 0.5)), 1e-6)
    with pytest.raises(TypeError):
        rkc.integrate(FakeMech(), T, P, [[0.5] * 3] * 4, 1e-6)
    with pytest.raises(ValueError):
        rkc.integrate(FakeMech(), np.full((4, 1), 1200.0), P, Y, 1e-6)
    with pytest.raises(TypeError):
        rkc.divergence(np.zeros(8, np.int64))


def test_binding_constants_match_the_header():
    txt = open(HDR).read()
    assert int(re.search(r"#define RKC_MAX_CELLS (\d+)", txt).group(1)) == rkc.MAX_CELLS == 2**31 - 2**20
    assert int(re.search(r"#define RKC_NCOUNTERS (\d+)", txt).group(1)) == rkc.NCOUNTERS


def test_every_mirrored_constant_matches_the_header():
    """Each RKC_<NAME> / RKC_SERVER_<NAME> define whose <NAME> the binding
    mirrors has the header's value."""
    txt = open(HDR).read()
    n = 0
    for name, val in re.findall(r"#define RKC_(\w+)\s+\(?(-?\d+)\)?", txt):
        if hasattr(rkc, name):
            assert getattr(rkc, name) == int(val), name
            n += 1
    for name, val in re.findall(r"RKC_(CNT_\w+) = (\d+)", txt):
        n += 1
        assert rkc.COUNTER_FIELDS[int(val)] is not None
    assert n >= 20


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes structures of the binding have the header's field offsets
    and sizes (a C program built against include/rkc.h prints them)."""
    structs = {"rkc_opts": rkc.Opts, "rkc_stats": rkc.Stats, "rkc_mech_desc": rkc.MechDesc}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rkc.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HDR), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(l.rsplit(" ", 1) for l in out if l.strip())
    for cname, cls in structs.items():
        assert int(got[cname + " size"]) == ct.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got[cname + "." + f]) == getattr(cls, f).offset, (cname, f)
