"""ctypes front end of the serial FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline leg of bench.py.  The product path never loads it.  It takes the
mechanism arrays as plain numpy arrays (the dict layout of the synthetic
generator) and shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

from . import build as _build

OK, UNDERFLOW, MAXSTEPS, NONFINITE, BADINPUT = 0, 1, 2, 3, 4
RKC, RKCK = 0, 1

_lib = None


class _Mech(ct.Structure):
    _fields_ = [("n_species", ct.c_int), ("n_reactions", ct.c_int),
                ("W", ct.c_void_p), ("nasa_low", ct.c_void_p), ("nasa_high", ct.c_void_p),
                ("T_mid", ct.c_void_p), ("reac", ct.c_void_p), ("prod", ct.c_void_p),
                ("A", ct.c_void_p), ("beta", ct.c_void_p), ("Ea", ct.c_void_p),
                ("pdep", ct.c_void_p), ("eff", ct.c_void_p), ("A0", ct.c_void_p),
                ("beta0", ct.c_void_p), ("Ea0", ct.c_void_p), ("troe", ct.c_void_p)]


class Counters(ct.Structure):
    _fields_ = [("n_rhs", ct.c_int32), ("n_steps", ct.c_int32), ("n_reject", ct.c_int32),
                ("n_sigma", ct.c_int32), ("s_max_used", ct.c_int32), ("s_hash", ct.c_int32),
                ("status", ct.c_int32), ("n_power_iter", ct.c_int32)]


COUNTER_FIELDS = [f[0] for f in Counters._fields_]


class Step(ct.Structure):
    _fields_ = [("t", ct.c_double), ("h", ct.c_double), ("err", ct.c_double),
                ("sigma", ct.c_double), ("y", ct.c_double * 3), ("s", ct.c_int32),
                ("new_sigma", ct.c_int32), ("accepted", ct.c_int32), ("pad", ct.c_int32)]


def _declare(L):
    """Argument and result types of the library's entry points."""
    L.orc_model_create.restype = ct.c_void_p
    L.orc_model_create.argtypes = [ct.POINTER(_Mech)]
    L.orc_model_destroy.argtypes = [ct.c_void_p]
    L.orc_rhs.argtypes = [ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_void_p]
    L.orc_rkc_coeffs.argtypes = [ct.c_int] + [ct.c_void_p] * 4
    L.orc_rkc_fixed_step.argtypes = [ct.c_void_p, ct.c_double, ct.c_void_p, ct.c_double,
                                     ct.c_int]
    L.orc_rkck_fixed_step.argtypes = [ct.c_void_p, ct.c_double, ct.c_void_p, ct.c_double,
                                      ct.c_void_p]
    L.orc_sigma.restype = ct.c_double
    L.orc_sigma.argtypes = [ct.c_void_p, ct.c_double, ct.c_void_p, ct.POINTER(ct.c_int)]
    L.orc_cell_trace.restype = ct.c_int
    L.orc_cell_trace.argtypes = [ct.c_void_p, ct.c_int, ct.c_double, ct.c_void_p,
                                 ct.c_double, ct.c_double, ct.c_double, ct.c_int, ct.c_int,
                                 ct.c_void_p, ct.c_void_p, ct.c_int, ct.POINTER(ct.c_int)]
    L.orc_integrate.argtypes = [ct.c_void_p, ct.c_int, ct.c_int, ct.c_void_p, ct.c_void_p,
                                ct.c_void_p, ct.c_double, ct.c_double, ct.c_double,
                                ct.c_int, ct.c_int, ct.c_void_p, ct.c_int]
    return L


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        _lib = _declare(ct.CDLL(path))
    return _lib


def load_variant(path):
    """A separately built copy of the oracle library (tests that plant a
    mistake, or change one rounding, in a copy of the source)."""
    return _declare(ct.CDLL(path))


def _p(a):
    return a.ctypes.data_as(ct.c_void_p)


class Model:
    """A mechanism loaded into the oracle (holds references to its arrays)."""

    def __init__(self, mech, library=None):
        L = library if library is not None else lib()
        self._L = L
        self.n_species = int(mech["n_species"])
        self.n_reactions = int(mech["n_reactions"])
        self._keep = {
            "W": np.ascontiguousarray(mech["W"], dtype=np.float64),
            "nasa_low": np.ascontiguousarray(mech["nasa_low"], dtype=np.float64),
            "nasa_high": np.ascontiguousarray(mech["nasa_high"], dtype=np.float64),
            "T_mid": np.ascontiguousarray(mech["T_mid"], dtype=np.float64),
            "reac": np.ascontiguousarray(mech["reac"], dtype=np.int32),
            "prod": np.ascontiguousarray(mech["prod"], dtype=np.int32),
            "A": np.ascontiguousarray(mech["A"], dtype=np.float64),
            "beta": np.ascontiguousarray(mech["beta"], dtype=np.float64),
            "Ea": np.ascontiguousarray(mech["Ea"], dtype=np.float64),
        }
        opt = {}
        if mech.get("pdep") is not None:
            opt = {"pdep": np.ascontiguousarray(mech["pdep"], dtype=np.int32),
                   "eff": np.ascontiguousarray(mech["eff"], dtype=np.float64),
                   "A0": np.ascontiguousarray(mech["A0"], dtype=np.float64),
                   "beta0": np.ascontiguousarray(mech["beta0"], dtype=np.float64),
                   "Ea0": np.ascontiguousarray(mech["Ea0"], dtype=np.float64),
                   "troe": np.ascontiguousarray(mech["troe"], dtype=np.float64)}
        self._keep.update(opt)
        k = self._keep
        pd = [_p(k[x]) if x in k else None for x in ("pdep", "eff", "A0", "beta0", "Ea0", "troe")]
        self._m = _Mech(self.n_species, self.n_reactions, _p(k["W"]), _p(k["nasa_low"]),
                        _p(k["nasa_high"]), _p(k["T_mid"]), _p(k["reac"]), _p(k["prod"]),
                        _p(k["A"]), _p(k["beta"]), _p(k["Ea"]), *pd)
        self._h = L.orc_model_create(ct.byref(self._m))

    def __del__(self):
        if getattr(self, "_h", None) and getattr(self, "_L", None) is not None:
            self._L.orc_model_destroy(self._h)
            self._h = None

    @property
    def N(self):
        return self.n_species + 1

    def rhs(self, T, P, Y):
        """f(y) for cells: returns [n][N] with column 0 = dT/dt, 1.. = dY/dt."""
        T = np.atleast_1d(np.asarray(T, dtype=np.float64))
        n = T.shape[0]
        y = np.empty((n, self.N))
        y[:, 0] = T
        y[:, 1:] = np.asarray(Y, dtype=np.float64).reshape(n, self.n_species)
        P = np.ascontiguousarray(np.broadcast_to(np.asarray(P, dtype=np.float64), (n,)))
        f = np.empty_like(y)
        self._L.orc_rhs(self._h, n, _p(P), _p(y), _p(f))
        return f

    def integrate(self, T, P, Y, dt, rtol=1e-6, atol=1e-10, method=RKC, s_max=1000,
                  max_steps=1000000, threads=None):
        """Returns (T_out, Y_out, counters structured array)."""
        T = np.array(T, dtype=np.float64, copy=True).reshape(-1)
        n = T.shape[0]
        Y = np.array(Y, dtype=np.float64, copy=True).reshape(n, self.n_species)
        P = np.ascontiguousarray(np.broadcast_to(np.asarray(P, dtype=np.float64), (n,)))
        cnt = (Counters * max(n, 1))()
        if threads is None:
            threads = min(os.cpu_count() or 1, 16)
        self._L.orc_integrate(self._h, int(method), n, _p(P), _p(T), _p(Y), float(dt),
                            float(rtol), float(atol), int(s_max), int(max_steps),
                            ct.cast(cnt, ct.c_void_p), int(threads))
        arr = np.ctypeslib.as_array(cnt)[:n]
        c = {f: np.array([getattr(x, f) for x in cnt[:n]], dtype=np.int64) for f in COUNTER_FIELDS}
        return T, Y, c

    def trace(self, y, P, dt, rtol=1e-6, atol=1e-10, method=RKC, s_max=1000,
              max_steps=1000000, cap=200000):
        """One cell (y = [T, Y...]) integrated over [0, dt] with every attempted
        step recorded.  Returns (y_out, counters dict, steps dict of arrays:
        t, h, err, sigma, y [n][3], s, new_sigma, accepted)."""
        y = np.array(y, dtype=np.float64, copy=True).reshape(-1)
        assert y.shape[0] == self.N
        buf = (Step * cap)()
        cnt = Counters()
        n = ct.c_int(0)
        self._L.orc_cell_trace(self._h, int(method), float(P), _p(y), float(dt), float(rtol),
                             float(atol), int(s_max), int(max_steps), ct.byref(cnt),
                             ct.cast(buf, ct.c_void_p), int(cap), ct.byref(n))
        m = min(n.value, cap)
        steps = {f: np.array([getattr(buf[i], f) for i in range(m)])
                 for f in ("t", "h", "err", "sigma", "s", "new_sigma", "accepted")}
        steps["y"] = np.array([list(buf[i].y) for i in range(m)]).reshape(m, 3)
        steps["accepted"] = steps["accepted"].astype(bool)
        steps["new_sigma"] = steps["new_sigma"].astype(bool)
        return y, {f: getattr(cnt, f) for f in COUNTER_FIELDS}, steps

    def rkc_fixed_step(self, y, P, h, s):
        y = np.array(y, dtype=np.float64, copy=True)
        self._L.orc_rkc_fixed_step(self._h, float(P), _p(y), float(h), int(s))
        return y

    def rkck_fixed_step(self, y, P, h):
        y = np.array(y, dtype=np.float64, copy=True)
        y4 = np.empty_like(y)
        self._L.orc_rkck_fixed_step(self._h, float(P), _p(y), float(h), _p(y4))
        return y, y4

    def sigma(self, y, P):
        y = np.ascontiguousarray(y, dtype=np.float64)
        it = ct.c_int(0)
        s = self._L.orc_sigma(self._h, float(P), _p(y), ct.byref(it))
        return s, it.value


def rkc_coeffs(s):
    """(mu_t[1..s], mu[2..s], nu[2..s], gam_t[2..s]) as arrays indexed by j."""
    a = [np.zeros(s + 1) for _ in range(4)]
    lib().orc_rkc_coeffs(int(s), *[_p(x) for x in a])
    return tuple(a)


def divergence(d, width=32):
    """Divergence measure D of Sec. 3.1 for consecutive runs of `width` cells:
    the run's total work over (run length x its largest work); 1 for a run
    whose work is all zero.  Plain loops over the definition."""
    d = [int(x) for x in d]
    out = []
    for first in range(0, len(d), width):
        run = d[first:first + width]
        mx = max(run)
        out.append(1.0 if mx == 0 else float(sum(run)) / (float(len(run)) * float(mx)))
    return np.array(out, dtype=np.float64)
