"""Python binding of the C ABI in include/rkc.h (argument marshalling only).

Every step of the integration runs in the HIP library librkc.so; this module
only converts numpy arrays or torch tensors into pointers.  If the library is
missing the import of `lib()` fails loudly: there is no CPU fallback.

Arrays:
  numpy arrays      -> host pointers (the library stages them on the device)
  torch GPU tensors -> device pointers (work is enqueued on the tensor's
                       current stream, or on the stream passed explicitly)
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librkc.so")

OK, EINVAL, ENOMEM, EDEVICE, ECELLS, ENOTSUP = 0, -1, -2, -3, -4, -5
CELL_OK, CELL_UNDERFLOW, CELL_MAXSTEPS, CELL_NONFINITE, CELL_BADINPUT = 0, 1, 2, 3, 4
RKC, RKCK = 0, 1
SCHED_AUTO, SCHED_PLAIN, SCHED_PERSISTENT = 0, 1, 2
PARAMS_AUTO, PARAMS_REGISTERS, PARAMS_LDS, PARAMS_GLOBAL = 0, 1, 2, 3
COEFS_TABLE, COEFS_RECURRENCE = 0, 1
LAYOUT_CELL_MAJOR, LAYOUT_SPECIES_MAJOR = 0, 1
NCOUNTERS = 8
MAX_CELLS = 2146435072          # RKC_MAX_CELLS: largest n_cells of one call
COUNTER_FIELDS = ["n_rhs", "n_steps", "n_reject", "n_sigma", "s_max_used", "s_hash", "status",
                  "n_power_iter"]

EXPORTED = ["rkc_opts_default", "rkc_mech_create", "rkc_mech_destroy", "rkc_mech_info",
            "rkc_rhs", "rkc_integrate", "rkc_integrate_device_noalloc", "rkc_autotune",
            "rkc_divergence", "rkc_graph_create", "rkc_graph_launch", "rkc_graph_destroy",
            "rkc_strerror"]
SERVER_EXPORTED = ["rkc_server_opts_default", "rkc_server_create", "rkc_server_destroy",
                   "rkc_server_register_mech", "rkc_server_submit", "rkc_server_poll",
                   "rkc_server_wait", "rkc_server_get_stats", "rkc_server_reset_stats"]


class MechDesc(ct.Structure):
    _fields_ = [("n_species", ct.c_int32), ("n_reactions", ct.c_int32),
                ("W", ct.c_void_p), ("nasa_low", ct.c_void_p), ("nasa_high", ct.c_void_p),
                ("T_mid", ct.c_void_p), ("reac", ct.c_void_p), ("prod", ct.c_void_p),
                ("A", ct.c_void_p), ("beta", ct.c_void_p), ("Ea", ct.c_void_p),
                ("pdep", ct.c_void_p), ("eff", ct.c_void_p), ("A0", ct.c_void_p),
                ("beta0", ct.c_void_p), ("Ea0", ct.c_void_p), ("troe", ct.c_void_p)]


PDEP_PLAIN, PDEP_THIRD_BODY, PDEP_LINDEMANN, PDEP_TROE = 0, 1, 2, 3


class Opts(ct.Structure):
    _fields_ = [("method", ct.c_int32), ("s_max", ct.c_int32), ("max_steps", ct.c_int32),
                ("lanes_per_cell", ct.c_int32), ("schedule", ct.c_int32),
                ("block_groups", ct.c_int32), ("grid_blocks", ct.c_int32),
                ("device_ptrs", ct.c_int32), ("stream", ct.c_void_p),
                ("cell_counters", ct.c_void_p), ("param_placement", ct.c_int32),
                ("stage_coefs", ct.c_int32), ("layout", ct.c_int32)]


class Stats(ct.Structure):
    _fields_ = [("n_rhs", ct.c_int64), ("n_steps", ct.c_int64), ("n_reject", ct.c_int64),
                ("n_sigma", ct.c_int64), ("n_power_iter", ct.c_int64),
                ("s_max_used", ct.c_int32), ("n_failed", ct.c_int32),
                ("worst_status", ct.c_int32), ("lanes_per_cell", ct.c_int32),
                ("schedule", ct.c_int32), ("grid_blocks", ct.c_int32),
                ("block_threads", ct.c_int32), ("lds_bytes", ct.c_int32),
                ("n_rhs_slots", ct.c_int64), ("param_placement", ct.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerOpts(ct.Structure):
    _fields_ = [("budget_bytes", ct.c_size_t), ("n_streams", ct.c_int32),
                ("max_batch_cells", ct.c_int32), ("lanes_per_cell", ct.c_int32),
                ("param_placement", ct.c_int32)]


class ServerStats(ct.Structure):
    _fields_ = [("submitted", ct.c_int64), ("completed", ct.c_int64),
                ("failed_requests", ct.c_int64), ("launches", ct.c_int64), ("cells", ct.c_int64),
                ("n_rhs", ct.c_int64), ("peak_bytes", ct.c_int64), ("peak_queue", ct.c_int64),
                ("mean_ms", ct.c_double), ("p50_ms", ct.c_double), ("p99_ms", ct.c_double),
                ("max_ms", ct.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class RkcError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (what, strerror(code), code))


_lib = None


def lib():
    """The loaded librkc.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librkc.so not built: run __graft_entry__.build() "
                               "or python paper_1309_2710_amd/build.py")
        # torch ships its own HIP runtime under the same soname; loading it first
        # makes it the single runtime of the process, shared with this library
        # (device pointers and streams from torch are then valid here).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ct.CDLL(LIB_PATH)
        L.rkc_opts_default.argtypes = [ct.POINTER(Opts)]
        L.rkc_mech_create.argtypes = [ct.POINTER(MechDesc), ct.POINTER(ct.c_void_p)]
        L.rkc_mech_destroy.argtypes = [ct.c_void_p]
        L.rkc_mech_info.argtypes = [ct.c_void_p] + [ct.POINTER(ct.c_int32)] * 4
        L.rkc_rhs.argtypes = [ct.c_void_p, ct.c_size_t, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                              ct.c_void_p, ct.POINTER(Opts)]
        L.rkc_integrate.argtypes = [ct.c_void_p, ct.c_size_t, ct.c_void_p, ct.c_void_p,
                                    ct.c_void_p, ct.c_double, ct.c_double, ct.c_double,
                                    ct.POINTER(Opts), ct.c_void_p, ct.POINTER(Stats)]
        L.rkc_integrate_device_noalloc.argtypes = [ct.c_void_p, ct.c_size_t, ct.c_void_p,
                                                   ct.c_void_p, ct.c_void_p, ct.c_double,
                                                   ct.c_double, ct.c_double, ct.POINTER(Opts),
                                                   ct.c_void_p]
        L.rkc_divergence.argtypes = [ct.c_size_t, ct.c_void_p, ct.c_int32, ct.c_int32,
                                     ct.c_void_p, ct.POINTER(Opts)]
        L.rkc_autotune.argtypes = [ct.c_void_p, ct.c_size_t, ct.c_void_p, ct.c_void_p,
                                    ct.c_void_p, ct.c_double, ct.c_double, ct.c_double,
                                    ct.POINTER(Opts), ct.POINTER(Opts), ct.POINTER(ct.c_float)]
        L.rkc_graph_create.argtypes = [ct.c_void_p, ct.c_size_t, ct.c_void_p, ct.c_void_p,
                                        ct.c_void_p, ct.c_double, ct.c_double, ct.c_double,
                                        ct.POINTER(Opts), ct.c_void_p, ct.POINTER(ct.c_void_p)]
        L.rkc_graph_launch.argtypes = [ct.c_void_p, ct.c_void_p]
        L.rkc_graph_destroy.argtypes = [ct.c_void_p]
        L.rkc_server_opts_default.argtypes = [ct.POINTER(ServerOpts)]
        L.rkc_server_create.argtypes = [ct.POINTER(ServerOpts), ct.POINTER(ct.c_void_p)]
        L.rkc_server_destroy.argtypes = [ct.c_void_p]
        L.rkc_server_register_mech.argtypes = [ct.c_void_p, ct.POINTER(MechDesc),
                                               ct.POINTER(ct.c_int32)]
        L.rkc_server_submit.argtypes = [ct.c_void_p, ct.c_int32, ct.c_size_t, ct.c_void_p,
                                        ct.c_void_p, ct.c_void_p, ct.c_double, ct.c_double,
                                        ct.c_double, ct.c_int32, ct.c_void_p,
                                        ct.POINTER(ct.c_uint64)]
        L.rkc_server_poll.argtypes = [ct.c_void_p, ct.c_uint64, ct.POINTER(ct.c_int32)]
        L.rkc_server_wait.argtypes = [ct.c_void_p, ct.c_uint64, ct.POINTER(ct.c_int32)]
        L.rkc_server_get_stats.argtypes = [ct.c_void_p, ct.POINTER(ServerStats)]
        L.rkc_server_reset_stats.argtypes = [ct.c_void_p]
        L.rkc_strerror.restype = ct.c_char_p
        L.rkc_strerror.argtypes = [ct.c_int]
        _lib = L
    return _lib


def strerror(code):
    try:
        return lib().rkc_strerror(int(code)).decode()
    except RuntimeError:
        return "code %d" % code


def _np_ptr(a):
    return a.ctypes.data_as(ct.c_void_p)


def _mech_desc(mech):
    """(rkc_mech_desc, arrays it points into) for a mechanism dict."""
    nS, nR = int(mech["n_species"]), int(mech["n_reactions"])
    keep = {
        "W": np.ascontiguousarray(mech["W"], np.float64),
        "nasa_low": np.ascontiguousarray(mech["nasa_low"], np.float64),
        "nasa_high": np.ascontiguousarray(mech["nasa_high"], np.float64),
        "T_mid": np.ascontiguousarray(mech["T_mid"], np.float64),
        "reac": np.ascontiguousarray(mech["reac"], np.int32),
        "prod": np.ascontiguousarray(mech["prod"], np.int32),
        "A": np.ascontiguousarray(mech["A"], np.float64),
        "beta": np.ascontiguousarray(mech["beta"], np.float64),
        "Ea": np.ascontiguousarray(mech["Ea"], np.float64),
    }
    opt = [None] * 6
    if mech.get("pdep") is not None:
        keep.update(pdep=np.ascontiguousarray(mech["pdep"], np.int32),
                    eff=np.ascontiguousarray(mech["eff"], np.float64),
                    A0=np.ascontiguousarray(mech["A0"], np.float64),
                    beta0=np.ascontiguousarray(mech["beta0"], np.float64),
                    Ea0=np.ascontiguousarray(mech["Ea0"], np.float64),
                    troe=np.ascontiguousarray(mech["troe"], np.float64))
        opt = [_np_ptr(keep[k]) for k in ["pdep", "eff", "A0", "beta0", "Ea0", "troe"]]
    d = MechDesc(nS, nR, *[_np_ptr(keep[k]) for k in
                           ["W", "nasa_low", "nasa_high", "T_mid", "reac", "prod", "A",
                            "beta", "Ea"]], *opt)
    return d, keep


class Mechanism:
    """A mechanism uploaded to the current HIP device (rkc_mech_create)."""

    def __init__(self, mech):
        L = lib()
        nS, nR = int(mech["n_species"]), int(mech["n_reactions"])
        d, keep = _mech_desc(mech)
        h = ct.c_void_p()
        rc = L.rkc_mech_create(ct.byref(d), ct.byref(h))
        if rc != OK:
            raise RkcError(rc, "rkc_mech_create")
        self._h = h
        self.n_species = nS
        self.n_reactions = nR

    @property
    def handle(self):
        return self._h

    def info(self):
        v = [ct.c_int32() for _ in range(4)]
        rc = lib().rkc_mech_info(self._h, *[ct.byref(x) for x in v])
        if rc != OK:
            raise RkcError(rc, "rkc_mech_info")
        return dict(zip(["n_species", "n_reactions", "n_units", "nnz"], [x.value for x in v]))

    def close(self):
        if getattr(self, "_h", None):
            lib().rkc_mech_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _check_shapes(mech, n, P, Y, layout=LAYOUT_CELL_MAJOR):
    """The C ABI takes bare pointers: check here that P is [n] and Y is
    [n][n_species] of this mechanism ([n_species][n] for the species-major
    layout)."""
    want = (n, mech.n_species) if layout == LAYOUT_CELL_MAJOR else (mech.n_species, n)
    if tuple(P.shape) != (n,) or tuple(Y.shape) != want:
        raise ValueError("shape mismatch: T [%d], P %s, Y %s for a mechanism with %d species"
                         % (n, tuple(P.shape), tuple(Y.shape), mech.n_species))


def _check_arrays(arrays, int32=False):
    """Every array handed to the C ABI as a bare pointer: all numpy (host) or
    all torch tensors on one GPU, C-contiguous, float64 (int32 for counts).
    Raises TypeError/ValueError otherwise; returns True for torch tensors."""
    dev = _is_torch(arrays[0])
    if dev:
        import torch
        want = torch.int32 if int32 else torch.float64
        d0 = arrays[0].device
        for a in arrays:
            if not _is_torch(a) or not a.is_cuda or a.device != d0:
                raise TypeError("expected torch tensors on one GPU device")
            if a.dtype != want or not a.is_contiguous():
                raise TypeError("expected contiguous %s tensors" % want)
    else:
        want = np.int32 if int32 else np.float64
        for a in arrays:
            if not isinstance(a, np.ndarray):
                raise TypeError("expected numpy arrays (or torch GPU tensors)")
            if a.dtype != want or not a.flags.c_contiguous:
                raise TypeError("expected C-contiguous %s arrays" % np.dtype(want).name)
    return dev


def _check_T(T):
    if len(T.shape) != 1:
        raise ValueError("T must be one-dimensional [n_cells]")


def make_opts(method=RKC, s_max=1000, max_steps=1000000, lanes_per_cell=0,
              schedule=SCHED_AUTO, block_groups=0, grid_blocks=0, device_ptrs=False,
              stream=None, cell_counters=None, param_placement=PARAMS_AUTO,
              stage_coefs=0, layout=LAYOUT_CELL_MAJOR):
    o = Opts()
    lib().rkc_opts_default(ct.byref(o))
    o.method = int(method)
    o.s_max = int(s_max)
    o.max_steps = int(max_steps)
    o.lanes_per_cell = int(lanes_per_cell)
    o.schedule = int(schedule)
    o.block_groups = int(block_groups)
    o.grid_blocks = int(grid_blocks)
    o.device_ptrs = 1 if device_ptrs else 0
    o.stream = stream
    o.cell_counters = cell_counters
    o.param_placement = int(param_placement)
    o.stage_coefs = int(stage_coefs)
    o.layout = int(layout)
    return o


def _stream_handle(stream, tensors):
    if stream is not None:
        return ct.c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)
    import torch
    return ct.c_void_p(torch.cuda.current_stream(tensors[0].device).cuda_stream)


def integrate(mech, T, P, Y, dt, rtol=1e-6, atol=1e-10, method=RKC, lanes_per_cell=0,
              schedule=SCHED_AUTO, block_groups=0, grid_blocks=0, s_max=1000,
              max_steps=1000000, counters=False, status=True, stats=False, stream=None,
              check=True, param_placement=PARAMS_AUTO, stage_coefs=0,
              layout=LAYOUT_CELL_MAJOR):
    """Integrate cells over [0, dt] in place.

    numpy inputs: T [n] and Y [n][nS] ([nS][n] with layout=LAYOUT_SPECIES_MAJOR)
    are overwritten in place (must be C-contiguous float64).  torch GPU
    inputs: the same, on the device.  Returns dict with optional 'status' [n]
    int32, 'counters' [n][8] int32, 'stats' (dict), 'rc'.
    """
    L = lib()
    dev = _check_arrays([T, P, Y])
    _check_T(T)
    n = int(T.shape[0])
    _check_shapes(mech, n, P, Y, layout)
    out = {}
    if dev:
        import torch
        st_t = torch.empty(n, dtype=torch.int32, device=T.device) if status else None
        cn_t = torch.empty((n, NCOUNTERS), dtype=torch.int32, device=T.device) if counters else None
        ptrs = [ct.c_void_p(a.data_ptr()) for a in (T, P, Y)]
        sp = ct.c_void_p(st_t.data_ptr()) if status else None
        cp = ct.c_void_p(cn_t.data_ptr()) if counters else None
        strm = _stream_handle(stream, [T])
    else:
        st_t = np.empty(n, np.int32) if status else None
        cn_t = np.empty((n, NCOUNTERS), np.int32) if counters else None
        ptrs = [_np_ptr(a) for a in (T, P, Y)]
        sp = _np_ptr(st_t) if status else None
        cp = _np_ptr(cn_t) if counters else None
        strm = ct.c_void_p(stream) if isinstance(stream, int) else None
    o = make_opts(method, s_max, max_steps, lanes_per_cell, schedule, block_groups, grid_blocks,
                  dev, strm, cp, param_placement, stage_coefs, layout)
    s = Stats()
    rc = L.rkc_integrate(mech.handle, n, ptrs[0], ptrs[1], ptrs[2], float(dt), float(rtol),
                         float(atol), ct.byref(o), sp, ct.byref(s) if stats else None)
    if check and rc not in (OK, ECELLS):
        raise RkcError(rc, "rkc_integrate")
    out["rc"] = rc
    if status:
        out["status"] = st_t
    if counters:
        out["counters"] = cn_t
    if stats:
        out["stats"] = s.as_dict()
    return out


def integrate_noalloc(mech, T, P, Y, dt, rtol=1e-6, atol=1e-10, method=RKC, lanes_per_cell=0,
                      schedule=SCHED_AUTO, block_groups=0, grid_blocks=0, s_max=1000,
                      max_steps=1000000, status=None, counters=None, stream=None,
                      param_placement=PARAMS_AUTO, stage_coefs=0, layout=LAYOUT_CELL_MAJOR,
                      check=True):
    """rkc_integrate_device_noalloc on torch GPU tensors, in place: no device
    memory is allocated by the library (status [n] and counters [n][8] int32
    tensors are optional outputs the caller owns).  Returns the C return code
    (raises on an error unless check is False)."""
    if not _check_arrays([T, P, Y]):
        raise TypeError("device arrays expected: torch GPU tensors")
    _check_T(T)
    n = int(T.shape[0])
    _check_shapes(mech, n, P, Y, layout)
    for a, shape in ((status, (n,)), (counters, (n, NCOUNTERS))):
        if a is not None and (not _check_arrays([a], int32=True) or tuple(a.shape) != shape):
            raise ValueError("status must be int32 [n_cells], counters int32 [n_cells][8]")
    o = make_opts(method, s_max, max_steps, lanes_per_cell, schedule, block_groups, grid_blocks,
                  True, _stream_handle(stream, [T]),
                  ct.c_void_p(counters.data_ptr()) if counters is not None else None,
                  param_placement, stage_coefs, layout)
    rc = lib().rkc_integrate_device_noalloc(
        mech.handle, n, ct.c_void_p(T.data_ptr()), ct.c_void_p(P.data_ptr()),
        ct.c_void_p(Y.data_ptr()), float(dt), float(rtol), float(atol), ct.byref(o),
        ct.c_void_p(status.data_ptr()) if status is not None else None)
    if check and rc != OK:
        raise RkcError(rc, "rkc_integrate_device_noalloc")
    return rc


def autotune(mech, T, P, Y, dt, rtol=1e-6, atol=1e-10, method=RKC, lanes_per_cell=0,
             param_placement=PARAMS_AUTO, layout=LAYOUT_CELL_MAJOR):
    """rkc_autotune on a sample of cells (numpy or torch GPU arrays, left
    unchanged).  Returns (dict of integrate() keyword arguments, best ms)."""
    dev = _is_torch(T)
    _check_shapes(mech, int(T.shape[0]), P, Y, layout)
    if dev:
        ptrs = [ct.c_void_p(a.data_ptr()) for a in (T, P, Y)]
        o = make_opts(method, lanes_per_cell=lanes_per_cell, device_ptrs=True,
                      stream=_stream_handle(None, [T]), param_placement=param_placement,
                      layout=layout)
    else:
        keep = [np.ascontiguousarray(a, np.float64) for a in (T, P, Y)]
        ptrs = [_np_ptr(a) for a in keep]
        o = make_opts(method, lanes_per_cell=lanes_per_cell, param_placement=param_placement,
                      layout=layout)
    t = Opts()
    ms = ct.c_float()
    rc = lib().rkc_autotune(mech.handle, int(T.shape[0]), *ptrs, float(dt), float(rtol),
                            float(atol), ct.byref(o), ct.byref(t), ct.byref(ms))
    if rc != OK:
        raise RkcError(rc, "rkc_autotune")
    return {"schedule": t.schedule, "block_groups": t.block_groups,
            "grid_blocks": t.grid_blocks, "lanes_per_cell": t.lanes_per_cell,
            "param_placement": t.param_placement}, ms.value


class Graph:
    """One recorded global step over device arrays (rkc_graph_create);
    launch() replays it on a stream.  The tensors must outlive the graph."""

    def __init__(self, mech, T, P, Y, dt, rtol=1e-6, atol=1e-10, method=RKC, lanes_per_cell=0,
                 schedule=SCHED_AUTO, block_groups=0, grid_blocks=0, s_max=1000,
                 max_steps=1000000, status=None, param_placement=PARAMS_AUTO,
                 layout=LAYOUT_CELL_MAJOR):
        if not _check_arrays([T, P, Y]):
            raise TypeError("a graph records device arrays: torch GPU tensors expected")
        _check_T(T)
        _check_shapes(mech, int(T.shape[0]), P, Y, layout)
        if status is not None and (not _check_arrays([status], int32=True)
                                   or tuple(status.shape) != (int(T.shape[0]),)):
            raise ValueError("status must be an int32 GPU tensor [n_cells]")
        o = make_opts(method, s_max, max_steps, lanes_per_cell, schedule, block_groups,
                      grid_blocks, True, None, None, param_placement, layout=layout)
        h = ct.c_void_p()
        rc = lib().rkc_graph_create(mech.handle, int(T.shape[0]), ct.c_void_p(T.data_ptr()),
                                    ct.c_void_p(P.data_ptr()), ct.c_void_p(Y.data_ptr()),
                                    float(dt), float(rtol), float(atol), ct.byref(o),
                                    ct.c_void_p(status.data_ptr()) if status is not None else None,
                                    ct.byref(h))
        if rc != OK:
            raise RkcError(rc, "rkc_graph_create")
        self._h = h
        self._keep = (mech, T, P, Y, status)

    def launch(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        rc = lib().rkc_graph_launch(self._h, ct.c_void_p(s.cuda_stream))
        if rc != OK:
            raise RkcError(rc, "rkc_graph_launch")

    def close(self):
        if getattr(self, "_h", None):
            lib().rkc_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def divergence(work, width=32, stride=1, stream=None):
    """Divergence measure D (Sec. 3.1) of runs of `width` consecutive cells.

    work: per-cell work counts, int32, numpy (host) or torch GPU tensor; a 2-D
    array of counters is read column 0 with its row stride.  Returns D as the
    same kind of array."""
    L = lib()
    n = int(work.shape[0])
    runs = (n + width - 1) // width
    if _check_arrays([work], int32=True):
        import torch
        st = int(work.stride(0)) if work.dim() == 2 else 1
        D = torch.empty(runs, dtype=torch.float64, device=work.device)
        o = make_opts(device_ptrs=True, stream=_stream_handle(stream, [work]))
        rc = L.rkc_divergence(n, ct.c_void_p(work.data_ptr()), st, int(width),
                              ct.c_void_p(D.data_ptr()), ct.byref(o))
    else:
        w = np.ascontiguousarray(work, np.int32)
        st = int(w.strides[0] // 4) if w.ndim == 2 else 1
        D = np.empty(runs, np.float64)
        rc = L.rkc_divergence(n, _np_ptr(w), st, int(width), _np_ptr(D), None)
    if rc != OK:
        raise RkcError(rc, "rkc_divergence")
    return D


def rhs(mech, T, P, Y, lanes_per_cell=0, stream=None, layout=LAYOUT_CELL_MAJOR):
    """Source term f [n][nS+1] (column 0 = dT/dt) for numpy or torch GPU inputs
    (Y [nS][n] and f [nS+1][n] with layout=LAYOUT_SPECIES_MAJOR)."""
    L = lib()
    _check_T(T)
    n = int(T.shape[0])
    _check_shapes(mech, n, P, Y, layout)
    N = mech.n_species + 1
    fshape = (n, N) if layout == LAYOUT_CELL_MAJOR else (N, n)
    if _is_torch(T):
        import torch
        _check_arrays([T, P, Y])
        f = torch.empty(fshape, dtype=torch.float64, device=T.device)
        ptrs = [ct.c_void_p(a.data_ptr()) for a in (T, P, Y, f)]
        o = make_opts(lanes_per_cell=lanes_per_cell, device_ptrs=True,
                      stream=_stream_handle(stream, [T]), layout=layout)
    else:
        f = np.empty(fshape, np.float64)
        # host inputs are copied by the call: any float array is converted first
        keep = [np.ascontiguousarray(a, np.float64) for a in (T, P, Y)]
        ptrs = [_np_ptr(a) for a in keep] + [_np_ptr(f)]
        o = make_opts(lanes_per_cell=lanes_per_cell, layout=layout)
    rc = L.rkc_rhs(mech.handle, n, *ptrs, ct.byref(o))
    if rc != OK:
        raise RkcError(rc, "rkc_rhs")
    return f


class Server:
    """Integration server (include/rkc_server.h) on the current HIP device.

    submit() takes numpy host arrays, which must stay alive and untouched
    until wait() returns for the request (the object keeps references)."""

    def __init__(self, budget_bytes=1 << 30, n_streams=4, max_batch_cells=1 << 20,
                 lanes_per_cell=0, param_placement=PARAMS_AUTO):
        L = lib()
        o = ServerOpts()
        L.rkc_server_opts_default(ct.byref(o))
        o.budget_bytes = int(budget_bytes)
        o.n_streams = int(n_streams)
        o.max_batch_cells = int(max_batch_cells)
        o.lanes_per_cell = int(lanes_per_cell)
        o.param_placement = int(param_placement)
        h = ct.c_void_p()
        rc = L.rkc_server_create(ct.byref(o), ct.byref(h))
        if rc != OK:
            raise RkcError(rc, "rkc_server_create")
        self._h = h
        self._live = {}
        self._nS = []

    def register(self, mech):
        d, keep = _mech_desc(mech)
        mid = ct.c_int32()
        rc = lib().rkc_server_register_mech(self._h, ct.byref(d), ct.byref(mid))
        if rc != OK:
            raise RkcError(rc, "rkc_server_register_mech")
        self._nS.append(int(mech["n_species"]))
        return mid.value

    def submit(self, mech_id, T, P, Y, dt, rtol=1e-6, atol=1e-10, method=RKC, status=None):
        if _check_arrays([T, P, Y]):
            raise TypeError("the server takes host (numpy) arrays")
        _check_T(T)
        n = int(T.shape[0])
        if tuple(P.shape) != (n,) or tuple(Y.shape) != (n, self._nS[mech_id]):
            raise ValueError("shape mismatch: T [%d], P %s, Y %s" % (n, P.shape, Y.shape))
        if status is not None and (_check_arrays([status], int32=True) or status.shape != (n,)):
            raise ValueError("status must be an int32 numpy array [n_cells]")
        rid = ct.c_uint64()
        rc = lib().rkc_server_submit(self._h, int(mech_id), n, _np_ptr(T), _np_ptr(P), _np_ptr(Y),
                                     float(dt), float(rtol), float(atol), int(method),
                                     _np_ptr(status) if status is not None else None,
                                     ct.byref(rid))
        if rc != OK:
            raise RkcError(rc, "rkc_server_submit")
        self._live[rid.value] = (T, P, Y, status)
        return rid.value

    def poll(self, rid):
        d = ct.c_int32()
        rc = lib().rkc_server_poll(self._h, rid, ct.byref(d))
        if rc != OK:
            raise RkcError(rc, "rkc_server_poll")
        return bool(d.value)

    def wait(self, rid):
        """(rc, n_failed); rc is OK or ECELLS (other codes raise)."""
        nf = ct.c_int32()
        rc = lib().rkc_server_wait(self._h, rid, ct.byref(nf))
        self._live.pop(rid, None)
        if rc not in (OK, ECELLS):
            raise RkcError(rc, "rkc_server_wait")
        return rc, nf.value

    def stats(self):
        s = ServerStats()
        rc = lib().rkc_server_get_stats(self._h, ct.byref(s))
        if rc != OK:
            raise RkcError(rc, "rkc_server_get_stats")
        return s.as_dict()

    def reset_stats(self):
        lib().rkc_server_reset_stats(self._h)

    def close(self):
        if getattr(self, "_h", None):
            lib().rkc_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
