"""ctypes binding of libnd.so with the names of include/nd.h.

Argument marshalling only: every step of the hot path runs in the HIP library.
Importing this module loads the library and fails loudly when it has not been
built (python -m paper_2410_19075_amd.build); there is no fallback.
"""
import ctypes
import os

import numpy as np

ND_OK = 0
ND_ERR_INVALID_ARG = -1
ND_ERR_OUT_OF_MEMORY = -2
ND_ERR_DEVICE = -3
ND_ERR_NOT_READY = -4
ND_ERR_NUMERIC = -5
ND_ERR_UNSUPPORTED = -6

ND_KURAMOTO, ND_FHN, ND_HH, ND_KURAMOTO_INERTIA = 0, 1, 2, 3
ND_RING, ND_CUBE3D, ND_CSR, ND_BALL3D, ND_DISK2D, ND_LINKS = 0, 1, 2, 3, 4, 5
ND_FP64, ND_FP32_BULK = 0, 1
ND_NOALLOC_MAX_NETS, ND_NOALLOC_MAX_WORK = 256, 262144  # nd_run_batch_noalloc limits (include/nd.h)
ND_MAX_PARAMS = 12
NVARS = {ND_KURAMOTO: 1, ND_FHN: 2, ND_HH: 4, ND_KURAMOTO_INERTIA: 2}

_c_i32, _c_i64, _c_dbl, _c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class nd_problem(ctypes.Structure):
    _fields_ = [("model", _c_i32), ("topo", _c_i32), ("precision", _c_i32), ("reserved", _c_i32),
                ("n", _c_i64), ("radius", _c_i64), ("n1", _c_i64), ("n2", _c_i64), ("n3", _c_i64),
                ("row_ptr", _c_vp), ("col", _c_vp), ("weight", _c_vp), ("nnz", _c_i64),
                ("per_elem", _c_vp), ("params", _c_dbl * ND_MAX_PARAMS)]


class nd_observe(ctypes.Structure):
    _fields_ = [("record_every", _c_i64), ("mv_start_step", _c_i64)]


class nd_kernel_config(ctypes.Structure):
    _fields_ = [("tile", _c_i32), ("block", _c_i32), ("grid", _c_i32), ("chunk", _c_i32), ("tile_y", _c_i32),
                ("tile_z", _c_i32)]


class nd_adaptive_stats(ctypes.Structure):
    _fields_ = [("t", _c_dbl), ("accepted", _c_i64), ("rejected", _c_i64), ("h_next", _c_dbl),
                ("failed", _c_i32), ("reserved", _c_i32)]


class nd_links_info(ctypes.Structure):
    _fields_ = [("v_bits", _c_i64), ("entries", _c_i64), ("d_bits", _c_i64), ("runs", _c_i64), ("bytes", _c_i64)]


class nd_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", _c_i64), ("max_slots", _c_i32), ("chunk_steps", _c_i32), ("grid", _c_i32),
                ("reserved", _c_i32)]


class nd_request_info(ctypes.Structure):
    _fields_ = [("state", _c_i32), ("status", _c_i32), ("steps_done", _c_i64), ("arrival", _c_dbl),
                ("admitted", _c_dbl), ("finished", _c_dbl)]


class nd_server_counters(ctypes.Structure):
    _fields_ = [("submitted", _c_i64), ("completed", _c_i64), ("failed", _c_i64), ("cancelled", _c_i64),
                ("queued", _c_i64), ("running", _c_i64), ("bytes_in_use", _c_i64), ("chunks", _c_i64),
                ("gpu_seconds", _c_dbl), ("osc_steps", _c_i64), ("active_seconds", _c_dbl)]


ND_REQ_QUEUED, ND_REQ_RUNNING, ND_REQ_DONE, ND_REQ_FAILED, ND_REQ_CANCELLED = range(5)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnd.so")
# One HIP runtime per process: PyTorch ships its own libamdhip64 / HSA runtime and
# references them under names that differ from libnd.so's, so if libnd.so were
# loaded first the process would hold two runtimes and the second could not open
# the device.  Loading torch first makes libnd.so bind to torch's runtime.
try:
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - torch is part of the supported stack
    pass
if not os.path.exists(LIB_PATH):
    raise ImportError(f"libnd.so is not built ({LIB_PATH}); run python -m paper_2410_19075_amd.build")
_lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.POINTER
_sig = {
    "nd_create": [_P(nd_problem), _P(_c_vp)],
    "nd_footprint": [_P(nd_problem), _P(_c_i64)],
    "nd_set_state": [_c_vp, _c_vp, _c_i64, _c_i32, _c_vp],
    "nd_run": [_c_vp, _c_dbl, _c_i64, _P(nd_observe), _c_vp],
    "nd_run_batch": [_P(_c_vp), _c_i32, _P(_c_dbl), _P(_c_i64), _P(nd_observe), _c_vp],
    "nd_run_batch_noalloc": [_P(_c_vp), _c_i32, _P(_c_dbl), _P(_c_i64), _P(nd_observe), _c_vp],
    "nd_run_adaptive": [_P(_c_vp), _c_i32, _P(_c_dbl), _P(_c_dbl), _c_dbl, _c_dbl, _c_i64, _P(nd_adaptive_stats),
                        _c_vp],
    "nd_run_adaptive_dense": [_P(_c_vp), _c_i32, _P(_c_dbl), _P(_c_dbl), _c_dbl, _c_dbl, _c_i64, _c_dbl, _c_vp,
                              _c_i64, _c_vp, _c_i64, _P(nd_adaptive_stats), _c_vp],
    "nd_get_state": [_c_vp, _c_vp, _c_i64, _c_i32, _c_vp],
    "nd_compress_links": [_c_i64, _c_vp, _c_vp, _c_vp, _c_i64, _c_vp, _c_i64, _c_vp, _c_i64, _c_vp, _c_i64,
                          _P(nd_links_info)],
    "nd_get_observables": [_c_vp, _c_vp, _c_i64, _c_vp, _c_i64, _c_i32, _c_vp],
    "nd_destroy": [_c_vp],
    "nd_sync": [_c_vp, _c_vp],
    "nd_get_config": [_c_vp, _P(nd_kernel_config)],
    "nd_set_config": [_c_vp, _P(nd_kernel_config)],
    "nd_server_create": [_P(nd_server_config), _P(_c_vp)],
    "nd_server_now": [_c_vp, _P(_c_dbl)],
    "nd_server_submit": [_c_vp, _P(nd_problem), _c_vp, _c_i64, _c_dbl, _c_i64, _P(nd_observe), _c_dbl,
                         _P(_c_i64)],
    "nd_server_pump": [_c_vp, _c_vp, _P(_c_i64)],
    "nd_server_info": [_c_vp, _c_i64, _P(nd_request_info)],
    "nd_server_result": [_c_vp, _c_i64, _c_vp, _c_i64, _c_vp, _c_i64],
    "nd_server_cancel": [_c_vp, _c_i64],
    "nd_server_stats": [_c_vp, _P(nd_server_counters)],
    "nd_server_destroy": [_c_vp],
    "nd_tune": [_P(nd_problem), _c_vp, _c_i64, _c_dbl, _c_i32, _c_vp, _P(nd_kernel_config), _P(_c_dbl)],
    "nd_tune_load": [ctypes.c_char_p],
    "nd_tune_save": [ctypes.c_char_p],
    "nd_tune_clear": [],
}
for _name, _args in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _c_i32
_lib.nd_status_str.argtypes = [_c_i32]
_lib.nd_status_str.restype = ctypes.c_char_p
_lib.nd_last_error.argtypes = []
_lib.nd_last_error.restype = ctypes.c_char_p


class NDError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.nd_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_lib.nd_status_str(status).decode()} ({status}): {msg}")


def _check(status, where, **extra):
    if status != ND_OK:
        err = NDError(status, where)
        for k, v in extra.items():
            setattr(err, k, v)
        raise err
    return status


def _buf(a, what, dtype="float64"):
    """(pointer, element count, on_device) of a contiguous torch tensor or numpy
    array of the dtype the C side reads (None -> (None, 0, None)).  The library
    copies count * sizeof(dtype) bytes, so anything else is refused here."""
    if a is None:
        return None, 0, None
    if hasattr(a, "data_ptr"):
        import torch
        if a.dtype != getattr(torch, dtype):
            raise TypeError(f"{what}: expected a torch.{dtype} tensor, got {a.dtype}")
        if not a.is_contiguous():
            raise ValueError(f"{what}: the tensor must be contiguous")
        return a.data_ptr(), a.numel(), bool(a.is_cuda)
    if not isinstance(a, np.ndarray):
        raise TypeError(f"{what}: expected a numpy array or a torch tensor, got {type(a).__name__}")
    if a.dtype != np.dtype(dtype):
        raise TypeError(f"{what}: expected a numpy {dtype} array, got {a.dtype}")
    if not a.flags.c_contiguous:
        raise ValueError(f"{what}: the array must be C-contiguous")
    if not a.flags.writeable and what.startswith("out"):
        raise ValueError(f"{what}: the array must be writeable")
    return a.ctypes.data, a.size, False


def _on_device(what, on_device, *places):
    """The copy direction of one call: every buffer on the same side, and an
    explicit on_device that matches where they are."""
    seen = {p for p in places if p is not None}
    if len(seen) > 1:
        raise ValueError(f"{what}: buffers on the host and on the device in one call")
    where = seen.pop() if seen else False
    if on_device is not None and bool(on_device) != where:
        raise ValueError(f"{what}: on_device={int(bool(on_device))} but the buffer is "
                         f"{'on the device' if where else 'in host memory'}")
    return int(where)


def _stream(stream):
    if stream is None:
        return None
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def problem(model, topo, n, params, precision=ND_FP64, radius=0, dims=(0, 0, 0), row_ptr=None, col=None,
            weight=None, per_elem=None):
    """Build an nd_problem.  The numpy arrays must stay alive until nd_create returns
    (the struct keeps references in `_keep`)."""
    p = nd_problem()
    p.model, p.topo, p.precision, p.reserved = model, topo, precision, 0
    p.n, p.radius = int(n), int(radius)
    p.n1, p.n2, p.n3 = (int(d) for d in dims)
    keep = []

    def arr(a, dt):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data

    p.row_ptr = arr(row_ptr, np.int64)
    p.col = arr(col, np.int32)
    p.weight = arr(weight, np.float64)
    p.nnz = 0 if row_ptr is None else int(np.asarray(row_ptr)[-1])
    p.per_elem = arr(per_elem, np.float64)
    for i, v in enumerate(params):
        p.params[i] = float(v)
    p._keep = keep
    return p


def nd_create(p):
    h = _c_vp()
    _check(_lib.nd_create(ctypes.byref(p), ctypes.byref(h)), "nd_create")
    return h.value


def nd_footprint(p):
    b = _c_i64()
    _check(_lib.nd_footprint(ctypes.byref(p), ctypes.byref(b)), "nd_footprint")
    return b.value


def nd_set_state(h, y, on_device=None, stream=None):
    ptr, n, dev = _buf(y, "nd_set_state y")
    on = _on_device("nd_set_state", on_device, dev)
    _check(_lib.nd_set_state(h, ptr, n, on, _stream(stream)), "nd_set_state")


def nd_get_state(h, y, on_device=None, stream=None):
    ptr, n, dev = _buf(y, "out: nd_get_state y")
    on = _on_device("nd_get_state", on_device, dev)
    _check(_lib.nd_get_state(h, ptr, n, on, _stream(stream)), "nd_get_state")


def observe(record_every=0, mv_start_step=-1):
    return nd_observe(int(record_every), int(mv_start_step))


def nd_run(h, dt, steps, obs=None, stream=None):
    _check(_lib.nd_run(h, float(dt), int(steps), ctypes.byref(obs) if obs is not None else None,
                       _stream(stream)), "nd_run")


def _batch_args(handles, dts, steps, obs):
    """Handle, dt and step arrays of a batch call (numpy buffers: a per-element
    ctypes conversion costs about a millisecond for thousands of networks)."""
    k = len(handles)
    hs = np.asarray([0 if h is None else h for h in handles], dtype=np.uintp)
    dd = np.ascontiguousarray(dts, dtype=np.float64)
    ss = np.ascontiguousarray(steps, dtype=np.int64)
    if dd.shape != (k,) or ss.shape != (k,):
        raise ValueError("dts and steps need one entry per handle")
    oo = (nd_observe * k)(*obs) if obs is not None else None
    return (k, hs, dd, ss, oo, hs.ctypes.data_as(_P(_c_vp)), dd.ctypes.data_as(_P(_c_dbl)),
            ss.ctypes.data_as(_P(_c_i64)))


def nd_run_batch(handles, dts, steps, obs=None, stream=None):
    k, _h, _d, _s, oo, hp, dp, sp = _batch_args(handles, dts, steps, obs)
    _check(_lib.nd_run_batch(hp, k, dp, sp, oo, _stream(stream)), "nd_run_batch")


def nd_run_batch_noalloc(handles, dts, steps, obs=None, stream=None):
    """nd_run_batch without any allocation (descriptor tables in the library's
    fixed per-GPU array; see include/nd.h)."""
    k, _h, _d, _s, oo, hp, dp, sp = _batch_args(handles, dts, steps, obs)
    _check(_lib.nd_run_batch_noalloc(hp, k, dp, sp, oo, _stream(stream)), "nd_run_batch_noalloc")


def nd_run_adaptive(handles, t_end, dt0, rtol, atol, max_steps=10 ** 7, stream=None):
    """Dormand-Prince 5(4) with step-size control on each network (FP64 rings of at
    most 1024 elements); returns one nd_adaptive_stats per network."""
    k = len(handles)
    hs = (_c_vp * k)(*handles)
    te = (_c_dbl * k)(*[float(x) for x in t_end])
    d0 = (_c_dbl * k)(*[float(x) for x in dt0])
    st = (nd_adaptive_stats * k)()
    _check(_lib.nd_run_adaptive(hs, k, te, d0, float(rtol), float(atol), int(max_steps), st, _stream(stream)),
           "nd_run_adaptive", stats=list(st))
    return list(st)


def nd_compress_links(n, row_ptr, col):
    """The library's compression of a binary coupling matrix given by rows:
    returns (V, d_ptr, d_pos, C, info)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    info = nd_links_info()
    _check(_lib.nd_compress_links(int(n), rp.ctypes.data, cl.ctypes.data if cl.size else None, None, 0, None, 0,
                                  None, 0, None, 0, ctypes.byref(info)), "nd_compress_links")
    V = np.empty(info.v_bits, dtype=np.int32)
    dptr = np.empty(info.entries + 1, dtype=np.int64)
    dpos = np.empty(info.d_bits, dtype=np.int32)
    C = np.empty(int(n), dtype=np.int32)
    _check(_lib.nd_compress_links(int(n), rp.ctypes.data, cl.ctypes.data if cl.size else None, V.ctypes.data, V.size,
                                  dptr.ctypes.data, dptr.size, dpos.ctypes.data, dpos.size, C.ctypes.data, C.size,
                                  ctypes.byref(info)), "nd_compress_links")
    return V, dptr, dpos, C, info


def nd_run_adaptive_dense(handles, t_end, dt0, rtol, atol, t_out, state_len=0, max_steps=10 ** 7, stream=None):
    """Dormand-Prince with dense output: returns (stats, R, Y) with R[i, k] the order
    parameter of network i at k * t_out and, when state_len (the largest nvars * n of
    the networks) is given, Y[i, k * nvars * n_i + v * n_i + j] its state there (NaN
    where a network does not reach the output)."""
    k = len(handles)
    hs = (_c_vp * k)(*handles)
    te = (_c_dbl * k)(*[float(x) for x in t_end])
    d0 = (_c_dbl * k)(*[float(x) for x in dt0])
    st = (nd_adaptive_stats * k)()
    # (a t_out <= 0 is passed on for the library to reject)
    outs = int(np.max(np.floor(np.asarray(t_end, dtype=np.float64) / t_out))) + 1 if k and t_out > 0 else 1
    R = np.empty((k, outs))
    ys = outs * int(state_len)
    Y = np.empty((k, ys)) if state_len else None
    _check(_lib.nd_run_adaptive_dense(hs, k, te, d0, float(rtol), float(atol), int(max_steps), float(t_out),
                                      R.ctypes.data, outs, Y.ctypes.data if Y is not None else None, ys, st,
                                      _stream(stream)), "nd_run_adaptive_dense", stats=list(st))
    return list(st), R, Y


def nd_get_observables(h, R=None, mean_vel=None, on_device=None, stream=None):
    pr, nr, dr = _buf(R, "out: nd_get_observables R")
    pm, nm, dm = _buf(mean_vel, "out: nd_get_observables mean_vel")
    on = _on_device("nd_get_observables", on_device, dr, dm)
    _check(_lib.nd_get_observables(h, pr, nr, pm, nm, on, _stream(stream)), "nd_get_observables")


def nd_sync(h, stream=None):
    _check(_lib.nd_sync(h, _stream(stream)), "nd_sync")


def nd_destroy(h):
    _check(_lib.nd_destroy(h), "nd_destroy")


def nd_get_config(h):
    c = nd_kernel_config()
    _check(_lib.nd_get_config(h, ctypes.byref(c)), "nd_get_config")
    return c


def nd_set_config(h, c):
    _check(_lib.nd_set_config(h, ctypes.byref(c)), "nd_set_config")


def nd_server_create(hbm_budget_bytes, max_slots=256, chunk_steps=64, grid=0):
    cfg = nd_server_config(int(hbm_budget_bytes), int(max_slots), int(chunk_steps), int(grid), 0)
    h = _c_vp()
    _check(_lib.nd_server_create(ctypes.byref(cfg), ctypes.byref(h)), "nd_server_create")
    return h.value


def nd_server_now(s):
    t = _c_dbl()
    _check(_lib.nd_server_now(s, ctypes.byref(t)), "nd_server_now")
    return t.value


def nd_server_submit(s, p, y0, dt, steps, obs=None, arrival=-1.0):
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    rid = _c_i64()
    _check(_lib.nd_server_submit(s, ctypes.byref(p), y0.ctypes.data, y0.size, float(dt), int(steps),
                                 ctypes.byref(obs) if obs is not None else None, float(arrival), ctypes.byref(rid)),
           "nd_server_submit")
    return rid.value


def nd_server_pump(s, stream=None):
    pending = _c_i64()
    _check(_lib.nd_server_pump(s, _stream(stream), ctypes.byref(pending)), "nd_server_pump")
    return pending.value


def nd_server_info(s, rid):
    info = nd_request_info()
    _check(_lib.nd_server_info(s, int(rid), ctypes.byref(info)), "nd_server_info")
    return info


def nd_server_result(s, rid, y, R=None):
    py, ny, dy = _buf(y, "out: nd_server_result y")
    pr, nr, dr = _buf(R, "out: nd_server_result R")
    if dy or dr:
        raise ValueError("nd_server_result copies into host memory (numpy arrays)")
    _check(_lib.nd_server_result(s, int(rid), py, ny, pr, nr), "nd_server_result")


def nd_server_cancel(s, rid):
    _check(_lib.nd_server_cancel(s, int(rid)), "nd_server_cancel")


def nd_server_stats(s):
    st = nd_server_counters()
    _check(_lib.nd_server_stats(s, ctypes.byref(st)), "nd_server_stats")
    return st


def nd_server_destroy(s):
    _check(_lib.nd_server_destroy(s), "nd_server_destroy")


def nd_tune(p, y0, dt, steps, stream=None):
    """Returns (best nd_kernel_config, ms per step)."""
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    best = nd_kernel_config()
    ms = _c_dbl()
    _check(_lib.nd_tune(ctypes.byref(p), y0.ctypes.data, y0.size, float(dt), int(steps), _stream(stream),
                        ctypes.byref(best), ctypes.byref(ms)), "nd_tune")
    return best, ms.value


def nd_tune_load(path):
    _check(_lib.nd_tune_load(os.fsencode(path)), "nd_tune_load")


def nd_tune_save(path):
    _check(_lib.nd_tune_save(os.fsencode(path)), "nd_tune_save")


def nd_tune_clear():
    _check(_lib.nd_tune_clear(), "nd_tune_clear")


def nd_status_str(s):
    return _lib.nd_status_str(s).decode()


def nd_last_error():
    return _lib.nd_last_error().decode()


# ------------------------------------------------------------ conveniences
def simulate(p, y0, dt, steps, record_every=0, mv_start_step=-1, stream=None):
    """Create a network, run it from host state y0 and return (y, R, mean_vel) as
    numpy arrays (all work on the GPU)."""
    h = nd_create(p)
    try:
        y0 = np.ascontiguousarray(y0, dtype=np.float64)
        nd_set_state(h, y0, on_device=0, stream=stream)
        nd_run(h, dt, steps, observe(record_every, mv_start_step), stream=stream)
        y = np.empty_like(y0)
        nd_get_state(h, y, on_device=0, stream=stream)
        R = np.empty(steps // record_every + 1) if record_every else None
        mv = np.empty(p.n) if mv_start_step >= 0 else None
        if R is not None or mv is not None:
            nd_get_observables(h, R, mv, on_device=0, stream=stream)
        return y, R, mv
    finally:
        nd_destroy(h)
