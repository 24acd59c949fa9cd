"""ctypes binding of libwsr.so (include/wsr.h): argument marshalling only.

Every function takes torch tensors for device buffers (float32 / int32, contiguous, on the
current HIP device) and host int64 offsets, and forwards raw pointers plus the current torch
stream to the C ABI.  All computation happens in the HIP kernels of the library; there is no
fallback: if the library is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwsr.so")

WSR_OK, WSR_ERR_INVALID, WSR_ERR_WORKSPACE, WSR_ERR_HIP, WSR_ERR_UNSUPPORTED = 0, -1, -2, -3, -4
WSR_PLAN_MERGE_HULL = 2
WSR_PLAN_MERGE_END = 4
WSR_STATUS_NONFINITE = 1
WSR_STEP_ETA_IN_DISPLACEMENT = 1
WSR_MAX_SEGMENT = 1 << 27
WSR_NOALLOC_SCRATCH_BYTES = 64 << 20
WSR_NOALLOC_MAX_SEGMENT = 1 << 21

EXPORTED = (
    "wsr_version", "wsr_status_string", "wsr_workspace_bytes", "wsr_prox_forward",
    "wsr_prox_backward", "wsr_plan_create", "wsr_plan_destroy", "wsr_plan_workspace_bytes",
    "wsr_prox_forward_batched", "wsr_prox_backward_batched", "wsr_trace_enable", "wsr_trace_collect",
    "wsr_prox_l1_forward", "wsr_prox_l1_forward_batched", "wsr_prox_step_batched",
    "wsr_segment_stats", "wsr_segment_stats_batched", "wsr_plan_autotune", "wsr_plan_merge_rounds",
    "wsr_plan_set_merge_rounds", "wsr_read_status", "wsr_plan_autotune_step", "wsr_prox_forward_noalloc",
    "wsr_plan_sort_routes", "wsr_plan_set_sort_routes",
)


class WsrError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        super().__init__("%s failed: %s (%d)" % (fn, _status_string(status), status))


_lib = None


def load():
    """Load libwsr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libwsr.so is not built; run `python -m paper_2311_03096_amd.build` "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    p, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
    f32 = ctypes.c_float
    sig = {
        "wsr_version": ([], i32),
        "wsr_status_string": ([i32], ctypes.c_char_p),
        "wsr_workspace_bytes": ([p, i64, ctypes.POINTER(sz)], i32),
        "wsr_prox_forward": ([p, p, p, i64, f32, p, p, p, sz, p], i32),
        "wsr_prox_forward_noalloc": ([p, p, p, i64, f32, p, p, p], i32),
        "wsr_prox_backward": ([p, p, p, i64, p, p, p, sz, p], i32),
        "wsr_prox_l1_forward": ([p, p, p, i64, f32, f32, f32, p, sz, p], i32),
        "wsr_prox_l1_forward_batched": ([p, p, p, p, f32, f32, f32, p, sz, p], i32),
        "wsr_prox_step_batched": ([p, p, p, f32, p, p, f32, f32, f32, i32, p, sz, p], i32),
        "wsr_segment_stats": ([p, p, i64, p, p, sz, p], i32),
        "wsr_plan_autotune": ([p, p, p, p, f32, p, sz, p], i32),
        "wsr_plan_merge_rounds": ([p, p], i32),
        "wsr_plan_set_merge_rounds": ([p, p], i32),
        "wsr_plan_sort_routes": ([p, p], i32),
        "wsr_plan_set_sort_routes": ([p, p], i32),
        "wsr_read_status": ([p, ctypes.POINTER(ctypes.c_uint32), i32, p], i32),
        "wsr_plan_autotune_step": ([p, p, p, f32, p, p, f32, f32, f32, i32, p, sz, p], i32),
        "wsr_segment_stats_batched": ([p, p, p, p, sz, p], i32),
        "wsr_plan_create": ([p, i64, i32, ctypes.POINTER(p)], i32),
        "wsr_plan_destroy": ([p], i32),
        "wsr_plan_workspace_bytes": ([p, ctypes.POINTER(sz)], i32),
        "wsr_prox_forward_batched": ([p, p, p, p, f32, p, p, p, sz, p], i32),
        "wsr_prox_backward_batched": ([p, p, p, p, p, p, sz, p], i32),
        "wsr_trace_enable": ([i32], i32),
        "wsr_trace_collect": ([i32, p, p, p, ctypes.POINTER(i32)], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _status_string(status):
    try:
        return load().wsr_status_string(int(status)).decode()
    except Exception:  # library not loadable: plain text
        return "status"


def _check(fn, rc):
    if rc != WSR_OK:
        raise WsrError(fn, rc)


class Plan:
    """A plan handle together with the layout it was created for (total length ``n`` and
    ``n_seg`` segments), so that the wrappers can check buffer sizes before any launch.  Passed
    to the C ABI as the raw handle (``_as_parameter_``)."""

    def __init__(self, handle, offsets):
        self._as_parameter_ = handle
        self.n = int(offsets[-1])
        self.n_seg = int(offsets.shape[0] - 1)


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _offsets(offsets):
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    if off.ndim != 1 or off.shape[0] < 1:
        raise ValueError("offsets must be a 1-D array of n_seg + 1 values")
    return off


def _n_of(offsets_or_plan):
    """Total length the buffers of a call must have (offsets[-1] or the plan's)."""
    if isinstance(offsets_or_plan, Plan):
        return offsets_or_plan.n
    if offsets_or_plan.shape[0] and offsets_or_plan[0] == 0 and np.all(np.diff(offsets_or_plan) >= 0):
        return int(offsets_or_plan[-1])
    return None  # invalid offsets: the library rejects them before reading any buffer


def _tensor(t, name, dtypes, numel=None, min_bytes=None, optional=False):
    """Reject a buffer the kernels would read or write out of bounds: wrong type or dtype, a size
    other than the layout's, or not contiguous.  Raises before any launch.  (Whether it is on the
    GPU is checked by ``_on_gpu`` after every buffer of the call has passed these checks.)"""
    if t is None:
        if optional:
            return
        raise ValueError("%s is required" % name)
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype not in dtypes:
        raise TypeError("%s must have dtype %s, not %s" % (name, " or ".join(str(d) for d in dtypes), t.dtype))
    if numel is not None and t.numel() != numel:
        raise ValueError("%s has %d elements; the segment layout needs %d" % (name, t.numel(), numel))
    if min_bytes is not None and t.numel() * t.element_size() < min_bytes:
        raise ValueError("%s holds %d bytes; at least %d are needed" % (name, t.numel() * t.element_size(),
                                                                       min_bytes))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def _on_gpu(**bufs):
    for name, t in bufs.items():
        if t is not None and not t.is_cuda:
            raise ValueError("%s must be on the GPU" % name)


def _f32():
    import torch
    return (torch.float32,)


def _i32():
    import torch
    return (torch.int32,)


def _words():
    import torch
    return (torch.int32, torch.uint32) if hasattr(torch, "uint32") else (torch.int32,)


def _bytes():
    import torch
    return (torch.uint8,)


def _check_values(n, **bufs):
    for name, t in bufs.items():
        _tensor(t, name, _f32(), numel=n)


def _check_saved(n, perm, mask):
    if (perm is None) != (mask is None):
        raise ValueError("saved_perm and saved_mask must both be given or both be None")
    _tensor(perm, "saved_perm", _i32(), numel=n, optional=True)
    _tensor(mask, "saved_mask", _words(), numel=(n + 31) // 32, optional=True)


def _check_lam(lam, n_seg, name="lambda"):
    _tensor(lam, name, _f32(), numel=n_seg, optional=True)


def _check_ws(ws):
    _tensor(ws, "workspace", _bytes(), optional=True)


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ws_args(ws):
    if ws is None:
        return None, 0
    return _ptr(ws), ws.numel() * ws.element_size()


def wsr_version():
    return load().wsr_version()


def wsr_status_string(status):
    return load().wsr_status_string(int(status)).decode()


def wsr_workspace_bytes(offsets):
    off = _offsets(offsets)
    n = ctypes.c_size_t(0)
    _check("wsr_workspace_bytes", load().wsr_workspace_bytes(off.ctypes.data_as(ctypes.c_void_p),
                                                             off.shape[0] - 1, ctypes.byref(n)))
    return n.value


def wsr_prox_forward(w, out, offsets, lam, saved_perm=None, saved_mask=None, ws=None, stream=None):
    off = _offsets(offsets)
    n = _n_of(off)
    _check_values(n, w=w, out=out)
    _check_saved(n, saved_perm, saved_mask)
    _check_ws(ws)
    _on_gpu(w=w, out=out, saved_perm=saved_perm, saved_mask=saved_mask, ws=ws)
    wp, wn = _ws_args(ws)
    _check("wsr_prox_forward", load().wsr_prox_forward(
        _ptr(w), _ptr(out), off.ctypes.data_as(ctypes.c_void_p), off.shape[0] - 1, float(lam),
        _ptr(saved_perm), _ptr(saved_mask), wp, wn, _stream(stream)))


def wsr_prox_forward_noalloc(w, out, offsets, lam, saved_perm=None, saved_mask=None, stream=None):
    """wsr_prox_forward with the library's fixed per-GPU scratch instead of a workspace (no
    allocation in the call; segments up to WSR_NOALLOC_MAX_SEGMENT)."""
    off = _offsets(offsets)
    n = _n_of(off)
    _check_values(n, w=w, out=out)
    _check_saved(n, saved_perm, saved_mask)
    _on_gpu(w=w, out=out, saved_perm=saved_perm, saved_mask=saved_mask)
    _check("wsr_prox_forward_noalloc", load().wsr_prox_forward_noalloc(
        _ptr(w), _ptr(out), off.ctypes.data_as(ctypes.c_void_p), off.shape[0] - 1, float(lam),
        _ptr(saved_perm), _ptr(saved_mask), _stream(stream)))


def wsr_prox_l1_forward(w, out, offsets, lam, beta, rho, ws=None, stream=None):
    off = _offsets(offsets)
    _check_values(_n_of(off), w=w, out=out)
    _check_ws(ws)
    _on_gpu(w=w, out=out, ws=ws)
    wp, wn = _ws_args(ws)
    _check("wsr_prox_l1_forward", load().wsr_prox_l1_forward(
        _ptr(w), _ptr(out), off.ctypes.data_as(ctypes.c_void_p), off.shape[0] - 1, float(lam),
        float(beta), float(rho), wp, wn, _stream(stream)))


def wsr_prox_backward(grad_out, grad_w, offsets, saved_perm, saved_mask, ws=None, stream=None):
    off = _offsets(offsets)
    n = _n_of(off)
    _check_values(n, grad_out=grad_out, grad_w=grad_w)
    _tensor(saved_perm, "saved_perm", _i32(), numel=n)
    _tensor(saved_mask, "saved_mask", _words(), numel=(n + 31) // 32 if n is not None else None)
    _check_ws(ws)
    _on_gpu(grad_out=grad_out, grad_w=grad_w, saved_perm=saved_perm, saved_mask=saved_mask, ws=ws)
    wp, wn = _ws_args(ws)
    _check("wsr_prox_backward", load().wsr_prox_backward(
        _ptr(grad_out), _ptr(grad_w), off.ctypes.data_as(ctypes.c_void_p), off.shape[0] - 1,
        _ptr(saved_perm), _ptr(saved_mask), wp, wn, _stream(stream)))


def wsr_plan_create(offsets, flags=0):
    """Create a plan; returns a ``Plan`` (the handle plus the layout's sizes)."""
    off = _offsets(offsets)
    h = ctypes.c_void_p()
    _check("wsr_plan_create", load().wsr_plan_create(off.ctypes.data_as(ctypes.c_void_p),
                                                     off.shape[0] - 1, int(flags), ctypes.byref(h)))
    return Plan(h, off)


def _plan(plan):
    if not isinstance(plan, Plan):
        raise TypeError("expected a Plan from wsr_plan_create")
    return plan


def wsr_plan_destroy(plan):
    _check("wsr_plan_destroy", load().wsr_plan_destroy(_plan(plan)))


def wsr_plan_workspace_bytes(plan):
    n = ctypes.c_size_t(0)
    _check("wsr_plan_workspace_bytes", load().wsr_plan_workspace_bytes(_plan(plan), ctypes.byref(n)))
    return n.value


def wsr_plan_autotune(plan, w, out, lam=None, lam_scalar=0.0, ws=None, stream=None):
    """Time the merge routes on ``w`` (``out`` is scratch and must not be ``w``)."""
    plan = _plan(plan)
    _check_values(plan.n, w=w, out=out)
    if w.data_ptr() == out.data_ptr():
        raise ValueError("the autotuner's output buffer must not alias w")
    _check_lam(lam, plan.n_seg)
    _check_ws(ws)
    _on_gpu(w=w, out=out, lam=lam, ws=ws)
    wp, wn = _ws_args(ws)
    _check("wsr_plan_autotune", load().wsr_plan_autotune(plan, _ptr(w), _ptr(out), _ptr(lam), float(lam_scalar),
                                                         wp, wn, _stream(stream)))


def wsr_plan_autotune_step(plan, w, grad, eta, scratch, alpha=None, alpha_scalar=0.0, beta=0.0, rho=0.0, flags=0,
                           ws=None, stream=None):
    """Time the merge routes on the proximal-gradient step's own launches (result to ``scratch``)."""
    plan = _plan(plan)
    _check_values(plan.n, w=w, grad=grad, scratch=scratch)
    if scratch.data_ptr() in (w.data_ptr(), grad.data_ptr()):
        raise ValueError("the autotuner's scratch buffer must alias neither w nor grad")
    _check_lam(alpha, plan.n_seg, "alpha")
    _check_ws(ws)
    _on_gpu(w=w, grad=grad, scratch=scratch, alpha=alpha, ws=ws)
    wp, wn = _ws_args(ws)
    _check("wsr_plan_autotune_step", load().wsr_plan_autotune_step(
        plan, _ptr(w), _ptr(grad), float(eta), _ptr(scratch), _ptr(alpha), float(alpha_scalar), float(beta),
        float(rho), int(flags), wp, wn, _stream(stream)))


def wsr_plan_merge_rounds(plan):
    """The plan's route per size class (2048, 4096, 8192, long): the cap on collision rounds
    (0 = hull merge only) or -1 = EndCollisions."""
    r = (ctypes.c_int32 * 4)()
    _check("wsr_plan_merge_rounds", load().wsr_plan_merge_rounds(_plan(plan), ctypes.cast(r, ctypes.c_void_p)))
    return list(r)


def wsr_plan_set_merge_rounds(plan, rounds):
    r = (ctypes.c_int32 * 4)(*[int(x) for x in rounds])
    _check("wsr_plan_set_merge_rounds", load().wsr_plan_set_merge_rounds(_plan(plan), ctypes.cast(r, ctypes.c_void_p)))


WSR_SORT_BUCKET = 0
WSR_SORT_RADIX = 1


def wsr_plan_sort_routes(plan):
    """The plan's sort route per short size class (2048, 4096, 8192): WSR_SORT_BUCKET or
    WSR_SORT_RADIX."""
    r = (ctypes.c_int32 * 3)()
    _check("wsr_plan_sort_routes", load().wsr_plan_sort_routes(_plan(plan), ctypes.cast(r, ctypes.c_void_p)))
    return list(r)


def wsr_plan_set_sort_routes(plan, routes):
    r = (ctypes.c_int32 * 3)(*[int(x) for x in routes])
    _check("wsr_plan_set_sort_routes", load().wsr_plan_set_sort_routes(_plan(plan), ctypes.cast(r, ctypes.c_void_p)))


def wsr_read_status(plan, clear=True, stream=None):
    """Synchronise the stream and return the plan's sticky status word (WSR_STATUS_NONFINITE bit)."""
    v = ctypes.c_uint32(0)
    _check("wsr_read_status", load().wsr_read_status(_plan(plan), ctypes.byref(v), 1 if clear else 0,
                                                     _stream(stream)))
    return v.value


def wsr_prox_forward_batched(plan, w, out, lam=None, lam_scalar=0.0, saved_perm=None, saved_mask=None,
                             ws=None, stream=None):
    plan = _plan(plan)
    _check_values(plan.n, w=w, out=out)
    _check_saved(plan.n, saved_perm, saved_mask)
    _check_lam(lam, plan.n_seg)
    _check_ws(ws)
    _on_gpu(w=w, out=out, lam=lam, saved_perm=saved_perm, saved_mask=saved_mask, ws=ws)
    wp, wn = _ws_args(ws)
    _check("wsr_prox_forward_batched", load().wsr_prox_forward_batched(
        plan, _ptr(w), _ptr(out), _ptr(lam), float(lam_scalar), _ptr(saved_perm), _ptr(saved_mask),
        wp, wn, _stream(stream)))


def wsr_prox_l1_forward_batched(plan, w, out, lam=None, lam_scalar=0.0, beta=0.0, rho=0.0, ws=None,
                                stream=None):
    plan = _plan(plan)
    _check_values(plan.n, w=w, out=out)
    _check_lam(lam, plan.n_seg)
    _check_ws(ws)
    _on_gpu(w=w, out=out, lam=lam, ws=ws)
    wp, wn = _ws_args(ws)
    _check("wsr_prox_l1_forward_batched", load().wsr_prox_l1_forward_batched(
        plan, _ptr(w), _ptr(out), _ptr(lam), float(lam_scalar), float(beta), float(rho), wp, wn,
        _stream(stream)))


def wsr_prox_step_batched(plan, w, grad, eta, out, alpha=None, alpha_scalar=0.0, beta=0.0, rho=0.0, flags=0,
                          ws=None, stream=None):
    plan = _plan(plan)
    _check_values(plan.n, w=w, grad=grad, out=out)
    _check_lam(alpha, plan.n_seg, "alpha")
    _check_ws(ws)
    _on_gpu(w=w, grad=grad, out=out, alpha=alpha, ws=ws)
    wp, wn = _ws_args(ws)
    _check("wsr_prox_step_batched", load().wsr_prox_step_batched(
        plan, _ptr(w), _ptr(grad), float(eta), _ptr(out), _ptr(alpha), float(alpha_scalar), float(beta),
        float(rho), int(flags), wp, wn, _stream(stream)))


STATS_RECORD_BYTES = 24  # wsr_segment_stats_t: float64 penalty, int64 distinct, int64 non-zero


def wsr_segment_stats(w, offsets, stats, ws=None, stream=None):
    """stats: a device buffer of n_seg records of (float64 penalty, int64 distinct non-zero,
    int64 non-zero), e.g. an int64 tensor of shape (n_seg, 3) viewed as needed."""
    off = _offsets(offsets)
    _check_values(_n_of(off), w=w)
    import torch
    _tensor(stats, "stats", (torch.int64, torch.float64, torch.uint8),
            min_bytes=STATS_RECORD_BYTES * (off.shape[0] - 1))
    _check_ws(ws)
    _on_gpu(w=w, stats=stats, ws=ws)
    wp, wn = _ws_args(ws)
    _check("wsr_segment_stats", load().wsr_segment_stats(
        _ptr(w), off.ctypes.data_as(ctypes.c_void_p), off.shape[0] - 1, _ptr(stats), wp, wn, _stream(stream)))


def wsr_segment_stats_batched(plan, w, stats, ws=None, stream=None):
    plan = _plan(plan)
    _check_values(plan.n, w=w)
    import torch
    _tensor(stats, "stats", (torch.int64, torch.float64, torch.uint8), min_bytes=STATS_RECORD_BYTES * plan.n_seg)
    _check_ws(ws)
    _on_gpu(w=w, stats=stats, ws=ws)
    wp, wn = _ws_args(ws)
    _check("wsr_segment_stats_batched", load().wsr_segment_stats_batched(
        plan, _ptr(w), _ptr(stats), wp, wn, _stream(stream)))


def stats_to_numpy(stats_host_bytes, n_seg):
    """Split the raw records (bytes or a uint8/int64 array on the host) into (penalty float64,
    distinct int64, nonzero int64) arrays."""
    rec = np.frombuffer(np.ascontiguousarray(stats_host_bytes).tobytes(), dtype=np.dtype(
        [("penalty", "<f8"), ("distinct", "<i8"), ("nonzero", "<i8")]), count=n_seg)
    return rec["penalty"].copy(), rec["distinct"].copy(), rec["nonzero"].copy()


def wsr_prox_backward_batched(plan, grad_out, grad_w, saved_perm, saved_mask, ws=None, stream=None):
    plan = _plan(plan)
    _check_values(plan.n, grad_out=grad_out, grad_w=grad_w)
    _tensor(saved_perm, "saved_perm", _i32(), numel=plan.n)
    _tensor(saved_mask, "saved_mask", _words(), numel=(plan.n + 31) // 32)
    _check_ws(ws)
    _on_gpu(grad_out=grad_out, grad_w=grad_w, saved_perm=saved_perm, saved_mask=saved_mask, ws=ws)
    wp, wn = _ws_args(ws)
    _check("wsr_prox_backward_batched", load().wsr_prox_backward_batched(
        plan, _ptr(grad_out), _ptr(grad_w), _ptr(saved_perm), _ptr(saved_mask), wp, wn, _stream(stream)))


def wsr_trace_enable(on=True):
    _check("wsr_trace_enable", load().wsr_trace_enable(1 if on else 0))


def wsr_trace_collect(max_entries=64):
    """Synchronise and return {kernel name: (launches, total ms)} for the traced launches."""
    names = ctypes.create_string_buffer(64 * max_entries)
    counts = (ctypes.c_int64 * max_entries)()
    total = (ctypes.c_double * max_entries)()
    n = ctypes.c_int(0)
    _check("wsr_trace_collect", load().wsr_trace_collect(max_entries, ctypes.cast(names, ctypes.c_void_p),
                                                         ctypes.cast(counts, ctypes.c_void_p),
                                                         ctypes.cast(total, ctypes.c_void_p), ctypes.byref(n)))
    res = {}
    for i in range(n.value):
        nm = names.raw[64 * i:64 * (i + 1)].split(b"\0", 1)[0].decode()
        res[nm] = (int(counts[i]), float(total[i]))
    return res
