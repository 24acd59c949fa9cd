"""CPU oracle for prox_{lambda R} -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library does not use it and
shares no code with it.

The arithmetic lives in ``wsr_oracle.c`` (plain C, FP64): sort, rank-dependent
shift, stack pool-adjacent-violators, scatter back (paper Sec. 4.1 and
Alg. prox), and Alg. prox's l1 and rewinding lines per cluster.  This module
only builds that file with gcc and marshals arguments.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wsr_oracle.c")
_LIB = os.path.join(_HERE, "libwsr_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile wsr_oracle.c into libwsr_oracle.so with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
             "-ffp-contract=off", _SRC, "-o", tmp, "-lpthread", "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        lib.wsr_oracle_prox_f64.argtypes = [i64, p, ctypes.c_double, p, p, p]
        lib.wsr_oracle_prox_f64.restype = ctypes.c_int
        lib.wsr_oracle_prox_segments_f32.argtypes = [i64, p, p, p, ctypes.c_int, p, p, p, ctypes.c_int]
        lib.wsr_oracle_prox_segments_f32.restype = ctypes.c_int
        lib.wsr_oracle_prox_l1_f64.argtypes = [i64, p, ctypes.c_double, ctypes.c_double, ctypes.c_double, p]
        lib.wsr_oracle_prox_l1_f64.restype = ctypes.c_int
        lib.wsr_oracle_prox_l1_segments_f32.argtypes = [i64, p, p, p, ctypes.c_int, ctypes.c_float,
                                                        ctypes.c_float, p, ctypes.c_int]
        lib.wsr_oracle_prox_l1_segments_f32.restype = ctypes.c_int
        lib.wsr_oracle_prox_step_segments_f32.argtypes = [i64, p, p, p, ctypes.c_float, p, ctypes.c_int,
                                                          ctypes.c_float, ctypes.c_float, ctypes.c_int, p,
                                                          ctypes.c_int]
        lib.wsr_oracle_prox_step_segments_f32.restype = ctypes.c_int
        lib.wsr_oracle_grad_step_f32.argtypes = [i64, p, p, ctypes.c_float, p]
        lib.wsr_oracle_grad_step_f32.restype = ctypes.c_int
        lib.wsr_oracle_segment_stats.argtypes = [i64, p, p, p, p, p]
        lib.wsr_oracle_segment_stats.restype = ctypes.c_int
        lib.wsr_oracle_vjp.argtypes = [i64, p, p, p, p, p]
        lib.wsr_oracle_vjp.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def prox_f64(w, lam: float):
    """One segment in FP64: returns (u, perm, start) with perm[k] = original index of rank k
    and start[k] = 1 where rank k begins a cluster."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    d = w.shape[0]
    u = np.empty(d, np.float64)
    perm = np.empty(d, np.int64)
    start = np.empty(d, np.uint8)
    rc = _load().wsr_oracle_prox_f64(d, _ptr(w), float(lam), _ptr(u), _ptr(perm), _ptr(start))
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)
    return u, perm, start


def prox_segments(w, lam, offsets=None, n_threads: int = 1):
    """Flat FP32 buffer with segment offsets (None = one segment).  ``lam`` is a scalar or one
    FP32 value per segment.  Returns (u FP64, perm_local int32, start uint8), each of length N:
    perm_local[o+k] = segment-local original index of rank k of the segment starting at o."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    n = w.shape[0]
    if offsets is None:
        offsets = np.array([0, n], np.int64)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n_seg = offsets.shape[0] - 1
    lam_arr = np.ascontiguousarray(np.atleast_1d(np.asarray(lam, dtype=np.float32)))
    per_seg = 1 if lam_arr.shape[0] == n_seg and n_seg != 1 else 0
    if per_seg == 0 and lam_arr.shape[0] != 1:
        raise ValueError("lam must be a scalar or have one value per segment")
    u = np.empty(n, np.float64)
    perm = np.empty(n, np.int32)
    start = np.empty(n, np.uint8)
    rc = _load().wsr_oracle_prox_segments_f32(n_seg, _ptr(offsets), _ptr(w), _ptr(lam_arr), per_seg,
                                              _ptr(u), _ptr(perm), _ptr(start), int(n_threads))
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)
    return u, perm, start


def prox_l1_f64(w, lam: float, beta: float, rho: float):
    """One segment in FP64, Alg. prox in full: prox of lam*R + beta*l1 with rewinding rho."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    out = np.empty(w.shape[0], np.float64)
    rc = _load().wsr_oracle_prox_l1_f64(w.shape[0], _ptr(w), float(lam), float(beta), float(rho), _ptr(out))
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)
    return out


def prox_l1_segments(w, lam, beta: float, rho: float, offsets=None, n_threads: int = 1):
    """Flat FP32 buffer with segment offsets, Alg. prox in full on every segment (lam scalar or
    per segment; beta and rho FP32 scalars).  Returns the FP64 output in the original order."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    n = w.shape[0]
    if offsets is None:
        offsets = np.array([0, n], np.int64)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n_seg = offsets.shape[0] - 1
    lam_arr = np.ascontiguousarray(np.atleast_1d(np.asarray(lam, dtype=np.float32)))
    per_seg = 1 if lam_arr.shape[0] == n_seg and n_seg != 1 else 0
    if per_seg == 0 and lam_arr.shape[0] != 1:
        raise ValueError("lam must be a scalar or have one value per segment")
    out = np.empty(n, np.float64)
    rc = _load().wsr_oracle_prox_l1_segments_f32(n_seg, _ptr(offsets), _ptr(w), _ptr(lam_arr), per_seg,
                                                 float(beta), float(rho), _ptr(out), int(n_threads))
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)
    return out


def prox_step_segments(w, grad, eta, alpha, beta, rho, offsets=None, eta_in_displacement=False,
                       n_threads: int = 1):
    """One proximal-gradient step per segment: z = fmaf(-eta, grad, w) in FP32, then Alg. prox in
    full with lambda = eta*alpha, beta' = eta*beta (FP32 products), or, with
    ``eta_in_displacement``, with alpha and beta unscaled and eta on the rewinding line.
    Returns the FP64 output in the original order."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    grad = np.ascontiguousarray(grad, dtype=np.float32)
    n = w.shape[0]
    if offsets is None:
        offsets = np.array([0, n], np.int64)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n_seg = offsets.shape[0] - 1
    a = np.ascontiguousarray(np.atleast_1d(np.asarray(alpha, dtype=np.float32)))
    per_seg = 1 if a.shape[0] == n_seg and n_seg != 1 else 0
    if per_seg == 0 and a.shape[0] != 1:
        raise ValueError("alpha must be a scalar or have one value per segment")
    out = np.empty(n, np.float64)
    rc = _load().wsr_oracle_prox_step_segments_f32(n_seg, _ptr(offsets), _ptr(w), _ptr(grad), float(eta),
                                                   _ptr(a), per_seg, float(beta), float(rho),
                                                   1 if eta_in_displacement else 0, _ptr(out), int(n_threads))
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)
    return out


def grad_step(w, grad, eta):
    """z = fmaf(-eta, grad, w) in FP32 (one rounding per element)."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    grad = np.ascontiguousarray(grad, dtype=np.float32)
    z = np.empty_like(w)
    rc = _load().wsr_oracle_grad_step_f32(w.shape[0], _ptr(w), _ptr(grad), float(eta), _ptr(z))
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)
    return z


def segment_stats(w, offsets=None):
    """Per segment: (R(w) FP64, distinct non-zero values, non-zero weights) as three arrays."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    if offsets is None:
        offsets = np.array([0, w.shape[0]], np.int64)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n_seg = offsets.shape[0] - 1
    pen = np.empty(n_seg, np.float64)
    nd = np.empty(n_seg, np.int64)
    nz = np.empty(n_seg, np.int64)
    rc = _load().wsr_oracle_segment_stats(n_seg, _ptr(offsets), _ptr(w), _ptr(pen), _ptr(nd), _ptr(nz))
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)
    return pen, nd, nz


def vjp(g, perm_local, start, offsets=None):
    """Per-cluster mean of the cotangent g (FP64), for the partition (perm_local, start)."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    n = g.shape[0]
    if offsets is None:
        offsets = np.array([0, n], np.int64)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    perm_local = np.ascontiguousarray(perm_local, dtype=np.int32)
    start = np.ascontiguousarray(start, dtype=np.uint8)
    out = np.empty(n, np.float64)
    rc = _load().wsr_oracle_vjp(offsets.shape[0] - 1, _ptr(offsets), _ptr(perm_local), _ptr(start),
                                _ptr(g), _ptr(out))
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)
    return out


def cluster_ids(perm_local, start, offsets=None):
    """Label every element (original order) with a global cluster number, clusters numbered in
    rank order segment by segment.  Pure bookkeeping on the oracle's own outputs."""
    perm_local = np.asarray(perm_local)
    start = np.asarray(start)
    n = perm_local.shape[0]
    if offsets is None:
        offsets = np.array([0, n], np.int64)
    ids = np.empty(n, np.int64)
    rank_label = np.cumsum(start.astype(np.int64)) - 1
    for s in range(len(offsets) - 1):
        o, e = int(offsets[s]), int(offsets[s + 1])
        ids[o + perm_local[o:e].astype(np.int64)] = rank_label[o:e]
    return ids
