"""Torch-facing wrappers over the C ABI: autograd prox and a batched per-step prox.

Torch supplies device memory and the stream; every step of the prox runs in the library's
HIP kernels.  Buffers for the saved state and the workspace are allocated here (the library
itself never allocates during a compute call).  Every buffer is checked against the segment
layout by the binding before any launch.
"""
from __future__ import annotations

import collections
import json
import os
import threading

import numpy as np
import torch

from . import _lib


def _mask_words(n):
    return (n + 31) // 32


def _workspace(nbytes, device):
    if nbytes == 0:
        return None
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _as_offsets(offsets, n):
    if offsets is None:
        offsets = np.array([0, n], dtype=np.int64)
    offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    if offsets.ndim != 1 or offsets.shape[0] < 1 or int(offsets[-1]) != n:
        raise ValueError("offsets must be n_seg + 1 values ending at the tensor's %d elements" % n)
    return offsets


# ------------------------------------------------------------------------------ tuning cache

def device_arch(device=None):
    """The GPU architecture name the tuning was measured on (e.g. 'gfx950:sramecc+:xnack-')."""
    props = torch.cuda.get_device_properties(device if device is not None else torch.cuda.current_device())
    return getattr(props, "gcnArchName", props.name)


def tuning_key(offsets, arch, flags=0, kind="forward"):
    """Key of a plan's tuning: the architecture, the call it was tuned for, the plan flags and the
    segment-length histogram (segments per short size class, and the long segments' lengths
    rounded up to a power of two)."""
    lens = np.diff(np.asarray(offsets, dtype=np.int64))
    classes = [int(np.count_nonzero((lens > lo) & (lens <= hi))) for lo, hi in ((0, 2048), (2048, 4096),
                                                                                  (4096, 8192))]
    longs = sorted(int(1 << int(np.ceil(np.log2(x)))) for x in lens[lens > 8192])
    return "%s|%s|%d|%s|%s" % (arch, kind, int(flags), ",".join(map(str, classes)), ",".join(map(str, longs)))


class TuningCache:
    """Routes found by the autotuner, persisted as JSON {key: {"rounds": [4 merge routes],
    "sort": [3 sort routes]}} and keyed by ``tuning_key`` so that a later run with the same
    architecture and segment layout reuses them without timing again (an entry of the older form,
    the 4 merge routes alone, reads with the bucket sort route).  Writes are atomic (temporary
    file + rename)."""

    def __init__(self, path=None):
        self.path = path or os.environ.get("WSR_TUNING_CACHE") or os.path.join(
            os.path.expanduser("~"), ".cache", "wsr", "tuning.json")
        self._lock = threading.Lock()

    def _read(self):
        try:
            with open(self.path) as f:
                data = json.load(f)
            return data if isinstance(data, dict) else {}
        except (OSError, ValueError):
            return {}

    @staticmethod
    def _ints(v, n):
        return isinstance(v, list) and len(v) == n and all(isinstance(x, int) for x in v)

    def get(self, key):
        """{"rounds": [4], "sort": [3]} stored under key, or None."""
        r = self._read().get(key)
        if self._ints(r, 4):
            return {"rounds": r, "sort": [0, 0, 0]}
        if isinstance(r, dict) and self._ints(r.get("rounds"), 4) and self._ints(r.get("sort"), 3):
            return {"rounds": r["rounds"], "sort": r["sort"]}
        return None

    def put(self, key, rounds, sort=(0, 0, 0)):
        with self._lock:
            data = self._read()
            data[key] = {"rounds": [int(x) for x in rounds], "sort": [int(x) for x in sort]}
            d = os.path.dirname(self.path)
            if d:
                os.makedirs(d, exist_ok=True)
            tmp = "%s.tmp%d" % (self.path, os.getpid())
            with open(tmp, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


# ------------------------------------------------------------------------------ batched plans

class BatchedProx:
    """All segments of a fixed segmentation in one batched call per step (plan created once).

    ``forward(w, out, lam)`` runs the batched prox; with ``save=True`` the saved permutation and
    cluster-start bits for ``backward`` are kept in this object.  ``capture()`` records one
    forward into a HIP graph (torch.cuda.CUDAGraph) for replay with ``replay()``.
    ``autotune=True`` times the merge and sort routes on the first call's inputs (wsr_plan_autotune, or
    wsr_plan_autotune_step for ``step``), into a scratch buffer; with ``tuning_cache`` (a
    ``TuningCache`` or a path) a stored tuning for the same architecture and segment layout is
    reused and a new one stored.  ``hull_only=True`` merges by the hull merge alone (for
    comparing routes).
    """

    def __init__(self, offsets, device="cuda", autotune=False, hull_only=False, tuning_cache=None):
        self.offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self.n = int(self.offsets[-1])
        self.n_seg = int(self.offsets.shape[0] - 1)
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.flags = _lib.WSR_PLAN_MERGE_HULL if hull_only else 0
        self.plan = _lib.wsr_plan_create(self.offsets, self.flags)
        self.tune_pending = bool(autotune)  # tuned on the first call's inputs
        if isinstance(tuning_cache, str):
            tuning_cache = TuningCache(tuning_cache)
        self.tuning_cache = tuning_cache
        self.ws = _workspace(_lib.wsr_plan_workspace_bytes(self.plan), self.device)
        self.perm = None
        self.mask = None
        self.graph = None

    def _saved_state(self):
        if self.perm is None:
            self.perm = torch.empty(self.n, dtype=torch.int32, device=self.device)
            self.mask = torch.empty(_mask_words(self.n), dtype=torch.int32, device=self.device)
        return self.perm, self.mask

    def _tune(self, kind, run):
        """Apply a cached tuning for this layout, or time the routes with ``run`` (synchronising:
        done before any graph capture) and store the result."""
        if not self.tune_pending:
            return
        key = tuning_key(self.offsets, device_arch(self.device), self.flags, kind) if self.tuning_cache else None
        cached = self.tuning_cache.get(key) if key else None
        if cached is not None:
            _lib.wsr_plan_set_merge_rounds(self.plan, cached["rounds"])
            _lib.wsr_plan_set_sort_routes(self.plan, cached["sort"])
        else:
            run()
            if key:
                self.tuning_cache.put(key, _lib.wsr_plan_merge_rounds(self.plan), _lib.wsr_plan_sort_routes(self.plan))
        self.tune_pending = False

    def merge_rounds(self):
        return _lib.wsr_plan_merge_rounds(self.plan)

    def sort_routes(self):
        return _lib.wsr_plan_sort_routes(self.plan)

    def forward(self, w, out, lam=None, lam_scalar=0.0, save=True):
        scratch = None
        if self.tune_pending:
            scratch = torch.empty_like(w)  # out may alias w: the routes are timed into scratch
            self._tune("forward", lambda: _lib.wsr_plan_autotune(self.plan, w, scratch, lam, lam_scalar, self.ws))
        perm, mask = self._saved_state() if save else (None, None)
        _lib.wsr_prox_forward_batched(self.plan, w, out, lam, lam_scalar, perm, mask, self.ws)

    def forward_l1(self, w, out, lam=None, lam_scalar=0.0, beta=0.0, rho=0.0):
        """Alg. prox in full (l1 and rewinding lines) over every segment; saves nothing."""
        _lib.wsr_prox_l1_forward_batched(self.plan, w, out, lam, lam_scalar, beta, rho, self.ws)

    def step(self, w, grad, eta, alpha=None, alpha_scalar=0.0, beta=0.0, rho=0.0, eta_in_displacement=False,
             out=None):
        """One proximal-gradient step w <- Prox(w - eta*grad) over every segment (in place unless
        ``out`` is given); ``alpha`` is a device tensor of per-segment coefficients or None."""
        out = w if out is None else out
        flags = _lib.WSR_STEP_ETA_IN_DISPLACEMENT if eta_in_displacement else 0
        if self.tune_pending:  # routes timed on the step's own launches, into scratch
            scratch = torch.empty_like(w)
            self._tune("step%d" % flags, lambda: _lib.wsr_plan_autotune_step(
                self.plan, w, grad, eta, scratch, alpha, alpha_scalar, beta, rho, flags, self.ws))
        _lib.wsr_prox_step_batched(self.plan, w, grad, eta, out, alpha, alpha_scalar, beta, rho, flags, self.ws)
        return out

    def backward(self, g, gw):
        if self.perm is None:
            raise RuntimeError("backward needs a forward with save=True first")
        _lib.wsr_prox_backward_batched(self.plan, g, gw, self.perm, self.mask, self.ws)

    def capture(self, w, out, lam=None, lam_scalar=0.0, save=True):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.forward(w, out, lam, lam_scalar, save)  # warm-up (and tuning) outside the graph
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.forward(w, out, lam, lam_scalar, save)
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def close(self):
        if self.plan is not None:
            _lib.wsr_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------------ autograd

_PLAN_CACHE_SIZE = 8
_plan_cache = collections.OrderedDict()
_plan_lock = threading.Lock()


def cached_plan(offsets, device):
    """A BatchedProx for this segment layout on this device, kept in a small LRU cache so that
    repeated calls (one per training step) reuse its plan and workspace."""
    offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    key = (str(device), offsets.tobytes())
    with _plan_lock:
        bp = _plan_cache.get(key)
        if bp is not None:
            _plan_cache.move_to_end(key)
            return bp
        bp = BatchedProx(offsets, device=device)
        _plan_cache[key] = bp
        while len(_plan_cache) > _PLAN_CACHE_SIZE:
            # an evicted plan is freed with its last reference (a pending backward holds one)
            _plan_cache.popitem(last=False)
        return bp


class ProxFunction(torch.autograd.Function):
    """u = prox_{lam R}(w) per segment; backward averages the cotangent within clusters.
    Both directions are the batched entry points over a cached plan (one launch per size class
    of short segments)."""

    @staticmethod
    def forward(ctx, w, lam, offsets):
        bp = cached_plan(offsets, w.device)
        n = w.numel()
        out = torch.empty_like(w)
        perm = torch.empty(n, dtype=torch.int32, device=w.device)
        mask = torch.empty(_mask_words(n), dtype=torch.int32, device=w.device)
        _lib.wsr_prox_forward_batched(bp.plan, w, out, None, lam, perm, mask, bp.ws)
        ctx.save_for_backward(perm, mask)
        ctx.bp = bp
        return out

    @staticmethod
    def backward(ctx, g):
        perm, mask = ctx.saved_tensors
        g = g.contiguous()
        gw = torch.empty_like(g)
        _lib.wsr_prox_backward_batched(ctx.bp.plan, g, gw, perm, mask, ctx.bp.ws)
        return gw, None, None


def prox(w, lam, offsets=None):
    """prox_{lam R} of a float32 GPU tensor; ``offsets`` (host, n_seg+1 int64) splits the
    flattened tensor into independent segments (default: one segment)."""
    flat = w.contiguous().view(-1)
    offsets = _as_offsets(offsets, flat.numel())
    return ProxFunction.apply(flat, float(lam), offsets).view(w.shape)


def prox_l1(w, lam, beta, rho=0.0, offsets=None):
    """Alg. prox in full on a float32 GPU tensor: prox of lam*R + beta*l1 with rewinding rho,
    per segment (the update of a proximal-gradient step; not differentiable here)."""
    flat = w.contiguous().view(-1)
    offsets = _as_offsets(offsets, flat.numel())
    out = torch.empty_like(flat)
    ws = _workspace(_lib.wsr_workspace_bytes(offsets), flat.device)
    _lib.wsr_prox_l1_forward(flat, out, offsets, lam, beta, rho, ws)
    return out.view(w.shape)


def segment_stats(w, offsets=None):
    """Per segment of a float32 GPU tensor: (R(w), distinct non-zero values, non-zero weights)
    as host numpy arrays (the ratio of the last two is the weight-sharing measure)."""
    flat = w.contiguous().view(-1)
    offsets = _as_offsets(offsets, flat.numel())
    n_seg = offsets.shape[0] - 1
    st = torch.empty((n_seg, 3), dtype=torch.int64, device=flat.device)
    ws = _workspace(_lib.wsr_workspace_bytes(offsets), flat.device)
    _lib.wsr_segment_stats(flat, offsets, st, ws)
    return _lib.stats_to_numpy(st.cpu().numpy(), n_seg)


def row_offsets(shapes):
    """Offsets of per-row segments for a list of 2-D weight shapes laid out back to back."""
    offs = [0]
    for rows, cols in shapes:
        for _ in range(rows):
            offs.append(offs[-1] + cols)
    return np.array(offs, dtype=np.int64)
