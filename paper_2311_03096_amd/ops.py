"""Torch-facing wrappers over the C ABI: autograd prox and a batched per-step prox.

Torch supplies device memory and the stream; every step of the prox runs in the library's
HIP kernels.  Buffers for the saved state and the workspace are allocated here (the library
itself never allocates during a compute call).
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib


def _mask_words(n):
    return (n + 31) // 32


def _workspace(nbytes, device):
    if nbytes == 0:
        return None
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _check_f32(t, name):
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError("%s must be a contiguous float32 tensor on the GPU" % name)


class ProxFunction(torch.autograd.Function):
    """u = prox_{lam R}(w) per segment; backward averages the cotangent within clusters."""

    @staticmethod
    def forward(ctx, w, lam, offsets):
        _check_f32(w, "w")
        n = w.numel()
        out = torch.empty_like(w)
        perm = torch.empty(n, dtype=torch.int32, device=w.device)
        mask = torch.empty(_mask_words(n), dtype=torch.int32, device=w.device)
        ws = _workspace(_lib.wsr_workspace_bytes(offsets), w.device)
        _lib.wsr_prox_forward(w, out, offsets, lam, perm, mask, ws)
        ctx.save_for_backward(perm, mask)
        ctx.offsets = offsets
        return out

    @staticmethod
    def backward(ctx, g):
        perm, mask = ctx.saved_tensors
        g = g.contiguous()
        gw = torch.empty_like(g)
        ws = _workspace(_lib.wsr_workspace_bytes(ctx.offsets), g.device)
        _lib.wsr_prox_backward(g, gw, ctx.offsets, perm, mask, ws)
        return gw, None, None


def prox(w, lam, offsets=None):
    """prox_{lam R} of a float32 GPU tensor; ``offsets`` (host, n_seg+1 int64) splits the
    flattened tensor into independent segments (default: one segment)."""
    flat = w.contiguous().view(-1)
    if offsets is None:
        offsets = np.array([0, flat.numel()], dtype=np.int64)
    offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    return ProxFunction.apply(flat, float(lam), offsets).view(w.shape)


def prox_l1(w, lam, beta, rho=0.0, offsets=None):
    """Alg. prox in full on a float32 GPU tensor: prox of lam*R + beta*l1 with rewinding rho,
    per segment (the update of a proximal-gradient step; not differentiable here)."""
    _check_f32(w.contiguous(), "w")
    flat = w.contiguous().view(-1)
    if offsets is None:
        offsets = np.array([0, flat.numel()], dtype=np.int64)
    offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    out = torch.empty_like(flat)
    ws = _workspace(_lib.wsr_workspace_bytes(offsets), flat.device)
    _lib.wsr_prox_l1_forward(flat, out, offsets, lam, beta, rho, ws)
    return out.view(w.shape)


def segment_stats(w, offsets=None):
    """Per segment of a float32 GPU tensor: (R(w), distinct non-zero values, non-zero weights)
    as host numpy arrays (the ratio of the last two is the weight-sharing measure)."""
    _check_f32(w.contiguous(), "w")
    flat = w.contiguous().view(-1)
    if offsets is None:
        offsets = np.array([0, flat.numel()], dtype=np.int64)
    offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
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


class BatchedProx:
    """All segments of a fixed segmentation in one batched call per step (plan created once).

    ``forward(w, out, lam)`` runs the batched prox; with ``save=True`` the saved permutation and
    cluster-start bits for ``backward`` are kept in this object.  ``capture()`` records one
    forward into a HIP graph (torch.cuda.CUDAGraph) for replay with ``replay()``.
    ``autotune=True`` times the merge routes on the first forward's weights (wsr_plan_autotune);
    ``hull_only=True`` merges by the hull merge alone (for comparing routes).
    """

    def __init__(self, offsets, device="cuda", autotune=False, hull_only=False):
        self.offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self.n = int(self.offsets[-1])
        self.device = torch.device(device)
        self.plan = _lib.wsr_plan_create(self.offsets, _lib.WSR_PLAN_MERGE_HULL if hull_only else 0)
        self.tune_pending = bool(autotune)  # tuned on the first forward's weights
        self.ws = _workspace(_lib.wsr_plan_workspace_bytes(self.plan), self.device)
        self.perm = torch.empty(self.n, dtype=torch.int32, device=self.device)
        self.mask = torch.empty(_mask_words(self.n), dtype=torch.int32, device=self.device)
        self.graph = None

    def forward(self, w, out, lam=None, lam_scalar=0.0, save=True):
        _check_f32(w, "w")
        _check_f32(out, "out")
        if self.tune_pending:  # synchronising: done before any graph capture
            _lib.wsr_plan_autotune(self.plan, w, out, lam, lam_scalar, self.ws)
            self.tune_pending = False
        _lib.wsr_prox_forward_batched(self.plan, w, out, lam, lam_scalar,
                                      self.perm if save else None, self.mask if save else None, self.ws)

    def forward_l1(self, w, out, lam=None, lam_scalar=0.0, beta=0.0, rho=0.0):
        """Alg. prox in full (l1 and rewinding lines) over every segment; saves nothing."""
        _check_f32(w, "w")
        _check_f32(out, "out")
        _lib.wsr_prox_l1_forward_batched(self.plan, w, out, lam, lam_scalar, beta, rho, self.ws)

    def step(self, w, grad, eta, alpha=None, alpha_scalar=0.0, beta=0.0, rho=0.0, eta_in_displacement=False,
             out=None):
        """One proximal-gradient step w <- Prox(w - eta*grad) over every segment (in place unless
        ``out`` is given); ``alpha`` is a device tensor of per-segment coefficients or None."""
        _check_f32(w, "w")
        _check_f32(grad, "grad")
        out = w if out is None else out
        if self.tune_pending:  # time the merge routes on these weights (scratch output, not w)
            scratch = torch.empty_like(w)
            _lib.wsr_plan_autotune(self.plan, w, scratch, alpha, float(alpha_scalar) * float(eta), self.ws)
            self.tune_pending = False
        _lib.wsr_prox_step_batched(self.plan, w, grad, eta, out, alpha, alpha_scalar, beta, rho,
                                   _lib.WSR_STEP_ETA_IN_DISPLACEMENT if eta_in_displacement else 0, self.ws)
        return out

    def backward(self, g, gw):
        _lib.wsr_prox_backward_batched(self.plan, g, gw, self.perm, self.mask, self.ws)

    def capture(self, w, out, lam=None, lam_scalar=0.0, save=True):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.forward(w, out, lam, lam_scalar, save)  # warm-up outside the graph
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
