"""Helpers for GPU parity tests: run the HIP library, compare with the CPU oracle.

Acceptance (per segment, scale = max |w| of the segment):
  * values: |u_gpu - u_oracle| <= 1e-5 * scale + 2 ulp(u)   (normwise relative 1e-5);
  * saved_perm: a permutation of the segment that sorts it (ties in any order);
  * partition: neighbours (in the oracle's rank order) are in the same cluster on both sides,
    except at near-ties: a boundary only one side has is excused when that side's two cluster
    values differ by less than 1e-6 * scale (the two y-averages are that close, so either
    decision is within the FP tolerance of the other);
  * cluster values are constant within each GPU cluster and non-decreasing in rank order.
"""
from __future__ import annotations

import os

import numpy as np
import torch

import oracle
import paper_2311_03096_amd as wsr

NTHREADS = max(1, min(16, os.cpu_count() or 1))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def mask_to_start(mask_words, n):
    bits = np.unpackbits(np.ascontiguousarray(mask_words).view(np.uint8), bitorder="little")
    return bits[:n].astype(np.uint8)


def seg_start_of_rank(offsets):
    lens = np.diff(offsets)
    return np.repeat(offsets[:-1], lens)


def gpu_forward(w, offsets, lam, save=True, batched=False, lam_arr=None, plan_flags=0, autotune=False):
    wt = dev(w)
    out = torch.empty_like(wt)
    n = w.shape[0]
    perm = torch.full((n,), -1, dtype=torch.int32, device="cuda") if save else None
    mask = torch.full(((n + 31) // 32,), -1, dtype=torch.int32, device="cuda") if save else None
    if batched:
        plan = wsr.wsr_plan_create(offsets, plan_flags)
        try:
            nb = wsr.wsr_plan_workspace_bytes(plan)
            ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
            la = dev(np.asarray(lam_arr, np.float32)) if lam_arr is not None else None
            if autotune:
                wsr.wsr_plan_autotune(plan, wt, out, la, lam, ws)
            wsr.wsr_prox_forward_batched(plan, wt, out, la, lam, perm, mask, ws)
            torch.cuda.synchronize()
        finally:
            wsr.wsr_plan_destroy(plan)
    else:
        nb = wsr.wsr_workspace_bytes(offsets)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
        wsr.wsr_prox_forward(wt, out, offsets, lam, perm, mask, ws)
        torch.cuda.synchronize()
    res = dict(out=out.cpu().numpy())
    if save:
        res["perm"] = perm.cpu().numpy()
        res["start"] = mask_to_start(mask.cpu().numpy(), n)
    return res


def gpu_backward(g, offsets, perm, start, batched=False):
    n = g.shape[0]
    words = np.packbits(np.concatenate([start, np.zeros((-n) % 32, np.uint8)]), bitorder="little").view(np.int32)
    gt, pt, mt = dev(g.astype(np.float32)), dev(perm.astype(np.int32)), dev(words)
    gw = torch.empty_like(gt)
    if batched:
        plan = wsr.wsr_plan_create(offsets)
        try:
            nb = wsr.wsr_plan_workspace_bytes(plan)
            ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
            wsr.wsr_prox_backward_batched(plan, gt, gw, pt, mt, ws)
            torch.cuda.synchronize()
        finally:
            wsr.wsr_plan_destroy(plan)
    else:
        nb = wsr.wsr_workspace_bytes(offsets)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
        wsr.wsr_prox_backward(gt, gw, offsets, pt, mt, ws)
        torch.cuda.synchronize()
    return gw.cpu().numpy()


def oracle_forward(w, offsets, lam):
    u, perm, start = oracle.prox_segments(w, lam, offsets, n_threads=NTHREADS)
    return dict(u=u, perm=perm, start=start)


def compare(w, offsets, g_res, o_res, rel_tol=1e-5, tie_rel=1e-6):
    """Return a stats dict; raises AssertionError on a violation."""
    w = np.asarray(w, np.float32)
    offsets = np.asarray(offsets, np.int64)
    n = w.shape[0]
    out = g_res["out"].astype(np.float64)
    u = o_res["u"]
    lens = np.diff(offsets)
    seg_of = np.repeat(np.arange(lens.shape[0]), lens)
    absw = np.abs(w.astype(np.float64))
    scale = np.ones(lens.shape[0])
    nz = lens > 0
    scale[nz] = np.maximum.reduceat(absw, offsets[:-1][nz])
    scale[(scale == 0) | ~np.isfinite(scale)] = 1.0
    sc = scale[seg_of]
    finite = np.isfinite(u)
    assert np.array_equal(np.isnan(out), ~finite), "NaN pattern differs"
    err = np.abs(out - u)
    err[~finite] = 0.0
    ulp = np.spacing(np.abs(u).astype(np.float32)).astype(np.float64)
    ulp[~finite] = 0.0
    bad = err > rel_tol * sc + 2 * ulp
    stats = dict(max_abs_err=float(err.max()) if n else 0.0,
                 max_rel_err=float((err / sc).max()) if n else 0.0,
                 n=n, n_seg=int(lens.shape[0]))
    assert not bad.any(), "value mismatch at %s: gpu %r oracle %r" % (
        np.nonzero(bad)[0][:5], out[bad][:5], u[bad][:5])
    if "perm" not in g_res:
        return stats
    perm = g_res["perm"].astype(np.int64)
    sstart = seg_start_of_rank(offsets)
    orig = sstart + perm
    # a permutation of each segment that sorts it
    assert np.all((perm >= 0) & (perm < np.repeat(lens, lens))), "perm out of range"
    cnt = np.bincount(orig, minlength=n)
    assert np.all(cnt == 1), "perm is not a permutation"
    first = np.zeros(n, bool)
    first[offsets[:-1][nz]] = True
    start = g_res["start"].astype(bool)
    # identity segments (lam = 0, d = 1, non-finite) may keep the identity permutation
    o_all = np.ones(lens.shape[0], bool)
    g_all = np.ones(lens.shape[0], bool)
    is_id = np.ones(lens.shape[0], bool)
    if nz.any():
        idx = offsets[:-1][nz]
        o_all[nz] = np.minimum.reduceat(o_res["start"].astype(np.uint8), idx) == 1
        g_all[nz] = np.minimum.reduceat(start.astype(np.uint8), idx) == 1
        is_id[nz] = np.minimum.reduceat((perm == np.arange(n) - sstart).astype(np.uint8), idx) == 1
    exempt = (o_all & g_all & is_id)[seg_of]
    xs = w[orig].astype(np.float64)
    dx = np.diff(xs)
    assert np.all((dx >= 0) | first[1:] | ~np.isfinite(dx) | exempt[1:]), "perm does not sort its segment"
    assert np.all(start[first]), "rank 0 of a segment must start a cluster"
    # cluster values constant inside a GPU cluster, non-decreasing across
    ov = out[orig]
    same = ~start[1:] & ~first[1:]
    fin = np.isfinite(ov[1:]) & np.isfinite(ov[:-1])
    assert np.all(ov[1:][same & fin] == ov[:-1][same & fin]), "value not constant in a cluster"
    # monotone along the ranks; a decrease is only allowed at a near-tie (both values within
    # the tie threshold, where the two neighbouring y-averages are equal to FP64 noise)
    dec = (ov[:-1] - ov[1:])
    dec[~(~first[1:] & fin) | exempt[1:]] = 0.0
    tau_r = tie_rel * sc[orig[1:]]
    stats_dec = float(dec.max()) if n > 1 else 0.0
    assert np.all(dec <= tau_r), "values decrease along the ranks by %g (max allowed %g) at %s" % (
        stats_dec, float(tau_r.min()) if n > 1 else 0.0, np.nonzero(dec > tau_r)[0][:5])
    # partition in the oracle's rank order
    cid = np.empty(n, np.int64)
    cid[orig] = np.cumsum(start)
    o_orig = sstart + o_res["perm"].astype(np.int64)
    o_start = o_res["start"].astype(bool)
    same_o = ~o_start[1:]
    same_g = cid[o_orig[1:]] == cid[o_orig[:-1]]
    mism = (same_o != same_g) & ~first[1:]
    tau = tie_rel * sc[o_orig[1:]]
    marg_o = np.abs(u[o_orig[1:]] - u[o_orig[:-1]])
    marg_g = np.abs(out[o_orig[1:]] - out[o_orig[:-1]])
    excused = np.where(~same_o, marg_o < tau, marg_g < tau + 2 * ulp[o_orig[1:]])
    unexcused = mism & ~excused
    stats.update(partition_mismatches=int(mism.sum()), unexcused=int(unexcused.sum()),
                 clusters=int(start.sum()), max_rank_decrease=stats_dec,
                 rank_decreases=int((dec > 0).sum()))
    assert not unexcused.any(), "partition differs at ranks %s" % (np.nonzero(unexcused)[0][:5] + 1)
    return stats


def gpu_forward_l1(w, offsets, lam, beta, rho, batched=False, lam_arr=None):
    """Alg. prox in full on the GPU (wsr_prox_l1_forward / _batched); returns the output."""
    wt = dev(w)
    out = torch.empty_like(wt)
    if batched:
        plan = wsr.wsr_plan_create(offsets)
        try:
            nb = wsr.wsr_plan_workspace_bytes(plan)
            ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
            la = dev(np.asarray(lam_arr, np.float32)) if lam_arr is not None else None
            wsr.wsr_prox_l1_forward_batched(plan, wt, out, la, lam, beta, rho, ws)
            torch.cuda.synchronize()
        finally:
            wsr.wsr_plan_destroy(plan)
    else:
        nb = wsr.wsr_workspace_bytes(offsets)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
        wsr.wsr_prox_l1_forward(wt, out, offsets, lam, beta, rho, ws)
        torch.cuda.synchronize()
    return out.cpu().numpy()


def gpu_step(w, grad, offsets, eta, alpha, beta, rho, variant=False, inplace=True, alpha_arr=None):
    """One proximal-gradient step on the GPU (wsr_prox_step_batched); returns (out, w after)."""
    wt, gt = dev(w), dev(grad)
    out = wt if inplace else torch.empty_like(wt)
    plan = wsr.wsr_plan_create(offsets)
    try:
        nb = wsr.wsr_plan_workspace_bytes(plan)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
        aa = dev(np.asarray(alpha_arr, np.float32)) if alpha_arr is not None else None
        wsr.wsr_prox_step_batched(plan, wt, gt, eta, out, aa, alpha, beta, rho,
                                  wsr.WSR_STEP_ETA_IN_DISPLACEMENT if variant else 0, ws)
        torch.cuda.synchronize()
    finally:
        wsr.wsr_plan_destroy(plan)
    return out.cpu().numpy(), wt.cpu().numpy()


def compare_l1(w, offsets, out, o_l1, o_plain, g_plain, beta, rho, rel_tol=1e-5, tie_rel=1e-6):
    """Check the GPU output of Alg. prox in full against the oracle's.

    o_plain / g_plain: the oracle's and the GPU's prox_{lam R} results with their partitions
    (the l1 call makes the same collisions as the plain forward).  Two kinds of element are left
    out of the value check, and counted: those whose prox_{lam R} value lies within
    1e-13 * d * scale of +-beta (the zero test is decided on an FP64 value on either side, from
    sums of d terms of size up to scale, so the two sides' values of u differ by far less than
    that band, and at the threshold either outcome is correct), and, when rho != 0, those
    whose cluster is not the same set of ranks on both sides (near-ties that the compare of the
    plain forward excuses; rewinding moves the output by rho times the mean velocity, which
    depends on the cluster's extent, so there the outputs differ by more than rounding).  ``rho``
    here is the coefficient of the mean velocity in the output's u - rho v form."""
    w = np.asarray(w, np.float32)
    offsets = np.asarray(offsets, np.int64)
    n = w.shape[0]
    out = np.asarray(out, np.float64)
    lens = np.diff(offsets)
    seg_of = np.repeat(np.arange(lens.shape[0]), lens)
    absw = np.abs(w.astype(np.float64))
    scale = np.ones(lens.shape[0])
    nz = lens > 0
    scale[nz] = np.maximum.reduceat(absw, offsets[:-1][nz])
    scale[(scale == 0) | ~np.isfinite(scale)] = 1.0
    sc = scale[seg_of]
    finite = np.isfinite(o_l1)
    assert np.array_equal(np.isnan(out), ~finite), "NaN pattern differs"
    u = o_plain["u"]
    band = 1e-13 * lens[seg_of].astype(np.float64) * sc
    near_zero_test = finite & (np.abs(np.abs(u) - float(np.float32(beta))) < band)
    other_cluster = np.zeros(n, bool)
    if rho != 0 and n:
        sstart = seg_start_of_rank(offsets)
        o_orig = sstart + o_plain["perm"].astype(np.int64)
        g_orig = sstart + g_plain["perm"].astype(np.int64)
        gid = np.empty(n, np.int64)
        gid[g_orig] = np.cumsum(g_plain["start"].astype(np.int64))
        o_first = np.nonzero(o_plain["start"])[0]
        g_seq = gid[o_orig]  # GPU cluster id of each rank, in the oracle's rank order
        lo = np.minimum.reduceat(g_seq, o_first)
        hi = np.maximum.reduceat(g_seq, o_first)
        o_size = np.diff(np.concatenate([o_first, [n]]))
        g_size = np.bincount(gid)[lo]
        same = (lo == hi) & (g_size == o_size)
        other_cluster[o_orig] = np.repeat(~same, o_size)
    skip = near_zero_test | other_cluster
    err = np.abs(out - o_l1)
    err[~finite | skip] = 0.0
    ulp = np.spacing(np.abs(o_l1).astype(np.float32)).astype(np.float64)
    ulp[~finite] = 0.0
    bad = err > rel_tol * sc + 2 * ulp
    assert not bad.any(), "value mismatch at %s: gpu %r oracle %r" % (
        np.nonzero(bad)[0][:5], out[bad][:5], o_l1[bad][:5])
    zeros_g = (out == 0.0) & finite & ~skip
    zeros_o = (o_l1 == 0.0) & finite & ~skip
    assert np.array_equal(zeros_g, zeros_o), "zeroed weights differ"
    return dict(n=n, max_abs_err=float(err.max()) if n else 0.0,
                max_rel_err=float((err / sc).max()) if n else 0.0, zeroed=int(zeros_o.sum()),
                skipped_zero_test=int(near_zero_test.sum()), skipped_partition=int(other_cluster.sum()))
