"""Helpers for GPU parity tests: run the HIP library, compare with the CPU oracle.

Acceptance (per segment, scale = max |w| of the segment):
  * values, normwise: |u_gpu - u_oracle| <= 1e-5 * scale + 2 ulp(u)   (the target's 1e-5);
  * values, elementwise: on every element whose GPU cluster and oracle cluster are the same set
    of ranks, the GPU's FP32 value is within 1 ulp of the oracle's FP64 value rounded to FP32;
    for values below 1e-3 * scale the forward error of the GPU's FP64 prefix sums
    (ELEMENT_FP64_ERR below) is allowed on top, since there an FP32 ulp is far below the FP64
    rounding of sums of the segment's size;
  * saved_perm: a permutation of the segment that sorts it (ties in any order);
  * partition: neighbours (in the oracle's rank order) are in the same cluster on both sides,
    except at near-ties: a boundary only one side has is excused when that side's two cluster
    values differ by less than 1e-6 * scale (the two y-averages are that close, so either
    decision is within the FP tolerance of the other);
  * cluster values are constant within each GPU cluster and non-decreasing in rank order;
  * optimality: the GPU output passes the certificate w - u in lam dR(u) (App. A.1 eq. prox_opt,
    Sec. 2 eq. subdiff_R) in the GPU's own rank order, with tolerance 1e-6 * scale.
Reported: max abs / normwise relative error, the max elementwise relative error over
|u| >= 1e-3 * scale, the max error in FP32 ulps on identical clusters, |sum u - sum w| per
segment, partition mismatches and the certificate's slacks.
"""
from __future__ import annotations

import os

import numpy as np
import torch

import oracle
import paper_2311_03096_amd as wsr
import pins

NTHREADS = max(1, min(16, os.cpu_count() or 1))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def mask_to_start(mask_words, n):
    bits = np.unpackbits(np.ascontiguousarray(mask_words).view(np.uint8), bitorder="little")
    return bits[:n].astype(np.uint8)


def autograd_saved_partition(u, offsets):
    """The partition saved by the prox's autograd node behind ``u`` (perm and cluster-start bits of
    the forward), as (perm, start) arrays."""
    node = u.grad_fn
    while node is not None and len(getattr(node, "saved_tensors", None) or ()) != 2:
        node = node.next_functions[0][0] if node.next_functions else None
    if node is None:
        raise ValueError("no prox node with a saved partition behind this tensor")
    perm, mask = node.saved_tensors
    n = int(np.asarray(offsets)[-1])
    return perm.cpu().numpy(), mask_to_start(mask.cpu().numpy(), n)


def seg_start_of_rank(offsets):
    lens = np.diff(offsets)
    return np.repeat(offsets[:-1], lens)


def gpu_forward(w, offsets, lam, save=True, batched=False, lam_arr=None, plan_flags=0, autotune=False,
                sort_routes=None):
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
            if sort_routes is not None:
                wsr.wsr_plan_set_sort_routes(plan, sort_routes)
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


def vjp_check(g, offsets, fw, gw):
    """Backward against the oracle VJP on the GPU's own partition (``fw``: perm and start of the
    forward), to 1 ulp of the FP32 rounding plus the forward error of the GPU's FP64 prefix sums
    of g (tree sums of at most 2^27 terms: 128 * 2^-53 * sum |g| over the segment, divided by the
    cluster's size).  Returns the max error in ulps."""
    offsets = np.asarray(offsets, np.int64)
    ref = oracle.vjp(np.asarray(g, np.float64), fw["perm"], fw["start"], offsets)
    lens = np.diff(offsets)
    seg_of = np.repeat(np.arange(lens.shape[0]), lens)
    G = np.zeros(lens.shape[0])
    nz = lens > 0
    G[nz] = np.add.reduceat(np.abs(np.asarray(g, np.float64)), offsets[:-1][nz])
    cid = np.cumsum(np.asarray(fw["start"], np.int64))  # GPU cluster of each rank
    csize_rank = np.bincount(cid)[cid]
    csize = np.empty_like(csize_rank)
    csize[np.repeat(offsets[:-1], lens) + np.asarray(fw["perm"], np.int64)] = csize_rank
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    tol = ulp + 128 * 2.0 ** -53 * G[seg_of] / csize
    err = np.abs(np.asarray(gw, np.float64) - ref)
    bad = err > tol
    max_ulps = float((err / np.maximum(ulp, 1e-300)).max()) if err.size else 0.0
    print("  backward vs oracle VJP on the GPU partition: max abs err %.3g, max ulps %.3g" % (
        float(err.max()) if err.size else 0.0, max_ulps), flush=True)
    assert not bad.any(), "backward mismatch at %s: gpu %r oracle %r" % (
        np.nonzero(bad)[0][:5], np.asarray(gw)[bad][:5], ref[bad][:5])
    return max_ulps


def oracle_forward(w, offsets, lam):
    u, perm, start = oracle.prox_segments(w, lam, offsets, n_threads=NTHREADS)
    return dict(u=u, perm=perm, start=start)


# Elementwise allowance beyond 1 ulp on identical clusters: the GPU forms a cluster value as
# c + (S_b - S_a)/(b - a) from FP64 prefix sums S of the centred sorted weights (tree sums of at
# most 2^27 terms), so |error| <= 2 * 64 * 2^-53 * sum_k |x_k - c| / (b - a); M below is that sum
# per segment (an upper bound of every |S_k|) plus lam * d / 4 for the closed-form velocity sums.
ELEMENT_FP64_ERR = 128 * 2.0 ** -53


def same_cluster(offsets, o_perm, o_start, g_perm, g_start):
    """Per element (original order): True where the GPU's cluster and the oracle's cluster are the
    same set of ranks; also the size of the oracle's cluster."""
    offsets = np.asarray(offsets, np.int64)
    n = int(offsets[-1])
    if n == 0:
        return np.zeros(0, bool), np.zeros(0, np.int64)
    sstart = seg_start_of_rank(offsets)
    o_orig = sstart + np.asarray(o_perm, np.int64)
    g_orig = sstart + np.asarray(g_perm, np.int64)
    gid = np.empty(n, np.int64)
    gid[g_orig] = np.cumsum(np.asarray(g_start, np.int64))
    o_first = np.nonzero(o_start)[0]
    g_seq = gid[o_orig]  # GPU cluster id of each rank, in the oracle's rank order
    lo = np.minimum.reduceat(g_seq, o_first)
    hi = np.maximum.reduceat(g_seq, o_first)
    o_size = np.diff(np.concatenate([o_first, [n]]))
    g_size = np.bincount(gid)[lo]
    same = (lo == hi) & (g_size == o_size)
    res = np.empty(n, bool)
    size = np.empty(n, np.int64)
    res[o_orig] = np.repeat(same, o_size)
    size[o_orig] = np.repeat(o_size, o_size)
    return res, size


def runs_as_clusters(offsets, o_perm, out):
    """GPU clusters read from an output without saved state: maximal runs of equal values along
    the oracle's rank order (the GPU writes one value per cluster).  Returns (perm, start)."""
    offsets = np.asarray(offsets, np.int64)
    n = int(offsets[-1])
    o_orig = seg_start_of_rank(offsets) + np.asarray(o_perm, np.int64)
    ov = np.asarray(out)[o_orig]
    start = np.ones(n, np.uint8)
    if n > 1:
        start[1:] = (ov[1:] != ov[:-1]).astype(np.uint8)
    first = offsets[:-1][np.diff(offsets) > 0]
    start[first] = 1
    return np.asarray(o_perm), start


def _per_segment(val, nseg):
    a = np.asarray(val, np.float64).reshape(-1)
    return np.full(nseg, float(a[0])) if a.shape[0] == 1 else a


def element_check(w, offsets, out, u, lam, same, csize, scale_el, o_perm, ref=None, extra=0.0):
    """Elementwise bar on identical clusters (see the module docstring); returns the stats.  ``u`` is
    the oracle's prox_{lam R} value (whose FP64 error the allowance bounds); ``ref`` (default u) the
    oracle value the output must match, with ``extra`` added to the allowance (per element)."""
    w = np.asarray(w, np.float32)
    offsets = np.asarray(offsets, np.int64)
    lens = np.diff(offsets)
    nseg = lens.shape[0]
    n = w.shape[0]
    seg_of = np.repeat(np.arange(nseg), lens)
    fin = np.isfinite(u) & np.isfinite(out)
    u32 = u.astype(np.float32)
    ulp = np.spacing(np.abs(u32)).astype(np.float64)
    # forward-error allowance of the GPU's FP64 sums, per segment: sum |x - c| with c the sorted
    # middle element (the centre the kernels subtract) plus the closed-form velocity sums
    wd = w.astype(np.float64)
    M = np.zeros(nseg)
    nz = lens > 0
    if nz.any():
        xs = wd[seg_start_of_rank(offsets) + np.asarray(o_perm, np.int64)]
        c = np.zeros(nseg)
        c[nz] = xs[offsets[:-1][nz] + lens[nz] // 2]
        dev = np.abs(wd - c[seg_of])
        dev[~np.isfinite(dev)] = 0.0
        M[nz] = np.add.reduceat(dev, offsets[:-1][nz])
    M = M + np.abs(_per_segment(lam, nseg)) * lens / 4.0
    allow = ELEMENT_FP64_ERR * M[seg_of] / np.maximum(csize, 1) + extra
    if ref is not None:
        u = np.asarray(ref, np.float64)
        fin = np.isfinite(u) & np.isfinite(out)
        u32 = u.astype(np.float32)
        ulp = np.spacing(np.abs(u32)).astype(np.float64)
    m = same & fin
    e32 = np.abs(out.astype(np.float64) - u32.astype(np.float64))
    ulps = np.zeros(n)
    ulps[m] = e32[m] / ulp[m]
    beyond = m & (e32 > ulp)
    big = m & (np.abs(u) >= 1e-3 * scale_el)
    # 1 ulp, strictly, for |u| >= 1e-3 * scale; below that the FP64 allowance as well
    bad = beyond & (big | (np.abs(out.astype(np.float64) - u) > ulp + allow))
    rel = np.zeros(n)
    rel[big] = np.abs(out.astype(np.float64)[big] - u[big]) / np.abs(u[big])
    st = dict(identical_cluster_elements=int(m.sum()), max_ulps=float(ulps.max()) if n else 0.0,
              beyond_1ulp=int(beyond.sum()), beyond_1ulp_large=int((beyond & big).sum()),
              max_elementwise_rel_err_large=float(rel.max()) if n else 0.0)
    assert not bad.any(), "elementwise error beyond 1 ulp + FP64 allowance at %s: gpu %r oracle %r" % (
        np.nonzero(bad)[0][:5], out[bad][:5], u[bad][:5])
    return st


def compare(w, offsets, g_res, o_res, rel_tol=1e-5, tie_rel=1e-6, lam=None):
    """Return a stats dict; raises AssertionError on a violation.  ``lam`` (scalar or per segment)
    enables the optimality certificate on the GPU output."""
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
    # momentum (Sec. 3): the sum of each segment is preserved
    if nz.any():
        wf = np.where(finite, w.astype(np.float64), 0.0)
        of = np.where(finite, out, 0.0)
        dsum = np.abs(np.add.reduceat(of, offsets[:-1][nz]) - np.add.reduceat(wf, offsets[:-1][nz]))
        stats["max_abs_sum_diff"] = float(dsum.max())
    g_perm, g_start = (g_res["perm"], g_res["start"]) if "perm" in g_res else runs_as_clusters(
        offsets, o_res["perm"], g_res["out"])
    same, csize = same_cluster(offsets, o_res["perm"], o_res["start"], g_perm, g_start)
    stats.update(element_check(w, offsets, g_res["out"], u, lam if lam is not None else 0.0, same, csize, sc,
                               o_res["perm"]))
    if lam is not None:
        cert = pins.kkt_certificate_segments(w, offsets, out, lam, tol_rel=tie_rel, perm=g_perm, start=g_start)
        stats["certificate"] = {k: v for k, v in cert.items() if k != "ok"}
        assert cert["ok"], "optimality certificate fails: %r" % cert
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


def step_reference(w, grad, off, eta, alpha, beta, rho, variant, alpha_arr=None):
    """The oracle's step output, and the plain prox_{lam R} of z = fmaf(-eta, grad, w) with the
    step's lambda on both sides (its partitions decide the near-tie excuses)."""
    f32 = np.float32
    a = np.asarray(alpha_arr, np.float32) if alpha_arr is not None else f32(alpha)
    o = oracle.prox_step_segments(w, grad, eta, a, beta, rho, off, eta_in_displacement=variant, n_threads=NTHREADS)
    z = oracle.grad_step(w, grad, eta)
    lam_eff = a if variant else (f32(eta) * a).astype(np.float32)
    beta_eff = beta if variant else float(f32(eta) * f32(beta))
    q = 1.0 - (eta if variant else 1.0) * (1.0 - rho)  # coefficient of v in u - q v
    lam_s = float(np.atleast_1d(lam_eff)[0])
    g_plain = gpu_forward(z, off, lam_s, batched=True, lam_arr=lam_eff if alpha_arr is not None else None)
    u, p, s = oracle.prox_segments(z, lam_eff, off, n_threads=NTHREADS)
    return o, z, dict(u=u, perm=p, start=s), g_plain, beta_eff, q, lam_eff


def compare_l1(w, offsets, out, o_l1, o_plain, g_plain, beta, rho, lam, rel_tol=1e-5, tie_rel=1e-6):
    """Check the GPU output of Alg. prox in full against the oracle's.

    o_plain / g_plain: the oracle's and the GPU's prox_{lam R} results with their partitions
    (the l1 call makes the same collisions as the plain forward).  The plain results are first
    checked with ``compare``, which requires every partition difference to be a near-tie (a
    boundary whose two cluster values differ by less than tie_rel * scale).  Two kinds of element
    are then left out of the l1 value check, and counted: those whose prox_{lam R} value lies
    within 1e-13 * d * scale of +-beta (the zero test is decided on an FP64 value on either side,
    from sums of d terms of size up to scale, so the two sides' values of u differ by far less
    than that band, and at the threshold either outcome is correct), and, when rho != 0, those
    whose cluster is not the same set of ranks on both sides (the near-ties just verified;
    rewinding moves the output by rho times the mean velocity, which depends on the cluster's
    extent, so there the outputs differ by more than rounding).  ``rho`` here is the coefficient
    of the mean velocity in the output's u - rho v form.  On identical clusters the output must be
    within 1 ulp of the oracle's FP64 value rounded to FP32, plus the FP64 allowance of the cluster
    value and the rounding of the epilogue's terms."""
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
    plain_stats = compare(w, offsets, g_plain, o_plain, rel_tol=rel_tol, tie_rel=tie_rel, lam=lam)
    finite = np.isfinite(o_l1)
    assert np.array_equal(np.isnan(out), ~finite), "NaN pattern differs"
    u = o_plain["u"]
    band = 1e-13 * lens[seg_of].astype(np.float64) * sc
    near_zero_test = finite & (np.abs(np.abs(u) - float(np.float32(beta))) < band)
    same, csize = (same_cluster(offsets, o_plain["perm"], o_plain["start"], g_plain["perm"], g_plain["start"])
                   if n else (np.zeros(0, bool), np.zeros(0, np.int64)))
    other_cluster = ~same if rho != 0 else np.zeros(n, bool)
    skip = near_zero_test | other_cluster
    err = np.abs(out - o_l1)
    err[~finite | skip] = 0.0
    ulp = np.spacing(np.abs(o_l1).astype(np.float32)).astype(np.float64)
    ulp[~finite] = 0.0
    bad = err > rel_tol * sc + 2 * ulp
    assert not bad.any(), "value mismatch at %s: gpu %r oracle %r" % (
        np.nonzero(bad)[0][:5], out[bad][:5], o_l1[bad][:5])
    # the soft threshold zeroes a cluster when |u| < beta (both sides decide it the same way on
    # their FP64 u; the near-threshold band is skipped above): those outputs are exactly zero on
    # both sides.  Any other exact zero comes from the rewinding line's cancellation (u - rho v of
    # a cluster whose weights are all zero is zero in exact arithmetic), which the GPU's FP64
    # prefix-sum form leaves as a rounding residue: there the other side must be zero up to FP64
    # rounding of the segment's scale.
    thr = finite & ~skip & (np.abs(u) < float(np.float32(beta)))
    assert np.all(out[thr] == 0.0) and np.all(o_l1[thr] == 0.0), "thresholded weights are not zero"
    rest = finite & ~skip & ~thr
    cancel = 1e-11 * sc
    zo, zg = rest & (o_l1 == 0.0), rest & (out == 0.0)
    assert np.all(np.abs(out[zo]) <= cancel[zo]) and np.all(np.abs(o_l1[zg]) <= cancel[zg]), \
        "zeroed weights differ beyond the rewinding's rounding"
    zeros_o = (o_l1 == 0.0) & finite & ~skip
    lam_el = _per_segment(lam, lens.shape[0])[seg_of]
    extra = 8 * 2.0 ** -53 * (np.abs(u) + np.abs(lam_el) + abs(float(beta)))
    est = element_check(w, offsets, out, u, lam, same & ~near_zero_test, csize, sc, o_plain["perm"],
                        ref=o_l1, extra=np.where(np.isfinite(extra), extra, 0.0))
    res = dict(n=n, max_abs_err=float(err.max()) if n else 0.0,
               max_rel_err=float((err / sc).max()) if n else 0.0, zeroed=int(zeros_o.sum()),
               skipped_zero_test=int(near_zero_test.sum()), skipped_partition=int((other_cluster & ~near_zero_test).sum()),
               plain_partition_mismatches=plain_stats.get("partition_mismatches", 0))
    res.update(est)
    return res
