"""Independent references that pin the oracle (test helpers; no GPU, no oracle imports).

Each function computes something the paper or plain mathematics fixes, by a route that
shares nothing with the oracle's sort + pool-adjacent-violators code:

* ``R_pairwise``        -- the penalty by its O(d^2) definition (Sec. 1, eq. reg).
* ``R_hyperplanes``     -- the penalty as the max over all orderings of the hyperplanes
                           h_pi (Sec. 2, eq. hyperplane / eq. r_alt).
* ``brute_force_prox``  -- exact minimiser of l*R(u) + 1/2||u-w||^2 by enumerating every
                           weak ordering of the output (ordered set partitions); on each
                           piece R is linear, so the restricted minimiser is closed form
                           (definition of prox, App. A.1; piecewise-linear R, Sec. 2).
* ``brute_force_prox_l1`` -- the same enumeration for alpha*R + beta*l1 (sign pattern and
                           zero block of the output enumerated as well).
* ``gcm_slopes``        -- isotonic regression of y as the slopes of the greatest convex
                           minorant of its cumulative-sum diagram, by a monotone-chain
                           lower hull with cross products (isotonic link, Sec. 1.2 and Sec. 3).
* ``naive_end_collisions`` -- repeated "rightmost collision" = last argmin of prefix averages
                           (Sec. 4.2 proposition rightmost_collision; Alg. end_collisions).
* ``kkt_certificate``   -- optimality check w - u in l*dR(u) (App. A.1 eq. prox_opt with the
                           subdifferential of Sec. 2 eq. subdiff_R, written as majorisation).
* ``kkt_certificate_segments`` -- the same certificate vectorised over the segments of a flat
                           buffer (GPU output at full size), in the GPU's own rank order.
* ``neighbour_collides`` -- the if-and-only-if condition for neighbours i, i+1 to collide
                           (App. C corollary "Neighbour collision").
"""
from __future__ import annotations

import itertools

import numpy as np


def R_pairwise(w) -> float:
    w = np.asarray(w, dtype=np.float64)
    d = w.shape[0]
    if d < 2:
        return 0.0
    diff = np.abs(w[:, None] - w[None, :])
    return float(np.triu(diff, 1).sum() / (d - 1))


def hyperplane_coeffs(order):
    """Coefficients of h_pi for the increasing ordering ``order`` (0-based element ids):
    element order[i] (1-based position i) gets (2i - d - 1)/(d - 1)."""
    d = len(order)
    c = np.zeros(d)
    for pos, e in enumerate(order, start=1):
        c[e] = (2 * pos - d - 1) / (d - 1)
    return c


def R_hyperplanes(w) -> float:
    w = np.asarray(w, dtype=np.float64)
    return max(float(hyperplane_coeffs(p) @ w) for p in itertools.permutations(range(len(w))))


def _set_partitions(items):
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for part in _set_partitions(rest):
        for i in range(len(part)):
            yield part[:i] + [[first] + part[i]] + part[i + 1:]
        yield [[first]] + part


def weak_orderings(d):
    """All ordered set partitions of range(d) (Fubini number many)."""
    for part in _set_partitions(list(range(d))):
        for blocks in itertools.permutations(part):
            yield blocks


def brute_force_prox(w, lam):
    """Exact prox by enumeration over weak orderings; d <= 7."""
    w = np.asarray(w, dtype=np.float64)
    d = w.shape[0]
    if d == 1 or lam == 0:
        return w.copy()
    coef = (2.0 * np.arange(d) + 1.0 - d) / (d - 1)  # rank k (0-based) -> (2(k+1)-d-1)/(d-1)
    best, best_u = np.inf, None
    for blocks in weak_orderings(d):
        r = 0
        vals = []
        for b in blocks:
            n = len(b)
            vals.append(w[list(b)].mean() - lam * coef[r:r + n].mean())
            r += n
        if any(vals[i] >= vals[i + 1] for i in range(len(vals) - 1)):
            continue  # not on this piece of R
        u = np.empty(d)
        for b, val in zip(blocks, vals):
            u[list(b)] = val
        obj = lam * R_pairwise(u) + 0.5 * float(((u - w) ** 2).sum())
        if obj < best:
            best, best_u = obj, u
    return best_u


def brute_force_prox_l1(w, alpha, beta):
    """Exact minimiser of alpha*R(u) + beta*||u||_1 + 1/2||u-w||^2 by enumeration; 2 <= d <= 6.

    A piece of the objective is fixed by a weak ordering of the output and by which of its
    blocks sit below zero, at zero, above zero: either one block is pinned at 0 (blocks before
    it negative, after it positive) or none is and a split point separates negative from
    positive blocks.  On a piece R and l1 are linear, so each free block's restricted
    minimiser is mean(w_g) - alpha*mean(coef over its ranks) - beta*sign_g.  The objective is
    strictly convex, so the best candidate that lies on its own piece is the minimiser
    (definition of prox, Sec. 1; the l1 prox as soft-thresholding, App. A.1 example)."""
    w = np.asarray(w, dtype=np.float64)
    d = w.shape[0]
    coef = (2.0 * np.arange(d) + 1.0 - d) / (d - 1)
    best, best_u = np.inf, None
    for blocks in weak_orderings(d):
        nb = len(blocks)
        pieces = [(z, z) for z in range(nb)] + [(None, s) for s in range(nb + 1)]
        for zero, split in pieces:
            r = 0
            vals = []
            ok = True
            for gi, b in enumerate(blocks):
                n = len(b)
                if zero is not None and gi == zero:
                    vals.append(0.0)
                else:
                    sgn = -1.0 if gi < split else 1.0
                    val = w[list(b)].mean() - alpha * coef[r:r + n].mean() - beta * sgn
                    if not (val * sgn > 0.0):
                        ok = False
                    vals.append(val)
                r += n
            if not ok or any(vals[i] >= vals[i + 1] for i in range(nb - 1)):
                continue
            u = np.empty(d)
            for b, val in zip(blocks, vals):
                u[list(b)] = val
            obj = alpha * R_pairwise(u) + beta * float(np.abs(u).sum()) + 0.5 * float(((u - w) ** 2).sum())
            if obj < best:
                best, best_u = obj, u
    return best_u


def gcm_slopes(y):
    """Isotonic (non-decreasing) regression of y via the lower convex hull of the
    cumulative-sum diagram (k, sum_{j<k} y_j), k = 0..d.  Collinear points are dropped."""
    y = np.asarray(y, dtype=np.float64)
    d = y.shape[0]
    S = np.concatenate([[0.0], np.cumsum(y)])
    hull = []
    for k in range(d + 1):
        while len(hull) >= 2:
            a, b = hull[-2], hull[-1]
            # drop b if it is on or above the segment a -> k (cross product <= 0)
            cross = (b - a) * (S[k] - S[a]) - (k - a) * (S[b] - S[a])
            if cross <= 0:
                hull.pop()
            else:
                break
        hull.append(k)
    out = np.empty(d)
    for a, b in zip(hull[:-1], hull[1:]):
        out[a:b] = (S[b] - S[a]) / (b - a)
    return out, hull


def naive_end_collisions(y):
    """Sec. 4.2: from the leftmost remaining particle i, everything up to the LAST argmin of
    the prefix averages of y[i:] sticks together; repeat from the next particle."""
    y = np.asarray(y, dtype=np.float64)
    d = y.shape[0]
    out = np.empty(d)
    starts = []
    i = 0
    while i < d:
        avg = np.cumsum(y[i:]) / np.arange(1, d - i + 1)
        m = avg.min()
        j = i + int(np.nonzero(avg == m)[0][-1])
        out[i:j + 1] = avg[j - i]
        starts.append(i)
        i = j + 1
    return out, starts


def shift(d, lam):
    """Rank-dependent velocities v_k = lam (d-1-2k)/(d-1), k = 0..d-1 (Alg. prox, line 'v <- ...')."""
    if d < 2:
        return np.zeros(d)
    k = np.arange(d, dtype=np.float64)
    return lam * (d - 1 - 2 * k) / (d - 1)


def kkt_certificate(w, u, lam, tol):
    """Check u == prox_{lam R}(w) through w - u in lam * dR(u).  Returns (ok, message).

    In the order of (u, w), u's tie groups C must be rank intervals on which u is constant, with
    u strictly increasing across groups; each group's value must equal the group's average of
    y = x + v; and every proper prefix (lowest-w elements) of a group must have average y >= u_C.
    The last two are majorisation by the permutahedron of the group's hyperplane coefficients."""
    w = np.asarray(w, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    d = w.shape[0]
    if d < 2 or lam == 0:
        ok = np.allclose(u, w, atol=tol, rtol=0)
        return ok, "identity case"
    order = np.lexsort((w, u))  # sort by u, then w
    x = w[order]
    uu = u[order]
    if np.any(np.diff(x) < 0):
        return False, "order of w not preserved by u"
    y = x + shift(d, lam)
    # groups: maximal runs of equal u
    cuts = np.nonzero(np.diff(uu) != 0)[0] + 1
    bounds = np.concatenate([[0], cuts, [d]])
    for a, b in zip(bounds[:-1], bounds[1:]):
        uc = uu[a]
        seg = y[a:b]
        if abs(seg.mean() - uc) > tol:
            return False, "group [%d,%d) value %.17g != avg y %.17g" % (a, b, uc, seg.mean())
        pref = np.cumsum(seg)[:-1] / np.arange(1, b - a)
        if pref.size and pref.min() < uc - tol:
            return False, "group [%d,%d) prefix average below value" % (a, b)
    return True, "ok"


def neighbour_collides(y, i):
    """Particles i and i+1 (0-based) collide iff max_{j<=i} avg(y[j..i]) >= min_{j>=i+1} avg(y[i+1..j])."""
    y = np.asarray(y, dtype=np.float64)
    left = np.cumsum(y[:i + 1][::-1]) / np.arange(1, i + 2)
    right = np.cumsum(y[i + 1:]) / np.arange(1, y.shape[0] - i)
    return left.max() >= right.min()


def kkt_certificate_segments(w, offsets, u, lam, tol_rel=1e-6, perm=None, start=None):
    """Vectorised form of ``kkt_certificate`` over every segment of a flat buffer, usable on
    GPU output at full size (App. A.1 eq. prox_opt with Sec. 2 eq. subdiff_R).

    Per segment s with d >= 2 and lam_s > 0, in the rank order (``perm``: segment-local indices
    in rank order, with ``start`` marking the first rank of every group; without them the order
    of (u, w) and the maximal runs of equal u), with v_k = lam (d-1-2k)/(d-1) and y = x + v:
      order     x non-decreasing along the ranks;
      constant  u equal inside a group;
      increase  group values non-decreasing along the ranks, up to tol (strictly increasing in
                exact arithmetic; a decrease below tol is a near-tie split);
      mean      group value = mean of y over the group, within tol;
      prefix    every proper prefix of a group has mean y >= group value - tol (majorisation:
                (w - u)/lam restricted to the group lies in the permutahedron of its
                hyperplane coefficients).
    Identity segments (d = 1 or lam = 0) must return w unchanged; segments holding a non-finite
    weight are skipped.  tol = tol_rel * max |w| of the segment.  Returns a dict of the worst
    slack per condition and ``ok``."""
    w = np.asarray(w, np.float32).astype(np.float64)
    u = np.asarray(u, np.float64)
    offsets = np.asarray(offsets, np.int64)
    n = w.shape[0]
    lens = np.diff(offsets)
    nseg = lens.shape[0]
    lam_s = np.asarray(lam, np.float64).reshape(-1)
    if lam_s.shape[0] != nseg:
        lam_s = np.full(nseg, float(lam_s[0]))
    res = dict(ok=True, order=0.0, constant=0, increase=0.0, mean=0.0, prefix=0.0, identity=0.0, groups=0)
    if n == 0:
        return res
    seg_of = np.repeat(np.arange(nseg), lens)
    seg_lo = np.repeat(offsets[:-1], lens)
    nz = lens > 0
    scale = np.ones(nseg)
    finite_seg = np.ones(nseg, bool)
    scale[nz] = np.maximum.reduceat(np.abs(w), offsets[:-1][nz])
    finite_seg[nz] = np.logical_and.reduceat(np.isfinite(w), offsets[:-1][nz])
    scale[~np.isfinite(scale) | (scale == 0)] = 1.0
    tol = tol_rel * scale
    ident_seg = (lens <= 1) | ~(lam_s > 0)
    ident = (ident_seg & finite_seg)[seg_of]
    if ident.any():
        res["identity"] = float(np.abs(u[ident] - w[ident]).max())
    if perm is not None:
        order = seg_lo + np.asarray(perm, np.int64)
        starts = np.asarray(start).astype(bool).copy()
    else:
        order = np.lexsort((w, u, seg_of))
        uo = u[order]
        starts = np.ones(n, bool)
        starts[1:] = uo[1:] != uo[:-1]
    first = np.zeros(n, bool)
    first[offsets[:-1][nz]] = True
    starts |= first
    act = ((~ident_seg) & finite_seg)[seg_of]  # per rank position (segments are contiguous)
    x = w[order]
    ur = u[order]
    k = (np.arange(n) - seg_lo).astype(np.float64)
    d = lens[seg_of].astype(np.float64)
    lam_r = lam_s[seg_of]
    v = np.where(act, lam_r * (d - 1.0 - 2.0 * k) / np.maximum(d - 1.0, 1.0), 0.0)
    tol_r = tol[seg_of]
    inner = act[1:] & ~first[1:]
    dx = np.diff(x)
    if inner.any():
        res["order"] = float(-np.min(np.where(inner, dx, 0.0)))
        same = inner & ~starts[1:]
        res["constant"] = int(np.count_nonzero(same & (ur[1:] != ur[:-1])))
        jump = inner & starts[1:]
        res["increase"] = float(np.max(np.where(jump, (ur[:-1] - ur[1:]) / tol_r[1:], -np.inf)))
    gs = np.nonzero(starts)[0]
    glen = np.diff(np.concatenate([gs, [n]]))
    gact = act[gs]
    res["groups"] = int(np.count_nonzero(gact))
    c = np.where(act, x + v - ur, 0.0)  # y - u: each group sums to ~0, so the running sum stays small
    cs = np.cumsum(c)
    base = np.concatenate([[0.0], cs])[gs]  # running sum before each group
    gsum = np.concatenate([cs[gs[1:] - 1], [cs[-1]]]) - base
    if gact.any():
        res["mean"] = float(np.max(np.abs(gsum / glen)[gact] / tol_r[gs][gact]))
    pref = cs - np.repeat(base, glen)
    plen = (np.arange(n) - np.repeat(gs, glen) + 1).astype(np.float64)
    last = np.zeros(n, bool)
    last[np.concatenate([gs[1:] - 1, [n - 1]])] = True
    proper = act & ~last
    if proper.any():
        res["prefix"] = float(np.max(np.where(proper, -(pref / plen) / tol_r, -np.inf)))
    res["ok"] = bool(res["order"] <= 0.0 and res["constant"] == 0 and res["increase"] <= 1.0
                     and res["mean"] <= 1.0 and res["prefix"] <= 1.0 and res["identity"] == 0.0)
    return res
