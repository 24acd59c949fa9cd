"""Seeded synthetic inputs shaped like the paper's workloads (no prox arithmetic here).

Every generator draws in FP64 with numpy.random.default_rng(seed) and casts to FP32, so the GPU
library and the CPU oracle see identical bits.  The paper trains on CIFAR10 / MNIST (Sec. 6);
those datasets and trained weights are not used: freshly initialised weights of the same shapes
stand in for them.

Each function returns a dict with
  w        float32 array (flat, segment-major)
  offsets  int64 array of n_seg + 1 segment offsets
  lam      float (prox scale = step size x penalty)
and, where relevant, ``g`` (upstream gradient, float32) and a short ``name``.
"""
from __future__ import annotations

import numpy as np


def _pack(name, w, offsets, lam, **extra):
    d = dict(name=name, w=np.ascontiguousarray(w, dtype=np.float32),
             offsets=np.ascontiguousarray(offsets, dtype=np.int64), lam=float(np.float32(lam)))
    d.update(extra)
    return d


def plain(d=4096, lam=0.1, seed=0):
    """One vector of N(0,1) weights."""
    rng = np.random.default_rng(seed)
    return _pack("plain_d%d" % d, rng.standard_normal(d), [0, d], lam)


def mlp_rows(lam=1e-3, seed=0, shapes=((4096, 3072), (4096, 4096), (10, 4096))):
    """All rows of a 3-layer MLP on 32x32x3 inputs (W1 4096x3072, W2 4096x4096, W3 10x4096),
    weights N(0, 1/fan_in), one segment per row (the paper's fully connected CIFAR10 net,
    Sec. 6.2 / App. E.2, with the layer widths of the batched workload)."""
    rng = np.random.default_rng(seed)
    parts, offs = [], [0]
    for rows, cols in shapes:
        parts.append(rng.standard_normal(rows * cols) / np.sqrt(cols))
        for _ in range(rows):
            offs.append(offs[-1] + cols)
    return _pack("mlp_rows_%d" % offs[-1], np.concatenate(parts), offs, lam)


def mlp_layers(lam=1e-3, seed=0, shapes=((4096, 3072), (4096, 4096), (10, 4096))):
    """The weights of ``mlp_rows`` (same draw) with one segment per weight matrix, the paper's
    per-layer application of R (App. E.1): segments of 12,582,912, 16,777,216 and 40,960."""
    case = mlp_rows(lam, seed, shapes)
    offs = [0]
    for rows, cols in shapes:
        offs.append(offs[-1] + rows * cols)
    return _pack("mlp_layers_%d" % offs[-1], case["w"], offs, lam)


def ica_worst_rows(rows=1024, d=4095, seed=0):
    """Rows holding the Sec. 4.1 worst case of ImminentCollisions recast as a prox input
    (lam = 1, d odd): (d+1)/2 equal weights and a slow ramp j(eps + 2/(d-1)), j = 1..d//2, with
    eps = 1/(4d), each row in its own random order.  Every row ends in one cluster after about
    d/2 collision rounds, the case the bounded-depth hull merge is for."""
    rng = np.random.default_rng(seed)
    eps = 1.0 / (4 * d)
    base = np.concatenate([np.zeros((d + 1) // 2), np.arange(1, d // 2 + 1) * (eps + 2.0 / (d - 1))])
    w = np.concatenate([base[rng.permutation(d)] for _ in range(rows)])
    return _pack("ica_worst_rows_%dx%d" % (rows, d), w, np.arange(rows + 1, dtype=np.int64) * d, 1.0)


def chain(d=1 << 24, lam=0.7, shuffle=False, seed=0):
    """Worst-case collision chain: sorted w_k = (k/(d-1))^2 (gaps grow, so clusters merge one at
    a time from one end).  All particles end in one cluster once
    lam >= (4d-5)/(6(d-1)) ~= 2/3; lam = 0.7 leaves a 5% margin."""
    k = np.arange(d, dtype=np.float64)
    w = (k / (d - 1.0)) ** 2
    if shuffle:
        w = w[np.random.default_rng(seed).permutation(d)]
    return _pack("chain_d%d%s" % (d, "_shuffled" if shuffle else ""), w, [0, d], lam)


def backward_rows(rows=1024, d=8192, lam=0.05, seed=0):
    """Batch of Laplace(0,1) rows with an N(0,1) upstream gradient."""
    rng = np.random.default_rng(seed)
    w = rng.laplace(0.0, 1.0, rows * d)
    g = rng.standard_normal(rows * d).astype(np.float32)
    return _pack("backward_%dx%d" % (rows, d), w, np.arange(rows + 1, dtype=np.int64) * d, lam, g=g)


def precision(d=1 << 26, lam=1e-4, seed=0):
    """Heavy cancellation: w = 1e3 + 1e-2 N(0,1) in FP32 (few distinct values, long tie groups)."""
    rng = np.random.default_rng(seed)
    return _pack("precision_d%d" % d, 1e3 + 1e-2 * rng.standard_normal(d), [0, d], lam)


def random_segments(lengths, dist="normal", lam=0.05, seed=0):
    """Uneven segments of the given lengths; dist in {normal, laplace, ties, sorted, mixed}."""
    rng = np.random.default_rng(seed)
    offs = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    n = int(offs[-1])
    if dist == "normal":
        w = rng.standard_normal(n)
    elif dist == "laplace":
        w = rng.laplace(0.0, 1.0, n)
    elif dist == "ties":
        w = rng.integers(-20, 21, n) / 8.0
    elif dist == "sorted":
        w = np.concatenate([np.sort(rng.standard_normal(b - a)) for a, b in zip(offs[:-1], offs[1:])]) \
            if n else np.zeros(0)
    else:
        w = rng.standard_normal(n) * rng.choice([1e-3, 1.0, 1e3], n)
    return _pack("segments_%s_%d" % (dist, n), w, offs, lam)
