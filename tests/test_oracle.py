"""Pins for the CPU oracle (runs without a GPU).

Each test checks the oracle against something fixed outside it: values printed in the
paper (tests/golden), brute-force minimisation of the prox objective, independent
characterisations (convex-minorant slopes, end collisions, the neighbour-collision
criterion, the optimality certificate), closed forms, and invariants of the flow.
"""
import os

import numpy as np
import pytest

import oracle
import pins

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _read_golden(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            rows[key] = np.array([float(v) for v in vals])
    return rows


# ----------------------------------------------------------------------------- golden values

def test_golden_counterexample_isotonic_link():
    """App. C counterexample: the paper's correct answer is the isotonic regression of y,
    and prox_R of the recast input equals it (isotonic link, Sec. 3)."""
    g = _read_golden("kearsley_counterexample.txt")
    y, x_star, x_wrong = g["y"], g["x_star"], g["x_wrong"]
    slopes, _ = pins.gcm_slopes(y)
    np.testing.assert_allclose(slopes, x_star, atol=1e-15)
    ends, _ = pins.naive_end_collisions(y)
    np.testing.assert_allclose(ends, x_star, atol=1e-15)
    # recast as a prox input: d = 4, lam = 0.3 gives v = [0.3, 0.1, -0.1, -0.3]; w = y - v
    lam = 0.3
    v = pins.shift(4, lam)
    np.testing.assert_allclose(v, [0.3, 0.1, -0.1, -0.3], atol=1e-16)
    w = y - v
    assert np.all(np.diff(w) > 0)
    u, perm, start = oracle.prox_f64(w, lam)
    np.testing.assert_allclose(u, x_star, atol=1e-14)
    assert np.max(np.abs(u - x_wrong)) > 1e-2
    assert list(start) == [1, 1, 0, 1]
    # any input order gives the same multiset of outputs, attached to the same weights
    rng = np.random.default_rng(0)
    p = rng.permutation(4)
    u2, _, _ = oracle.prox_f64(w[p], lam)
    np.testing.assert_allclose(u2, x_star[p], atol=1e-14)


def test_golden_d3_hyperplanes():
    """Sec. 2 example: the six printed (signs, hyperplane) pairs are consistent, are exactly the
    hyperplanes of eq. hyperplane, and R is their pointwise maximum."""
    rows = []
    with open(os.path.join(GOLDEN, "d3_hyperplanes.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                _, signs, coef = [s.strip() for s in line.split(";")]
                rows.append((np.array([1.0 if s == "+" else -1.0 for s in signs.split()]),
                             np.array([float(c) for c in coef.split()])))
    assert len(rows) == 6
    terms = np.array([[1, -1, 0], [0, 1, -1], [1, 0, -1]], dtype=float)  # w1-w2, w2-w3, w1-w3
    for signs, coef in rows:
        np.testing.assert_allclose(0.5 * signs @ terms, coef)
    import itertools
    from_eq = {tuple(pins.hyperplane_coeffs(p)) for p in itertools.permutations(range(3))}
    assert {tuple(c) for _, c in rows} == from_eq
    rng = np.random.default_rng(1)
    for _ in range(50):
        w = rng.normal(size=3)
        assert abs(max(c @ w for _, c in rows) - pins.R_pairwise(w)) < 1e-12


@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_R_pairwise_equals_max_hyperplane(d):
    rng = np.random.default_rng(d)
    for _ in range(20):
        w = rng.normal(size=d)
        if rng.random() < 0.3:
            w[rng.integers(d)] = w[0]
        assert abs(pins.R_hyperplanes(w) - pins.R_pairwise(w)) < 1e-12


# ----------------------------------------------------------------------------- brute force

def _random_case(rng, d):
    kind = rng.integers(4)
    if kind == 0:
        w = rng.normal(size=d)
    elif kind == 1:
        w = rng.integers(-2, 3, size=d).astype(float)  # many ties
    elif kind == 2:
        w = rng.laplace(size=d)
    else:
        w = np.sort(rng.normal(size=d)) * rng.choice([0.01, 1.0, 100.0])
    lam = float(rng.choice([0.0, 1e-3, 0.05, 0.3, 1.0, 5.0])) * float(np.abs(w).max() + 1.0)
    return w, lam


def test_brute_force_small_d():
    rng = np.random.default_rng(2)
    n = 0
    for d in [1, 2, 3, 4, 5, 6]:
        for _ in range(25 if d < 6 else 12):
            w, lam = _random_case(rng, d)
            u, _, _ = oracle.prox_f64(w, lam)
            ub = pins.brute_force_prox(w, lam)
            np.testing.assert_allclose(u, ub, atol=1e-9 * (1 + np.abs(w).max()), err_msg=f"{w} {lam}")
            n += 1
    assert n > 100


def test_brute_force_d7():
    rng = np.random.default_rng(3)
    for _ in range(3):
        w, lam = _random_case(rng, 7)
        u, _, _ = oracle.prox_f64(w, lam)
        np.testing.assert_allclose(u, pins.brute_force_prox(w, lam), atol=1e-9 * (1 + np.abs(w).max()))


# ----------------------------------------------------------------------------- other algorithms

def test_gcm_and_end_collisions_agree():
    """Sorted oracle output = slopes of the convex minorant of y's cumulative sums = end
    collisions; cluster starts agree (coarsest partition)."""
    rng = np.random.default_rng(4)
    for trial in range(30):
        d = int(rng.integers(2, 400))
        w, lam = _random_case(rng, d)
        if lam == 0:
            lam = 0.1
        u, perm, start = oracle.prox_f64(w, lam)
        x = w[perm]
        y = x + pins.shift(d, lam)
        gcm, hull = pins.gcm_slopes(y)
        eca, eca_starts = pins.naive_end_collisions(y)
        tol = 1e-10 * (1 + np.abs(w).max())
        np.testing.assert_allclose(u[perm], gcm, atol=tol)
        np.testing.assert_allclose(u[perm], eca, atol=tol)


def test_exact_arithmetic_partitions_identical():
    """With dyadic inputs and lam/(d-1) dyadic every sum is exact in FP64, so the three
    independent routes must give the identical (coarsest) partition, ties included."""
    rng = np.random.default_rng(5)
    for trial in range(60):
        d = int(rng.integers(2, 200))
        w = rng.integers(-8, 9, size=d).astype(float) * 0.25
        lam = (d - 1) * 0.125 * float(rng.integers(0, 5))
        if lam == 0:
            continue
        u, perm, start = oracle.prox_f64(w, lam)
        y = w[perm] + pins.shift(d, lam)
        _, hull = pins.gcm_slopes(y)
        _, eca_starts = pins.naive_end_collisions(y)
        assert list(np.nonzero(start)[0]) == hull[:-1]
        assert list(np.nonzero(start)[0]) == eca_starts


def test_neighbour_collision_criterion():
    rng = np.random.default_rng(6)
    for trial in range(20):
        d = int(rng.integers(2, 120))
        w, lam = _random_case(rng, d)
        if lam == 0:
            lam = 0.2
        u, perm, start = oracle.prox_f64(w, lam)
        y = w[perm] + pins.shift(d, lam)
        # only check boundaries whose decision is not a near-tie
        for i in range(d - 1):
            left = np.cumsum(y[:i + 1][::-1]) / np.arange(1, i + 2)
            right = np.cumsum(y[i + 1:]) / np.arange(1, d - i)
            if abs(left.max() - right.min()) < 1e-9 * (1 + np.abs(w).max()):
                continue
            assert bool(start[i + 1]) == (not pins.neighbour_collides(y, i))


@pytest.mark.parametrize("dist", ["normal", "laplace", "ties", "sorted_quadratic", "offset"])
def test_kkt_certificate(dist):
    rng = np.random.default_rng(7)
    d = 20000
    if dist == "normal":
        w, lam = rng.normal(size=d), 0.1
    elif dist == "laplace":
        w, lam = rng.laplace(size=d), 5.0
    elif dist == "ties":
        w, lam = rng.integers(-50, 50, size=d).astype(float), 0.5
    elif dist == "sorted_quadratic":
        w, lam = (np.arange(d) / (d - 1.0)) ** 2, 0.4
    else:
        w, lam = 1e3 + 1e-2 * rng.normal(size=d), 1e-4
    u, _, _ = oracle.prox_f64(w, lam)
    ok, msg = pins.kkt_certificate(w, u, lam, tol=1e-9 * (1 + np.abs(w).max()))
    assert ok, msg


def _kkt_case(seed=21):
    rng = np.random.default_rng(seed)
    lens = [1, 2, 7, 300, 5000, 0, 2048, 40]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    w = np.concatenate([rng.normal(size=lens[0] + lens[1] + lens[2]), rng.laplace(size=lens[3]),
                        1e3 + 1e-2 * rng.normal(size=lens[4]), rng.integers(-9, 9, lens[6]) / 4.0,
                        rng.normal(size=lens[7])]).astype(np.float32)
    lam = np.array([0.3, 0.2, 0.5, 1.0, 1e-4, 0.1, 0.25, 0.0], np.float32)
    return w, off, lam


def test_kkt_certificate_segments_accepts_oracle_output():
    """The vectorised certificate accepts the oracle's output on a layout with identity segments
    (d = 1, lam = 0), an empty segment, a precision-stress segment and tie groups, both in the
    oracle's rank order and in the (u, w) order; and it agrees with the per-segment loop form."""
    w, off, lam = _kkt_case()
    u, perm, start = oracle.prox_segments(w, lam, off)
    for kw in (dict(perm=perm, start=start), {}):
        r = pins.kkt_certificate_segments(w, off, u, lam, tol_rel=1e-9, **kw)
        assert r["ok"], r
    for s in range(len(off) - 1):
        a, b = off[s], off[s + 1]
        if b - a >= 2 and lam[s] > 0:
            ok, msg = pins.kkt_certificate(w[a:b].astype(np.float64), u[a:b], float(lam[s]), 1e-9 * 1e3)
            assert ok, msg


def test_kkt_certificate_segments_rejects_mistakes():
    """Plausible mistakes in a prox output each fail one condition: a wrong lambda, a shifted
    cluster value, two clusters merged, one cluster split, the shift v with the wrong sign, and a
    changed identity segment."""
    w, off, lam = _kkt_case()
    u, perm, start = oracle.prox_segments(w, lam, off)
    seg = 3  # the Laplace segment (many clusters of several ranks)
    a, b = off[seg], off[seg + 1]
    tol = 1e-9

    def bad(u2, **kw):
        r = pins.kkt_certificate_segments(w, off, u2, lam, tol_rel=tol, **kw)
        return not r["ok"]

    u_lam, _, _ = oracle.prox_segments(w, lam * np.float32(1.01), off)
    assert bad(u_lam) and bad(u_lam, perm=perm, start=start)
    u2 = u.copy()
    o = a + perm[a:b].astype(np.int64)  # original indices in rank order
    cid = np.cumsum(start[a:b]) - 1
    big = np.bincount(cid)
    c = int(np.argmax(big))  # the largest cluster
    members = o[cid == c]
    u2[members] += 1e-3
    assert bad(u2) and bad(u2, perm=perm, start=start)
    # merge clusters c and c+1 into one with their joint mean value
    u3 = u.copy()
    both = o[(cid == c) | (cid == c + 1)]
    u3[both] = u[both].mean()
    assert bad(u3)
    # split the largest cluster in two at its middle rank, each half at its own mean of y
    x = w[o].astype(np.float64)
    d = b - a
    v = lam[seg] * (d - 1 - 2 * np.arange(d)) / (d - 1)
    y = x + v
    idx = np.nonzero(cid == c)[0]
    h = idx[: len(idx) // 2]
    t = idx[len(idx) // 2:]
    u4 = u.copy()
    u4[o[h]] = y[h].mean()
    u4[o[t]] = y[t].mean()
    st4 = start.copy()
    st4[a + t[0]] = 1
    assert bad(u4) and bad(u4, perm=perm, start=st4)
    # v with the wrong sign: isotonic regression of x - v instead of x + v
    yw = x - v
    u5 = u.copy()
    u5[o] = np.maximum.accumulate(yw)  # any monotone fit of the wrong y
    assert bad(u5)
    # identity segment changed
    u6 = u.copy()
    u6[off[7]] += 1e-6
    assert bad(u6, perm=perm, start=start)


# ----------------------------------------------------------------------------- closed forms

def test_closed_form_d2():
    rng = np.random.default_rng(8)
    for _ in range(200):
        a, b = rng.normal(size=2)
        lam = abs(rng.normal())
        u, _, _ = oracle.prox_f64(np.array([a, b]), lam)
        lo, hi = min(a, b), max(a, b)
        if hi - lo <= 2 * lam:
            exp = np.array([(a + b) / 2] * 2)
        else:
            exp = np.array([a + lam, b - lam]) if a < b else np.array([a - lam, b + lam])
        np.testing.assert_allclose(u, exp, atol=1e-14)


def test_closed_form_no_collision():
    rng = np.random.default_rng(9)
    d = 1000
    x = np.cumsum(rng.uniform(1.0, 2.0, size=d))
    lam = 0.49 * (d - 1) * 1.0 / 2  # all gaps >= 1 > 2 lam/(d-1)
    p = rng.permutation(d)
    w = x[p]
    u, _, start = oracle.prox_f64(w, lam)
    np.testing.assert_allclose(u, w + pins.shift(d, lam)[np.argsort(np.argsort(w))], atol=1e-12)
    assert start.all()


def test_closed_form_large_lambda_one_cluster():
    rng = np.random.default_rng(10)
    d = 777
    w = rng.normal(size=d)
    maxgap = np.diff(np.sort(w)).max()
    lam = (d - 1) * maxgap / 2 * 1.0001
    u, _, start = oracle.prox_f64(w, lam)
    np.testing.assert_allclose(u, w.mean(), atol=1e-13)
    assert start.sum() == 1


@pytest.mark.parametrize("d", [101, 1001, 4001])
def test_ica_worst_case_all_collide(d):
    """Sec. 4.1 worst case: y = [1, 1-2/(d-1), ..., 0, e, 2e, ..., floor(d/2) e] -- the paper states
    all particles eventually collide.  Recast as a prox input with lam = 1 (d odd)."""
    eps = 1.0 / (4 * d)
    half = (d + 1) // 2
    j = np.arange(1, d // 2 + 1)
    w = np.concatenate([np.zeros(half), j * (eps + 2.0 / (d - 1))])
    y = np.sort(w) + pins.shift(d, 1.0)
    np.testing.assert_allclose(y[:half], 1 - 2 * np.arange(half) / (d - 1), atol=1e-12)
    np.testing.assert_allclose(y[half:], j * eps, atol=1e-12)
    u, _, start = oracle.prox_f64(w, 1.0)
    assert start.sum() == 1
    np.testing.assert_allclose(u, w.mean(), atol=1e-14)


def test_worst_case_chain_one_cluster():
    """Sorted w_k = (k/(d-1))^2: all particles end in one cluster iff
    lam >= (4d-5)/(6(d-1)) (prefix averages of y decrease to the end)."""
    d = 4096
    w = (np.arange(d) / (d - 1.0)) ** 2
    lam_min = (4 * d - 5) / (6.0 * (d - 1))
    u, _, start = oracle.prox_f64(w, lam_min * 1.05)
    assert start.sum() == 1
    np.testing.assert_allclose(u, w.mean(), atol=1e-14)
    u, _, start = oracle.prox_f64(w, lam_min * 0.95)
    assert start.sum() > 1


def test_tie_groups_closed_form():
    """Weights on a coarse grid with lam far below the grid spacing: the clusters are exactly
    the tie groups and u = value + lam (d-1-a-b)/(d-1) for the group's rank range [a, b]."""
    rng = np.random.default_rng(11)
    d = 50000
    w = np.round(rng.normal(size=d) * 20) / 16.0
    lam = 1e-4
    u, perm, start = oracle.prox_f64(w, lam)
    x = w[perm]
    assert np.array_equal(np.nonzero(start)[0], np.nonzero(np.concatenate([[True], np.diff(x) != 0]))[0])
    starts = np.nonzero(start)[0]
    ends = np.concatenate([starts[1:], [d]]) - 1
    for a, b in zip(starts[:50], ends[:50]):
        np.testing.assert_allclose(u[perm[a:b + 1]], x[a] + lam * (d - 1 - a - b) / (d - 1), atol=1e-12)


# ----------------------------------------------------------------------------- invariants

def test_invariants():
    rng = np.random.default_rng(12)
    for _ in range(40):
        d = int(rng.integers(2, 3000))
        w, lam = _random_case(rng, d)
        u, perm, start = oracle.prox_f64(w, lam)
        s = 1 + np.abs(w).max()
        assert abs(u.sum() - w.sum()) < 1e-9 * s * d ** 0.5  # momentum (Sec. 3)
        assert np.all(np.diff(u[np.argsort(w, kind='stable')]) >= 0)  # order preserved (Sec. 4.2 fact 1)
        assert np.all(np.abs(u - w) <= lam * (1 + 1e-12) + 1e-12 * s)
        assert u.min() >= w.min() - 1e-12 * s and u.max() <= w.max() + 1e-12 * s
        # weight sharing preserved: equal weights stay equal (Sec. 3 lemma)
        for v in np.unique(w)[:5]:
            assert np.ptp(u[w == v]) == 0
        p = rng.permutation(d)
        up, _, _ = oracle.prox_f64(w[p], lam)
        np.testing.assert_allclose(up, u[p], atol=1e-12 * s)
        c = float(rng.normal())
        np.testing.assert_allclose(oracle.prox_f64(w + c, lam)[0], u + c, atol=1e-9 * (s + abs(c)))
        np.testing.assert_allclose(oracle.prox_f64(-w, lam)[0], -u, atol=1e-12 * s)
        sc = float(rng.uniform(0.1, 10))
        np.testing.assert_allclose(oracle.prox_f64(sc * w, lam)[0], sc * oracle.prox_f64(w, lam / sc)[0],
                                   atol=1e-9 * s * sc)


def test_semigroup():
    """prox_{(a+b)R} = prox_{bR} o prox_{aR}: the prox is the time-1 flow of an autonomous ODE
    (Sec. 3, eq. prox_ode and theorem prox_R), so flows compose."""
    rng = np.random.default_rng(13)
    for _ in range(30):
        d = int(rng.integers(2, 2000))
        w, lam = _random_case(rng, d)
        a = lam * float(rng.uniform(0, 1))
        b = lam - a
        u = oracle.prox_f64(w, lam)[0]
        u2 = oracle.prox_f64(oracle.prox_f64(w, a)[0], b)[0]
        np.testing.assert_allclose(u2, u, atol=1e-9 * (1 + np.abs(w).max()))


# ----------------------------------------------------------------------------- gradient

def test_vjp_structure_and_finite_differences():
    rng = np.random.default_rng(14)
    d = 2000
    for trial in range(6):
        w = rng.laplace(size=d)
        lam = [0.05, 5.0][trial % 2]
        u, perm, start = oracle.prox_f64(w, lam)
        pl = perm.astype(np.int32)
        g = rng.normal(size=d)
        jg = oracle.vjp(g, pl, start)
        np.testing.assert_allclose(oracle.vjp(jg, pl, start), jg, atol=1e-12)  # J^2 = J
        np.testing.assert_allclose(oracle.vjp(np.ones(d), pl, start), 1.0, atol=1e-12)  # J 1 = 1
        h = rng.normal(size=d)
        assert abs(h @ jg - g @ oracle.vjp(h, pl, start)) < 1e-9 * d  # symmetric
        # central finite differences along a random direction; mask elements whose cluster
        # membership changes between w - eps v, w, w + eps v (a kink is crossed there)
        eps = 1e-6
        vdir = rng.normal(size=d)
        up, pp, sp = oracle.prox_f64(w + eps * vdir, lam)
        um, pm, sm = oracle.prox_f64(w - eps * vdir, lam)
        ids0 = oracle.cluster_ids(pl, start)
        idp = oracle.cluster_ids(pp.astype(np.int32), sp)
        idm = oracle.cluster_ids(pm.astype(np.int32), sm)

        def members(ids):
            out = {}
            for i, c in enumerate(ids):
                out.setdefault(c, []).append(i)
            return {i: tuple(out[c]) for i, c in enumerate(ids)}
        m0, mp, mm = members(ids0), members(idp), members(idm)
        keep = np.array([m0[i] == mp[i] == mm[i] for i in range(d)])
        assert keep.mean() > 0.5
        fd = (up - um) / (2 * eps)
        jv = oracle.vjp(vdir, pl, start)
        assert np.max(np.abs(fd - jv)[keep]) < 1e-6


# ----------------------------------------------------------------------------- segments API

def test_segments_match_single_and_threads():
    rng = np.random.default_rng(15)
    lens = [0, 1, 2, 5, 100, 3072, 4096, 7, 0, 1]
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    w = rng.normal(size=offsets[-1]).astype(np.float32)
    lam = rng.uniform(0, 0.1, size=len(lens)).astype(np.float32)
    u1, p1, s1 = oracle.prox_segments(w, lam, offsets, n_threads=1)
    u4, p4, s4 = oracle.prox_segments(w, lam, offsets, n_threads=4)
    assert np.array_equal(u1, u4) and np.array_equal(p1, p4) and np.array_equal(s1, s4)
    for s, (a, b) in enumerate(zip(offsets[:-1], offsets[1:])):
        if b == a:
            continue
        u, perm, start = oracle.prox_f64(w[a:b].astype(np.float64), float(lam[s]))
        np.testing.assert_array_equal(u1[a:b], u)
        np.testing.assert_array_equal(p1[a:b], perm)
        np.testing.assert_array_equal(s1[a:b], start)


def test_nonfinite_and_bad_args():
    u, perm, start = oracle.prox_f64(np.array([1.0, np.nan, 2.0]), 0.1)
    assert np.isnan(u).all()
    with pytest.raises(ValueError):
        oracle.prox_f64(np.array([1.0, 2.0]), -1.0)
    with pytest.raises(ValueError):
        oracle.prox_segments(np.zeros(4, np.float32), 0.1, np.array([0, 3, 2, 4]))


# ----------------------------------------------------------------------------- l1 and rewinding
# Alg. prox in full: the clusters of prox_{lam R}, then its l1 and rewinding lines per cluster.

def _l1_case(rng, d):
    w, lam = _random_case(rng, d)
    beta = float(rng.choice([0.0, 0.05, 0.2, 0.6])) * float(np.abs(w).max() + 1e-3) * float(rng.uniform(0.5, 1.5))
    return w, lam, beta


def test_l1_brute_force_small_d():
    """rho = 0: the output is the exact minimiser of lam*R + beta*l1 + 1/2||u - w||^2, found by
    enumeration (pins the decomposition proposition and the soft-threshold lines)."""
    rng = np.random.default_rng(21)
    n = 0
    for d in [2, 3, 4, 5]:
        for _ in range(20):
            w, lam, beta = _l1_case(rng, d)
            out = oracle.prox_l1_f64(w, lam, beta, 0.0)
            ub = pins.brute_force_prox_l1(w, lam, beta)
            np.testing.assert_allclose(out, ub, atol=1e-9 * (1 + np.abs(w).max()), err_msg=f"{w} {lam} {beta}")
            n += 1
    w, lam, beta = _l1_case(rng, 6)
    np.testing.assert_allclose(oracle.prox_l1_f64(w, lam, beta, 0.0), pins.brute_force_prox_l1(w, lam, beta),
                               atol=1e-9 * (1 + np.abs(w).max()))
    assert n == 80


def test_l1_rewinding_from_brute_force():
    """rho in (0, 1]: before the rewinding line the output splits as x + v, x the mean weight of
    each surviving cluster, zero on zeroed ones; rewinding returns x + (1 - rho) v.  x is taken
    from the groups of the brute-force minimiser, so nothing here comes from the oracle."""
    rng = np.random.default_rng(22)
    for d in [3, 4, 5]:
        for _ in range(12):
            w, lam, beta = _l1_case(rng, d)
            P = pins.brute_force_prox_l1(w, lam, beta)
            vals, inv = np.unique(P, return_inverse=True)
            for rho in [0.25, 0.98, 1.0]:
                exp = np.empty(d)
                for gi, val in enumerate(vals):
                    m = inv == gi
                    xbar = w[m].mean()
                    exp[m] = 0.0 if val == 0.0 else xbar + (1.0 - rho) * (val - xbar)
                np.testing.assert_allclose(oracle.prox_l1_f64(w, lam, beta, rho), exp,
                                           atol=1e-9 * (1 + np.abs(w).max()), err_msg=f"{w} {lam} {beta} {rho}")


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.98, 1.0])
def test_l1_closed_form_without_weight_sharing(rho):
    """lam = 0 (and d = 1 for any lam): the rewound l1 prox of the rewinding section's example,
    sign(w) (|w| - (1 - rho) beta) where |w| > beta, else 0; rho = 0 is soft-thresholding
    (App. A.1 example)."""
    rng = np.random.default_rng(23)
    w = rng.normal(size=2000)
    beta = 0.5
    exp = np.where(np.abs(w) > beta, w - (1.0 - rho) * beta * np.sign(w), 0.0)
    np.testing.assert_allclose(oracle.prox_l1_f64(w, 0.0, beta, rho), exp, atol=1e-15)
    for x in [-2.0, -0.3, 0.0, 0.4, 1.7]:
        got = oracle.prox_l1_f64(np.array([x]), 0.7, beta, rho)[0]
        assert got == (0.0 if abs(x) < beta else x - (1.0 - rho) * beta * np.sign(x))
    if rho == 0.0:
        np.testing.assert_allclose(exp, np.sign(w) * np.maximum(np.abs(w) - beta, 0.0), atol=1e-15)


def test_l1_reductions_and_invariants():
    rng = np.random.default_rng(24)
    for _ in range(30):
        d = int(rng.integers(2, 3000))
        w, lam, beta = _l1_case(rng, d)
        s = 1 + np.abs(w).max()
        u = oracle.prox_f64(w, lam)[0]
        # beta = 0, rho = 0: prox_{lam R} itself
        np.testing.assert_allclose(oracle.prox_l1_f64(w, lam, 0.0, 0.0), u, atol=1e-12 * s)
        rho = float(rng.uniform())
        # beta = 0: the velocities of a cluster sum to its displacement and all of them to zero
        # (momentum, Sec. 3), so every rho keeps the sum of the weights
        assert abs(oracle.prox_l1_f64(w, lam, 0.0, rho).sum() - w.sum()) < 1e-9 * s * d ** 0.5
        out = oracle.prox_l1_f64(w, lam, beta, rho)
        # the zeroed weights are exactly those whose prox_{lam R} value is below beta in size
        np.testing.assert_array_equal(out == 0.0, np.abs(u) < beta)
        # odd symmetry and positive homogeneity of lam*R + beta*l1
        np.testing.assert_allclose(oracle.prox_l1_f64(-w, lam, beta, rho), -out, atol=1e-12 * s)
        np.testing.assert_allclose(oracle.prox_l1_f64(2.0 * w, 2.0 * lam, 2.0 * beta, rho), 2.0 * out,
                                   atol=1e-12 * s)
        # rho = 0 equals soft-thresholding of prox_{lam R} (decomposition proposition)
        np.testing.assert_allclose(oracle.prox_l1_f64(w, lam, beta, 0.0),
                                   np.sign(u) * np.maximum(np.abs(u) - beta, 0.0), atol=1e-12 * s)


def test_l1_segments_match_single_and_threads():
    rng = np.random.default_rng(25)
    lens = [0, 1, 2, 5, 100, 3072, 4096, 7, 0, 1]
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    w = rng.normal(size=offsets[-1]).astype(np.float32)
    lam = rng.uniform(0, 0.1, size=len(lens)).astype(np.float32)
    beta, rho = np.float32(0.3), np.float32(0.75)
    o1 = oracle.prox_l1_segments(w, lam, beta, rho, offsets, n_threads=1)
    o4 = oracle.prox_l1_segments(w, lam, beta, rho, offsets, n_threads=4)
    assert np.array_equal(o1, o4)
    for s, (a, b) in enumerate(zip(offsets[:-1], offsets[1:])):
        if b > a:
            np.testing.assert_array_equal(
                o1[a:b], oracle.prox_l1_f64(w[a:b].astype(np.float64), float(lam[s]), float(beta), float(rho)))


def test_l1_nonfinite_and_bad_args():
    assert np.isnan(oracle.prox_l1_f64(np.array([1.0, np.inf, 2.0]), 0.1, 0.5, 0.5)).all()
    for lam, beta, rho in [(-1.0, 0.1, 0.0), (0.1, -0.1, 0.0), (0.1, 0.1, 1.5), (0.1, 0.1, -0.5),
                           (0.1, np.nan, 0.0), (0.1, 0.1, np.nan), (0.1, np.inf, 0.0)]:
        with pytest.raises(ValueError):
            oracle.prox_l1_f64(np.array([1.0, 2.0]), lam, beta, rho)


# ----------------------------------------------------------------------------- proximal-gradient step

def _rewound(P, w, kappa_one_minus_rho):
    """x + k (P - x) per group of equal entries of the brute-force minimiser P, zero on its zero
    group (x = mean weight of the group): the rewinding split of Alg. prox."""
    vals, inv = np.unique(P, return_inverse=True)
    exp = np.empty(P.shape[0])
    for gi, val in enumerate(vals):
        m = inv == gi
        xbar = w[m].mean()
        exp[m] = 0.0 if val == 0.0 else xbar + kappa_one_minus_rho * (val - xbar)
    return exp


def test_step_against_brute_force():
    """z = w - eta*g (exact here: eta = 1/2 or 1/4 and weights and gradients of similar size,
    so the FP32 gradient step has one rounding on both routes); the step is the prox of
    eta*(alpha R + beta l1) at z with rewinding, or, with eta on the rewinding line, the prox of
    alpha R + beta l1 at z with x + eta (1 - rho) v."""
    rng = np.random.default_rng(26)
    for d in [2, 3, 4, 5]:
        for _ in range(10):
            w = rng.normal(size=d).astype(np.float32)
            g = rng.normal(size=d).astype(np.float32)
            eta = float(rng.choice([0.5, 0.25]))
            alpha = np.float32(rng.choice([0.0, 0.1, 0.5, 2.0]))
            beta = np.float32(rng.choice([0.0, 0.1, 0.4]))
            rho = float(np.float32(rng.choice([0.0, 0.5, 0.98])))
            z = (w.astype(np.float64) - eta * g.astype(np.float64)).astype(np.float32).astype(np.float64)
            off = np.array([0, d], np.int64)
            tol = 1e-9 * (1 + np.abs(z).max())
            got = oracle.prox_step_segments(w, g, eta, alpha, beta, rho, off)
            P = pins.brute_force_prox_l1(z, float(np.float32(eta * alpha)), float(np.float32(eta * beta)))
            np.testing.assert_allclose(got, _rewound(P, z, 1.0 - rho), atol=tol)
            got = oracle.prox_step_segments(w, g, eta, alpha, beta, rho, off, eta_in_displacement=True)
            P = pins.brute_force_prox_l1(z, float(alpha), float(beta))
            np.testing.assert_allclose(got, _rewound(P, z, eta * (1.0 - rho)), atol=tol)


def test_step_modes_agree_at_unit_eta_and_per_segment_alpha():
    rng = np.random.default_rng(27)
    lens = [0, 1, 5, 300, 4096, 7]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    w = rng.normal(size=off[-1]).astype(np.float32)
    g = rng.normal(size=off[-1]).astype(np.float32)
    alpha = rng.uniform(0, 0.2, size=len(lens)).astype(np.float32)
    a = oracle.prox_step_segments(w, g, 1.0, alpha, 0.2, 0.5, off)
    b = oracle.prox_step_segments(w, g, 1.0, alpha, 0.2, 0.5, off, eta_in_displacement=True, n_threads=3)
    np.testing.assert_array_equal(a, b)
    # with a zero gradient the standard step is Alg. prox with eta folded into the coefficients
    eta = np.float32(0.3)
    c = oracle.prox_step_segments(w, np.zeros_like(g), eta, alpha, 0.2, 0.5, off)
    np.testing.assert_array_equal(c, oracle.prox_l1_segments(w, (eta * alpha).astype(np.float32),
                                                             np.float32(eta * np.float32(0.2)), 0.5, off))
    with pytest.raises(ValueError):
        oracle.prox_step_segments(w, g, -1.0, alpha, 0.2, 0.5, off)
    # the gradient step alone: one rounding of w - eta*g.  eta*g is exact in FP64; rounding the
    # FP64 difference to FP32 gives the correctly rounded result unless that difference is itself
    # halfway between two FP32 values (FP32 midpoints are FP64 numbers, so the exact value lies
    # on the same side of every midpoint as its FP64 rounding)
    z = oracle.grad_step(w, g, eta)
    r64 = w.astype(np.float64) - np.float64(eta) * g.astype(np.float64)
    r32 = r64.astype(np.float32)
    nb = np.where(r64 > r32, np.nextafter(r32, np.float32(np.inf)), np.nextafter(r32, np.float32(-np.inf)))
    ok = r64 != (r32.astype(np.float64) + nb.astype(np.float64)) / 2
    assert ok.mean() > 0.99
    np.testing.assert_array_equal(z[ok], r32[ok])


# ----------------------------------------------------------------------------- segment statistics

def test_segment_penalty_against_definitions():
    """R from the sorted order (App. B) against the O(d^2) pairwise definition (Sec. 1, eq. reg)
    and, for d <= 6, the maximum over all orderings of the hyperplanes (Sec. 2)."""
    rng = np.random.default_rng(30)
    lens = [0, 1, 2, 3, 5, 6, 40, 1000, 1999]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    w = np.concatenate([rng.normal(size=n) if i % 2 else rng.integers(-3, 4, size=n)
                        for i, n in enumerate(lens)]).astype(np.float32)
    pen, _, _ = oracle.segment_stats(w, off)
    for s, (a, b) in enumerate(zip(off[:-1], off[1:])):
        x = w[a:b].astype(np.float64)
        ref = pins.R_pairwise(x) if b - a >= 2 else 0.0
        np.testing.assert_allclose(pen[s], ref, rtol=1e-12, atol=1e-12)
        if 2 <= b - a <= 6:
            np.testing.assert_allclose(pen[s], pins.R_hyperplanes(x), rtol=1e-12, atol=1e-12)


def test_segment_counts_and_invariants():
    rng = np.random.default_rng(31)
    w = np.round(rng.normal(size=5000) * 4) / 4  # many ties and exact zeros
    w[:7] = -0.0
    w = w.astype(np.float32)
    pen, nd, nz = oracle.segment_stats(w)
    v = w[w != 0]
    assert nz[0] == v.size and nd[0] == np.unique(v).size
    # translation and permutation invariance, positive homogeneity, R = 0 on a constant vector
    c = np.float32(0.5)
    np.testing.assert_allclose(oracle.segment_stats(w + c)[0], pen, rtol=1e-12)
    np.testing.assert_allclose(oracle.segment_stats(w[rng.permutation(w.size)])[0], pen, rtol=1e-12)
    np.testing.assert_allclose(oracle.segment_stats(np.float32(-2) * w)[0], 2 * pen, rtol=1e-12)
    assert oracle.segment_stats(np.full(10, 3.0, np.float32))[0][0] == 0.0
    # chain w_k = (k/(d-1))^2: R = 1/(d-1) sum_{i>j} (w_i - w_j) in exact rationals, from the
    # FP32 inputs themselves (every float is a rational)
    from fractions import Fraction
    d = 64
    x = np.array([(k / (d - 1)) ** 2 for k in range(d)], np.float32)
    wk = [Fraction(float(v)) for v in x]
    exact = sum(wk[i] - wk[j] for i in range(d) for j in range(i)) / (d - 1)
    np.testing.assert_allclose(oracle.segment_stats(x)[0][0], float(exact), rtol=1e-14)
    pen, nd, nz = oracle.segment_stats(np.array([1.0, np.nan, 2.0], np.float32))
    assert np.isnan(pen[0]) and nd[0] == -1 and nz[0] == -1
