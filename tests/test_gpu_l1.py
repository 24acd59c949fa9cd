"""GPU parity of Alg. prox in full (l1 and rewinding lines) through the C ABI, against the
oracle's wsr_oracle_prox_l1_* on the same seeded inputs.

The collisions are those of the plain forward; the cases cover both kernel paths (one
workgroup per segment, device-wide for long segments), the batched entry point with
per-segment lambdas, the identity segments (lambda = 0, d = 1) where only the l1 rule acts,
non-finite segments, and the paper's rewinding value rho = 0.98.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected only where a GPU exists
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2311_03096_amd as wsr  # noqa: E402
from gpu_util import NTHREADS, compare_l1, dev, gpu_forward, gpu_forward_l1, gpu_step, step_reference  # noqa: E402
from paper_2311_03096_amd import workloads  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check_l1(case, beta, rho, batched=False, lam_arr=None):
    w, off, lam = case["w"], case["offsets"], case["lam"]
    beta, rho = float(np.float32(beta)), float(np.float32(rho))
    _say("l1 case", case.get("name"), "n", w.shape[0], "segments", off.shape[0] - 1, "beta", beta,
         "rho", rho, "batched", batched)
    lam_o = np.asarray(lam_arr, np.float32) if lam_arr is not None else lam
    out = gpu_forward_l1(w, off, lam, beta, rho, batched=batched, lam_arr=lam_arr)
    g_plain = gpu_forward(w, off, lam, batched=batched, lam_arr=lam_arr)
    u, p, s = oracle.prox_segments(w, lam_o, off, n_threads=NTHREADS)
    o_l1 = oracle.prox_l1_segments(w, lam_o, beta, rho, off, n_threads=NTHREADS)
    st = compare_l1(w, off, out, o_l1, dict(u=u, perm=p, start=s), g_plain, beta, rho, lam_o)
    _say("  stats", st)
    return out, st


@pytest.mark.parametrize("beta,rho", [(0.0, 0.0), (0.3, 0.0), (0.3, 0.5), (0.05, 0.98), (0.0, 1.0), (2.5, 0.5)])
def test_l1_d4096(beta, rho):
    _check_l1(workloads.plain(4096, 0.1), beta, rho)


@pytest.mark.parametrize("d", [1, 2, 65, 2049, 4097, 8192, 8193, 50000, 100003])
@pytest.mark.parametrize("dist", ["normal", "ties", "laplace"])
def test_l1_sizes(d, dist):
    lam = {"normal": 0.05, "ties": 0.5, "laplace": 2.0}[dist]
    case = workloads.random_segments([d], dist, lam, seed=d + 1)
    beta = 0.2 * float(np.abs(case["w"]).max())
    _check_l1(case, beta, 0.98)


@pytest.mark.parametrize("rho", [0.0, 0.98])
def test_l1_long_typical(rho):
    case = workloads.random_segments([(1 << 20) + 777], "normal", 0.1, seed=31)
    _, st = _check_l1(case, 0.5, rho)
    assert st["zeroed"] > 0


def test_l1_chain_one_cluster():
    case = workloads.chain(d=1 << 20)
    out, _ = _check_l1(case, 0.1, 0.5)
    assert np.ptp(out) == 0.0  # one cluster: one value


def test_l1_batched_equals_plain_and_per_segment_lambda():
    lens = [0, 1, 2, 3, 17, 64, 65, 1000, 2048, 2049, 3072, 4096, 4097, 8192, 8193, 20000, 0, 5, 33, 7000]
    case = workloads.random_segments(lens, "mixed", 0.05, seed=5)
    beta = 0.1 * float(np.abs(case["w"]).max())
    o1, _ = _check_l1(case, beta, 0.98, batched=False)
    o2, _ = _check_l1(case, beta, 0.98, batched=True)
    assert np.array_equal(o1, o2)
    lam_arr = np.linspace(0.0, 2.0, len(lens)).astype(np.float32)
    _check_l1(case, beta, 0.25, batched=True, lam_arr=lam_arr)


def test_l1_identity_and_nonfinite_segments():
    lens = [1, 3000, 1, 9000, 50, 20000]
    case = workloads.random_segments(lens, "normal", 0.0, seed=6)
    w = case["w"].copy()
    off = case["offsets"]
    w[off[4] + 7] = np.nan  # the fifth segment holds a NaN
    w[off[5] + 19999] = np.inf  # the last one an infinity (long segment)
    case = dict(case, w=w)
    for rho in (0.0, 0.6):
        # lambda = 0 on every segment: the elementwise rule of the rewinding section's example
        out, _ = _check_l1(case, 0.4, rho)
        ok = np.isfinite(w)
        seg_bad = np.zeros(w.shape[0], bool)
        for s in (4, 5):
            seg_bad[off[s]:off[s + 1]] = True
        x = w.astype(np.float64)
        b, r = float(np.float32(0.4)), float(np.float32(rho))  # the library takes FP32 arguments
        exp = np.where(np.abs(x) < b, 0.0, x - (1 - r) * b * np.sign(x))
        m = ok & ~seg_bad
        ulp = np.spacing(np.abs(exp[m]).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(out[m] - exp[m]) <= ulp)  # one FP32 rounding of the FP64 value
        assert np.isnan(out[seg_bad]).all()
    lam_arr = np.array([0.3, 0.0, 1.0, 0.0, 0.2, 0.05], np.float32)
    _check_l1(case, 0.4, 0.6, batched=True, lam_arr=lam_arr)


def test_l1_mlp_rows_batched():
    case = workloads.mlp_rows()
    _, st = _check_l1(case, 0.01, 0.98, batched=True)
    assert st["zeroed"] > 0


# ----------------------------------------------------------------------------- proximal-gradient step

def _check_step(case, eta, alpha, beta, rho, variant, inplace=True, alpha_arr=None, seed=0):
    w, off = case["w"], case["offsets"]
    f32 = np.float32
    eta, alpha, beta, rho = float(f32(eta)), float(f32(alpha)), float(f32(beta)), float(f32(rho))
    _say("step case", case.get("name"), "n", w.shape[0], "segments", off.shape[0] - 1, "eta", eta, "alpha",
         alpha, "beta", beta, "rho", rho, "variant", variant, "inplace", inplace)
    grad = np.random.default_rng(seed).standard_normal(w.shape[0]).astype(np.float32)
    out, w_after = gpu_step(w, grad, off, eta, alpha, beta, rho, variant, inplace, alpha_arr)
    if not inplace:
        assert np.array_equal(w_after, w)
    o, z, o_plain, g_plain, beta_eff, q, lam_eff = step_reference(w, grad, off, eta, alpha, beta, rho, variant,
                                                                   alpha_arr)
    st = compare_l1(z, off, out, o, o_plain, g_plain, beta_eff, q, lam_eff)
    _say("  stats", st)
    return out, st


@pytest.mark.parametrize("variant", [False, True])
def test_step_mlp_rows_in_place(variant):
    case = workloads.mlp_rows()
    # the paper's CIFAR10 setting has learning rate 0.1 and rho = 0.98
    _check_step(case, 0.1, 1e-2 if not variant else 1e-3, 0.1 if not variant else 0.01, 0.98, variant)


@pytest.mark.parametrize("variant", [False, True])
def test_step_mixed_segments_per_segment_alpha(variant):
    lens = [0, 1, 2, 65, 2049, 4096, 8192, 8193, 20000, 3, 100003]
    case = workloads.random_segments(lens, "mixed", 0.05, seed=9)
    alpha_arr = np.linspace(0.0, 0.5, len(lens)).astype(np.float32)
    _check_step(case, 0.25, 0.0, 0.05, 0.5, variant, inplace=False, alpha_arr=alpha_arr, seed=1)
    _check_step(case, 0.25, 0.2, 0.05, 0.5, variant, inplace=True, seed=2)


@pytest.mark.parametrize("eta", [0.0, 1.0, 3.0])
def test_step_eta_edges(eta):
    """eta = 0: the standard step is the identity (lambda = beta' = 0), the variant keeps the
    cluster means; eta = 1: both forms coincide; eta = 3 > 1/(1 - rho): the variant moves the
    clusters past their prox values."""
    case = workloads.random_segments([3000, 9000], "normal", 0.1, seed=10)
    o1, _ = _check_step(case, eta, 0.3, 0.2, 0.5, False, seed=3)
    o2, _ = _check_step(case, eta, 0.3, 0.2, 0.5, True, seed=3)
    if eta == 0.0:
        assert np.array_equal(o1, case["w"])
    if eta == 1.0:
        np.testing.assert_allclose(o1, o2, rtol=0, atol=1e-6)


def test_ops_batched_step_autotuned_in_place():
    """The torch wrapper: a plan tuned on the first step's weights, an in-place step, the
    statistics of the result."""
    from paper_2311_03096_amd.ops import BatchedProx, row_offsets, segment_stats
    off = row_offsets([(300, 3072), (2, 20000)])
    rng = np.random.default_rng(50)
    w0 = (rng.standard_normal(off[-1]) / 50).astype(np.float32)
    g0 = rng.standard_normal(off[-1]).astype(np.float32)
    w = torch.from_numpy(w0).cuda()
    bp = BatchedProx(off, autotune=True)
    try:
        bp.step(w, torch.from_numpy(g0).cuda(), eta=0.1, alpha_scalar=1e-2, beta=0.1, rho=0.98)
        torch.cuda.synchronize()
        assert not bp.tune_pending
    finally:
        bp.close()
    got = w.cpu().numpy()
    o, z, o_plain, g_plain, beta_eff, q, lam_eff = step_reference(w0, g0, off, 0.1, 1e-2, 0.1, 0.98, False)
    st = compare_l1(z, off, got, o, o_plain, g_plain, beta_eff, q, lam_eff)
    _say("  stats", st)
    R, nd, nz = segment_stats(w, off)
    Ro, ndo, nzo = oracle.segment_stats(got, off)
    np.testing.assert_allclose(R, Ro, rtol=1e-9)
    assert np.array_equal(nd, ndo) and np.array_equal(nz, nzo)


def test_step_aliasing_and_nonfinite_gradient():
    """out may alias the gradient; a non-finite gradient entry makes its segment NaN (the step's
    input there is non-finite), the other segments are unaffected."""
    lens = [3000, 9000, 4096, 20000]
    case = workloads.random_segments(lens, "normal", 0.05, seed=51)
    w0, off = case["w"], case["offsets"]
    g0 = np.random.default_rng(52).standard_normal(w0.shape[0]).astype(np.float32)
    g0[off[1] + 17] = np.nan   # second segment (long)
    g0[off[2] + 5] = np.inf    # third segment (short)
    o = oracle.prox_step_segments(w0, g0, 0.2, np.float32(0.05), 0.1, 0.5, off, n_threads=NTHREADS)
    wt, gt = dev(w0), dev(g0)
    plan = wsr.wsr_plan_create(off)
    try:
        nb = wsr.wsr_plan_workspace_bytes(plan)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
        wsr.wsr_prox_step_batched(plan, wt, gt, 0.2, gt, None, 0.05, 0.1, 0.5, 0, ws)  # out = grad
        torch.cuda.synchronize()
    finally:
        wsr.wsr_plan_destroy(plan)
    got = gt.cpu().numpy()
    assert np.isnan(got[off[1]:off[2]]).all() and np.isnan(got[off[2]:off[3]]).all()
    o2, z, o_plain, g_plain, beta_eff, q, lam_eff = step_reference(w0, g0, off, 0.2, 0.05, 0.1, 0.5, False)
    assert np.array_equal(np.isnan(o), np.isnan(o2))
    st = compare_l1(z, off, got, o2, o_plain, g_plain, beta_eff, q, lam_eff)
    _say("  stats", st)
    assert np.array_equal(wt.cpu().numpy(), w0)  # w untouched


def test_sticky_nonfinite_status():
    """A plan's status word records a non-finite input weight from any batched forward-type call
    (short or long segment) until it is read and cleared."""
    lens = [3000, 20000]
    case = workloads.random_segments(lens, "normal", 0.05, seed=53)
    off = case["offsets"]
    w_ok = dev(case["w"])
    plan = wsr.wsr_plan_create(off)
    try:
        nb = wsr.wsr_plan_workspace_bytes(plan)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
        out = torch.empty_like(w_ok)
        wsr.wsr_prox_forward_batched(plan, w_ok, out, None, 0.05, None, None, ws)
        assert wsr.wsr_read_status(plan) == 0
        for where in (off[0] + 5, off[1] + 19999):  # short segment, then long segment
            w_bad = w_ok.clone()
            w_bad[int(where)] = float("nan")
            wsr.wsr_prox_forward_batched(plan, w_bad, out, None, 0.05, None, None, ws)
            wsr.wsr_prox_forward_batched(plan, w_ok, out, None, 0.05, None, None, ws)  # sticky
            assert wsr.wsr_read_status(plan, clear=False) == wsr.WSR_STATUS_NONFINITE
            assert wsr.wsr_read_status(plan) == wsr.WSR_STATUS_NONFINITE
            assert wsr.wsr_read_status(plan) == 0
        g = torch.zeros_like(w_ok)
        g[7] = float("inf")
        wsr.wsr_prox_step_batched(plan, w_ok, g, 0.1, out, None, 0.1, 0.0, 0.0, 0, ws)
        assert wsr.wsr_read_status(plan) == wsr.WSR_STATUS_NONFINITE
        wsr.wsr_prox_l1_forward_batched(plan, w_ok, out, None, 0.05, 0.1, 0.5, ws)
        assert wsr.wsr_read_status(plan) == 0
    finally:
        wsr.wsr_plan_destroy(plan)


def _random_layout(seed):
    rng = np.random.default_rng(2000 + seed)
    nseg = int(rng.integers(1, 41))
    kinds = rng.choice(["tiny", "short", "long"], nseg, p=[0.3, 0.5, 0.2])
    lens = [int(rng.integers(0, 40)) if k == "tiny" else int(rng.integers(40, 8193)) if k == "short"
            else int(rng.integers(8193, 150000)) for k in kinds]
    dist = ["normal", "laplace", "ties", "sorted", "mixed"][seed % 5]
    lam = float(10.0 ** rng.uniform(-4, 0))
    case = workloads.random_segments(lens, dist, lam, seed=seed)
    scale = float(np.abs(case["w"]).max()) if case["w"].size else 1.0
    beta = float(rng.choice([0.0, 0.01, 0.1, 0.5])) * scale
    rho = float(rng.choice([0.0, 0.5, 0.98, 1.0]))
    return case, beta, rho, rng


@pytest.mark.parametrize("seed", list(range(5)) + [28, 32])  # 28, 32: beta = 0, rho = 1, clusters of zeros
def test_l1_and_step_random_layouts(seed):
    """Seeded random layouts (1-40 segments, 1 to ~150k weights each, every distribution):
    Alg. prox in full through the plain and batched entry points, and one proximal-gradient step
    in both forms, against the oracle."""
    case, beta, rho, rng = _random_layout(seed)
    _check_l1(case, beta, rho, batched=bool(seed % 2))
    eta = float(rng.choice([0.05, 0.1, 1.0]))
    _check_step(case, eta, case["lam"] / eta, beta / eta, rho, variant=bool(seed % 2), inplace=bool(seed % 3),
                seed=seed)
