"""GPU tests of the torch-facing layer and the plan API: batched autograd through a cached plan,
an autotuned in-place forward, the step's autotuner, the persisted tuning, and the stream-local
status read.  Results are checked against the CPU oracle."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected only where a GPU exists
    pytest.skip("no GPU", allow_module_level=True)

import paper_2311_03096_amd as wsr  # noqa: E402
from gpu_util import (autograd_saved_partition, compare, compare_l1, dev, gpu_forward, oracle_forward,  # noqa: E402
                      step_reference, vjp_check)
from paper_2311_03096_amd import ops, workloads  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_autograd_batched_rows_and_plan_cache():
    """prox() on a row-segmented layer runs the batched entry points over a cached plan: forward
    and backward against the oracle, and a second call reuses the same plan."""
    off = ops.row_offsets([(300, 3072), (40, 4096), (2, 20000)])
    rng = np.random.default_rng(60)
    w0 = (rng.standard_normal(off[-1]) / 50).astype(np.float32)
    g0 = rng.standard_normal(off[-1]).astype(np.float32)
    lam = 1e-3
    w = torch.from_numpy(w0).cuda().requires_grad_(True)
    u = ops.prox(w, lam, off)
    gp, gs = autograd_saved_partition(u, off)  # read before backward frees it
    u.backward(torch.from_numpy(g0).cuda())
    bp = ops.cached_plan(off, w.device)
    u2 = ops.prox(w.detach(), lam, off)
    assert ops.cached_plan(off, w.device) is bp
    assert torch.equal(u.detach(), u2)
    o = oracle_forward(w0, off, lam)
    out = u.detach().cpu().numpy()
    _say("  forward", compare(w0, off, dict(out=out), o, lam=lam))
    _say("  with the saved partition", compare(w0, off, dict(out=out, perm=gp, start=gs), o, lam=lam))
    vjp_check(g0, off, dict(perm=gp, start=gs), w.grad.cpu().numpy())


def test_autotuned_forward_in_place():
    """BatchedProx(autotune=True).forward(w, w): the routes are timed into a scratch buffer, so
    the in-place result is the prox applied once."""
    case = workloads.random_segments([3000] * 100 + [4096] * 50 + [30000], "normal", 0.05, seed=61)
    off = case["offsets"]
    w = dev(case["w"])
    bp = ops.BatchedProx(off, autotune=True)
    try:
        bp.forward(w, w, lam_scalar=case["lam"], save=False)
        torch.cuda.synchronize()
        assert not bp.tune_pending
        _say("  tuned routes", bp.merge_rounds())
    finally:
        bp.close()
    o = oracle_forward(case["w"], off, case["lam"])
    _say("  stats", compare(case["w"], off, dict(out=w.cpu().numpy()), o, lam=case["lam"]))


def test_autotune_rejects_aliasing():
    case = workloads.random_segments([3000, 20000], "normal", 0.05, seed=62)
    w = dev(case["w"])
    plan = wsr.wsr_plan_create(case["offsets"])
    try:
        lib = wsr.load()
        import ctypes
        p = ctypes.c_void_p(w.data_ptr())
        rc = lib.wsr_plan_autotune(plan, p, p, None, ctypes.c_float(0.05), None, 0, None)
        assert rc == wsr.WSR_ERR_INVALID
    finally:
        wsr.wsr_plan_destroy(plan)


@pytest.mark.parametrize("variant", [False, True])
def test_autotune_step_then_step(variant):
    """The step's autotuner times the step's own launches (into scratch, w and grad untouched);
    the tuned plan's step matches the oracle."""
    case = workloads.random_segments([3072] * 200 + [4096] * 100 + [50000], "normal", 0.05, seed=63)
    off = case["offsets"]
    w0 = case["w"]
    g0 = np.random.default_rng(64).standard_normal(w0.shape[0]).astype(np.float32)
    eta, alpha, beta, rho = 0.1, (1e-2 if not variant else 1e-3), (0.1 if not variant else 0.01), 0.98
    w, g = dev(w0), dev(g0)
    plan = wsr.wsr_plan_create(off)
    try:
        nb = wsr.wsr_plan_workspace_bytes(plan)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
        scratch = torch.empty_like(w)
        flags = wsr.WSR_STEP_ETA_IN_DISPLACEMENT if variant else 0
        wsr.wsr_plan_autotune_step(plan, w, g, eta, scratch, None, alpha, beta, rho, flags, ws)
        _say("  tuned routes", wsr.wsr_plan_merge_rounds(plan))
        assert np.array_equal(w.cpu().numpy(), w0) and np.array_equal(g.cpu().numpy(), g0)
        wsr.wsr_prox_step_batched(plan, w, g, eta, w, None, alpha, beta, rho, flags, ws)
        torch.cuda.synchronize()
    finally:
        wsr.wsr_plan_destroy(plan)
    o, z, o_plain, g_plain, beta_eff, q, lam_eff = step_reference(w0, g0, off, np.float32(eta), np.float32(alpha),
                                                                  np.float32(beta), np.float32(rho), variant)
    _say("  stats", compare_l1(z, off, w.cpu().numpy(), o, o_plain, g_plain, beta_eff, q, lam_eff))


def test_tuning_cache_round_trip(tmp_path):
    """A plan tuned once stores its routes under the architecture and segment-length histogram; a
    new plan of the same layout takes them from the cache without timing, and gives the same
    result."""
    case = workloads.random_segments([4096] * 64 + [20000], "normal", 0.05, seed=65)
    off = case["offsets"]
    path = str(tmp_path / "tuning.json")
    w = dev(case["w"])
    out1, out2 = torch.empty_like(w), torch.empty_like(w)
    a = ops.BatchedProx(off, autotune=True, tuning_cache=path)
    a.forward(w, out1, lam_scalar=case["lam"])
    key = ops.tuning_key(off, ops.device_arch(), 0, "forward")
    stored = ops.TuningCache(path).get(key)
    assert stored == {"rounds": a.merge_rounds(), "sort": a.sort_routes()}
    # a different stored tuning is applied as is, with no timing (the plan's routes become it)
    forced, forced_sort = [6, 0, 16, 0], [1, 1, 0]
    ops.TuningCache(path).put(key, forced, forced_sort)
    b = ops.BatchedProx(off, autotune=True, tuning_cache=path)
    b.forward(w, out2, lam_scalar=case["lam"])
    assert b.merge_rounds() == forced and b.sort_routes() == forced_sort and not b.tune_pending
    torch.cuda.synchronize()
    assert torch.equal(out1, out2)  # every route gives the same result
    a.close()
    b.close()


@pytest.mark.parametrize("dist", ["normal", "quantised", "ties"])
def test_sort_routes_give_the_same_bits(dist):
    """The short classes' two sort routes (the bucket-rank sort, with the radix sort when a bucket
    overflows; the radix sort alone) give identical outputs, permutations and cluster starts (both
    order by value, then index) on spread-out, quantised and tie-heavy rows of every size class,
    matching the oracle; the autotuned routes give the same bits again."""
    lens = [17, 1, 2049] + [2048] * 30 + [3072] * 30 + [4096] * 30 + [6000] * 10 + [8192] * 6
    case = workloads.random_segments(lens, "ties" if dist == "ties" else "normal", 1e-3, seed=66)
    w = case["w"]
    if dist == "quantised":  # 1/64 steps: a few equal weights per value
        w = (np.round(w.astype(np.float64) * 64) / 64).astype(np.float32)
    off, lam = case["offsets"], case["lam"]
    a = gpu_forward(w, off, lam, batched=True, sort_routes=[wsr.WSR_SORT_BUCKET] * 3)
    b = gpu_forward(w, off, lam, batched=True, sort_routes=[wsr.WSR_SORT_RADIX] * 3)
    c = gpu_forward(w, off, lam, batched=True, autotune=True)
    for k in ("out", "perm", "start"):
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k
    _say("sort routes", dist, "clusters", int(a["start"].sum()))
    compare(w, off, a, oracle_forward(w, off, lam), lam=lam)


def test_sort_routes_l1_step_and_stats():
    """The batched l1 forward, proximal-gradient step and segment statistics give the same bits
    under both sort routes, on tie-heavy rows (where the routes differ most in time)."""
    lens = [2048] * 20 + [4096] * 20 + [7000] * 5 + [3]
    case = workloads.random_segments(lens, "normal", 1e-3, seed=67)
    w_np = (np.round(case["w"].astype(np.float64) * 32) / 32).astype(np.float32)
    off = case["offsets"]
    g_np = np.random.default_rng(68).standard_normal(w_np.shape[0]).astype(np.float32)
    w, g = dev(w_np), dev(g_np)
    res = []
    for route in (wsr.WSR_SORT_BUCKET, wsr.WSR_SORT_RADIX):
        plan = wsr.wsr_plan_create(off)
        try:
            wsr.wsr_plan_set_sort_routes(plan, [route] * 3)
            assert wsr.wsr_plan_sort_routes(plan) == [route] * 3
            nb = wsr.wsr_plan_workspace_bytes(plan)
            ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
            o1, o2 = torch.empty_like(w), torch.empty_like(w)
            wsr.wsr_prox_l1_forward_batched(plan, w, o1, None, 0.05, 0.01, 0.5, ws)
            wsr.wsr_prox_step_batched(plan, w, g, 0.1, o2, None, 1e-2, 0.01, 0.98, 0, ws)
            st = torch.full((len(lens), 3), -7, dtype=torch.int64, device="cuda")  # every record written
            wsr.wsr_segment_stats_batched(plan, w, st, ws)
            torch.cuda.synchronize()
            res.append((o1.cpu().numpy(), o2.cpu().numpy(), st.cpu().numpy()))
        finally:
            wsr.wsr_plan_destroy(plan)
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    with pytest.raises(wsr.WsrError):
        plan = wsr.wsr_plan_create(off)
        try:
            wsr.wsr_plan_set_sort_routes(plan, [0, 2, 0])
        finally:
            wsr.wsr_plan_destroy(plan)


def test_phase_clock_build():
    """The measurement build libwsr_phases.so gives the regular library's bits, and its phase
    timestamps are written for every short segment, in order, at the slots of its workgroup."""
    import ctypes
    import os
    lens = [2048] * 30 + [1] + [4096] * 30 + [7000] * 10 + [30000]
    case = workloads.random_segments(lens, "normal", 0.05, seed=69)
    off = np.ascontiguousarray(case["offsets"], dtype=np.int64)
    w = dev(case["w"])
    ref = torch.empty_like(w)
    plan = wsr.wsr_plan_create(off)
    try:
        nb = wsr.wsr_plan_workspace_bytes(plan)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        wsr.wsr_prox_forward_batched(plan, w, ref, None, case["lam"], None, None, ws)
    finally:
        wsr.wsr_plan_destroy(plan)
    lib = ctypes.CDLL(os.path.join(os.path.dirname(wsr.__file__), "libwsr_phases.so"))
    p, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.wsr_plan_create.argtypes = [p, i64, ctypes.c_int, ctypes.POINTER(p)]
    lib.wsr_plan_destroy.argtypes = [p]
    lib.wsr_prox_forward_batched.argtypes = [p, p, p, p, ctypes.c_float, p, p, p, ctypes.c_size_t, p]
    lib.wsr_phase_clock_buffer.argtypes = [p, i64]
    slots = lib.wsr_phase_clock_slots()
    n_short = len(lens) - 1
    clocks = torch.zeros(n_short * slots, dtype=torch.int64, device="cuda")
    out = torch.empty_like(w)
    stream = p(torch.cuda.current_stream().cuda_stream)
    assert lib.wsr_phase_clock_buffer(None, 5) == wsr.WSR_ERR_INVALID
    assert lib.wsr_phase_clock_buffer(p(clocks.data_ptr()), n_short) == 0
    h = p()
    assert lib.wsr_plan_create(off.ctypes.data, len(lens), 0, ctypes.byref(h)) == 0
    try:
        rc = lib.wsr_prox_forward_batched(h, p(w.data_ptr()), p(out.data_ptr()), None, case["lam"], None, None,
                                          p(ws.data_ptr()), nb, stream)
        assert rc == 0
        torch.cuda.synchronize()
    finally:
        lib.wsr_phase_clock_buffer(None, 0)
        lib.wsr_plan_destroy(h)
    assert torch.equal(out.view(torch.int32), ref.view(torch.int32))
    t = clocks.view(n_short, slots).cpu().numpy()
    done = t[:, 5] > 0
    assert done.sum() == n_short - 1  # the d = 1 segment leaves before the sort
    assert np.all(t[~done, :2] > 0) and np.all(t[~done, 2:] == 0)
    assert np.all(np.diff(t[done, :6], axis=1) >= 0)
    assert np.all(t[:, 6:] == 0)


def test_phase_clock_build_merge_and_backward():
    """The measurement build's long-segment forward gives the regular bits and writes the merge
    launches' timestamps in order; its batched backward gives the regular bits and writes the
    backward's phase timestamps in order."""
    import ctypes
    import os
    lib = ctypes.CDLL(os.path.join(os.path.dirname(wsr.__file__), "libwsr_phases.so"))
    p, i64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
    lib.wsr_prox_forward.argtypes = [p, p, p, i64, ctypes.c_float, p, p, p, sz, p]
    lib.wsr_workspace_bytes.argtypes = [p, i64, ctypes.POINTER(sz)]
    lib.wsr_phase_merge_clock_buffer.argtypes = [p]
    lib.wsr_phase_clock_buffer.argtypes = [p, i64]
    lib.wsr_plan_create.argtypes = [p, i64, ctypes.c_int, ctypes.POINTER(p)]
    lib.wsr_plan_destroy.argtypes = [p]
    lib.wsr_prox_forward_batched.argtypes = [p, p, p, p, ctypes.c_float, p, p, p, ctypes.c_size_t, p]
    lib.wsr_prox_backward_batched.argtypes = [p, p, p, p, p, p, ctypes.c_size_t, p]
    stream = p(torch.cuda.current_stream().cuda_stream)
    # one long segment of 2^20 + 777 weights: 257 hull tiles, levels in three merge launches
    case = workloads.plain((1 << 20) + 777, 0.05, seed=70)
    off = np.ascontiguousarray(case["offsets"], dtype=np.int64)
    w = dev(case["w"])
    ref = torch.empty_like(w)
    out = torch.empty_like(w)
    nb = sz()
    assert lib.wsr_workspace_bytes(off.ctypes.data, 1, ctypes.byref(nb)) == 0
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    wsr.wsr_prox_forward(w, ref, off, case["lam"], None, None, ws)
    clk = torch.zeros(4 * 4096 * 16, dtype=torch.int64, device="cuda")
    assert lib.wsr_phase_merge_clock_buffer(p(clk.data_ptr())) == 0
    try:
        assert lib.wsr_prox_forward(p(w.data_ptr()), p(out.data_ptr()), off.ctypes.data, 1, case["lam"], None, None,
                                    p(ws.data_ptr()), nb.value, stream) == 0
        torch.cuda.synchronize()
    finally:
        lib.wsr_phase_merge_clock_buffer(None)
    assert torch.equal(out.view(torch.int32), ref.view(torch.int32))
    t = clk.view(4, 4096, 16).cpu().numpy()
    launches = [li for li in range(4) if (t[li, :, 0] > 0).any()]
    assert launches == [0, 1, 2]  # 257 tiles: levels 1-4, 5-8, 9
    for li in launches:
        a = t[li][t[li, :, 0] > 0]
        nlev = int((a[0, 1:5] > 0).sum())
        assert nlev >= 1 and np.all(a[:, 1:1 + nlev] > 0)
        assert np.all(np.diff(a[:, :1 + nlev], axis=1) >= 0)
        assert np.all(a[:, 13] >= a[:, nlev])
    # the batched backward of short rows
    lens = [4096] * 40 + [3000] * 20
    case = workloads.random_segments(lens, "normal", 1e-3, seed=71)
    off = np.ascontiguousarray(case["offsets"], dtype=np.int64)
    w = dev(case["w"])
    g = dev(np.random.default_rng(72).standard_normal(off[-1]).astype(np.float32))
    out = torch.empty_like(w)
    perm = torch.empty(off[-1], dtype=torch.int32, device="cuda")
    mask = torch.empty((int(off[-1]) + 31) // 32, dtype=torch.int32, device="cuda")
    gw_ref, gw = torch.empty_like(g), torch.empty_like(g)
    h = p()
    assert lib.wsr_plan_create(off.ctypes.data, len(lens), 0, ctypes.byref(h)) == 0
    slots = lib.wsr_phase_clock_slots()
    clocks = torch.zeros(len(lens) * slots, dtype=torch.int64, device="cuda")
    try:
        assert lib.wsr_prox_forward_batched(h, p(w.data_ptr()), p(out.data_ptr()), None, case["lam"],
                                            p(perm.data_ptr()), p(mask.data_ptr()), None, 0, stream) == 0
        assert lib.wsr_prox_backward_batched(h, p(g.data_ptr()), p(gw_ref.data_ptr()), p(perm.data_ptr()),
                                             p(mask.data_ptr()), None, 0, stream) == 0
        assert lib.wsr_phase_clock_buffer(p(clocks.data_ptr()), len(lens)) == 0
        assert lib.wsr_prox_backward_batched(h, p(g.data_ptr()), p(gw.data_ptr()), p(perm.data_ptr()),
                                             p(mask.data_ptr()), None, 0, stream) == 0
        torch.cuda.synchronize()
    finally:
        lib.wsr_phase_clock_buffer(None, 0)
        lib.wsr_plan_destroy(h)
    assert torch.equal(gw.view(torch.int32), gw_ref.view(torch.int32))
    tb = clocks.view(len(lens), slots).cpu().numpy()
    assert np.all(tb[:, :5] > 0) and np.all(np.diff(tb[:, :5], axis=1) >= 0) and np.all(tb[:, 5:] == 0)


def test_read_status_on_its_stream():
    """The status read synchronises only the stream it is given: work on that stream is covered."""
    case = workloads.random_segments([3000, 20000], "normal", 0.05, seed=66)
    off = case["offsets"]
    w_bad = dev(case["w"])
    w_bad[17] = float("nan")
    plan = wsr.wsr_plan_create(off)
    s = torch.cuda.Stream()
    try:
        nb = wsr.wsr_plan_workspace_bytes(plan)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
        out = torch.empty_like(w_bad)
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            wsr.wsr_prox_forward_batched(plan, w_bad, out, None, 0.05, None, None, ws)
        assert wsr.wsr_read_status(plan, clear=True, stream=s.cuda_stream) == wsr.WSR_STATUS_NONFINITE
        assert wsr.wsr_read_status(plan, clear=False, stream=s.cuda_stream) == 0
    finally:
        torch.cuda.synchronize()
        wsr.wsr_plan_destroy(plan)


def test_per_row_and_batched_equal_gpu_forward():
    """The plain entry point (one launch per row) and the batched one give identical bits."""
    case = workloads.random_segments([4096] * 32 + [3072] * 32, "laplace", 0.05, seed=67)
    a = gpu_forward(case["w"], case["offsets"], case["lam"], batched=False)
    b = gpu_forward(case["w"], case["offsets"], case["lam"], batched=True)
    for k in ("out", "perm", "start"):
        assert np.array_equal(a[k], b[k])
