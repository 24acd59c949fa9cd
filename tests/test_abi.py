"""C-ABI contract tests that need no GPU: the library loads, exports every symbol that
include/wsr.h declares, and rejects bad arguments on the host before enqueuing anything."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2311_03096_amd as wsr
from paper_2311_03096_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = ctypes.c_void_p(256)  # never dereferenced: only used in calls that must fail validation


def _declared_symbols():
    with open(os.path.join(ROOT, "include", "wsr.h")) as f:
        txt = f.read()
    return sorted(set(re.findall(r"WSR_API\s+[\w\s\*]+?\b(wsr_\w+)\s*\(", txt)))


def test_header_matches_exports():
    declared = _declared_symbols()
    assert len(declared) == 25
    lib = wsr.load()
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTED) == declared


def test_version_and_status_strings():
    assert wsr.wsr_version() >= 100
    for code in (0, -1, -2, -3, -4):
        assert wsr.wsr_status_string(code)
    assert wsr.wsr_status_string(12345) == "unknown status"


def test_workspace_sizes():
    assert wsr.wsr_workspace_bytes([0, 8192]) == 0
    assert wsr.wsr_workspace_bytes([0, 0, 3, 4099, 12291]) == 0
    a = wsr.wsr_workspace_bytes([0, 8193])
    b = wsr.wsr_workspace_bytes([0, 1 << 20])
    c = wsr.wsr_workspace_bytes([0, 5, 1 << 20, (1 << 20) + 9000])
    assert 0 < a < b and b == c
    assert b >= (1 << 20) * 16  # two key and two index buffers at least
    with pytest.raises(wsr.WsrError) as e:
        wsr.wsr_workspace_bytes([0, (1 << 27) + 1])
    assert e.value.status == wsr.WSR_ERR_UNSUPPORTED


def _fwd(off, lam=0.1, w=FAKE, out=FAKE, perm=None, mask=None, ws=None, ws_bytes=0):
    off = np.ascontiguousarray(off, dtype=np.int64)
    return wsr.load().wsr_prox_forward(w, out, off.ctypes.data_as(ctypes.c_void_p), off.shape[0] - 1,
                                       ctypes.c_float(lam), perm, mask, ws, ws_bytes, None)


def test_forward_argument_errors():
    E = wsr.WSR_ERR_INVALID
    assert _fwd([1, 4]) == E  # offsets[0] != 0
    assert _fwd([0, 4, 2]) == E  # decreasing
    assert _fwd([0, 4], lam=-1.0) == E
    assert _fwd([0, 4], lam=float("nan")) == E
    assert _fwd([0, 4], lam=float("inf")) == E
    assert _fwd([0, 4], w=None) == E
    assert _fwd([0, 4], out=None) == E
    assert _fwd([0, 4], perm=FAKE, mask=None) == E  # saved state must be both or neither
    assert _fwd([0, 4], perm=None, mask=FAKE) == E
    assert _fwd([0, 1 << 20]) == wsr.WSR_ERR_WORKSPACE  # long segment needs workspace
    need = wsr.wsr_workspace_bytes([0, 1 << 20])
    assert _fwd([0, 1 << 20], ws=FAKE, ws_bytes=need - 1) == wsr.WSR_ERR_WORKSPACE
    assert _fwd([0, (1 << 27) + 1]) == wsr.WSR_ERR_UNSUPPORTED
    off = np.array([0, 4], np.int64)
    assert wsr.load().wsr_prox_forward(FAKE, FAKE, None, 1, ctypes.c_float(0.1), None, None, None, 0,
                                       None) == E
    assert wsr.load().wsr_prox_forward(FAKE, FAKE, off.ctypes.data_as(ctypes.c_void_p), -1,
                                       ctypes.c_float(0.1), None, None, None, 0, None) == E


def test_l1_forward_argument_errors():
    lib = wsr.load()
    off = np.array([0, 4], np.int64)
    po = off.ctypes.data_as(ctypes.c_void_p)
    E = wsr.WSR_ERR_INVALID
    f = ctypes.c_float

    def l1(beta, rho, lam=0.1, w=FAKE):
        return lib.wsr_prox_l1_forward(w, FAKE, po, 1, f(lam), f(beta), f(rho), None, 0, None)

    for beta, rho in [(-0.1, 0.0), (float("nan"), 0.0), (float("inf"), 0.0), (0.1, -0.01), (0.1, 1.01),
                      (0.1, float("nan"))]:
        assert l1(beta, rho) == E
    assert l1(0.1, 0.5, lam=-1.0) == E
    assert l1(0.1, 0.5, w=None) == E
    big = np.array([0, 1 << 20], np.int64)
    assert lib.wsr_prox_l1_forward(FAKE, FAKE, big.ctypes.data_as(ctypes.c_void_p), 1, f(0.1), f(0.1), f(0.5),
                                   None, 0, None) == wsr.WSR_ERR_WORKSPACE
    assert lib.wsr_prox_l1_forward_batched(None, FAKE, FAKE, None, f(0.1), f(0.1), f(0.5), None, 0, None) == E
    assert lib.wsr_prox_l1_forward_batched(FAKE, FAKE, FAKE, None, f(0.1), f(-1.0), f(0.5), None, 0, None) == E


def test_step_argument_errors():
    lib = wsr.load()
    E = wsr.WSR_ERR_INVALID
    f = ctypes.c_float

    def step(plan=FAKE, w=FAKE, g=FAKE, eta=0.1, out=FAKE, alpha=None, a=0.1, beta=0.1, rho=0.5, flags=0):
        return lib.wsr_prox_step_batched(plan, w, g, f(eta), out, alpha, f(a), f(beta), f(rho), flags, None, 0,
                                         None)

    assert step(plan=None) == E
    assert step(w=None) == E
    assert step(g=None) == E
    assert step(out=None) == E
    assert step(flags=2) == E
    assert step(eta=-1.0) == E
    assert step(eta=float("nan")) == E
    assert step(beta=-0.5) == E
    assert step(rho=1.5) == E
    assert step(a=-1.0) == E
    assert step(a=float("inf")) == E


def test_stats_argument_errors():
    lib = wsr.load()
    E = wsr.WSR_ERR_INVALID
    off = np.array([0, 4], np.int64)
    po = off.ctypes.data_as(ctypes.c_void_p)
    assert lib.wsr_segment_stats(None, po, 1, FAKE, None, 0, None) == E
    assert lib.wsr_segment_stats(FAKE, po, 1, None, None, 0, None) == E
    bad = np.array([0, 5, 3], np.int64)
    assert lib.wsr_segment_stats(FAKE, bad.ctypes.data_as(ctypes.c_void_p), 2, FAKE, None, 0, None) == E
    big = np.array([0, 1 << 20], np.int64)
    assert lib.wsr_segment_stats(FAKE, big.ctypes.data_as(ctypes.c_void_p), 1, FAKE, None, 0,
                                 None) == wsr.WSR_ERR_WORKSPACE
    assert lib.wsr_segment_stats_batched(None, FAKE, FAKE, None, 0, None) == E


def test_backward_argument_errors():
    lib = wsr.load()
    off = np.array([0, 4], np.int64)
    po = off.ctypes.data_as(ctypes.c_void_p)
    E = wsr.WSR_ERR_INVALID
    assert lib.wsr_prox_backward(FAKE, FAKE, po, 1, None, FAKE, None, 0, None) == E
    assert lib.wsr_prox_backward(FAKE, FAKE, po, 1, FAKE, None, None, 0, None) == E
    assert lib.wsr_prox_backward(FAKE, FAKE, po, 1, FAKE, FAKE, None, 0, None) == E  # aliasing
    assert lib.wsr_prox_backward(None, FAKE, po, 1, FAKE, FAKE, None, 0, None) == E
    big = np.array([0, 1 << 20], np.int64)
    assert lib.wsr_prox_backward(FAKE, ctypes.c_void_p(512), big.ctypes.data_as(ctypes.c_void_p), 1, FAKE,
                                 FAKE, None, 0, None) == wsr.WSR_ERR_WORKSPACE


def test_plan_argument_errors():
    lib = wsr.load()
    off = np.array([1, 4], np.int64)
    h = ctypes.c_void_p()
    assert lib.wsr_plan_create(off.ctypes.data_as(ctypes.c_void_p), 1, 0, ctypes.byref(h)) == wsr.WSR_ERR_INVALID
    off = np.array([0, 4], np.int64)
    assert lib.wsr_plan_create(off.ctypes.data_as(ctypes.c_void_p), 1, 0, None) == wsr.WSR_ERR_INVALID
    assert lib.wsr_plan_create(off.ctypes.data_as(ctypes.c_void_p), 1, 8, ctypes.byref(h)) == wsr.WSR_ERR_INVALID
    assert lib.wsr_plan_create(off.ctypes.data_as(ctypes.c_void_p), 1, 1, ctypes.byref(h)) == wsr.WSR_ERR_INVALID
    both = wsr.WSR_PLAN_MERGE_HULL | wsr.WSR_PLAN_MERGE_END
    assert lib.wsr_plan_create(off.ctypes.data_as(ctypes.c_void_p), 1, both, ctypes.byref(h)) == wsr.WSR_ERR_INVALID
    assert lib.wsr_plan_autotune(None, FAKE, FAKE, None, ctypes.c_float(0.1), None, 0, None) == wsr.WSR_ERR_INVALID
    assert lib.wsr_plan_merge_rounds(None, FAKE) == wsr.WSR_ERR_INVALID
    assert lib.wsr_plan_set_merge_rounds(None, FAKE) == wsr.WSR_ERR_INVALID
    assert lib.wsr_plan_sort_routes(None, FAKE) == wsr.WSR_ERR_INVALID
    assert lib.wsr_plan_set_sort_routes(None, FAKE) == wsr.WSR_ERR_INVALID
    assert lib.wsr_read_status(None, None, 0, None) == wsr.WSR_ERR_INVALID
    f = ctypes.c_float
    assert lib.wsr_plan_autotune_step(None, FAKE, FAKE, f(0.1), ctypes.c_void_p(512), None, f(0.1), f(0.0), f(0.0), 0,
                                      None, 0, None) == wsr.WSR_ERR_INVALID
    assert lib.wsr_plan_destroy(None) == wsr.WSR_ERR_INVALID
    n = ctypes.c_size_t()
    assert lib.wsr_plan_workspace_bytes(None, ctypes.byref(n)) == wsr.WSR_ERR_INVALID
    assert lib.wsr_prox_forward_batched(None, FAKE, FAKE, None, ctypes.c_float(0.1), None, None, None, 0,
                                        None) == wsr.WSR_ERR_INVALID
    assert lib.wsr_prox_backward_batched(None, FAKE, FAKE, FAKE, FAKE, None, 0, None) == wsr.WSR_ERR_INVALID


@pytest.mark.gpu
def test_plan_merge_routes():
    """The route a plan records: the default cap of collision rounds, or 0 (hull merge only).
    Creating a plan uploads its offsets, so this needs a device."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("plan creation uploads offsets to a device")
    p0 = wsr.wsr_plan_create([0, 100, 5000, 20000])
    p1 = wsr.wsr_plan_create([0, 100, 5000, 20000], wsr.WSR_PLAN_MERGE_HULL)
    try:
        assert wsr.wsr_plan_merge_rounds(p0) == [6, 6, 6, 6]
        assert wsr.wsr_plan_merge_rounds(p1) == [0, 0, 0, 0]
        wsr.wsr_plan_set_merge_rounds(p0, [0, 16, 2, 6])
        assert wsr.wsr_plan_merge_rounds(p0) == [0, 16, 2, 6]
        with pytest.raises(wsr.WsrError):
            wsr.wsr_plan_set_merge_rounds(p0, [0, 65, 2, 6])
        wsr.wsr_plan_set_merge_rounds(p0, [-1, 6, 6, 6])  # EndCollisions for the 2048 class
        assert wsr.wsr_plan_merge_rounds(p0) == [-1, 6, 6, 6]
        with pytest.raises(wsr.WsrError):
            wsr.wsr_plan_set_merge_rounds(p0, [-2, 6, 6, 6])
        with pytest.raises(wsr.WsrError):
            wsr.wsr_plan_set_merge_rounds(p0, [6, 6, 6, -1])  # no EndCollisions for long segments
        p2 = wsr.wsr_plan_create([0, 100, 5000, 20000], wsr.WSR_PLAN_MERGE_END)
        assert wsr.wsr_plan_merge_rounds(p2) == [-1, -1, -1, 6]
        wsr.wsr_plan_destroy(p2)
    finally:
        wsr.wsr_plan_destroy(p0)
        wsr.wsr_plan_destroy(p1)


def test_trace_collect_arguments():
    lib = wsr.load()
    n = ctypes.c_int(0)
    assert lib.wsr_trace_collect(-1, None, None, None, ctypes.byref(n)) == wsr.WSR_ERR_INVALID
    assert lib.wsr_trace_collect(4, None, None, None, ctypes.byref(n)) == wsr.WSR_ERR_INVALID
    assert lib.wsr_trace_collect(0, None, None, None, None) == wsr.WSR_ERR_INVALID
    assert wsr.wsr_trace_collect() == {}  # nothing recorded


def test_workloads_shapes():
    from paper_2311_03096_amd import workloads
    m = workloads.mlp_rows()
    assert m["offsets"].shape[0] - 1 == 8202 and m["offsets"][-1] == 29401088
    assert m["w"].dtype == np.float32
    c = workloads.chain(d=4096)
    assert np.all(np.diff(c["w"]) >= 0) and c["lam"] == np.float32(0.7)
    b = workloads.backward_rows(rows=4, d=16)
    assert b["g"].shape == (64,)


# ----------------------------------------------------------------------------- binding checks
# The ctypes binding rejects every buffer the kernels could read or write out of bounds (wrong
# dtype, wrong length for the segment layout, non-contiguous, not on the GPU) before any call
# into the library.  These run on CPU tensors: each mismatch must be named before the device check.

def _t(n, dtype=None):
    import torch
    return torch.zeros(n, dtype=dtype or torch.float32)


def test_binding_rejects_bad_buffers_plain():
    import torch
    off = np.array([0, 100, 300], np.int64)
    cases = [
        (dict(w=_t(300, torch.float64)), TypeError, "dtype"),
        (dict(w=_t(299)), ValueError, "elements"),
        (dict(out=_t(301)), ValueError, "elements"),
        (dict(w=_t(600)[::2]), ValueError, "contiguous"),
        (dict(saved_perm=_t(300, torch.int32)), ValueError, "both"),
        (dict(saved_perm=_t(300, torch.int64), saved_mask=_t(10, torch.int32)), TypeError, "dtype"),
        (dict(saved_perm=_t(299, torch.int32), saved_mask=_t(10, torch.int32)), ValueError, "elements"),
        (dict(saved_perm=_t(300, torch.int32), saved_mask=_t(9, torch.int32)), ValueError, "elements"),
        (dict(ws=_t(16, torch.float32)), TypeError, "dtype"),
        (dict(), ValueError, "GPU"),  # right sizes, but host memory
    ]
    for over, exc, word in cases:
        args = dict(w=_t(300), out=_t(300), saved_perm=None, saved_mask=None, ws=None)
        args.update(over)
        with pytest.raises(exc, match=word):
            _lib.wsr_prox_forward(args["w"], args["out"], off, 0.1, args["saved_perm"], args["saved_mask"],
                                  args["ws"])
    with pytest.raises(ValueError, match="elements"):
        _lib.wsr_prox_backward(_t(300), _t(300), off, _t(300, torch.int32), _t(11, torch.int32))
    with pytest.raises(ValueError, match="elements"):
        _lib.wsr_prox_l1_forward(_t(300), _t(30), off, 0.1, 0.1, 0.5)
    with pytest.raises(ValueError, match="bytes"):
        _lib.wsr_segment_stats(_t(300), off, _t(5, torch.int64))  # needs 2 records of 24 bytes


def test_binding_rejects_bad_buffers_batched():
    import torch
    plan = _lib.Plan(ctypes.c_void_p(256), np.array([0, 100, 300], np.int64))  # never dereferenced
    assert plan.n == 300 and plan.n_seg == 2
    with pytest.raises(ValueError, match="elements"):
        _lib.wsr_prox_forward_batched(plan, _t(300), _t(200), None, 0.1)
    with pytest.raises(ValueError, match="elements"):  # one lambda per segment
        _lib.wsr_prox_forward_batched(plan, _t(300), _t(300), _t(3), 0.1)
    with pytest.raises(TypeError, match="dtype"):
        _lib.wsr_prox_forward_batched(plan, _t(300), _t(300), _t(2, torch.float64), 0.1)
    with pytest.raises(ValueError, match="elements"):
        _lib.wsr_prox_backward_batched(plan, _t(300), _t(300), _t(299, torch.int32), _t(10, torch.int32))
    with pytest.raises(ValueError, match="elements"):
        _lib.wsr_prox_step_batched(plan, _t(300), _t(301), 0.1, _t(300))
    with pytest.raises(ValueError, match="elements"):
        _lib.wsr_prox_step_batched(plan, _t(300), _t(300), 0.1, _t(300), alpha=_t(1))
    with pytest.raises(ValueError, match="elements"):
        _lib.wsr_prox_l1_forward_batched(plan, _t(3), _t(300))
    with pytest.raises(ValueError, match="bytes"):
        _lib.wsr_segment_stats_batched(plan, _t(300), _t(47, torch.uint8))
    w = _t(300)
    with pytest.raises(ValueError, match="alias"):
        _lib.wsr_plan_autotune(plan, w, w, None, 0.1)
    with pytest.raises(ValueError, match="alias"):
        _lib.wsr_plan_autotune_step(plan, w, _t(300), 0.1, w)
    with pytest.raises(TypeError, match="Plan"):
        _lib.wsr_prox_forward_batched(ctypes.c_void_p(256), _t(300), _t(300), None, 0.1)


def test_tuning_key_and_cache(tmp_path):
    from paper_2311_03096_amd.ops import TuningCache, tuning_key
    off = np.concatenate([[0], np.cumsum([100, 3000, 3000, 5000, 20000, 1 << 20])]).astype(np.int64)
    k = tuning_key(off, "gfx950", 0, "forward")
    assert k == "gfx950|forward|0|1,2,1|32768,1048576"
    assert tuning_key(off, "gfx950", 0, "step0") != k
    assert tuning_key(off[:-1], "gfx950", 0, "forward") != k
    cache = TuningCache(str(tmp_path / "sub" / "tuning.json"))
    assert cache.get(k) is None
    cache.put(k, [6, 64, -1, 16], [0, 1, 0])
    assert TuningCache(cache.path).get(k) == {"rounds": [6, 64, -1, 16], "sort": [0, 1, 0]}
    cache.put("other", [0, 0, 0, 0])
    assert cache.get(k)["rounds"] == [6, 64, -1, 16] and cache.get("other") == {"rounds": [0, 0, 0, 0],
                                                                                "sort": [0, 0, 0]}
    import json
    with open(cache.path) as f:
        data = json.load(f)
    data["old"] = [2, 2, 2, 0]  # the older form: merge routes alone
    with open(cache.path, "w") as f:
        json.dump(data, f)
    assert cache.get("old") == {"rounds": [2, 2, 2, 0], "sort": [0, 0, 0]}
    with open(cache.path, "w") as f:
        f.write("not json")
    assert cache.get(k) is None  # a damaged file is ignored, not fatal


def test_noalloc_limits_on_host():
    """The fixed scratch of the allocation-free forward holds the workspace of every segment up to
    WSR_NOALLOC_MAX_SEGMENT; a longer one is rejected before any device call."""
    assert wsr.wsr_workspace_bytes([0, wsr.WSR_NOALLOC_MAX_SEGMENT]) <= wsr.WSR_NOALLOC_SCRATCH_BYTES
    assert wsr.wsr_workspace_bytes([0, 4 * wsr.WSR_NOALLOC_MAX_SEGMENT]) > wsr.WSR_NOALLOC_SCRATCH_BYTES
    lib = wsr.load()
    for d, want in ((4 * wsr.WSR_NOALLOC_MAX_SEGMENT, wsr.WSR_ERR_WORKSPACE), ((1 << 27) + 1, wsr.WSR_ERR_UNSUPPORTED)):
        off = np.array([0, d], np.int64)
        assert lib.wsr_prox_forward_noalloc(FAKE, FAKE, off.ctypes.data_as(ctypes.c_void_p), 1, ctypes.c_float(0.1),
                                            None, None, None) == want
    off = np.array([0, 5, 3], np.int64)
    assert lib.wsr_prox_forward_noalloc(FAKE, FAKE, off.ctypes.data_as(ctypes.c_void_p), 2, ctypes.c_float(0.1),
                                        None, None, None) == wsr.WSR_ERR_INVALID
