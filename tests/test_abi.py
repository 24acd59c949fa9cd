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
    assert len(declared) == 21
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
        wsr.wsr_workspace_bytes([0, (1 << 26) + 1])
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
    assert _fwd([0, (1 << 26) + 1]) == wsr.WSR_ERR_UNSUPPORTED
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
    assert lib.wsr_read_status(None, None, 0) == wsr.WSR_ERR_INVALID
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
