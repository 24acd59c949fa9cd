"""GPU test of the allocation-free forward (wsr_prox_forward_noalloc, through the C ABI): it
must give exactly what wsr_prox_forward gives with a caller's workspace, on two calls in a row
(the second with a smaller input, so stale scratch contents from the first would show), and the
oracle's result; a segment beyond the fixed scratch is rejected on the host."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected only where a GPU exists
    pytest.skip("no GPU", allow_module_level=True)

import paper_2311_03096_amd as wsr  # noqa: E402
from gpu_util import compare, dev, gpu_forward, mask_to_start, oracle_forward  # noqa: E402
from paper_2311_03096_amd import workloads  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _noalloc(case, save=True):
    w = dev(case["w"])
    out = torch.full_like(w, float("nan"))
    n = w.numel()
    perm = torch.full((n,), -1, dtype=torch.int32, device="cuda") if save else None
    mask = torch.full(((n + 31) // 32,), -1, dtype=torch.int32, device="cuda") if save else None
    wsr.wsr_prox_forward_noalloc(w, out, case["offsets"], case["lam"], perm, mask)
    torch.cuda.synchronize()
    res = dict(out=out.cpu().numpy())
    if save:
        res["perm"] = perm.cpu().numpy()
        res["start"] = mask_to_start(mask.cpu().numpy(), n)
    return res


@pytest.mark.parametrize("save", [True, False])
def test_noalloc_matches_workspace_forward_twice(save):
    first = workloads.random_segments([wsr.WSR_NOALLOC_MAX_SEGMENT, 3000, 50000, 17], "normal", 0.05, seed=80)
    second = workloads.random_segments([300001, 4096, 9000], "laplace", 0.5, seed=81)  # smaller
    assert second["w"].shape[0] < first["w"].shape[0]
    for case in (first, second):
        _say("noalloc case", case["name"], "n", case["w"].shape[0], "save", save)
        got = _noalloc(case, save)
        ref = gpu_forward(case["w"], case["offsets"], case["lam"], save=save)
        for k in got:
            assert np.array_equal(got[k], ref[k]), k
        o = oracle_forward(case["w"], case["offsets"], case["lam"])
        _say("  stats", compare(case["w"], case["offsets"], got, o, lam=case["lam"]))


def test_noalloc_rejects_beyond_scratch():
    d = wsr.WSR_NOALLOC_MAX_SEGMENT * 2
    w = torch.zeros(d, dtype=torch.float32, device="cuda")
    with pytest.raises(wsr.WsrError) as e:
        wsr.wsr_prox_forward_noalloc(w, w, np.array([0, d], np.int64), 0.1)
    assert e.value.status == wsr.WSR_ERR_WORKSPACE
