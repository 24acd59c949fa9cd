"""Benchmark of the prox_R hot path on one MI355X.

A step = one full pass of the path over the workload: forward (sort, rank shift, cluster
merge, scatter, saved permutation and cluster-start bits) then backward (cluster averages of an
upstream gradient).  Default workload: the worst-case collision chain, one segment of
d = 2^24 FP32 weights w_k = (k/(d-1))^2 with lam = 0.7 (every particle ends in one cluster).

Prints one JSON line: elements/s over the timed steps, the roofline of the dominant kernel
(HIP-event durations measured live on the library's stream; a sort pass is charged its share of
the sort's one key + index round trip), the CPU oracle on the host as a reference, and extra
figures, each the median of >= 50 timed reps after >= 10 warm-ups: one row per workload (plain
d = 4096, the shuffled chain, a typical N(0,1) vector of 2^24, the 1024 x 8192 backward rows, the
d = 2^26 precision vector with its FP32 negative control), the batched MLP rows (graph-captured
batched launches versus per-row launches), Alg. prox in full, segment statistics, the merge
routes and the per-layer segmentation.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "prox_R elements/s + % HBM roofline at d=2^24; batched vs per-row launch speedup"
WORKLOAD_TEXT = {
    "chain": "worst-case collision chain: one FP32 segment d=2^24, w_k=(k/(d-1))^2, lam=0.7 "
             "(one final cluster); step = forward with saved state + backward",
    "typical": "one N(0,1) FP32 segment d=2^24, lam=0.1; step = forward with saved state + backward",
}

# Algorithmic HBM bytes per element that each kernel must move (compulsory traffic of its role
# in the path; see the design notes).  "el" = elements of the segment(s) the launch covers.  A
# segment too long for on-chip memory needs one out-of-core key + index round trip for its sort
# (SORT_ROUND_TRIP_B per element, once per sort): it is spread over the sort's scatter passes, so
# each scatter launch is charged its share; the histogram passes and the extra passes of a
# multi-pass sort are not compulsory.  The rate of one scatter pass moving key + index once is
# reported beside it as ``achieved_per_pass``.
SORT_ROUND_TRIP_B = 16.0
KERNEL_BYTES_PER_EL = {
    "radix_hist": 0.0,          # histogram reads: not compulsory (inside the sort's round trip)
    "radix_rowscan": 0.0,
    "big_tile_hull": 4.0,       # read sorted key (hull vertices are bookkeeping)
    "big_apply": 12.125,        # read sorted key + perm 8 B, write value 4 B, start bit
    "big_bwd_tile": 12.0,       # read perm 4 + gradient 4, write gathered gradient 4
    "big_bwd_apply": 12.125,    # read gathered gradient 4 + perm 4 + bit, write gradient 4
    "prox_fwd_small_4096": 12.125,  # read w, write u + perm + bit
    "prox_bwd_small_4096": 12.125,  # read g + perm + bit, write gradient
    "prox_fwd_small_8192": 12.125,
    "prox_bwd_small_8192": 12.125,
    "prox_fwd_small_2048": 12.125,
    "prox_bwd_small_2048": 12.125,
}
SORT_KERNELS = ("radix_scatter", "radix_hist", "radix_rowscan")
MED_REPS, MED_WARMUP = 50, 10  # extra figures: median of >= 50 timed reps after >= 10 warm-ups


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the typical and batched figures")
    ap.add_argument("--rounds", default="", help="with --workload mlp: the batched plan's merge routes as four "
                    "collision-round caps (2048,4096,8192,long classes) instead of autotuning them")
    ap.add_argument("--workload", choices=["chain", "typical", "mlp", "shuffled", "backward", "precision"],
                    default="chain",
                    help="chain (default, the headline), or run one workload only (for profiling): the typical "
                         "d=2^24 vector, the batched MLP rows, the shuffled chain, the 1024x8192 backward "
                         "rows, the d=2^26 precision vector")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="BYTES",
                    help="first run one plain device copy of BYTES bytes (HBM counter calibration)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Step:
    """Buffers and the fwd+bwd step of one workload through the C ABI."""

    def __init__(self, case, batched=False, autotune=False, rounds=None):
        import torch
        import paper_2311_03096_amd as wsr
        self.wsr, self.torch = wsr, torch
        self.case = case
        self.n = case["w"].shape[0]
        self.offsets = case["offsets"]
        self.lam = case["lam"]
        self.w = torch.from_numpy(case["w"]).cuda()
        self.out = torch.empty_like(self.w)
        self.perm = torch.empty(self.n, dtype=torch.int32, device="cuda")
        self.mask = torch.empty((self.n + 31) // 32, dtype=torch.int32, device="cuda")
        g = case.get("g")
        if g is None:
            g = np.random.default_rng(123).standard_normal(self.n).astype(np.float32)
        self.g = torch.from_numpy(g).cuda()
        self.gw = torch.empty_like(self.g)
        self.batched = batched
        if batched:
            self.plan = wsr.wsr_plan_create(self.offsets)
            nb = wsr.wsr_plan_workspace_bytes(self.plan)
        else:
            self.plan = None
            nb = wsr.wsr_workspace_bytes(self.offsets)
        self.ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
        self.rounds = None
        if batched and rounds is not None:  # merge routes given (e.g. an earlier run's tuning)
            wsr.wsr_plan_set_merge_rounds(self.plan, rounds)
            self.rounds = wsr.wsr_plan_merge_rounds(self.plan)
        elif batched and autotune:  # merge route per size class, timed on these weights (synchronises)
            wsr.wsr_plan_autotune(self.plan, self.w, self.out, None, self.lam, self.ws)
            self.rounds = wsr.wsr_plan_merge_rounds(self.plan)

    def __call__(self):
        wsr = self.wsr
        if self.batched:
            wsr.wsr_prox_forward_batched(self.plan, self.w, self.out, None, self.lam, self.perm, self.mask, self.ws)
            wsr.wsr_prox_backward_batched(self.plan, self.g, self.gw, self.perm, self.mask, self.ws)
        else:
            wsr.wsr_prox_forward(self.w, self.out, self.offsets, self.lam, self.perm, self.mask, self.ws)
            wsr.wsr_prox_backward(self.g, self.gw, self.offsets, self.perm, self.mask, self.ws)


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return e0.elapsed_time(e1) / steps, wall


def copy_bandwidth(nbytes=1 << 28, reps=10):
    """Device-copy bandwidth (read + write bytes per second) of one plain elementwise kernel over
    nbytes, the practical ceiling next to the 8 TB/s HBM peak."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    ms, _ = time_steps(lambda: torch.mul(src, 1.0, out=dst), reps, 2)
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def trace_kernels(fn, reps):
    import torch
    import paper_2311_03096_amd as wsr
    torch.cuda.synchronize()
    wsr.wsr_trace_collect()
    wsr.wsr_trace_enable(True)
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    wsr.wsr_trace_enable(False)
    return wsr.wsr_trace_collect()


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE / WRITE_SIZE summary of this
    workload (calibrated against a plain copy kernel); None when there is none or the kernel
    sources changed since it was taken."""
    from paper_2311_03096_amd.prof_summary import read_traffic
    return read_traffic(os.path.join(ROOT, "profiles", "traffic_%s.md" % workload), workload, kernel)


def roofline(trace, n_el, steps, workload, sorts_per_step=1):
    """Dominant kernel by total time; achieved = algorithmic bytes per launch / mean duration.
    A radix scatter launch is charged its share of the sort's one round trip
    (SORT_ROUND_TRIP_B * n_el * sorts / scatter launches); ``achieved_per_pass`` gives the rate of
    that pass moving key + index once (16 B/el)."""
    name, (cnt, tot) = max(trace.items(), key=lambda kv: kv[1][1])
    avg_ms = tot / cnt
    if name == "radix_scatter":
        bpl = SORT_ROUND_TRIP_B * n_el * sorts_per_step * steps / cnt
    elif name in KERNEL_BYTES_PER_EL:
        bpl = KERNEL_BYTES_PER_EL[name] * n_el
    else:
        return dict(kernel=name, launches_per_step=cnt / steps, avg_ms=avg_ms, bound="hbm", achieved=None,
                    peak=HBM_PEAK_GBS, unit="GB/s", frac=None, traffic=None)
    ach = bpl / (avg_ms * 1e-3) / 1e9
    tr = measured_traffic(workload, name)
    res = dict(kernel=name, launches_per_step=cnt / steps, avg_ms=round(avg_ms, 5),
               bytes_per_el=round(bpl / n_el, 4), algorithmic_bytes_per_launch=bpl, bound="hbm",
               achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(ach / HBM_PEAK_GBS, 4),
               traffic=None if tr is None else round(tr))
    if name == "radix_scatter":
        per_pass = SORT_ROUND_TRIP_B * n_el / (avg_ms * 1e-3) / 1e9
        res["achieved_per_pass"] = round(per_pass, 1)
        res["frac_per_pass"] = round(per_pass / HBM_PEAK_GBS, 4)
    if tr is not None:
        res["traffic_unit"] = "HBM bytes per launch"
        res["traffic_over_algorithmic"] = round(tr / bpl, 3) if bpl else None
    return res


def median_ms(fn, reps=MED_REPS, warmup=MED_WARMUP):
    """Median over ``reps`` single-call timings (HIP events on the current stream, which the
    library's calls use) after ``warmup`` untimed calls."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in evs]))


def step_fraction(n_el, ms, bpe, copy_gbs):
    gbs = bpe * n_el / (ms * 1e-3) / 1e9
    return dict(bytes_per_el=bpe, GBps=round(gbs, 1), frac_peak=round(gbs / HBM_PEAK_GBS, 4),
                frac_copy=round(gbs / copy_gbs, 4) if copy_gbs else None)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


VALU_PEAK_WAVE_INSTR = 256 * 2.4e9  # one wave64 VALU instruction per clock per CU (4 SIMDs x 16 lanes)


def alu_roofline(kernel, avg_ms, workload):
    """The issue-rate bound of a kernel that is not HBM-bound: its VALU wave-instructions per
    launch (committed rocprofv3 counter summary, matched by kernel source hash) over its mean
    launch time, against one wave64 VALU instruction per clock per CU; the LDS instructions
    per launch are given beside it."""
    if not kernel or not avg_ms:
        return None
    from paper_2311_03096_amd import prof_summary as ps
    c = ps.read_counters(os.path.join(ROOT, "profiles", "counters_%s.md" % workload), workload, kernel)
    if c is None:
        return None
    achieved = c["valu"] / (avg_ms * 1e-3)
    return dict(kernel=kernel, bound="alu", unit="wave64 VALU instr/s", achieved=achieved,
                peak=VALU_PEAK_WAVE_INSTR, frac=round(achieved / VALU_PEAK_WAVE_INSTR, 4),
                valu_per_launch=c["valu"], lds_per_launch=c["lds"],
                valu_floor_ms=round(c["valu"] / VALU_PEAK_WAVE_INSTR * 1e3, 4))


def cpu_baseline(case, step=None):
    """Oracle forward + VJP over the whole workload on the host (one thread), on the same upstream
    gradient as the GPU step.  With ``step`` (the GPU step's buffers after the timed region) the
    oracle's last results also give the accuracy of the GPU results."""
    import oracle
    w, off, lam = case["w"], case["offsets"], case["lam"]
    g = np.random.default_rng(123).standard_normal(w.shape[0]).astype(np.float32).astype(np.float64)
    reps, t0 = 0, time.perf_counter()
    while True:  # whole steps until about 10 s of CPU work
        u, perm, start = oracle.prox_segments(w, lam, off, n_threads=1)
        vg = oracle.vjp(g, perm, start, off)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= 10.0:
            break
    res = dict(value=float(reps * w.shape[0] / dt), unit="elements/s", cores=1, kind="oracle",
               sample="%d full fwd+vjp steps of %s (%d elements each), FP64 sort + stack PAV, 1 thread, "
               "%.1f s" % (reps, case["name"], w.shape[0], dt), host_cpu=_cpu_model())
    acc = accuracy(case, step, u, perm, start, vg) if step is not None else None
    return res, acc


def accuracy(case, step, u, perm, start, vg=None):
    """Errors of a GPU step's results against the FP64 oracle's (u, perm, start, and the VJP vg):
    max abs and normwise relative error, the max elementwise relative error over |u| >= 1e-3 max|w|,
    |sum u - sum w|, cluster counts, permutation equality, and the backward's errors."""
    w = case["w"]
    out = step.out.cpu().numpy().astype(np.float64)
    words = step.mask.cpu().numpy().view(np.uint8)
    start_g = np.unpackbits(words, bitorder="little")[:w.shape[0]]
    scale = float(np.abs(w).max())
    err = np.abs(out - u)
    big = np.abs(u) >= 1e-3 * scale
    acc = dict(workload=case["name"], max_abs_err=float(err.max()), max_rel_err=float(err.max() / scale),
               max_elementwise_rel_err_large=float((err[big] / np.abs(u[big])).max()) if big.any() else 0.0,
               abs_sum_diff=float(abs(out.sum() - w.astype(np.float64).sum())),
               clusters_gpu=int(start_g.sum()), clusters_oracle=int(start.sum()),
               permutation_equal=bool(np.array_equal(step.perm.cpu().numpy(), perm)),
               cluster_starts_differing=int((start_g != start).sum()))
    if vg is not None:
        gw = step.gw.cpu().numpy().astype(np.float64)
        gerr = np.abs(gw - vg)
        acc.update(grad_max_abs_err=float(gerr.max()),
                   grad_max_rel_err=float(gerr.max() / max(float(np.abs(vg).max()), 1e-30)))
    return acc


def config_line(name, case, copy_gbs, kind="fwd_bwd", batched=False, long_sort=False, oracle_check=False,
                cpu_threads=0, cpu_runs=5):
    """One row of the per-workload table: the median step time (>= 50 reps after >= 10 warm-ups),
    elements/s, the whole step's fraction of HBM peak under the algorithmic bytes (24.25 B/el for
    forward with saved state + backward, 12.125 B/el for the backward alone; plus the sort's
    16 B/el round trip for a segment too long for on-chip memory), and the dominant kernel with its
    own fraction.  ``oracle_check``: errors against the FP64 oracle; ``cpu_threads`` > 0: the
    oracle's forward + VJP timed on that many host threads (median of ``cpu_runs`` runs)."""
    import torch
    import oracle
    step = Step(case, batched=batched)
    n = step.n
    if kind == "bwd":  # the saved state of one forward, then the backward alone
        if batched:
            step.wsr.wsr_prox_forward_batched(step.plan, step.w, step.out, None, step.lam, step.perm, step.mask,
                                              step.ws)
            fn = lambda: step.wsr.wsr_prox_backward_batched(step.plan, step.g, step.gw, step.perm, step.mask,
                                                            step.ws)
        else:
            step.wsr.wsr_prox_forward(step.w, step.out, step.offsets, step.lam, step.perm, step.mask, step.ws)
            fn = lambda: step.wsr.wsr_prox_backward(step.g, step.gw, step.offsets, step.perm, step.mask, step.ws)
        bpe = 12.125
    else:
        fn = step
        bpe = 24.25
    ms = median_ms(fn)
    tr = trace_kernels(fn, 3)
    roof = roofline(tr, n, 3, name, sorts_per_step=1 if (long_sort and kind != "bwd") else 0)
    res = dict(workload=case["name"], elements=n, segments=int(case["offsets"].shape[0] - 1), lam=case["lam"],
               step=("backward" if kind == "bwd" else "forward with saved state + backward"),
               ms_median=round(ms, 5), elements_per_s=n / (ms * 1e-3),
               step_fraction=step_fraction(n, ms, bpe, copy_gbs), dominant_kernel=roof,
               kernel_ms_per_step={k: round(v[1] / 3, 4) for k, v in tr.items()})
    if long_sort and kind != "bwd":
        res["step_fraction_with_sort_round_trip"] = step_fraction(n, ms, bpe + SORT_ROUND_TRIP_B, copy_gbs)
    if kind == "bwd":
        res["ms_median_forward_and_backward"] = round(median_ms(step), 5)
    if oracle_check or cpu_threads:
        torch.cuda.synchronize()
        w, off, lam = case["w"], case["offsets"], case["lam"]
        g = step.g.cpu().numpy().astype(np.float64)
        nthr = cpu_threads or 1
        times = []
        for _ in range(cpu_runs if cpu_threads else 1):
            t0 = time.perf_counter()
            u, perm, start = oracle.prox_segments(w, lam, off, n_threads=nthr)
            vg = oracle.vjp(g, perm, start, off)
            times.append(time.perf_counter() - t0)
        if cpu_threads:
            t = float(np.median(times))
            what = ("median of %d fwd+vjp runs over the whole workload, %.3f s each" % (len(times), t)
                    if len(times) > 1 else "one fwd+vjp run over the whole workload, %.3f s" % t)
            res["cpu_oracle"] = dict(value=n / t, unit="elements/s", cores=nthr, kind="oracle", sample=what)
        if kind != "bwd":
            step()  # results of one whole step for the accuracy check
        torch.cuda.synchronize()
        res["accuracy"] = accuracy(case, step, u, perm, start, vg)
    return res


def fp32_prefix_control(case):
    """Negative control for the precision workload: cluster values formed from a plain sequential
    FP32 prefix sum of the sorted weights (the clusters are the FP32 tie groups here, so each
    value is S[b] - S[a] over its group, divided by its size, plus the group's mean velocity),
    against the same formula in FP64 -- the error the FP64 sums of the kernels avoid."""
    w = np.sort(case["w"])
    d = w.shape[0]
    lam = float(case["lam"])
    edges = np.concatenate([[0], np.nonzero(np.diff(w))[0] + 1, [d]])
    a, b = edges[:-1], edges[1:]
    S32 = np.concatenate([[np.float32(0)], np.cumsum(w, dtype=np.float32)])
    S64 = np.concatenate([[0.0], np.cumsum(w.astype(np.float64))])
    v = lam * (d - a - b) / (d - 1.0)  # mean velocity of ranks [a, b)
    u32 = (S32[b].astype(np.float64) - S32[a].astype(np.float64)) / (b - a) + v
    u64 = (S64[b] - S64[a]) / (b - a) + v
    return dict(what="cluster values of the FP32 tie groups from a sequential FP32 prefix sum vs FP64",
                groups=int(a.shape[0]), max_abs_err=float(np.abs(u32 - u64).max()),
                max_rel_err=float(np.abs(u32 - u64).max() / np.abs(w).max()))


def batched_vs_per_row(steps, warmup, per_row=True, rounds=None, cpu_threads=0):
    """MLP rows (8202 segments, 29.4M weights): fwd+bwd, graph-captured batched launches (plan
    autotuned once on these weights, outside the timed region) vs per-row launches of the plain
    entry points on the same stream.  Medians of >= 50 reps (10 for the per-row launches, which
    take ~0.2 s a step) after >= 10 warm-ups (2 per-row)."""
    import torch
    from paper_2311_03096_amd import workloads
    case = workloads.mlp_rows()
    n = case["w"].shape[0]
    b = Step(case, batched=True, autotune=True, rounds=rounds)
    p = Step(case, batched=False) if per_row else None
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b()
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b()
    ms_graph = median_ms(graph.replay, max(MED_REPS, steps), max(MED_WARMUP, warmup))
    ms_batched = median_ms(b, max(MED_REPS, steps), max(MED_WARMUP, warmup))
    ms_rows = median_ms(p, 10, 2) if per_row else float("nan")
    tr = trace_kernels(b, 3)
    roof = roofline({k: v for k, v in tr.items() if k.startswith("prox_fwd")}, n, 3, "mlp_rows")
    copy_gbs = copy_bandwidth()
    roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4) if roof.get("achieved") else None
    bwd = {k: v for k, v in tr.items() if k.startswith("prox_bwd")}
    roof_b = roofline(bwd, n, 3, "mlp_rows") if bwd else None
    res = dict(workload="mlp_rows 4096x3072 + 4096x4096 + 10x4096, per-row segments, lam=1e-3",
               fwd_kernel_alu_roofline=alu_roofline(roof.get("kernel"), roof.get("avg_ms"), "mlp_rows"),
               elements=n, ms_per_step_graph=round(ms_graph, 4), ms_per_step_batched=round(ms_batched, 4),
               ms_per_step_per_row=round(ms_rows, 4), elements_per_s_graph=n / (ms_graph * 1e-3),
               speedup_graph_vs_per_row=round(ms_rows / ms_graph, 2), fwd_kernel_roofline=roof,
               bwd_kernel_roofline=roof_b, copy_GBps=round(copy_gbs, 1),
               step_fraction_graph=step_fraction(n, ms_graph, 24.25, copy_gbs),
               kernel_ms_per_step={k: round(v[1] / 3, 4) for k, v in tr.items()},
               autotuned_merge_rounds=b.rounds, timing="median of >= 50 reps after >= 10 warm-ups")
    if cpu_threads:
        import oracle
        g = b.g.cpu().numpy().astype(np.float64)
        times = []
        for _ in range(5):
            t0 = time.perf_counter()
            u, perm, start = oracle.prox_segments(case["w"], case["lam"], case["offsets"], n_threads=cpu_threads)
            vg = oracle.vjp(g, perm, start, case["offsets"])
            times.append(time.perf_counter() - t0)
        t = float(np.median(times))
        res["cpu_oracle"] = dict(value=n / t, unit="elements/s", cores=cpu_threads, kind="oracle",
                                 sample="median of 5 fwd+vjp runs over the 8202 rows, rows split across "
                                        "threads, %.3f s each" % t)
        graph.replay()
        torch.cuda.synchronize()
        res["accuracy"] = accuracy(case, b, u, perm, start, vg)
    return res


def l1_figures(steps, warmup):
    """Alg. prox in full (l1 and rewinding lines, the update of a proximal-gradient step) next
    to the plain inference forward on the same inputs: MLP rows batched and graph-captured, and
    one N(0,1) vector of 2^24 weights."""
    import torch
    import paper_2311_03096_amd as wsr
    from paper_2311_03096_amd import workloads
    res = {}
    case = workloads.mlp_rows()
    off = case["offsets"]
    w = torch.from_numpy(case["w"]).cuda()
    out = torch.empty_like(w)
    plan = wsr.wsr_plan_create(off)
    try:
        nb = wsr.wsr_plan_workspace_bytes(plan)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
        beta, rho = 0.01, 0.98
        fns = dict(
            l1=lambda: wsr.wsr_prox_l1_forward_batched(plan, w, out, None, case["lam"], beta, rho, ws),
            plain=lambda: wsr.wsr_prox_forward_batched(plan, w, out, None, case["lam"], None, None, ws))
        ms = {}
        for k, fn in fns.items():
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                fn()
            torch.cuda.current_stream().wait_stream(s)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                fn()
            ms[k] = median_ms(g.replay)
        n = w.numel()
        res["mlp_rows"] = dict(workload="mlp_rows, lam=1e-3, beta=0.01, rho=0.98, batched + hipGraph, no saved state",
                               ms_l1=round(ms["l1"], 4), ms_plain_forward=round(ms["plain"], 4),
                               elements_per_s_l1=n / (ms["l1"] * 1e-3))
        # one proximal-gradient step of every row (out of place, so every timed step sees the
        # same weights): gradient step fused into the prox kernels' loads
        grad = torch.from_numpy(np.random.default_rng(7).standard_normal(n).astype(np.float32)).cuda()
        fn = lambda: wsr.wsr_prox_step_batched(plan, w, grad, 0.1, out, None, 1e-2, 0.1, 0.98, 0, ws)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            fn()
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        ms_step = median_ms(g.replay)
        res["mlp_rows_step"] = dict(
            workload="mlp_rows: w <- Prox(w - 0.1 grad), alpha=1e-2, beta=0.1, rho=0.98, batched + hipGraph",
            ms=round(ms_step, 4), elements_per_s=n / (ms_step * 1e-3),
            hbm_frac_12B=round(12.0 * n / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
    finally:
        wsr.wsr_plan_destroy(plan)
    d = 1 << 24
    case = workloads.plain(d, 0.1, seed=1)
    off = case["offsets"]
    w = torch.from_numpy(case["w"]).cuda()
    out = torch.empty_like(w)
    nb = wsr.wsr_workspace_bytes(off)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    ms_l1 = median_ms(lambda: wsr.wsr_prox_l1_forward(w, out, off, case["lam"], 0.5, 0.98, ws))
    ms_pl = median_ms(lambda: wsr.wsr_prox_forward(w, out, off, case["lam"], None, None, ws))
    res["typical_d2p24"] = dict(workload="one N(0,1) vector d=2^24, lam=0.1, beta=0.5, rho=0.98",
                                ms_l1=round(ms_l1, 4), ms_plain_forward=round(ms_pl, 4),
                                elements_per_s_l1=d / (ms_l1 * 1e-3))
    return res


def stats_figures(steps, warmup):
    """Per-segment R(w) and the weight-sharing counts: MLP rows batched, one 2^24 vector."""
    import torch
    import paper_2311_03096_amd as wsr
    from paper_2311_03096_amd import workloads
    res = {}
    case = workloads.mlp_rows()
    off = case["offsets"]
    w = torch.from_numpy(case["w"]).cuda()
    st = torch.empty((off.shape[0] - 1, 3), dtype=torch.int64, device="cuda")
    plan = wsr.wsr_plan_create(off)
    try:
        nb = wsr.wsr_plan_workspace_bytes(plan)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
        ms = median_ms(lambda: wsr.wsr_segment_stats_batched(plan, w, st, ws))
    finally:
        wsr.wsr_plan_destroy(plan)
    res["mlp_rows"] = dict(workload="R(w) and counts of each of the 8202 MLP rows, batched", ms=round(ms, 4),
                           elements_per_s=w.numel() / (ms * 1e-3))
    d = 1 << 24
    case = workloads.plain(d, 0.1, seed=1)
    off = case["offsets"]
    w = torch.from_numpy(case["w"]).cuda()
    st = torch.empty((1, 3), dtype=torch.int64, device="cuda")
    ws = torch.empty(wsr.wsr_workspace_bytes(off), dtype=torch.uint8, device="cuda")
    ms = median_ms(lambda: wsr.wsr_segment_stats(w, off, st, ws))
    res["typical_d2p24"] = dict(workload="R(w) and counts of one N(0,1) vector d=2^24", ms=round(ms, 4),
                                elements_per_s=d / (ms * 1e-3))
    return res


def lds_probe_figures():
    """LDS throughput on this device (the bound of the short-segment kernels next to VALU):
    conflict-free 4-byte reads, random 4-byte reads, random 4-byte atomics, from the probes of
    libwsr_probe.so (measurement only)."""
    import ctypes
    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2311_03096_amd", "libwsr_probe.so"))
    lib.wsr_lds_probe.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.wsr_lds_probe_shape.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    nt, nw = ctypes.c_int(), ctypes.c_int()
    lib.wsr_lds_probe_shape(ctypes.byref(nt), ctypes.byref(nw))
    blocks, rounds = 4 * 256, 512  # 8 accesses per lane per round
    out = torch.zeros(blocks, dtype=torch.int32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    res = dict(workgroups=blocks, threads=nt.value, accesses_per_thread=rounds * 8)
    for kind, name, nbytes in ((0, "read4_conflict_free", 4), (1, "read4_random", 4), (2, "atomic4_random", 4)):
        fn = lambda: lib.wsr_lds_probe(kind, rounds, blocks, ctypes.c_void_p(out.data_ptr()), stream)
        assert fn() == 0
        ms = time_steps(fn, 5, 1)[0]
        accesses = blocks * nt.value * rounds * 8
        res[name] = dict(ms=round(ms, 4), G_accesses_per_s=round(accesses / (ms * 1e-3) / 1e9, 1),
                         TBps=round(accesses * nbytes / (ms * 1e-3) / 1e12, 2),
                         bytes_per_clk_per_cu=round(accesses * nbytes / (ms * 1e-3) / 256 / 2.4e9, 1))
    return res


def merge_route_figures(steps, warmup):
    """The merge routes side by side (inference forward, batched): ImminentCollisions rounds with
    the hull merge as fallback (default), the hull merge alone, EndCollisions (short segments),
    and the autotuned choice, on training-like rows, on rows of the collision worst case, and on
    one long N(0,1) vector."""
    import torch
    import paper_2311_03096_amd as wsr
    from paper_2311_03096_amd import workloads
    res = {}
    cases = [("mlp_rows", workloads.mlp_rows()), ("ica_worst_rows_1024x4095", workloads.ica_worst_rows(1024, 4095)),
             ("typical_d2p24", workloads.plain(1 << 24, 0.1, seed=1))]
    for name, case in cases:
        off = case["offsets"]
        w = torch.from_numpy(case["w"]).cuda()
        out = torch.empty_like(w)
        row = {}
        for route in ("default", "hull_only", "end_collisions", "autotuned"):
            if route == "end_collisions" and name.startswith("typical"):
                continue  # one long segment: EndCollisions is a short-segment route
            flags = {"hull_only": wsr.WSR_PLAN_MERGE_HULL, "end_collisions": wsr.WSR_PLAN_MERGE_END}.get(route, 0)
            plan = wsr.wsr_plan_create(off, flags)
            try:
                nb = wsr.wsr_plan_workspace_bytes(plan)
                ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
                if route == "autotuned":
                    wsr.wsr_plan_autotune(plan, w, out, None, case["lam"], ws)
                    row["autotuned_rounds"] = wsr.wsr_plan_merge_rounds(plan)
                    row["autotuned_sort"] = wsr.wsr_plan_sort_routes(plan)
                fn = lambda: wsr.wsr_prox_forward_batched(plan, w, out, None, case["lam"], None, None, ws)
                reps = 5 if route == "end_collisions" and name == "mlp_rows" else MED_REPS  # ~0.1 s a call
                row["ms_" + route] = round(median_ms(fn, reps, 2 if reps < MED_REPS else MED_WARMUP), 4)
            finally:
                wsr.wsr_plan_destroy(plan)
        res[name] = row
    return res


def quantised_rows(w):
    """The MLP rows' weights rounded to 1/64 of their scale (1/sqrt(3072))."""
    scale = np.sqrt(3072.0) * 64.0
    return (np.round(w.astype(np.float64) * scale) / scale).astype(np.float32)


def sort_route_figures():
    """The short classes' sort routes side by side (inference forward, batched, default merge
    route): the bucket-rank sort (the radix sort when a bucket overflows), the radix sort alone,
    and the autotuned choice, on the MLP rows and on the same rows quantised to 1/64 of the
    weights' scale (a few hundred distinct values per row: many equal weights, as in weights that
    are already shared)."""
    import torch
    import paper_2311_03096_amd as wsr
    from paper_2311_03096_amd import workloads
    base = workloads.mlp_rows()
    quant = quantised_rows(base["w"])
    res = {}
    for name, w_np in (("mlp_rows", base["w"]), ("mlp_rows_quantised_1_64", quant)):
        w = torch.from_numpy(w_np).cuda()
        out = torch.empty_like(w)
        row = dict(distinct_values_first_row=int(np.unique(w_np[:3072]).shape[0]))
        for route in ("bucket", "radix", "autotuned"):
            plan = wsr.wsr_plan_create(base["offsets"])
            try:
                nb = wsr.wsr_plan_workspace_bytes(plan)
                ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
                if route == "autotuned":
                    wsr.wsr_plan_autotune(plan, w, out, None, base["lam"], ws)
                    row["autotuned_sort"] = wsr.wsr_plan_sort_routes(plan)
                    row["autotuned_rounds"] = wsr.wsr_plan_merge_rounds(plan)
                else:
                    wsr.wsr_plan_set_sort_routes(plan, [wsr.WSR_SORT_RADIX if route == "radix" else wsr.WSR_SORT_BUCKET] * 3)
                fn = lambda: wsr.wsr_prox_forward_batched(plan, w, out, None, base["lam"], None, None, ws)
                row["ms_" + route] = round(median_ms(fn), 4)
            finally:
                wsr.wsr_plan_destroy(plan)
        res[name] = row
    return res


PHASES = ("load_and_key", "sort", "prefix_sums", "collisions_and_values", "stores")
BWD_PHASES = ("load_and_stage", "gather_and_scan", "cluster_values", "stores")


def phase_summary(t, names, tick_us, cus):
    """Per-phase mean / median duration and share of the workgroups' lifetimes, the launch span
    and the resident workgroups per CU (mean and maximum) from one launch's timestamps
    (t[workgroup, mark], ticks; workgroups that did not reach the last mark are left out)."""
    k = len(names) + 1
    t = t[:, :k]
    t = t[t[:, -1] > 0] * tick_us
    dur = np.diff(t, axis=1)
    life = t[:, -1] - t[:, 0]
    span = t[:, -1].max() - t[:, 0].min()
    ev = np.concatenate([np.stack([t[:, 0], np.ones(len(t))], 1), np.stack([t[:, -1], -np.ones(len(t))], 1)])
    ev = ev[np.lexsort((ev[:, 1], ev[:, 0]))]  # at equal times, ends before starts
    row = dict(span_us=round(float(span), 1), workgroup_us_mean=round(float(life.mean()), 2),
               in_flight_per_cu=round(float(life.sum() / span / cus), 2),
               in_flight_max_per_cu=round(float(np.cumsum(ev[:, 1]).max() / cus), 2))
    for i, ph in enumerate(names):
        row[ph] = dict(us_mean=round(float(dur[:, i].mean()), 2), us_median=round(float(np.median(dur[:, i])), 2),
                       share=round(float(dur[:, i].sum() / life.sum()), 3))
    return row


def phase_clock_figures():
    """Where the short-segment kernels spend their time: the measurement build libwsr_phases.so
    (the same kernels, with one thread of each workgroup reading the device wall clock after the
    barrier that closes each phase) on the MLP rows and on the same rows quantised to 1/64: the
    forward under both sort routes, and the backward (inference forward / backward, batched,
    default merge route).  Per phase: the mean and median over workgroups of its duration and its
    share of a workgroup's lifetime; per launch: the span from the first start to the last end
    and the mean and maximum number of workgroups resident per CU; and the launch time of the
    regular build next to the timestamped one."""
    import ctypes
    import torch
    from paper_2311_03096_amd import workloads
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2311_03096_amd", "libwsr_phases.so"))
    p, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.wsr_plan_create.argtypes = [p, i64, ctypes.c_int, ctypes.POINTER(p)]
    lib.wsr_plan_destroy.argtypes = [p]
    lib.wsr_plan_set_sort_routes.argtypes = [p, p]
    lib.wsr_prox_forward_batched.argtypes = [p, p, p, p, ctypes.c_float, p, p, p, ctypes.c_size_t, p]
    lib.wsr_prox_backward_batched.argtypes = [p, p, p, p, p, p, ctypes.c_size_t, p]
    lib.wsr_phase_clock_buffer.argtypes = [p, i64]
    lib.wsr_phase_clock_rate_khz.argtypes = [ctypes.POINTER(ctypes.c_int)]
    lib.wsr_phase_occupancy.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    slots = lib.wsr_phase_clock_slots()
    occ = ctypes.c_int()
    if lib.wsr_phase_occupancy(1, ctypes.byref(occ)) != 0:
        raise RuntimeError("wsr_phase_occupancy failed")
    khz = ctypes.c_int()
    if lib.wsr_phase_clock_rate_khz(ctypes.byref(khz)) != 0 or khz.value <= 0:
        raise RuntimeError("no wall-clock rate")
    tick_us = 1e3 / khz.value
    base = workloads.mlp_rows()
    off = np.ascontiguousarray(base["offsets"], dtype=np.int64)
    nseg = off.shape[0] - 1
    clocks = torch.zeros(nseg * slots, dtype=torch.int64, device="cuda")
    stream = p(torch.cuda.current_stream().cuda_stream)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    res = dict(workload="mlp_rows, lam=1e-3, batched", workgroups=nseg, clock_mhz=khz.value / 1e3,
               occupancy_limit_per_cu=occ.value)

    def check(rc, what):
        if rc != 0:
            raise RuntimeError("%s: %d" % (what, rc))

    def timed(fn):
        """(ms of the regular launch, ms with timestamps, the last launch's timestamps)."""
        lib.wsr_phase_clock_buffer(None, 0)
        ms_plain = median_ms(fn, 20, 5)
        clocks.zero_()
        check(lib.wsr_phase_clock_buffer(p(clocks.data_ptr()), nseg), "wsr_phase_clock_buffer")
        ms_clocked = median_ms(fn, 20, 5)  # the last call's timestamps stay in the buffer
        torch.cuda.synchronize()
        lib.wsr_phase_clock_buffer(None, 0)
        t = clocks.view(nseg, slots).cpu().numpy().astype(np.float64)
        return ms_plain, ms_clocked, t

    g = torch.from_numpy(np.random.default_rng(3).standard_normal(off[-1]).astype(np.float32)).cuda()
    gw = torch.empty_like(g)
    perm = torch.empty(off[-1], dtype=torch.int32, device="cuda")
    mask = torch.empty((int(off[-1]) + 31) // 32 + 1, dtype=torch.int32, device="cuda")
    for name, w_np in (("mlp_rows", base["w"]), ("mlp_rows_quantised_1_64", quantised_rows(base["w"]))):
        w = torch.from_numpy(w_np).cuda()
        out = torch.empty_like(w)
        for route, rname in ((0, "bucket"), (1, "radix")):
            plan = p()
            check(lib.wsr_plan_create(off.ctypes.data, nseg, 0, ctypes.byref(plan)), "wsr_plan_create")
            try:
                check(lib.wsr_plan_set_sort_routes(plan, (ctypes.c_int32 * 3)(route, route, route)),
                      "wsr_plan_set_sort_routes")
                fwd = lambda: check(lib.wsr_prox_forward_batched(plan, p(w.data_ptr()), p(out.data_ptr()), None,
                                                                 base["lam"], None, None, None, 0, stream), "forward")
                ms_plain, ms_clocked, t = timed(fwd)
                row = dict(ms_regular_build=round(ms_plain, 4), ms_timestamped=round(ms_clocked, 4))
                row.update(phase_summary(t, PHASES, tick_us, cus))
                res[name + "_" + rname] = row
                if name == "mlp_rows" and route == 0:  # the backward on this forward's saved state
                    check(lib.wsr_prox_forward_batched(plan, p(w.data_ptr()), p(out.data_ptr()), None, base["lam"],
                                                       p(perm.data_ptr()), p(mask.data_ptr()), None, 0, stream),
                          "forward with saved state")
                    bwd = lambda: check(lib.wsr_prox_backward_batched(plan, p(g.data_ptr()), p(gw.data_ptr()),
                                                                      p(perm.data_ptr()), p(mask.data_ptr()), None, 0,
                                                                      stream), "backward")
                    ms_plain, ms_clocked, t = timed(bwd)
                    row = dict(ms_regular_build=round(ms_plain, 4), ms_timestamped=round(ms_clocked, 4))
                    row.update(phase_summary(t, BWD_PHASES, tick_us, cus))
                    res["mlp_rows_backward"] = row
            finally:
                lib.wsr_plan_destroy(plan)
    return res


def merge_clock_figures():
    """The tile merge tree of one long segment (d = 2^24: 4096 hull tiles, 12 levels in three
    launches of 4), timed inside the kernels by the measurement build libwsr_phases.so, on the
    chain and on N(0,1) weights: per launch and level the span to the level's end, the longest
    bridge search among its merges, the mean time per level spent before the searches (junction
    windows) and after them (range updates and prefix rebuild), and the end of the launch's
    work (the last launch also writes references to every tile's neighbouring surviving vertices)."""
    import ctypes
    import torch
    from paper_2311_03096_amd import workloads
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2311_03096_amd", "libwsr_phases.so"))
    p, i64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
    lib.wsr_prox_forward.argtypes = [p, p, p, i64, ctypes.c_float, p, p, p, sz, p]
    lib.wsr_workspace_bytes.argtypes = [p, i64, ctypes.POINTER(sz)]
    lib.wsr_phase_merge_clock_buffer.argtypes = [p]
    lib.wsr_phase_clock_rate_khz.argtypes = [ctypes.POINTER(ctypes.c_int)]
    khz = ctypes.c_int()
    if lib.wsr_phase_clock_rate_khz(ctypes.byref(khz)) != 0 or khz.value <= 0:
        raise RuntimeError("no wall-clock rate")
    tick_us = 1e3 / khz.value
    nl, ng, ns = 4, 4096, 16  # launches, workgroups, words per workgroup (the build's layout)
    clk = torch.zeros(nl * ng * ns, dtype=torch.int64, device="cuda")
    res = {}
    for name, case in (("chain_d2p24", workloads.chain(1 << 24, 0.7)),
                       ("typical_d2p24", workloads.plain(1 << 24, 0.1, seed=1))):
        off = np.ascontiguousarray(case["offsets"], dtype=np.int64)
        n = off.shape[0] - 1
        nb = sz()
        if lib.wsr_workspace_bytes(off.ctypes.data, n, ctypes.byref(nb)) != 0:
            raise RuntimeError("wsr_workspace_bytes failed")
        ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        w = torch.from_numpy(case["w"]).cuda()
        out = torch.empty_like(w)
        stream = p(torch.cuda.current_stream().cuda_stream)

        def fwd():
            rc = lib.wsr_prox_forward(p(w.data_ptr()), p(out.data_ptr()), off.ctypes.data, n, float(case["lam"]),
                                      None, None, p(ws.data_ptr()), nb.value, stream)
            if rc != 0:
                raise RuntimeError("wsr_prox_forward: %d" % rc)
        for _ in range(3):
            fwd()
        clk.zero_()
        if lib.wsr_phase_merge_clock_buffer(p(clk.data_ptr())) != 0:
            raise RuntimeError("wsr_phase_merge_clock_buffer failed")
        try:
            fwd()
            torch.cuda.synchronize()
        finally:
            lib.wsr_phase_merge_clock_buffer(None)
        t = clk.view(nl, ng, ns).cpu().numpy().astype(np.float64)
        row = {}
        for li in range(nl):
            a = t[li]
            a = a[a[:, 0] > 0]
            if len(a) == 0:
                continue
            t0 = a[:, 0].min()
            lv = []
            for l in range(4):
                if not (a[:, 1 + l] > 0).any():
                    break
                lv.append(dict(end_us=round(float((a[:, 1 + l].max() - t0) * tick_us), 2),
                               bridge_max_us=round(float(a[:, 5 + l].max() * tick_us), 2)))
            row["launch%d" % li] = dict(workgroups=len(a), levels=lv,
                                        before_searches_us_per_level=round(float(a[:, 15].mean() * tick_us / len(lv)), 2),
                                        after_searches_us_per_level=round(float(a[:, 14].mean() * tick_us / len(lv)), 2),
                                        end_of_work_us=round(float((a[:, 13].max() - t0) * tick_us), 2))
        res[name] = row
        del ws, w, out
        torch.cuda.empty_cache()
    return res


def nproc():
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


def config_table(copy_gbs):
    """The per-workload rows (single-GPU workloads of the benchmark configurations and the
    variants that exercise the sort): median timings, fractions, dominant kernels, errors."""
    from paper_2311_03096_amd import workloads
    d = 1 << 24
    rows = {}
    rows["plain_d4096"] = config_line("plain_d4096", workloads.plain(4096, 0.1), copy_gbs, oracle_check=True,
                                      cpu_threads=1)
    log("plain d=4096", rows["plain_d4096"])
    rows["chain_d2p24_shuffled"] = config_line("chain_d2p24_shuffled", workloads.chain(d, 0.7, shuffle=True),
                                               copy_gbs, long_sort=True)
    log("shuffled chain", rows["chain_d2p24_shuffled"])
    rows["typical_d2p24"] = config_line("typical_d2p24", workloads.plain(d, 0.1, seed=1), copy_gbs, long_sort=True)
    log("typical", rows["typical_d2p24"])
    rows["backward_rows_1024x8192"] = config_line("backward_rows_1024x8192",
                                                  workloads.backward_rows(1024, 8192, 0.05), copy_gbs, kind="bwd",
                                                  batched=True, oracle_check=True, cpu_threads=nproc())
    log("backward rows", rows["backward_rows_1024x8192"])
    prec = workloads.precision(1 << 26, 1e-4)
    rows["precision_d2p26"] = config_line("precision_d2p26", prec, copy_gbs, long_sort=True, oracle_check=True,
                                          cpu_threads=1, cpu_runs=1)  # ~10 s a run
    rows["precision_d2p26"]["fp32_prefix_sum_control"] = fp32_prefix_control(prec)
    log("precision", rows["precision_d2p26"])
    return rows


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the prox path here is single-GPU (segments would "
              "shard across GPUs with no exchange); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2311_03096_amd as wsr
    from paper_2311_03096_amd import workloads
    wsr.load()  # fails loudly when the HIP library is missing
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calib > 0:
        n = args.copy_calib // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)  # one elementwise kernel: reads 4n bytes, writes 4n bytes
        torch.cuda.synchronize()
        log("copy calibration kernel: %d bytes read, %d bytes written" % (4 * n, 4 * n))
        del src, dst

    d = 1 << 24
    if args.workload == "mlp":
        rounds = [int(x) for x in args.rounds.split(",")] if args.rounds else None
        res = batched_vs_per_row(max(5, args.steps), args.warmup, per_row=not args.no_extra, rounds=rounds)
        print(json.dumps(res), flush=True)
        return
    if args.workload in ("shuffled", "backward", "precision"):  # one workload's row (for profiling)
        copy_gbs = copy_bandwidth()
        if args.workload == "shuffled":
            res = config_line("chain_d2p24_shuffled", workloads.chain(d, 0.7, shuffle=True), copy_gbs, long_sort=True)
        elif args.workload == "backward":
            res = config_line("backward_rows_1024x8192", workloads.backward_rows(1024, 8192, 0.05), copy_gbs,
                              kind="bwd", batched=True)
        else:
            res = config_line("precision_d2p26", workloads.precision(1 << 26, 1e-4), copy_gbs, long_sort=True)
        print(json.dumps(res), flush=True)
        return
    case = workloads.chain(d, 0.7) if args.workload == "chain" else workloads.plain(d, 0.1, seed=1)
    log("workload", case["name"], "steps", args.steps, "warmup", args.warmup)
    step = Step(case)
    ms, wall = time_steps(step, args.steps, args.warmup)
    tr = trace_kernels(step, 3)
    roof = roofline(tr, d, 3, {"chain": "chain_d2p24", "typical": "typical_d2p24"}[args.workload])
    log("ms/step", ms, "trace", tr)
    copy_gbs = copy_bandwidth()
    roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4) if roof.get("achieved") else None
    extra = dict(kernel_ms_per_step={k: round(v[1] / 3, 4) for k, v in tr.items()},
                 wall_ms_per_step=round(wall, 4), copy_GBps=round(copy_gbs, 1),
                 step_fraction=step_fraction(d, ms, 24.25, copy_gbs),
                 step_fraction_with_sort_round_trip=step_fraction(d, ms, 24.25 + SORT_ROUND_TRIP_B, copy_gbs),
                 ms_median=round(median_ms(step), 5))
    if not args.no_extra:
        extra["configs"] = config_table(copy_gbs)
        extra["batched_mlp_rows"] = batched_vs_per_row(max(5, args.steps), args.warmup, cpu_threads=nproc())
        log("batched", extra["batched_mlp_rows"])
        extra["prox_l1_rewinding"] = l1_figures(max(5, args.steps), args.warmup)
        log("l1", extra["prox_l1_rewinding"])
        extra["segment_stats"] = stats_figures(max(5, args.steps), args.warmup)
        log("stats", extra["segment_stats"])
        try:  # a measurement aside: its absence must not cost the bench line
            extra["lds_probe"] = lds_probe_figures()
        except Exception as e:  # noqa: BLE001
            extra["lds_probe"] = dict(error=str(e))
        log("lds probe", extra["lds_probe"])
        extra["merge_routes"] = merge_route_figures(max(5, args.steps), args.warmup)
        log("merge routes", extra["merge_routes"])
        extra["sort_routes"] = sort_route_figures()
        log("sort routes", extra["sort_routes"])
        try:
            extra["phase_clocks"] = phase_clock_figures()
        except Exception as e:  # noqa: BLE001
            extra["phase_clocks"] = dict(error=str(e))
        log("phase clocks", extra["phase_clocks"])
        try:
            extra["merge_clocks"] = merge_clock_figures()
        except Exception as e:  # noqa: BLE001
            extra["merge_clocks"] = dict(error=str(e))
        log("merge clocks", extra["merge_clocks"])
        lay = workloads.mlp_layers()
        st = Step(lay, batched=True)
        ms_l = median_ms(st)
        extra["mlp_per_layer"] = dict(workload="the MLP's weights, one segment per layer (12.6M, 16.8M, 41K), "
                                      "lam=1e-3, fwd+bwd, batched", ms_median=round(ms_l, 4),
                                      elements_per_s=lay["w"].shape[0] / (ms_l * 1e-3),
                                      step_fraction=step_fraction(lay["w"].shape[0], ms_l, 24.25, copy_gbs))
        log("per-layer", extra["mlp_per_layer"])
    res = dict(metric=METRIC, value=d / (ms * 1e-3), unit="elements/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(ms, 4), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload=WORKLOAD_TEXT[args.workload], d=d, lam=float(case["lam"]),
                           parallelism="single GPU"),
               roofline=roof)
    if not args.no_cpu:
        res["cpu_baseline"], res["accuracy"] = cpu_baseline(case, step)
        log("cpu", res["cpu_baseline"], res["accuracy"])
    res["extra"] = extra
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
