"""MI355X (gfx950) library for the proximal map of the weight-sharing penalty
R(w) = 1/(d-1) sum_{i>j} |w_i - w_j|  ("Weight-Sharing Regularization", AISTATS 2024).

The C ABI (include/wsr.h, libwsr.so) does the work in hand-written HIP kernels; this package
is its ctypes binding (same names) plus torch wrappers for autograd and batched steps.
"""
from ._lib import (Plan, WSR_ERR_HIP, WSR_ERR_INVALID, WSR_ERR_UNSUPPORTED, WSR_ERR_WORKSPACE,
                   WSR_MAX_SEGMENT, WSR_OK, WSR_PLAN_MERGE_END, WSR_PLAN_MERGE_HULL, WsrError, load,
                   wsr_plan_autotune, wsr_plan_autotune_step, wsr_plan_create, wsr_plan_destroy, wsr_plan_merge_rounds,
                   wsr_plan_set_merge_rounds, wsr_plan_sort_routes, wsr_plan_set_sort_routes, WSR_SORT_BUCKET,
                   WSR_SORT_RADIX, wsr_read_status, WSR_STATUS_NONFINITE,
                   wsr_plan_workspace_bytes,
                   wsr_prox_backward, wsr_prox_backward_batched, wsr_prox_forward, wsr_prox_forward_noalloc,
                   WSR_NOALLOC_MAX_SEGMENT, WSR_NOALLOC_SCRATCH_BYTES,
                   wsr_prox_forward_batched, wsr_prox_l1_forward, wsr_prox_l1_forward_batched,
                   wsr_prox_step_batched, WSR_STEP_ETA_IN_DISPLACEMENT, wsr_segment_stats,
                   wsr_segment_stats_batched, stats_to_numpy,
                   wsr_status_string, wsr_trace_collect,
                   wsr_trace_enable, wsr_version, wsr_workspace_bytes)

__all__ = [
    "load", "WsrError", "wsr_version", "wsr_status_string", "wsr_workspace_bytes",
    "wsr_prox_forward", "wsr_prox_forward_noalloc", "WSR_NOALLOC_MAX_SEGMENT", "WSR_NOALLOC_SCRATCH_BYTES",
    "wsr_prox_backward", "wsr_plan_create", "wsr_plan_destroy",
    "wsr_plan_workspace_bytes", "wsr_prox_forward_batched", "wsr_prox_backward_batched",
    "wsr_prox_l1_forward", "wsr_prox_l1_forward_batched", "wsr_prox_step_batched",
    "WSR_STEP_ETA_IN_DISPLACEMENT", "wsr_segment_stats", "wsr_segment_stats_batched", "stats_to_numpy",
    "wsr_trace_enable", "wsr_trace_collect",
    "WSR_OK", "WSR_ERR_INVALID", "WSR_ERR_WORKSPACE", "WSR_ERR_HIP", "WSR_ERR_UNSUPPORTED",
    "WSR_PLAN_MERGE_HULL", "WSR_PLAN_MERGE_END", "WSR_MAX_SEGMENT", "wsr_plan_autotune", "wsr_plan_autotune_step",
    "wsr_plan_merge_rounds", "Plan",
    "wsr_plan_set_merge_rounds", "wsr_plan_sort_routes", "wsr_plan_set_sort_routes", "WSR_SORT_BUCKET",
    "WSR_SORT_RADIX", "wsr_read_status", "WSR_STATUS_NONFINITE",
]
