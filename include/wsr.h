/*
 * wsr.h -- C ABI of the MI355X (gfx950) library for the proximal map of the
 * weight-sharing penalty
 *
 *     R_d(w) = 1/(d-1) * sum_{i>j} |w_i - w_j|                (paper Sec. 1, eq. reg)
 *     prox_{lam R_d}(w) = argmin_u  lam*R_d(u) + 1/2 ||u - w||^2   (Sec. 1; App. A.1)
 *
 * computed as: sort -> rank-dependent shift -> cluster merging -> scatter back
 * (Alg. prox without its l1 lines; Sec. 3 particle model; Sec. 4 collision
 * algorithms).  lam is "step size x penalty" (eta * alpha in the proximal-gradient
 * update, Sec. 1 and App. A.1 eq. pgd).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - A flat FP32 buffer of N = offsets[n_seg] weights is split into n_seg segments
 *   [offsets[s], offsets[s+1]).  Each segment is an independent prox problem with its
 *   own normalisation 1/(d_s - 1) (the paper applies R per layer, App. E.1; rows of a
 *   weight matrix are just shorter segments).  offsets[0] must be 0, offsets must be
 *   non-decreasing, every segment must satisfy d_s <= WSR_MAX_SEGMENT.
 * - Device pointers are plain device addresses (hipMalloc / torch CUDA tensors) on
 *   the current HIP device; "stream" is a hipStream_t passed as void* (NULL = the
 *   null stream).  Every compute call only enqueues work on that stream, returns
 *   without synchronising (the exceptions, wsr_plan_autotune, wsr_read_status and
 *   wsr_trace_collect, say so), and allocates no memory: scratch comes from the caller's
 *   workspace "ws" of "ws_bytes" bytes (device memory, any contents, 256-byte
 *   aligned), sized with the matching *_workspace_bytes call.  Two calls that
 *   overlap in time on different streams must not share a workspace.
 * - Outputs may alias inputs only where stated.
 * - Saved state for the backward pass (both pointers NULL = inference, no save):
 *     saved_perm[N]  int32: at flat position offsets[s] + k, the segment-local index
 *                    of the weight with rank k in segment s (ascending order).
 *     saved_mask[ceil(N/32)] uint32: bit (p % 32) of word p / 32 is set iff flat
 *                    position p = offsets[s] + k starts a cluster (rank k is the first
 *                    rank of its group of equal outputs).
 *   The forward call overwrites every word of saved_mask.
 * - Semantics of special segments: d_s == 0 is skipped; d_s == 1 or lam == 0 gives
 *   the identity (every weight its own cluster); a segment holding a NaN or +-Inf
 *   weight gets NaN outputs (every weight its own cluster).  In these cases saved_perm
 *   holds some permutation of the segment.  A lambda read from device memory that is
 *   not > 0 (negative, zero or NaN) also gives the identity.
 * - Clusters are the coarsest partition: neighbouring ranks whose exact outputs
 *   are equal share a cluster (merge when avg_y(lower) >= avg_y(upper), Sec. 4.1).
 *   Results are deterministic: the same inputs give bit-identical outputs.
 *
 * Errors: argument errors are detected on the host before anything is enqueued and
 * return WSR_ERR_INVALID (bad pointer, size, offsets or lambda), WSR_ERR_WORKSPACE
 * (workspace too small) or WSR_ERR_UNSUPPORTED (segment longer than
 * WSR_MAX_SEGMENT).  A failing HIP launch returns WSR_ERR_HIP.  Calls never abort.
 */
#ifndef WSR_H
#define WSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define WSR_API __attribute__((visibility("default")))
#else
#define WSR_API
#endif

#define WSR_OK 0
#define WSR_ERR_INVALID (-1)
#define WSR_ERR_WORKSPACE (-2)
#define WSR_ERR_HIP (-3)
#define WSR_ERR_UNSUPPORTED (-4)

/* longest supported segment (elements): 2^27, above the paper's largest layers (~1e8 weights) */
#define WSR_MAX_SEGMENT ((int64_t)1 << 27)

/* Library version as 10000*major + 100*minor + patch. */
WSR_API int wsr_version(void);

/* Static description of a status code; never NULL. */
WSR_API const char* wsr_status_string(int status);

/*
 * Workspace bytes needed by wsr_prox_forward / wsr_prox_backward for these host
 * offsets (n_seg + 1 entries).  Segments short enough to be solved inside one
 * workgroup need none; longer ones need scratch for a device-wide sort and the
 * cross-tile cluster merge, sized for the longest segment (segments are processed
 * one after another).  Writes the size to *bytes.
 */
WSR_API int wsr_workspace_bytes(const int64_t* h_offsets, int64_t n_seg, size_t* bytes);

/*
 * Forward prox, one lambda for all segments (Alg. prox lines sort / shift /
 * collisions / repeat_interleave / scatter; l1 lines not applied).
 *   w[N]          device, input weights (flat, segment-major)
 *   out[N]        device, prox values in the original order; may alias w
 *   h_offsets     HOST array of n_seg + 1 int64 segment offsets
 *   lambda        prox scale, finite and >= 0
 *   saved_perm, saved_mask   device, both NULL (inference) or both non-NULL
 *   ws, ws_bytes  device workspace, >= wsr_workspace_bytes(h_offsets, n_seg)
 * Segments are launched one after another (one launch per short segment; this is
 * the per-row path that the batched entry point is compared against).
 */
WSR_API int wsr_prox_forward(const float* w, float* out, const int64_t* h_offsets, int64_t n_seg,
                     float lambda, int32_t* saved_perm, uint32_t* saved_mask, void* ws,
                     size_t ws_bytes, void* stream);

/*
 * wsr_prox_forward without a workspace argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Long
 * segments use a fixed scratch array of WSR_NOALLOC_SCRATCH_BYTES in device memory, one per GPU,
 * created with the library's code object and held until the process ends; the call itself
 * allocates nothing.  Limit: a segment whose workspace (wsr_workspace_bytes) exceeds the scratch
 * returns WSR_ERR_WORKSPACE before anything is enqueued; every segment of up to
 * WSR_NOALLOC_MAX_SEGMENT elements fits.  All calls on one GPU share its scratch: calls that
 * overlap in time on one GPU (other streams, other host threads) race and must be ordered by the
 * caller.  The scratch needs no clearing (every word the kernels read is written first in the
 * same call).  Arguments, results and errors otherwise as in wsr_prox_forward.
 */
#define WSR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
#define WSR_NOALLOC_MAX_SEGMENT ((int64_t)1 << 21)
WSR_API int wsr_prox_forward_noalloc(const float* w, float* out, const int64_t* h_offsets, int64_t n_seg,
                                     float lambda, int32_t* saved_perm, uint32_t* saved_mask, void* stream);

/*
 * Forward of Alg. prox in full: the proximal map of lambda*R_d + beta*l1 with rewinding rho
 * (Sec. 1, prox of the combined penalty; App. "combining weight-sharing and sparsity" for its
 * decomposition; Sec. "rewinding" and Alg. prox, l1 and rewinding lines).  The collisions are
 * those of wsr_prox_forward; then every cluster C = ranks [a, b) of prox_{lambda R} with value
 * u_C, mean weight x_C and mean velocity v_C = lambda (d - a - b)/(d - 1) (u_C = x_C + v_C) gets
 *     0                                          if |u_C| < beta
 *     x_C + (1 - rho) (v_C - beta sign(u_C))     otherwise,
 * decided and evaluated in FP64, rounded once to FP32.  rho = 0 gives prox_{lambda R + beta l1}
 * (soft-thresholding of prox_{lambda R}); beta = rho = 0 gives prox_{lambda R}; rho = 1 keeps
 * the mean weight of every surviving cluster.  Segments that wsr_prox_forward leaves unchanged
 * (d_s == 1, lambda == 0) get the elementwise rule with v = 0; non-finite segments get NaN.
 *   beta          finite, >= 0
 *   rho           in [0, 1]
 * Other arguments as in wsr_prox_forward.  No state is saved: this is the update of a
 * proximal-gradient step, not a differentiable layer.
 */
WSR_API int wsr_prox_l1_forward(const float* w, float* out, const int64_t* h_offsets, int64_t n_seg,
                                float lambda, float beta, float rho, void* ws, size_t ws_bytes,
                                void* stream);

/*
 * Backward of the prox: grad_w = J^T grad_out, where on the piece of the map picked
 * by the saved partition J averages within each cluster (J is symmetric and
 * idempotent).  Not in the paper: it follows from Alg. prox's repeat_interleave of
 * cluster averages, with the partition held fixed.
 *   grad_out[N]   device, upstream gradient (original order)
 *   grad_w[N]     device, result (original order); must not alias grad_out
 *   saved_perm, saved_mask   device, as written by the matching forward call
 */
WSR_API int wsr_prox_backward(const float* grad_out, float* grad_w, const int64_t* h_offsets,
                      int64_t n_seg, const int32_t* saved_perm, const uint32_t* saved_mask,
                      void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ batched */

typedef struct wsr_plan wsr_plan; /* opaque, owned by the library */

/*
 * Plan for a fixed segmentation: validates and uploads the offsets (one hipMalloc,
 * done here and never during compute calls), groups segments by size class and
 * records the launch schedule used by the batched calls, so that a whole optimizer
 * step of prox calls is a fixed sequence of launches (hipGraph-capturable).
 *   flags: 0, or WSR_PLAN_MERGE_HULL to merge clusters by the bounded-depth hull merge
 *   only (Sec. 4.3 search collisions on hulls), without the ImminentCollisions rounds
 *   (Sec. 4.1) that the default route tries first; results are identical, only the time
 *   differs (for comparing the two routes).
 * On success *plan receives a new plan; free it with wsr_plan_destroy (which returns
 * WSR_ERR_INVALID for a NULL plan).
 */
#define WSR_PLAN_MERGE_HULL 2
/* WSR_PLAN_MERGE_END: short segments merge by EndCollisions (Sec. 4.2, Alg. end_collisions: the
 * rightmost collision found by a block-wide reduction, one round per cluster: fast with few
 * clusters, slow with many); long segments keep the default route.  Not combinable with
 * WSR_PLAN_MERGE_HULL.  For comparing routes; results are identical. */
#define WSR_PLAN_MERGE_END 4
WSR_API int wsr_plan_create(const int64_t* h_offsets, int64_t n_seg, int flags, wsr_plan** plan);
WSR_API int wsr_plan_destroy(wsr_plan* plan);

/*
 * Autotuner: times the merge routes of every size class of the plan on the caller's weights
 * (the batched forward of that class alone, without saved state: a warm-up launch and three
 * timed ones per route) and keeps the fastest route of each class in the plan for every later
 * batched call; then, for each short class, the radix sort route against the bucket sort route
 * with that merge route (see wsr_plan_sort_routes).  Routes of the short classes: a cap of 0 (hull merge only), 2, 6, 16 or 64
 * ImminentCollisions rounds before the hull merge, and EndCollisions (Sec. 4.2) when a probe over
 * the class's first segments finds it no slower than 1.5x the default route there; long
 * segments: a cap of 0, 6 or 16, timed on the longest one.  Synchronises the stream; not for use
 * under graph capture.
 *   w[N]      device weights of the plan's layout; out[N] device scratch (overwritten), which must
 *             not alias w (WSR_ERR_INVALID)
 *   d_lambda, lambda_scalar, ws, ws_bytes, stream   as in wsr_prox_forward_batched
 */
WSR_API int wsr_plan_autotune(wsr_plan* plan, const float* w, float* out, const float* d_lambda,
                              float lambda_scalar, void* ws, size_t ws_bytes, void* stream);

/*
 * Autotuner for the proximal-gradient step: as wsr_plan_autotune, but each candidate route is
 * timed on the launches of wsr_prox_step_batched itself (gradient step fused into the load, the
 * lambda and l1 options of the chosen form), so the routes are chosen for the input the step's
 * collisions actually see, z = fmaf(-eta, grad, w), and its lambda (eta*alpha, or alpha in the
 * variant).  Arguments as in wsr_prox_step_batched; the result goes to scratch[N], which must
 * alias neither w nor grad (WSR_ERR_INVALID).  Synchronises the stream.
 */
WSR_API int wsr_plan_autotune_step(wsr_plan* plan, const float* w, const float* grad, float eta,
                                   float* scratch, const float* d_alpha, float alpha_scalar, float beta,
                                   float rho, int flags, void* ws, size_t ws_bytes, void* stream);

/* The plan's route per size class (2048, 4096, 8192, long): the cap on collision rounds before
 * the hull merge (0 = hull merge only), or -1 = EndCollisions.  Writes 4 values. */
WSR_API int wsr_plan_merge_rounds(const wsr_plan* plan, int32_t* rounds);

/* Sets the 4 routes (short classes -1..64, long 0..64), e.g. to reuse what wsr_plan_autotune
 * found in an earlier run without timing again.  Host only; WSR_ERR_INVALID for a value out of
 * range. */
WSR_API int wsr_plan_set_merge_rounds(wsr_plan* plan, const int32_t* rounds);

/*
 * Sort route per short size class (2048, 4096, 8192), the sort step of Alg. prox for segments
 * that fit one workgroup: WSR_SORT_BUCKET (default) sorts by value buckets and ranks inside each
 * bucket, taking the LDS radix sort only when a bucket overflows; WSR_SORT_RADIX takes the LDS
 * radix sort at once.  Both give the same sorted order (by value, then index), so results are
 * identical; the bucket sort is faster on spread-out weights, the radix sort on rows with many
 * equal weights (quantised or already shared).  wsr_plan_autotune and wsr_plan_autotune_step time
 * the radix route against the bucket route with each class's chosen merge route and keep the
 * faster.  wsr_plan_sort_routes writes 3 values; wsr_plan_set_sort_routes sets them (host only;
 * WSR_ERR_INVALID for another value).  The batched forward, l1 forward, step and statistics use
 * them; the per-segment entry points use the bucket route.
 */
#define WSR_SORT_BUCKET 0
#define WSR_SORT_RADIX 1
WSR_API int wsr_plan_sort_routes(const wsr_plan* plan, int32_t* routes);
WSR_API int wsr_plan_set_sort_routes(wsr_plan* plan, const int32_t* routes);

/*
 * Sticky status of a plan's batched calls (forward, l1 forward, step): bit WSR_STATUS_NONFINITE
 * is set on the device when any segment held a NaN or +-Inf input weight (that segment's
 * outputs are NaN, as documented above) and stays set until read with clear != 0.  Enqueues the
 * read (and the clear) on `stream` and synchronises that stream only: the word covers the calls
 * ordered before it on that stream (calls on other streams must have completed or be ordered
 * before it by events).  Writes the word to *flags.  Not for use under graph capture.
 */
#define WSR_STATUS_NONFINITE 1u
WSR_API int wsr_read_status(const wsr_plan* plan, uint32_t* flags, int clear, void* stream);

/* A plan may be used by calls on any stream, but calls that overlap in time must not share a
 * workspace; wsr_plan_autotune(_step), wsr_plan_set_merge_rounds and wsr_plan_set_sort_routes
 * change the plan and must not run while other calls with the same plan are being issued from
 * another host thread. */

/* Workspace bytes needed by the batched calls of this plan. */
WSR_API int wsr_plan_workspace_bytes(const wsr_plan* plan, size_t* bytes);

/*
 * Batched forward over every segment of the plan: all short segments in one launch
 * per size class, long segments through the device-wide path.
 *   d_lambda      device array of n_seg FP32 lambdas, or NULL to use lambda_scalar for
 *                 every segment (values are read by the kernels, so they may change
 *                 between replays of a captured graph)
 * Other arguments as in wsr_prox_forward.
 */
WSR_API int wsr_prox_forward_batched(const wsr_plan* plan, const float* w, float* out,
                             const float* d_lambda, float lambda_scalar, int32_t* saved_perm,
                             uint32_t* saved_mask, void* ws, size_t ws_bytes, void* stream);

/* Batched form of wsr_prox_l1_forward: lambdas as in wsr_prox_forward_batched, one beta and one
 * rho for every segment. */
WSR_API int wsr_prox_l1_forward_batched(const wsr_plan* plan, const float* w, float* out,
                                        const float* d_lambda, float lambda_scalar, float beta,
                                        float rho, void* ws, size_t ws_bytes, void* stream);

/*
 * One proximal-gradient step over every segment of the plan (Sec. 1 update of w with step size
 * eta and the prox of alpha*R + beta*l1; App. A.1 eq. pgd), with Alg. prox in full:
 *     z   = fmaf(-eta, grad, w)               elementwise, FP32, one rounding
 *     out = Alg. prox of z, per segment
 * flags = 0: the prox of eta*(alpha_s R + beta l1) with rewinding rho, i.e. wsr_prox_l1_forward
 *            with lambda = eta*alpha_s and beta' = eta*beta (both FP32 products);
 * flags = WSR_STEP_ETA_IN_DISPLACEMENT: the variant of the experiments appendix (MNIST on a
 *            torus) that multiplies the learning rate into the remaining displacement instead of
 *            into alpha and beta: collisions and the zero test use alpha_s and beta, and the
 *            rewinding line becomes x_C += eta (1 - rho) v_C.
 *   w[N], grad[N] device inputs;  out[N] device output, may alias w or grad (in-place update)
 *   eta           finite, >= 0
 *   d_alpha       device array of n_seg FP32 alphas, or NULL to use alpha_scalar everywhere
 *   beta, rho     as in wsr_prox_l1_forward
 * Short segments take the gradient step inside the prox kernel's load; long segments write z
 * to out first (one extra elementwise pass) and run the device-wide path in place.  No state
 * is saved.  Other arguments as in wsr_prox_forward_batched.
 */
#define WSR_STEP_ETA_IN_DISPLACEMENT 1
WSR_API int wsr_prox_step_batched(const wsr_plan* plan, const float* w, const float* grad, float eta,
                                  float* out, const float* d_alpha, float alpha_scalar, float beta,
                                  float rho, int flags, void* ws, size_t ws_bytes, void* stream);

/* Batched backward over every segment of the plan (see wsr_prox_backward). */
WSR_API int wsr_prox_backward_batched(const wsr_plan* plan, const float* grad_out, float* grad_w,
                              const int32_t* saved_perm, const uint32_t* saved_mask, void* ws,
                              size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ statistics */

/*
 * Per-segment statistics of a weight buffer, each from the segment's sorted order:
 *   penalty           R_d(w_s) = 1/(d-1) sum_k (2k - d + 1) x_k for the sorted x (App. B: R in
 *                     O(d log d); Sec. 1 eq. reg), FP64 (centred FP64 sums); 0 for d <= 1
 *   distinct_nonzero  number of distinct non-zero values   } the weight-sharing measure of the
 *   nonzero           number of non-zero weights           } CIFAR10 table is their ratio
 * -0 counts as zero.  A segment holding a NaN or +-Inf weight gets penalty NaN and counts -1;
 * an empty segment gets zeros.
 */
typedef struct {
  double penalty;
  int64_t distinct_nonzero;
  int64_t nonzero;
} wsr_segment_stats_t;

/*
 *   w[N]          device, weights (flat, segment-major)
 *   d_stats       device array of n_seg wsr_segment_stats_t, every entry written
 *   ws, ws_bytes  as for wsr_prox_forward (same size: wsr_workspace_bytes)
 * Segments are processed one after another (one launch per short segment).
 */
WSR_API int wsr_segment_stats(const float* w, const int64_t* h_offsets, int64_t n_seg,
                              wsr_segment_stats_t* d_stats, void* ws, size_t ws_bytes, void* stream);

/* Batched form over the plan's segments (one launch per size class; workspace as
 * wsr_plan_workspace_bytes). */
WSR_API int wsr_segment_stats_batched(const wsr_plan* plan, const float* w, wsr_segment_stats_t* d_stats,
                                      void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ tracing */

/*
 * Per-kernel timing for measurement (not used by the compute path itself).
 * wsr_trace_enable(1) creates a pool of HIP events (allocation: call it outside graph
 * capture); while enabled, every kernel the library launches is bracketed by two events
 * recorded on the stream it is launched on.  wsr_trace_enable(0) stops recording.
 * wsr_trace_collect synchronises the recorded events and writes, for up to max_entries
 * distinct kernel names, the name (NUL-terminated, at most 63 chars, in names[i*64]),
 * the number of launches and their summed duration in milliseconds; *n_out receives the
 * number of entries written.  Collecting clears the recorded launches.  Launches beyond the
 * pool size (4096 per collect) are not recorded.
 */
WSR_API int wsr_trace_enable(int on);
WSR_API int wsr_trace_collect(int max_entries, char* names, int64_t* counts, double* total_ms,
                              int* n_out);

#ifdef __cplusplus
}
#endif

#endif /* WSR_H */
