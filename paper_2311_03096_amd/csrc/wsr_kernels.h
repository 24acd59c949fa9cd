// wsr_kernels.h -- kernel entry points and launch descriptors shared by the host code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wsr {

// ImminentCollisions rounds tried before the hull merge by default (typical weights converge
// in 2-4 rounds).
constexpr int kIcaRounds = 6;
// SegArgs::merge_rounds value selecting the EndCollisions route (short segments only).
constexpr int kRouteEnd = -2;

// Which segment a workgroup of the short-segment kernels solves.  Batched launches give a
// schedule (sched[blockIdx.x] = segment id) over device offsets; single-segment launches give
// (start, d) directly.  lambda comes from lam_arr[segment] when lam_arr != nullptr.
// l1 = 1: the forward applies Alg. prox's l1 and rewinding lines (beta, rho, rewinding-line
// scale kappa) to every cluster.  grad != nullptr: the forward's input is the gradient step
// fmaf(-eta, grad, w), and the segment's lambda is multiplied by lam_mul (FP32).
struct SegArgs {
  const int64_t* offsets;
  const int32_t* sched;
  const float* lam_arr;
  float lam_scalar;
  int64_t start;
  int d;
  int seg_id;
  float beta = 0.0f;
  float rho = 0.0f;
  int l1 = 0;
  float kappa = 1.0f;
  const float* grad = nullptr;
  float eta = 0.0f;
  float lam_mul = 1.0f;
  int merge_rounds = -1;  // cap on ImminentCollisions rounds before the hull merge (-1: default,
                          // 0: hull merge only), or kRouteEnd: EndCollisions
  uint32_t* status = nullptr;  // sticky status word: bit 0 is OR-ed in for a non-finite segment
  int sort_route = 0;  // kSortBucket: bucket-rank sort (the radix sort when a bucket overflows),
                       // kSortRadix: the LDS radix sort only
#ifdef WSR_PHASE_CLOCKS
  unsigned long long* clocks = nullptr;  // phase timestamps (measurement build only, see below)
#endif
};

// Measurement build (WSR_PHASE_CLOCKS): thread 0 of each workgroup of the short-segment forward
// records the device wall clock right after the barrier that closes each phase, at
// clocks[block * kPhaseSlots + mark]: 0 start, 1 weights loaded and keyed, 2 sorted, 3 prefix
// sums, 4 collisions and cluster values, 5 stores issued; the backward: 0 start, 1 cotangent,
// perm and mask staged, 2 gathered and scanned, 3 cluster values, 4 stores issued.  The regular
// build has no such code.
constexpr int kPhaseSlots = 8;
#ifdef WSR_PHASE_CLOCKS
#define WSR_PHASE_MARK(args, m)                                                              \
  do {                                                                                       \
    if (threadIdx.x == 0 && (args).clocks)                                                   \
      (args).clocks[(int64_t)blockIdx.x * kPhaseSlots + (m)] = wall_clock64();               \
  } while (0)
#else
#define WSR_PHASE_MARK(args, m) \
  do {                          \
  } while (0)
#endif

// Sort routes of the short-segment kernels.
constexpr int kSortBucket = 0;
constexpr int kSortRadix = 1;

// Bits of the sticky status word of a plan.
constexpr uint32_t kStatusNonFinite = 1u;

// Per-segment statistics (layout of wsr_segment_stats_t): R(w), the number of distinct non-zero
// values and the number of non-zero weights.
struct SegStats {
  double penalty;
  long long distinct;
  long long nonzero;
};

template <int TMAX, int NT>
__global__ void k_seg_stats_small(SegArgs args, const float* w, SegStats* stats);
template <int TMAX, int NT, bool END>
__global__ void k_prox_fwd_small(SegArgs args, const float* w, float* out, int32_t* perm_out,
                                 uint32_t* mask_out);
template <int TMAX, int NT>
__global__ void k_prox_bwd_small(SegArgs args, const float* gin, float* gout, const int32_t* perm_in,
                                 const uint32_t* mask_in);
__global__ void k_zero_u32(uint32_t* p, int64_t n);

}  // namespace wsr
