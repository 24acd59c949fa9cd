// wsr_lds_probe.hip -- LDS throughput probes for the roofline of the short-segment kernels
// (measurement only; not part of the prox path).  Each workgroup fills a 32 KB LDS buffer and
// then runs a fixed number of rounds of one access pattern:
//   kind 0: conflict-free 4-byte reads (lane-consecutive addresses),
//   kind 1: random 4-byte reads (a hashed word per lane, the pattern of the bucket-rank scans),
//   kind 2: random 4-byte LDS atomic adds (the pattern of the bucket counters).
// Every address stays inside the buffer (masked index); results are folded into one word per
// workgroup so the compiler keeps every access.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kProbeThreads = 512;
constexpr int kProbeWords = 8192;  // 32 KB of LDS per workgroup

__global__ __launch_bounds__(kProbeThreads) void k_lds_probe(int kind, int rounds, uint32_t* out) {
  __shared__ alignas(16) uint32_t buf[kProbeWords];
  const int tid = threadIdx.x;
  for (int i = tid; i < kProbeWords; i += kProbeThreads) buf[i] = (uint32_t)i * 2654435761u;
  __syncthreads();
  uint32_t acc = 0u;
  // each round issues 8 LDS accesses per lane at immediate offsets (64 words apart) from a
  // per-lane base, so the loop spends about one VALU instruction per access and LDS is the
  // limit; the base stays below kSpan (every address inside the buffer) and moves by 512 words
  // each round, so no access is loop-invariant
  constexpr int kSpan = kProbeWords - 512;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  // kind 0: consecutive lanes read consecutive words (no bank conflicts); kinds 1, 2: a hashed
  // word per lane
  int base = kind == 0 ? (wave * 64 + lane) % kSpan
                       : (int)((((uint32_t)tid * 2654435761u) ^ (blockIdx.x * 40503u)) % (uint32_t)kSpan);
  if (kind != 2) {
    for (int r = 0; r < rounds; ++r) {
      const uint32_t* p = buf + base;
#pragma unroll
      for (int k = 0; k < 8; ++k) acc += p[64 * k];
      base += 512;
      if (base >= kSpan) base -= kSpan;
    }
  } else {
    for (int r = 0; r < rounds; ++r) {
      uint32_t* p = buf + base;
#pragma unroll
      for (int k = 0; k < 8; ++k) atomicAdd(p + 64 * k, 1u);
      base += 512;
      if (base >= kSpan) base -= kSpan;
    }
    __syncthreads();
    acc = buf[tid];
  }
  // the result decides a store, so no access can be dropped; the value is never expected
  if (acc == 0x9E3779B9u) out[blockIdx.x] = acc;
}

}  // namespace

// Launch `blocks` workgroups of the probe on `stream`; out[blocks] is written only in the
// (never expected) case that a workgroup's folded result equals a fixed constant.
// kind: 0, 1 or 2 (above); rounds > 0.  Returns 0, -1 for bad arguments, -3 for a HIP error.
extern "C" __attribute__((visibility("default"))) int wsr_lds_probe(int kind, int rounds, int blocks, void* out,
                                                                    void* stream) {
  if (kind < 0 || kind > 2 || rounds <= 0 || blocks <= 0 || !out) return -1;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_lds_probe, dim3(blocks), dim3(kProbeThreads), 0, (hipStream_t)stream, kind, rounds,
                     (uint32_t*)out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// Threads per workgroup and LDS words per workgroup of the probe (to convert counts to bytes).
extern "C" __attribute__((visibility("default"))) int wsr_lds_probe_shape(int* threads, int* words) {
  if (!threads || !words) return -1;
  *threads = kProbeThreads;
  *words = kProbeWords;
  return 0;
}
