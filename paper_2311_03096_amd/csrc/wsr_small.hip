// wsr_small.hip -- prox_{lam R} of segments that fit one workgroup (d <= TMAX), everything in LDS.
//
// One workgroup solves one segment end to end (Alg. prox without its l1 lines):
//   1. coalesced load of the FP32 weights, order-preserving u32 keys, non-finite check;
//   2. stable LSD radix sort in LDS (4 passes of 8 bits; wave-level digit matching with
//      ballots, per-wave counters, block scan), index payload; a pass whose digit is the same
//      for every key is skipped;
//   3. centred FP64 prefix sums S_k = sum_{j<k}(x_j - c) + lam k(d-k)/(d-1)  (rank shift of
//      Alg. prox; sum v in closed form);
//   4. collisions = lower hull of (k, S_k): per-thread stack hulls then bridge merges
//      (Sec. 4.1 pool adjacent violators, Sec. 4.3 search collisions);
//   5. cluster values, scatter back to original order in LDS (Alg. prox repeat_interleave +
//      scatter), coalesced stores of out / saved perm / cluster-start bits.
// The backward kernel averages the upstream gradient within each saved cluster.
#include "wsr_device.h"
#include "wsr_kernels.h"

namespace wsr {

template <int TMAX, int NT>
struct FwdSmem {
  static constexpr int E = TMAX / NT;
  static constexpr int NW = NT / kWave;
  union {
    uint32_t key[TMAX];  // sort keys; sorted keys after the sort
    float cval[TMAX];    // per-cluster values (output phase)
    float g[TMAX];       // backward: upstream gradient by original index
  } a;
  uint16_t idx[TMAX];  // payload: segment-local original index (perm after the sort)
  union {
    double S[TMAX + 1];  // prefix sums (forward) / G (backward)
    float outv[TMAX];    // results by original index (output phase)
  } c;
  union {
    uint32_t wcnt[NW][256];
    struct {
      uint16_t vert[NT * (E + 1)];
      int cnt[NT];
      int mres[NT];
    } h;
  } d;
  uint32_t lmask[TMAX / 32 + 2];
  double dred[NW + 1];
  int ired[NW + 1];
  int flag[4];  // one slot per radix pass: "every key has the same digit"
};

__device__ __forceinline__ void resolve_segment(const SegArgs& a, int64_t* start, int* d, float* lam) {
  if (a.sched) {
    const int s = a.sched[blockIdx.x];
    const int64_t o = a.offsets[s];
    *start = o;
    *d = (int)(a.offsets[s + 1] - o);
    *lam = a.lam_arr ? a.lam_arr[s] : a.lam_scalar;
  } else {
    *start = a.start;
    *d = a.d;
    *lam = a.lam_arr ? a.lam_arr[a.seg_id] : a.lam_scalar;
  }
}

// Stable block radix sort of the register-held items (wave-striped layout:
// position p = wave*64*IPT + r*64 + lane).  On return sm.a.key / sm.idx hold the sorted items.
template <int TMAX, int NT>
__device__ void block_radix_sort(FwdSmem<TMAX, NT>& sm, uint32_t (&k)[TMAX / NT],
                                 uint16_t (&ix)[TMAX / NT], int d) {
  constexpr int IPT = TMAX / NT;
  constexpr int NW = NT / kWave;
  constexpr int DPT = (256 + NT - 1) / NT;  // digits per thread in the digit scan
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wv = tid / kWave;
  const int wbase = wv * kWave * IPT;
  const int nr = min(IPT, max(0, (d - wbase + kWave - 1) / kWave));
  int counted = 0;
  for (int w = 0; w < NW; ++w) counted += kWave * min(IPT, max(0, (d - w * kWave * IPT + kWave - 1) / kWave));

  // initial order = original index order
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    if (r < nr) {
      const int p = wbase + r * kWave + lane;
      sm.a.key[p] = k[r];
      sm.idx[p] = ix[r];
    }
  }
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = pass * 8;
    for (int j = lane; j < 256; j += kWave) sm.d.wcnt[wv][j] = 0u;
    uint16_t rk[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      if (r < nr) {
        const uint32_t dg = (k[r] >> shift) & 255u;
        const uint64_t peers = match_digit8(dg);
        const uint32_t base = sm.d.wcnt[wv][dg];
        const int nbelow = __popcll(peers & lanemask_lt());
        if (nbelow == 0) sm.d.wcnt[wv][dg] = base + (uint32_t)__popcll(peers);
        rk[r] = (uint16_t)(base + nbelow);
      }
    }
    if (tid == 0) sm.flag[pass] = 0;
    __syncthreads();
    // digit offsets: per wave exclusive within a digit, digits exclusive across the block
    uint32_t tot[DPT];
    uint32_t mysum = 0;
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int dg = tid * DPT + q;
      uint32_t run = 0;
      if (dg < 256) {
        for (int w = 0; w < NW; ++w) {
          const uint32_t c = sm.d.wcnt[w][dg];
          sm.d.wcnt[w][dg] = run;
          run += c;
        }
      }
      tot[q] = run;
      mysum += run;
    }
    int dtotal;
    const int dbase = block_excl_scan<NT, int>((int)mysum, sm.ired, &dtotal);
    uint32_t acc = (uint32_t)dbase;
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int dg = tid * DPT + q;
      if (dg < 256) {
        if ((int)tot[q] == counted) sm.flag[pass] = 1;  // every key has this digit: identity pass
        for (int w = 0; w < NW; ++w) sm.d.wcnt[w][dg] += acc;
      }
      acc += tot[q];
    }
    __syncthreads();
    if (sm.flag[pass]) continue;  // uniform across the block; the slot is never rewritten
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      if (r < nr) {
        const uint32_t dg = (k[r] >> shift) & 255u;
        const int np = (int)sm.d.wcnt[wv][dg] + rk[r];
        sm.a.key[np] = k[r];
        sm.idx[np] = ix[r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      if (r < nr) {
        const int p = wbase + r * kWave + lane;
        k[r] = sm.a.key[p];
        ix[r] = sm.idx[p];
      }
    }
    __syncthreads();
  }
}

// Given the cluster-start list vert[0..ncl] (ranks, vert[ncl] == d) and per-cluster values
// cval[0..ncl), write res[idx[k]] = cval[cluster of k] for all ranks k < d (blocked ranges).
template <int NT, int E>
__device__ __forceinline__ void scatter_cluster_values(const uint16_t* vert, int ncl, const float* cval,
                                                       const uint16_t* idx, float* res, int d) {
  const int k0 = threadIdx.x * E;
  if (k0 >= d) return;
  // cluster of k0: last i with vert[i] <= k0
  int lo = 0, hi = ncl;  // vert[lo] <= k0 < vert[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (vert[mid] <= k0)
      lo = mid;
    else
      hi = mid;
  }
  int cid = lo;
  int next = vert[cid + 1];
  float v = cval[cid];
  const int k1 = min(k0 + E, d);
  for (int k = k0; k < k1; ++k) {
    while (k >= next) {
      ++cid;
      next = vert[cid + 1];
      v = cval[cid];
    }
    res[idx[k]] = v;
  }
}

template <int TMAX, int NT>
__global__ __launch_bounds__(NT) void k_prox_fwd_small(SegArgs args, const float* w, float* out,
                                                       int32_t* perm_out, uint32_t* mask_out) {
  constexpr int IPT = TMAX / NT;
  constexpr int E = IPT;
  __shared__ FwdSmem<TMAX, NT> sm;
  int64_t start;
  int d;
  float lam;
  resolve_segment(args, &start, &d, &lam);
  if (d <= 0) return;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wv = tid / kWave;
  const int wbase = wv * kWave * IPT;
  const int off = (int)(start & 31);

  for (int j = tid; j < TMAX / 32 + 2; j += NT) sm.lmask[j] = 0u;
  uint32_t k[IPT];
  uint16_t ix[IPT];
  int bad = 0;
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const int p = wbase + r * kWave + lane;
    if (p < d) {
      const float f = w[start + p];
      bad |= !isfinite(f);
      k[r] = float_to_key(f);
    } else {
      k[r] = 0xFFFFFFFFu;
    }
    ix[r] = (uint16_t)p;
  }
  const bool nonfinite = __syncthreads_or(bad) != 0;
  if (nonfinite || d == 1 || !(lam > 0.0f)) {
    // identity (or NaN) segment: every weight its own cluster, perm = identity
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      const int p = wbase + r * kWave + lane;
      if (p < d) {
        out[start + p] = nonfinite ? __builtin_nanf("") : key_to_float(k[r]);
        if (perm_out) perm_out[start + p] = p;
        atomicOr(&sm.lmask[(p + off) >> 5], 1u << ((p + off) & 31));
      }
    }
    __syncthreads();
    if (mask_out) store_mask_words<NT>(mask_out, start, d, sm.lmask);
    return;
  }

  block_radix_sort<TMAX, NT>(sm, k, ix, d);

  // centred FP64 prefix sums S_k (blocked: thread t owns ranks [tE, tE+E))
  const double c = (double)key_to_float(sm.a.key[d >> 1]);
  const double lamd = (double)lam / (double)(d - 1);
  const int k0 = tid * E;
  double xs[E];
  double lsum = 0.0;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int kk = k0 + i;
    xs[i] = kk < d ? (double)key_to_float(sm.a.key[kk]) - c : 0.0;
    lsum += xs[i];
  }
  double Xk = block_excl_scan<NT, double>(lsum, sm.dred, (double*)nullptr);
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int kk = k0 + i;
    if (kk <= d) sm.c.S[kk] = Xk + lamd * (double)kk * (double)(d - kk);
    Xk += xs[i];
  }
  if (tid == NT - 1 && d == TMAX) sm.c.S[TMAX] = Xk;  // X_d (the shift term vanishes at k = d)
  __syncthreads();

  tile_hull<NT, E>(sm.c.S, d, sm.d.h.vert, sm.d.h.cnt, sm.d.h.mres);

  // cluster values: c + (S_b - S_a)/(b - a) for consecutive hull vertices a < b
  const int nv = sm.d.h.cnt[0];
  const uint16_t* vert = sm.d.h.vert;
  for (int i = tid; i < nv - 1; i += NT) {
    const int a = vert[i], b = vert[i + 1];
    sm.a.cval[i] = (float)(c + (sm.c.S[b] - sm.c.S[a]) / (double)(b - a));
    atomicOr(&sm.lmask[(a + off) >> 5], 1u << ((a + off) & 31));
  }
  __syncthreads();
  scatter_cluster_values<NT, E>(vert, nv - 1, sm.a.cval, sm.idx, sm.c.outv, d);
  __syncthreads();
  for (int i = tid; i < d; i += NT) out[start + i] = sm.c.outv[i];
  if (perm_out)
    for (int i = tid; i < d; i += NT) perm_out[start + i] = sm.idx[i];
  if (mask_out) store_mask_words<NT>(mask_out, start, d, sm.lmask);
}

template <int TMAX, int NT>
__global__ __launch_bounds__(NT) void k_prox_bwd_small(SegArgs args, const float* gin, float* gout,
                                                       const int32_t* perm_in, const uint32_t* mask_in) {
  constexpr int E = TMAX / NT;
  __shared__ FwdSmem<TMAX, NT> sm;
  int64_t start;
  int d;
  float lam;
  resolve_segment(args, &start, &d, &lam);
  if (d <= 0) return;
  const int tid = threadIdx.x;
  const int off = (int)(start & 31);
  const int nwords = (off + d + 31) >> 5;
  const int64_t g0 = start >> 5;
  for (int i = tid; i < d; i += NT) {
    sm.a.g[i] = gin[start + i];
    int p = perm_in[start + i];
    sm.idx[i] = (uint16_t)min(max(p, 0), d - 1);
  }
  for (int j = tid; j < nwords; j += NT) sm.lmask[j] = mask_in[g0 + j];
  __syncthreads();
  // gathered cotangent in rank order, cluster starts, FP64 prefix sums
  const int k0 = tid * E;
  float gk[E];
  double lsum = 0.0;
  int lst = 0;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int kk = k0 + i;
    gk[i] = 0.0f;
    if (kk < d) {
      gk[i] = sm.a.g[sm.idx[kk]];
      lsum += (double)gk[i];
      const int b = kk + off;
      lst += (kk == 0) || ((sm.lmask[b >> 5] >> (b & 31)) & 1u);
    }
  }
  int ncl;
  const int cbase = block_excl_scan<NT, int>(lst, sm.ired, &ncl);
  double G = block_excl_scan<NT, double>(lsum, sm.dred, (double*)nullptr);
  int ci = cbase;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int kk = k0 + i;
    if (kk <= d) sm.c.S[kk] = G;
    if (kk < d) {
      const int b = kk + off;
      if ((kk == 0) || ((sm.lmask[b >> 5] >> (b & 31)) & 1u)) sm.d.h.vert[ci++] = (uint16_t)kk;
      G += (double)gk[i];
    }
  }
  if (tid == NT - 1 && d == TMAX) sm.c.S[TMAX] = G;
  if (tid == 0) sm.d.h.vert[ncl] = (uint16_t)d;
  __syncthreads();
  for (int i = tid; i < ncl; i += NT) {
    const int a = sm.d.h.vert[i], b = sm.d.h.vert[i + 1];
    sm.a.cval[i] = (float)((sm.c.S[b] - sm.c.S[a]) / (double)(b - a));
  }
  __syncthreads();
  scatter_cluster_values<NT, E>(sm.d.h.vert, ncl, sm.a.cval, sm.idx, sm.c.outv, d);
  __syncthreads();
  for (int i = tid; i < d; i += NT) gout[start + i] = sm.c.outv[i];
}

// Zero a word array (used for the saved cluster-start mask before OR-ing boundary words).
__global__ void k_zero_u32(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = i; j < n; j += stride) p[j] = 0u;
}

#define WSR_INSTANTIATE_SMALL(TM, NTH)                                                          \
  template __global__ void k_prox_fwd_small<TM, NTH>(SegArgs, const float*, float*, int32_t*,   \
                                                      uint32_t*);                               \
  template __global__ void k_prox_bwd_small<TM, NTH>(SegArgs, const float*, float*,             \
                                                      const int32_t*, const uint32_t*);

WSR_INSTANTIATE_SMALL(2048, 128)
WSR_INSTANTIATE_SMALL(4096, 256)
WSR_INSTANTIATE_SMALL(8192, 512)

}  // namespace wsr
