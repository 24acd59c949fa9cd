// wsr_small.hip -- prox_{lam R} of segments that fit one workgroup (d <= TMAX), everything in LDS.
//
// One workgroup solves one segment end to end (Alg. prox; its l1 and rewinding lines when
// SegArgs::l1 is set), E = TMAX/NT = 8 ranks per thread:
//   1. coalesced load of the FP32 weights, order-preserving u32 keys, non-finite check;
//   2. sort with index payload: bucket-rank sort (value buckets, LDS atomics, rank = bucket start
//      + smaller keys of the bucket), or a stable LSD radix sort in LDS (4 passes of 8 bits,
//      ballot digit matching) when buckets are too full;
//   3. centred FP64 prefix sums S_k = sum_{j<k}(x_j - c) + lam k(d-k)/(d-1)  (rank shift of
//      Alg. prox; sum v in closed form);
//   4. collisions = lower hull of (k, S_k): ImminentCollisions rounds (Sec. 4.1), else per-thread
//      stack hulls and bridge merges (Sec. 4.3 search collisions);
//   5. cluster values, written to the original order in LDS (Alg. prox repeat_interleave +
//      scatter), coalesced stores of out / saved perm / cluster-start bits.
// The backward kernel averages the upstream gradient within each saved cluster.
#include "wsr_device.h"
#include "wsr_kernels.h"

namespace wsr {

// Bucket sort: longest bucket handled (longer ones take the radix sort), and the sentinel padding
// after the bucket-ordered keys that lets a rank scan run past its bucket's end.
constexpr int kBucketMax = 48;
constexpr int kRankPad = 64;

// LDS of the forward kernel, sized so that three workgroups of the 4096 class share a CU.  The
// prefix sums use the transposed rank layout; the other arrays indexed by rank are flat (a
// thread's E = 8 consecutive ranks are read as 16-byte words).  Arrays whose lifetimes do not
// overlap share storage: the bucket sort's scratch, the collision rounds' exchange slots and the
// hull merge's scratch are live one after another, with a barrier between each two.
template <int TMAX, int NT>
struct FwdSmem {
  static constexpr int E = TMAX / NT;
  static constexpr int NW = NT / kWave;
  using SL = RankT<NT, E>;
  // (16-byte aligned: blocks of ranks are read and written as 16-byte words)
  union alignas(16) {
    double S[SL::kSize];  // prefix sums S_0..S_d (layout SL)
    float outv[TMAX];    // results by original index (after the collision rounds)
    struct {
      uint32_t key[TMAX + 1];          // 2*TMAX 16-bit bucket counters in pairs, then starts;
                                       // the sorted keys once the starts are read
      uint32_t tkey[TMAX + kRankPad];  // keys in bucket order, sentinel-padded
    } bs;
    struct {
      uint32_t key[TMAX + 1];  // keys by position; the sorted keys after the last pass
      uint32_t wcnt[NW][256];
    } rs;
  } c;
  alignas(16) uint16_t idx[TMAX];  // original index of each rank
  union {
    struct {
      uint16_t vert[NT * (E + 1)];
      int16_t cnt[NT];
      int16_t mres[NT];
    } h;                  // hull merge (collision rounds not converged)
    uint16_t tidx[TMAX];     // bucket sort: indices in bucket order
    WaveBound wb[2 * NW];    // collision rounds: wave exchange slots, two sets
  } d;
  uint32_t lmask[TMAX / 32 + 2];
  union {
    long long lred[NW + 1];  // bucket sort: counter scan
    double dred[NW + 1];     // prefix sums (barriers separate the two scans)
  } sc;
  int tiecnt;  // bucket sort: sum over keys of the smaller keys in their bucket
  int ired[NW + 1];
  uint32_t ured[2 * NW];
  int flag[4];  // one slot per radix pass: "every key has the same digit"
};

// gfx950 allocates LDS to workgroups in granules of 1280 bytes (128 per CU): three 4096-key
// forward workgroups share a CU only while the rounded size is at most 42 granules.  At 43 the
// timestamps of the measurement build show at most two resident per CU.
static_assert(3 * ((sizeof(FwdSmem<4096, 512>) + 1279) / 1280) <= 128, "three 4096-key forward workgroups per CU");

struct SegView {
  int64_t start;
  int d;
  float lam;
};

__device__ __forceinline__ SegView resolve_segment(const SegArgs& a) {
  if (a.sched) {
    const int s = a.sched[blockIdx.x];
    const int64_t o = a.offsets[s];
    return SegView{o, (int)(a.offsets[s + 1] - o), (a.lam_arr ? a.lam_arr[s] : a.lam_scalar) * a.lam_mul};
  }
  return SegView{a.start, a.d, (a.lam_arr ? a.lam_arr[a.seg_id] : a.lam_scalar) * a.lam_mul};
}

// Waves per SIMD the forward kernel is compiled for (register budget): the 4096 class fits
// three workgroups of 8 waves per CU by LDS, so it keeps its registers to 6 waves per SIMD.
constexpr int fwd_waves_per_simd(int tmax) { return tmax == 4096 ? 6 : 1; }

// Stable block radix sort of the register-held items (wave-striped layout:
// position p = wave*64*IPT + r*64 + lane).  On return sm.c.rs.key / sm.idx hold the sorted items.
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
      sm.c.rs.key[p] = k[r];
      sm.idx[p] = ix[r];
    }
  }
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = pass * 8;
    for (int j = lane; j < 256; j += kWave) sm.c.rs.wcnt[wv][j] = 0u;
    uint16_t rk[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      if (r < nr) {
        const uint32_t dg = (k[r] >> shift) & 255u;
        const uint64_t peers = match_digit8(dg);
        const uint32_t base = sm.c.rs.wcnt[wv][dg];
        const int nbelow = popc_below(peers);
        if (nbelow == 0) sm.c.rs.wcnt[wv][dg] = base + (uint32_t)__popcll(peers);
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
          const uint32_t c = sm.c.rs.wcnt[w][dg];
          sm.c.rs.wcnt[w][dg] = run;
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
        for (int w = 0; w < NW; ++w) sm.c.rs.wcnt[w][dg] += acc;
      }
      acc += tot[q];
    }
    __syncthreads();
    if (sm.flag[pass]) continue;  // uniform across the block; the slot is never rewritten
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      if (r < nr) {
        const uint32_t dg = (k[r] >> shift) & 255u;
        const int np = (int)sm.c.rs.wcnt[wv][dg] + rk[r];
        sm.c.rs.key[np] = k[r];
        sm.idx[np] = ix[r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      if (r < nr) {
        const int p = wbase + r * kWave + lane;
        k[r] = sm.c.rs.key[p];
        ix[r] = sm.idx[p];
      }
    }
    __syncthreads();
  }
}

// Before the sort (and a barrier): per-wave key range in sm.ured, zeroed counters and tie count.
template <int TMAX, int NT>
__device__ __forceinline__ void bucket_sort_prologue(FwdSmem<TMAX, NT>& sm, const uint32_t (&k)[TMAX / NT], int d) {
  constexpr int IPT = TMAX / NT;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wv = tid / kWave;
  const int wbase = wv * kWave * IPT;
  uint32_t kmn = 0xFFFFFFFFu, kmx = 0u;
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const int p = wbase + r * kWave + lane;
    if (p < d) {
      kmn = min(kmn, k[r]);
      kmx = max(kmx, k[r]);
    }
  }
  kmn = wave_min_u32(kmn);
  kmx = wave_max_u32(kmx);
  if (lane == 0) {
    sm.ured[2 * wv] = kmn;
    sm.ured[2 * wv + 1] = kmx;
  }
  for (int j = tid; j < TMAX + 1; j += NT) sm.c.bs.key[j] = 0u;
  if (tid == 0) sm.tiecnt = 0;
}

// Bucket-rank sort of the register-held items (any layout) into sm.c.bs.key / sm.idx; requires
// bucket_sort_prologue and a barrier before it.
// Keys are spread over NB = 2*TMAX buckets by a monotone map of their value over [min, max].  One
// atomic pass counts the keys per bucket (16-bit counters, two to a word) and gives each key a
// slot inside its bucket; a scan turns counts into bucket starts; keys are placed in bucket
// order.  A key's rank is its bucket's start plus the number of keys of its bucket that are
// smaller: since buckets are monotone in value, every key past the end of the bucket (and the
// sentinel padding) is larger, so the count scans a fixed number of slots with no bound checks.
// Equal keys would share a rank; that shows as fewer smaller-key counts than key pairs sharing a
// bucket, and then all ranks are recomputed in (key, index) order.  The result is the same total
// order the stable radix sort produces.  Returns false (sorted arrays untouched) when some bucket holds more than
// kBucketMax keys, so that skewed or tie-heavy segments keep a bounded cost by taking the radix
// sort instead.
template <int TMAX, int NT>
__device__ bool block_bucket_sort(FwdSmem<TMAX, NT>& sm, const uint32_t (&k)[TMAX / NT],
                                  const uint16_t (&ix)[TMAX / NT], int d) {
  constexpr int IPT = TMAX / NT;
  constexpr int NW = NT / kWave;
  constexpr int NB = 2 * TMAX;
  constexpr int WPT = TMAX / NT;  // counter words (bucket pairs) per thread in the scan
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wv = tid / kWave;
  const int wbase = wv * kWave * IPT;
  uint32_t* cnt2 = sm.c.bs.key;
  const uint16_t* st16 = reinterpret_cast<const uint16_t*>(sm.c.bs.key);
  uint32_t* tkey = sm.c.bs.tkey;
  uint16_t* tidx = sm.d.tidx;

  uint32_t kmn = sm.ured[0];
  uint32_t kmx = sm.ured[1];
  for (int w = 1; w < NW; ++w) {
    kmn = min(kmn, sm.ured[2 * w]);
    kmx = max(kmx, sm.ured[2 * w + 1]);
  }
  if (kmn == kmx) {  // every key equal: index order is sorted
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      const int p = wbase + r * kWave + lane;
      if (p < d) {
        cnt2[ix[r]] = k[r];
        sm.idx[ix[r]] = ix[r];
      }
    }
    __syncthreads();
    return true;
  }
  const float mn = key_to_float(kmn);
  const float scale = (float)NB / (key_to_float(kmx) - mn);
  if (!(scale > 0.0f) || isinf(scale)) return false;  // uniform: range overflow or denormal span
  int bk[IPT];
  uint16_t loc[IPT];
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const int p = wbase + r * kWave + lane;
    bk[r] = 0;
    loc[r] = 0;
    if (p < d) {
      const int b = (int)((key_to_float(k[r]) - mn) * scale);
      bk[r] = min(max(b, 0), NB - 1);
      const int sh = (bk[r] & 1) * 16;
      loc[r] = (uint16_t)(atomicAdd(&cnt2[bk[r] >> 1], 1u << sh) >> sh);
    }
  }
  __syncthreads();
  // counts -> bucket starts; thread t owns counter words [t*WPT, (t+1)*WPT)
  // (the high half of the scanned word counts the key pairs sharing a bucket, sum c(c-1)/2: with
  // distinct keys exactly one key of each pair is the smaller)
  uint32_t c[WPT];
  load_u32_block<WPT>(cnt2, tid * WPT, c);
  int sum = 0;
  int pairs = 0;
  int cmax = 0;
#pragma unroll
  for (int i = 0; i < WPT; ++i) {
    const int c0 = (int)(c[i] & 0xFFFFu), c1 = (int)(c[i] >> 16);
    sum += c0 + c1;
    pairs += ((c0 * (c0 - 1)) >> 1) + ((c1 * (c1 - 1)) >> 1);
    cmax = max(cmax, max(c0, c1));
  }
  cmax = (int)wave_max_u32((uint32_t)cmax);
  long long tot2;
  const long long run2 =
      block_excl_scan<NT, long long, false>((long long)sum | ((long long)pairs << 32), sm.sc.lred, &tot2);
  int run = (int)(run2 & 0xFFFFFFFFll);
  const int total = (int)(tot2 & 0xFFFFFFFFll);
  const int pairs_total = (int)(tot2 >> 32);
  if (lane == 0) sm.ured[wv] = (uint32_t)cmax;
#pragma unroll
  for (int i = 0; i < WPT; ++i) {
    const int c0 = (int)(c[i] & 0xFFFFu), c1 = (int)(c[i] >> 16);
    c[i] = (uint32_t)run | ((uint32_t)(run + c0) << 16);
    run += c0 + c1;
  }
#pragma unroll
  for (int q = 0; q < WPT / 4; ++q)
    *reinterpret_cast<uint4*>(cnt2 + tid * WPT + 4 * q) = make_uint4(c[4 * q], c[4 * q + 1], c[4 * q + 2], c[4 * q + 3]);
  if (tid == NT - 1) cnt2[TMAX] = (uint32_t)total;  // start of the (empty) bucket NB
  for (int j = tid; j < kRankPad; j += NT) tkey[d + j] = 0xFFFFFFFFu;  // above every finite key
  __syncthreads();
  cmax = (int)sm.ured[0];
  for (int w = 1; w < NW; ++w) cmax = max(cmax, (int)sm.ured[w]);
  if (cmax > kBucketMax) return false;  // uniform
  int lo[IPT];
  int jmax = 0;  // longest bucket among the thread's items
#pragma unroll
  for (int r = 0; r < IPT; ++r) {  // loads unconditional (bk = 0 for padding) so they overlap
    const int p = wbase + r * kWave + lane;
    const int s0 = (int)st16[bk[r]];
    const int s1 = (int)st16[bk[r] + 1];
    lo[r] = p < d ? s0 : 0;
    jmax = max(jmax, p < d ? s1 - s0 : 0);
  }
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const int p = wbase + r * kWave + lane;
    if (p < d) tkey[lo[r] + loc[r]] = k[r];
  }
  __syncthreads();
  // rank = bucket start + smaller keys of the bucket; the items advance together, two slots a
  // step (one paired read per item, all issued before the compares), and the sentinel padding
  // covers the overrun of the last step
  int rank[IPT];
  const uint32_t* kp[IPT];
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    rank[r] = lo[r];
    kp[r] = tkey + lo[r];
  }
  for (int j = 0; j < jmax; j += 2) {
    uint32_t q0[IPT], q1[IPT];  // every item's pair in flight before any compare
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      q0[r] = kp[r][j];
      q1[r] = kp[r][j + 1];
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r) rank[r] += (q0[r] < k[r] ? 1 : 0) + (q1[r] < k[r] ? 1 : 0);
  }
  int below = 0;
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const int p = wbase + r * kWave + lane;
    if (p < d) {
      below += rank[r] - lo[r];
      cnt2[rank[r]] = k[r];
      sm.idx[rank[r]] = ix[r];
    }
  }
  below = wave_sum(below);
  if (lane == 0) atomicAdd(&sm.tiecnt, below);
  __syncthreads();
  if (sm.tiecnt != pairs_total) {
    // equal keys (they shared ranks above): order each bucket by (key, index) instead; an equal
    // key is always in the same bucket, and the padding never equals a finite key
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      const int p = wbase + r * kWave + lane;
      if (p < d) tidx[lo[r] + loc[r]] = ix[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IPT; ++r) rank[r] = lo[r];
    for (int j = 0; j < jmax; ++j) {
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const uint32_t kj = tkey[lo[r] + j];
        const uint16_t ij = tidx[min(lo[r] + j, TMAX - 1)];
        rank[r] += (kj < k[r]) | ((kj == k[r]) & (ij < ix[r]));
      }
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      const int p = wbase + r * kWave + lane;
      if (p < d) {
        cnt2[rank[r]] = k[r];
        sm.idx[rank[r]] = ix[r];
      }
    }
    __syncthreads();
  }
  return true;
}

// Given the hull vertices vert[0..ncl] (ranks, vert[ncl] == d) of S, the output
// fin(offset + (S_b - S_a)/(b - a), a, b) of the cluster [a, b) of every rank of the thread's
// blocked range, into val[i] for rank k0 + i < d (the caller stages them by original index).
template <int NT, int E, typename SL, typename Fin>
__device__ __forceinline__ void cluster_values(const uint16_t* vert, int ncl, const double* S, double offset, int d,
                                               Fin fin, float (&val)[E]) {
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
  int a = vert[lo];
  int b = vert[lo + 1];
  float v = fin(offset + (S[SL::at(b)] - S[SL::at(a)]) / (double)(b - a), a, b);
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int k = k0 + i;
    if (k < d) {
      while (k >= b) {
        ++lo;
        a = b;
        b = vert[lo + 1];
        v = fin(offset + (S[SL::at(b)] - S[SL::at(a)]) / (double)(b - a), a, b);
      }
      val[i] = v;
    }
  }
}

// EndCollisions (Sec. 4.2: the rightmost collision ends the cluster that starts at a; it is the
// last b in (a, d] minimising the average of y over [a, b), i.e. the next vertex of the lower
// hull of (k, S_k); Alg. end_collisions), repeated from a = 0 until b = d: one block-wide
// reduction per cluster, so it is fast when the clusters are few and slow when they are many.
// Later candidates win ties (rightmost), and a candidate q beats an earlier p exactly when p is
// not strictly below the segment a -> q (the predicate of every other route).  sv[0..E] are the
// thread's S values; red holds NT/64 ints.  Writes the hull vertices to vert (vert[0] = 0, the
// last = d) and returns their number.  All threads must call.
template <int NT, int E, typename SL>
__device__ int end_collisions(const double* S, const double (&sv)[E + 1], int d, uint16_t* vert, int* red) {
  constexpr int NW = NT / kWave;
  const int tid = threadIdx.x;
  const int k0 = tid * E;
  int a = 0, nv = 0;
  if (tid == 0) vert[0] = 0;
  while (a < d) {
    const double sa = S[SL::at(a)];
    int best = -1;
    double sbest = 0.0;
#pragma unroll
    for (int i = 1; i <= E; ++i) {
      const int b = k0 + i;
      if (b > a && b <= d && (best < 0 || !below(a, sa, best, sbest, b, sv[i]))) {
        best = b;
        sbest = sv[i];
      }
    }
    // wave: butterfly over the lanes (both partners combine the same pair, so all agree)
    for (int m = 1; m < kWave; m <<= 1) {
      const int ob = __shfl_xor(best, m, kWave);
      const double os = __shfl_xor(sbest, m, kWave);
      if (ob >= 0) {
        if (best < 0) {
          best = ob;
          sbest = os;
        } else {
          const bool lo_mine = best < ob;
          const int p = lo_mine ? best : ob, q = lo_mine ? ob : best;
          const double sp = lo_mine ? sbest : os, sq = lo_mine ? os : sbest;
          const bool q_wins = !below(a, sa, p, sp, q, sq);
          best = q_wins ? q : p;
          sbest = q_wins ? sq : sp;
        }
      }
    }
    if (lane_id() == 0) red[tid / kWave] = best;
    __syncthreads();
    // block: the waves' winners in rank order, the same sequence in every thread
    int w = -1;
    double sw = 0.0;
    for (int j = 0; j < NW; ++j) {
      const int p = red[j];
      if (p < 0) continue;
      const double sp = S[SL::at(p)];
      if (w < 0 || !below(a, sa, w, sw, p, sp)) {
        w = p;
        sw = sp;
      }
    }
    __syncthreads();  // red is written again in the next round
    a = w;
    ++nv;
    if (tid == 0) vert[nv] = (uint16_t)a;
  }
  __syncthreads();
  return nv + 1;
}

template <int TMAX, int NT, bool END>
__global__ __launch_bounds__(NT, fwd_waves_per_simd(TMAX)) void k_prox_fwd_small(SegArgs args, const float* w, float* out,
                                                       int32_t* perm_out, uint32_t* mask_out) {
  constexpr int IPT = TMAX / NT;
  constexpr int E = IPT;
  __shared__ FwdSmem<TMAX, NT> sm;
  const SegView seg = resolve_segment(args);
  const int64_t start = seg.start;
  const int d = seg.d;
  const float lam = seg.lam;
  if (d <= 0) return;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wv = tid / kWave;
  const int wbase = wv * kWave * IPT;
  const int off = (int)(start & 31);
  WSR_PHASE_MARK(args, 0);

  for (int j = tid; j < TMAX / 32 + 2; j += NT) sm.lmask[j] = 0u;
  uint32_t k[IPT];
  uint16_t ix[IPT];
  float f[IPT];
#pragma unroll
  for (int r = 0; r < IPT; ++r) {  // all loads in flight before any use
    const int p = wbase + r * kWave + lane;
    f[r] = p < d ? w[start + p] : 0.0f;
  }
  if (args.grad) {  // proximal-gradient step: the input is w - eta * grad, one FP32 rounding
    float gv[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      const int p = wbase + r * kWave + lane;
      gv[r] = p < d ? args.grad[start + p] : 0.0f;
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r) f[r] = __builtin_fmaf(-args.eta, gv[r], f[r]);
  }
  int bad = 0;
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const int p = wbase + r * kWave + lane;
    bad |= (p < d) & !isfinite(f[r]);
    k[r] = p < d ? float_to_key(f[r]) : 0xFFFFFFFFu;
    ix[r] = (uint16_t)p;
  }
  bucket_sort_prologue<TMAX, NT>(sm, k, d);  // shares the barrier below
  const bool nonfinite = __syncthreads_or(bad) != 0;
  WSR_PHASE_MARK(args, 1);
  if (nonfinite && tid == 0 && args.status) atomicOr(args.status, kStatusNonFinite);
  if (nonfinite || d == 1 || !(lam > 0.0f)) {
    // identity (or NaN) segment: every weight its own cluster, perm = identity
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      const int p = wbase + r * kWave + lane;
      if (p < d) {
        const float x = key_to_float(k[r]);
        out[start + p] = nonfinite ? __builtin_nanf("")
                                   : (args.l1 ? L1Rewind(args.beta, args.rho, args.kappa)((double)x, 0.0) : x);
        if (perm_out) perm_out[start + p] = p;
        atomicOr(&sm.lmask[(p + off) >> 5], 1u << ((p + off) & 31));
      }
    }
    __syncthreads();
    if (mask_out) store_mask_words<NT>(mask_out, start, d, sm.lmask);
    return;
  }

  if (args.sort_route == kSortRadix || !block_bucket_sort<TMAX, NT>(sm, k, ix, d))
    block_radix_sort<TMAX, NT>(sm, k, ix, d);
  WSR_PHASE_MARK(args, 2);

  // centred FP64 prefix sums S_k (blocked: thread t owns ranks [tE, tE+E)); S overwrites the
  // sorted keys, so every key is read before the block scan's barriers
  using SL = typename FwdSmem<TMAX, NT>::SL;
  const uint32_t* skey = sm.c.bs.key;
  const double c = (double)key_to_float(skey[d >> 1]);
  const double lamd = (double)lam / (double)(d - 1);
  const int k0 = tid * E;
  uint32_t kv[E];
  load_u32_block<E>(skey, k0, kv);  // ranks past d hold stale words, masked below
  double xs[E];
  double lsum = 0.0;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    xs[i] = k0 + i < d ? (double)key_to_float(kv[i]) - c : 0.0;
    lsum += xs[i];
  }
  double Xk = block_excl_scan<NT, double, false>(lsum, sm.sc.dred, (double*)nullptr);
  double sv[E + 1];
#pragma unroll
  for (int i = 0; i <= E; ++i) {
    const int kk = k0 + i;
    sv[i] = Xk + lamd * (double)kk * (double)(d - kk);
    if (i < E) {
      if (kk <= d) sm.c.S[SL::at(kk)] = sv[i];
      Xk += xs[i];
    }
  }
  if (tid == NT - 1 && d == TMAX) sm.c.S[SL::at(TMAX)] = sv[E];  // X_d (the shift term vanishes at k = d)
  __syncthreads();
  WSR_PHASE_MARK(args, 3);

  // collisions: ImminentCollisions rounds (converge in a few rounds on typical weights), else
  // the bounded-depth hull merge; or, in the END instantiation (a route the caller chooses),
  // EndCollisions
  uint32_t bm;
  Cand lc, rc;
  if (!END &&
      ica_rounds<NT, E, SL>(sm.c.S, sv, d, args.merge_rounds < 0 ? kIcaRounds : args.merge_rounds, &bm, &lc, &rc,
                            sm.d.wb)) {
    if (bm) {
      const int b0 = k0 + off;
      const uint64_t wide = (uint64_t)bm << (b0 & 31);
      atomicOr(&sm.lmask[b0 >> 5], (uint32_t)wide);
      if (wide >> 32) atomicOr(&sm.lmask[(b0 >> 5) + 1], (uint32_t)(wide >> 32));
    }
    // S is no longer read once the rounds have converged: the results take its place
    uint16_t ixr[E];
    load_u16_block<E>(sm.idx, k0, ixr);
    if (args.l1)
      walk_values<E>(bm, sv, lc, rc, d, c, ixr, sm.c.outv, L1Value{L1Rewind(args.beta, args.rho, args.kappa), lamd, d});
    else
      walk_values<E>(bm, sv, lc, rc, d, c, ixr, sm.c.outv);
  } else {
    int nv;
    if constexpr (END) {
      nv = end_collisions<NT, E, SL>(sm.c.S, sv, d, sm.d.h.vert, sm.ired);
    } else {
      __syncthreads();  // the rounds' last reads of the exchange slots, which the hull overwrites
      tile_hull<NT, E, SL, int16_t>(sm.c.S, d, sm.d.h.vert, sm.d.h.cnt, sm.d.h.mres);
      nv = sm.d.h.cnt[0];
    }
    const uint16_t* vert = sm.d.h.vert;
    for (int i = tid; i < nv - 1; i += NT) {
      const int a = vert[i];
      atomicOr(&sm.lmask[(a + off) >> 5], 1u << ((a + off) & 31));
    }
    // values in registers while S holds the sums, then by original index into LDS over S (the
    // stores below are lane-consecutive)
    float val[E];
    if (args.l1)
      cluster_values<NT, E, SL>(vert, nv - 1, sm.c.S, c, d, L1Value{L1Rewind(args.beta, args.rho, args.kappa), lamd, d},
                                val);
    else
      cluster_values<NT, E, SL>(vert, nv - 1, sm.c.S, c, d, PlainValue(), val);
    __syncthreads();  // every read of S is done
    uint16_t ixr[E];
    load_u16_block<E>(sm.idx, k0, ixr);
#pragma unroll
    for (int i = 0; i < E; ++i)
      if (k0 + i < d) sm.c.outv[ixr[i]] = val[i];
  }
  __syncthreads();
  WSR_PHASE_MARK(args, 4);
  // fixed trip count (TMAX / NT) so every LDS read is issued before the stores wait on them
  float* const og = out + start;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int i = tid + r * NT;
    if (i < d) og[i] = sm.c.outv[i];
  }
  if (perm_out) {
    int32_t* const pg = perm_out + start;
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = tid + r * NT;
      if (i < d) pg[i] = sm.idx[i];
    }
  }
  if (mask_out) store_mask_words<NT>(mask_out, start, d, sm.lmask);
  WSR_PHASE_MARK(args, 5);
}

// Statistics of one segment from its sorted order (App. B): R(w) = 1/(d-1) sum_k (2k-d+1) x_k,
// summed in FP64 over the centred values x_k - c (the weights 2k-d+1 sum to zero, so centring
// changes nothing but the rounding), and the counts of non-zero weights and of distinct non-zero
// values (a rank counts when its value differs from the previous rank's).  The sort is the
// forward kernel's.  Non-finite segment: penalty NaN, counts -1.
template <int TMAX, int NT>
__global__ __launch_bounds__(NT, fwd_waves_per_simd(TMAX)) void k_seg_stats_small(SegArgs args, const float* w,
                                                                                  SegStats* stats) {
  constexpr int IPT = TMAX / NT;
  constexpr int E = IPT;
  __shared__ FwdSmem<TMAX, NT> sm;
  const SegView seg = resolve_segment(args);
  const int sid = args.sched ? args.sched[blockIdx.x] : args.seg_id;
  const int64_t start = seg.start;
  const int d = seg.d;
  if (d <= 0) return;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wv = tid / kWave;
  const int wbase = wv * kWave * IPT;
  uint32_t k[IPT];
  uint16_t ix[IPT];
  float f[IPT];
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const int p = wbase + r * kWave + lane;
    f[r] = p < d ? w[start + p] : 0.0f;
  }
  int bad = 0;
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const int p = wbase + r * kWave + lane;
    bad |= (p < d) & !isfinite(f[r]);
    k[r] = p < d ? float_to_key(f[r]) : 0xFFFFFFFFu;
    ix[r] = (uint16_t)p;
  }
  bucket_sort_prologue<TMAX, NT>(sm, k, d);  // shares the barrier below
  const bool nonfinite = __syncthreads_or(bad) != 0;
  if (nonfinite) {
    if (tid == 0) stats[sid] = SegStats{__builtin_nan(""), -1, -1};
    return;
  }
  if (args.sort_route == kSortRadix || !block_bucket_sort<TMAX, NT>(sm, k, ix, d))
    block_radix_sort<TMAX, NT>(sm, k, ix, d);
  const uint32_t* skey = sm.c.bs.key;
  const double c = (double)key_to_float(skey[d >> 1]);
  const int k0 = tid * E;
  uint32_t kv[E];
  load_u32_block<E>(skey, k0, kv);  // ranks past d hold stale words, masked below
  float prev = (k0 > 0 && k0 <= d) ? key_to_float(skey[k0 - 1]) : 0.0f;
  double lsum = 0.0;
  long long cnt = 0;  // non-zero weights in the high half, distinct non-zero values in the low
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int kk = k0 + i;
    if (kk < d) {
      const float x = key_to_float(kv[i]);
      lsum += (double)(2 * kk - d + 1) * ((double)x - c);
      if (x != 0.0f) cnt += (1ll << 32) + ((kk == 0 || x != prev) ? 1 : 0);
      prev = x;
    }
  }
  double total;
  (void)block_excl_scan<NT, double, false>(lsum, sm.sc.dred, &total);
  __syncthreads();  // the counter scan below reuses the same LDS slots
  long long ctot;
  (void)block_excl_scan<NT, long long, false>(cnt, sm.sc.lred, &ctot);
  if (tid == 0)
    stats[sid] = SegStats{d > 1 ? total / (double)(d - 1) : 0.0, ctot & 0xFFFFFFFFll, ctot >> 32};
}

template <int TMAX, int NT>
struct BwdSmem {
  static constexpr int NW = NT / kWave;
  float g[TMAX];                   // upstream gradient by original index, then results
  alignas(16) uint16_t idx[TMAX];  // saved permutation (rank -> original index)
  uint32_t lmask[TMAX / 32 + 2];
  double dred[NW + 1];
  Cand shL[NW], shR[NW];
  int shF[NW];
};

// Eight waves per SIMD (64 VGPRs): the kernel waits mostly for its loads, so as many segments
// as the registers allow are in flight (four 4096-class or two 8192-class workgroups per CU).
template <int TMAX, int NT>
__global__ __launch_bounds__(NT, 8) void k_prox_bwd_small(SegArgs args, const float* gin, float* gout,
                                                       const int32_t* perm_in, const uint32_t* mask_in) {
  constexpr int E = TMAX / NT;
  __shared__ BwdSmem<TMAX, NT> sm;
  const SegView seg = resolve_segment(args);
  const int64_t start = seg.start;
  const int d = seg.d;
  const float lam = seg.lam;
  if (d <= 0) return;
  const int tid = threadIdx.x;
  const int off = (int)(start & 31);
  const int nwords = (off + d + 31) >> 5;
  const int64_t g0 = start >> 5;
  WSR_PHASE_MARK(args, 0);
  // every load of the thread in flight before the LDS stores (fixed trip count TMAX / NT)
  {
    const float* const gg = gin + start;
    const int32_t* const pg = perm_in + start;
    float gv[E];
    int32_t pv[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = tid + r * NT;
      gv[r] = i < d ? gg[i] : 0.0f;
      pv[r] = i < d ? pg[i] : 0;
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = tid + r * NT;
      if (i < d) {
        sm.g[i] = gv[r];
        sm.idx[i] = (uint16_t)min(max(pv[r], 0), d - 1);
      }
    }
  }
  for (int j = tid; j < nwords; j += NT) sm.lmask[j] = mask_in[g0 + j];
  __syncthreads();
  WSR_PHASE_MARK(args, 1);
  // cotangent in rank order, cluster starts of the thread's ranks, FP64 prefix sums G (registers)
  const int k0 = tid * E;
  float gk[E];
  double lsum = 0.0;
  uint32_t bm = 0;
  {
    uint16_t ixr[E];
    load_u16_block<E>(sm.idx, k0, ixr);  // ranks past d hold stale entries, not used
    // the start bits of ranks k0 .. k0+E-1 lie in two mask words (words past the segment's end
    // hold stale bits, masked below)
    const int b0 = k0 + off;
    const uint64_t mw = (uint64_t)sm.lmask[b0 >> 5] | ((uint64_t)sm.lmask[(b0 >> 5) + 1] << 32);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int kk = k0 + i;
      const float gv = sm.g[kk < d ? ixr[i] : 0];  // unconditional gather
      const uint32_t st = (kk == 0) | (uint32_t)((mw >> ((b0 & 31) + i)) & 1u);
      gk[i] = kk < d ? gv : 0.0f;
      lsum += (double)gk[i];
      bm |= (kk < d ? st : 0u) << i;
    }
  }
  double total;
  double G = block_excl_scan_lean<NT>(lsum, sm.dred, &total);
  WSR_PHASE_MARK(args, 2);
  double sv[E + 1];
  Cand mineL{-1, 0.0}, mineR{-1, 0.0};
#pragma unroll
  for (int i = 0; i <= E; ++i) {
    sv[i] = G;
    if (i < E) {
      if ((bm >> i) & 1u) {
        if (mineR.pos < 0) mineR = Cand{k0 + i, G};
        mineL = Cand{k0 + i, G};
      }
      G += (double)gk[i];
    }
  }
  Cand lc, rc;
  carry_exchange<NT>(mineL, mineR, false, Cand{d, total}, sm.shL, sm.shR, sm.shF, &lc, &rc);
  uint16_t ixw[E];  // read again here rather than held through the scans
  load_u16_block<E>(sm.idx, k0, ixw);
  walk_values<E>(bm, sv, lc, rc, d, 0.0, ixw, sm.g);  // every gather above is done (block scan)
  __syncthreads();
  WSR_PHASE_MARK(args, 3);
  float* const og = gout + start;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int i = tid + r * NT;
    if (i < d) og[i] = sm.g[i];
  }
  WSR_PHASE_MARK(args, 4);
}

// Zero a word array (used for the saved cluster-start mask before OR-ing boundary words).
__global__ void k_zero_u32(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = i; j < n; j += stride) p[j] = 0u;
}

#define WSR_INSTANTIATE_SMALL(TM, NTH)                                                          \
  template __global__ void k_seg_stats_small<TM, NTH>(SegArgs, const float*, SegStats*);         \
  template __global__ void k_prox_fwd_small<TM, NTH, false>(SegArgs, const float*, float*,       \
                                                             int32_t*, uint32_t*);              \
  template __global__ void k_prox_fwd_small<TM, NTH, true>(SegArgs, const float*, float*,        \
                                                            int32_t*, uint32_t*);               \
  template __global__ void k_prox_bwd_small<TM, NTH>(SegArgs, const float*, float*,             \
                                                      const int32_t*, const uint32_t*);

WSR_INSTANTIATE_SMALL(2048, 256)
WSR_INSTANTIATE_SMALL(4096, 512)
WSR_INSTANTIATE_SMALL(8192, 1024)

}  // namespace wsr
