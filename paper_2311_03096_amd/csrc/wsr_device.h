// wsr_device.h -- device building blocks shared by the gfx950 kernels.
//
// Geometry used throughout.  For a segment of d weights sorted ascending (x_0 <= ... <= x_{d-1}),
// the particle of rank k gets the velocity v_k = lam (d-1-2k)/(d-1) (Alg. prox, shift line;
// Sec. 2 eq. hyperplane) and the destination y_k = x_k + v_k.  With the centred prefix sums
//     S_k = sum_{j<k} (x_j - c) + sum_{j<k} v_j = X_k + lam k (d-k)/(d-1),   k = 0..d,
// the sticky-particle collisions of Sec. 3/4 (pool adjacent violators on y, merging on >=)
// produce exactly the edges of the lower convex hull of the points P_k = (k, S_k) with collinear
// points dropped: the cluster of ranks [a, b) is the hull edge P_a -> P_b and its value is
//     c + (S_b - S_a) / (b - a)                        (avg y of the cluster, Sec. 4.2 fact 3).
// The closed form of sum v follows from the rank shift; c is any constant (the sorted median is
// used) and only makes the FP64 sums short.
//
// Hull building blocks:
//   - below(a, b, c): point b strictly below the segment a -> c.  "not below" is the paper's
//     imminent-collision test y-avg(left) >= y-avg(right) (Sec. 4.1) on blocks [a,b) and [b,c).
//   - leaf hulls: each thread runs the sequential stack algorithm on E consecutive ranks.
//   - bridge(L, R): merging two solved neighbours changes one chain at their junction; the
//     merged cluster [i*, j*] is found by searching for the first left vertex whose rightmost
//     collision crosses the junction (Sec. 4.3 theorem search_collision; Alg. search_collisions
//     Merge and RightmostCollision), with galloping searches so that short bridges cost O(1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wsr {

constexpr int kWave = 64;

// Order-preserving map FP32 -> u32 (IEEE total order on non-NaN values; -0 < +0).
__device__ __forceinline__ uint32_t float_to_key(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_to_float(uint32_t k) {
  uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __uint_as_float(u);
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// LDS arrays indexed by rank are read in blocks of 16 consecutive ranks per thread; one pad
// word per 16 entries spreads those blocks over the LDS banks (unpadded, all lanes of a wave
// would hit the same one or two banks).
__device__ __forceinline__ int rpad(int k) { return k + (k >> 4); }
constexpr int rpad_size(int n) { return n + (n >> 4) + 1; }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// Lanes of the wave holding the same 8-bit digit (all 64 lanes must be active).  Per bit b the
// lanes whose bit differs from this lane's are ballot(b) ^ B, with B = 0 or all ones from this
// lane's bit; the peers are the lanes that differ in no bit.  Each bit costs a sign-extending bit
// extract, a compare for the ballot and one three-input bit operation per mask half.
__device__ __forceinline__ uint64_t match_digit8(uint32_t dg) {
  uint32_t dlo = 0u, dhi = 0u;  // lanes that differ in some bit so far
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint32_t B = (uint32_t)(-(int32_t)((dg >> b) & 1u));
    const uint64_t m = __builtin_amdgcn_uicmp(B, 0u, 33);  // ballot(B != 0): one compare
    dlo |= (uint32_t)m ^ B;
    dhi |= (uint32_t)(m >> 32) ^ B;
  }
  return ~(((uint64_t)dhi << 32) | dlo);
}

// base + i for an index below 2^30 / sizeof(T), formed as a 32-bit byte offset so a uniform base
// stays in scalar registers (one vector address register, no 64-bit vector arithmetic).
template <typename T>
__device__ __forceinline__ T* at_u32(T* base, uint32_t i) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint32_t)(i * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ const T* at_u32(const T* base, uint32_t i) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)(i * (uint32_t)sizeof(T)));
}

// Number of set bits of m at lanes below this one (the mbcnt instructions, which take the mask
// per lane).
__device__ __forceinline__ int popc_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Cross-lane moves through DPP (data-parallel primitives: a VALU operand modifier, no LDS round
// trip).  A lane whose source lane is out of range keeps `old`.  Every lane of the wave must be
// active.  CTRL: 0x110+n row_shr:n (within 16-lane rows), 0x142 row_bcast:15 (lane 15 of a row to
// the next row), 0x143 row_bcast:31 (lane 31 to rows 2 and 3), 0x138 wave_shr:1.
template <int CTRL, int ROW_MASK, typename T>
__device__ __forceinline__ T dpp(T v, T old) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROW_MASK, 0xF, false);
}

// Wave-inclusive scan with an associative op and its identity (Hillis-Steele inside each row of
// 16 lanes, then the row totals; App. A.2).
template <typename T, typename Op>
__device__ __forceinline__ T wave_incl_scan_op(T v, T id, Op op) {
  v = op(v, dpp<0x111, 0xF>(v, id));
  v = op(v, dpp<0x112, 0xF>(v, id));
  v = op(v, dpp<0x114, 0xF>(v, id));
  v = op(v, dpp<0x118, 0xF>(v, id));
  v = op(v, dpp<0x142, 0xA>(v, id));
  v = op(v, dpp<0x143, 0xC>(v, id));
  return v;
}
__device__ __forceinline__ double wave_incl_scan(double v) {
  return wave_incl_scan_op(v, 0.0, [](double a, double b) { return a + b; });
}
__device__ __forceinline__ int wave_incl_scan(int v) {
  return wave_incl_scan_op(v, 0, [](int a, int b) { return a + b; });
}
__device__ __forceinline__ long long wave_incl_scan(long long v) {
  return wave_incl_scan_op(v, 0ll, [](long long a, long long b) { return a + b; });
}
// Wave-uniform sum (the scan's last lane, read into scalar registers).
__device__ __forceinline__ int wave_sum(int v) {
  return __builtin_amdgcn_readlane(wave_incl_scan(v), kWave - 1);
}
// The exclusive form: each lane gets the inclusive value of the lane below (lane 0: id).
template <typename T>
__device__ __forceinline__ T wave_shift_up(T v, T id) {
  return dpp<0x138, 0xF>(v, id);
}
// Wave-uniform min / max (the scan's last lane, read into a scalar register).
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  const uint32_t m = wave_incl_scan_op(v, 0u, [](uint32_t a, uint32_t b) { return a > b ? a : b; });
  return (uint32_t)__builtin_amdgcn_readlane((int)m, kWave - 1);
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  const uint32_t m = wave_incl_scan_op(v, 0xFFFFFFFFu, [](uint32_t a, uint32_t b) { return a < b ? a : b; });
  return (uint32_t)__builtin_amdgcn_readlane((int)m, kWave - 1);
}
// Wave-uniform bitwise OR / AND.
__device__ __forceinline__ uint32_t wave_or_u32(uint32_t v) {
  const uint32_t m = wave_incl_scan_op(v, 0u, [](uint32_t a, uint32_t b) { return a | b; });
  return (uint32_t)__builtin_amdgcn_readlane((int)m, kWave - 1);
}
__device__ __forceinline__ uint32_t wave_and_u32(uint32_t v) {
  const uint32_t m = wave_incl_scan_op(v, 0xFFFFFFFFu, [](uint32_t a, uint32_t b) { return a & b; });
  return (uint32_t)__builtin_amdgcn_readlane((int)m, kWave - 1);
}

// Block-wide exclusive scan; sh must hold NT/64 + 1 values.  Every thread of the block must call.
// Summation order is fixed (waves in order), so results are deterministic.  TRAIL = false leaves
// out the closing barrier: the caller must then not write sh again before another barrier.
template <int NT, typename T, bool TRAIL = true>
__device__ __forceinline__ T block_excl_scan(T v, T* sh, T* total) {
  constexpr int NW = NT / kWave;
  const int lane = lane_id();
  const int wv = threadIdx.x / kWave;
  T inc = wave_incl_scan(v);
  T exc = wave_shift_up(inc, T(0));
  if (lane == kWave - 1) sh[wv] = inc;
  __syncthreads();
  T base = T(0), tot = T(0);
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const T t = sh[w];
    if (w < wv) base += t;
    tot += t;
  }
  if (total) *total = tot;
  if (TRAIL) __syncthreads();
  return base + exc;
}

// block_excl_scan of doubles (no closing barrier, as TRAIL = false) for kernels short of
// registers: the cross-wave sums come from one LDS read per lane and lane reads instead of one
// LDS read per wave held in registers; the summation order is the same, so are the bits.
template <int NT>
__device__ __forceinline__ double block_excl_scan_lean(double v, double* sh, double* total) {
  constexpr int NW = NT / kWave;
  const int lane = lane_id();
  const int wv = threadIdx.x / kWave;
  const double inc = wave_incl_scan(v);
  const double exc = wave_shift_up(inc, 0.0);
  if (lane == kWave - 1) sh[wv] = inc;
  __syncthreads();
  const long long mb = __double_as_longlong(lane < NW ? sh[lane] : 0.0);
  double base = 0.0, tot = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int lo = __builtin_amdgcn_readlane((int)(mb & 0xFFFFFFFFll), w);
    const int hi = __builtin_amdgcn_readlane((int)(mb >> 32), w);
    const double t = __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
    if (w < wv) base += t;
    tot += t;
  }
  if (total) *total = tot;
  return base + exc;
}

// Layouts of LDS arrays indexed by rank (prefix sums S): rank-padded (blocks of 16 ranks per
// thread spread over the banks) or transposed.
struct RankPadded {
  __device__ static __forceinline__ int at(int k) { return rpad(k); }
};
// Transposed: the E ranks of thread t sit E rows apart, rank k at (k mod E)(NT+1) + k/E, so the
// lanes of a wave touching their i-th rank hit consecutive words.  Holds ranks 0..NT*E
// (E*(NT+1) entries).
template <int NT, int E>
struct RankT {
  static_assert((E & (E - 1)) == 0, "E must be a power of two");
  static constexpr int kSize = E * (NT + 1);
  __device__ static __forceinline__ int at(int k) { return (k & (E - 1)) * (NT + 1) + k / E; }
};

// Point b strictly below the segment a -> c (a < b < c); positions are ranks, s* are S values.
__device__ __forceinline__ bool below(int a, double sa, int b, double sb, int c, double sc) {
  return (sb - sa) * (double)(c - b) < (sc - sb) * (double)(b - a);
}

// Sequential stack hull of points lo..hi (inclusive) of S; writes vertex ranks to st, returns count.
template <typename SI>
__device__ __forceinline__ int leaf_hull(const double* S, int lo, int hi, uint16_t* st) {
  int n = 0;
  int p0 = 0, p1 = 0;  // top and second-from-top ranks
  double s0 = 0.0, s1 = 0.0;
  for (int k = lo; k <= hi; ++k) {
    const double sk = S[SI::at(k)];
    while (n >= 2 && !below(p1, s1, p0, s0, k, sk)) {
      --n;  // collision: the top block sticks to the incoming one
      p0 = p1;
      s0 = s1;
      if (n >= 2) {
        p1 = st[n - 2];
        s1 = S[SI::at(p1)];
      }
    }
    st[n++] = (uint16_t)k;
    p1 = p0;
    s1 = s0;
    p0 = k;
    s0 = sk;
  }
  return n;
}

// Generic vertex accessor interface for bridge(): V.pos(i), V.s(i) for the left chain L (indices
// 0..p) and the right chain R (0..q), with L(p) == R(0) the shared junction point.
// Returns the merged chain as L[0..istar] ++ R[jstar..q].  No-bridge result: istar = p, jstar = 1.
template <typename LV, typename RV>
__device__ void bridge(const LV& L, int p, const RV& R, int q, int* istar, int* jstar) {
  if (q <= 0) {  // right chain is a single point: nothing to merge
    *istar = p;
    *jstar = 1;
    return;
  }
  if (p <= 0) {  // left chain is a single point
    *istar = 0;
    *jstar = 1;
    return;
  }
  // Tangent from the point (qa, qs) to R, excluding R(0): first j >= 1 with R(j) strictly below
  // the segment Q -> R(j+1) (j = q when none): the rightmost collision of Q inside R.
  auto tangent = [&](int qa, double qs) -> int {
    auto f = [&](int j) -> bool {
      if (j >= q) return true;
      return below(qa, qs, R.pos(j), R.s(j), R.pos(j + 1), R.s(j + 1));
    };
    int lo = 0, hi = 1, step = 1;
    while (!f(hi)) {
      lo = hi;
      step <<= 1;
      hi = min(lo + step, q);
    }
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (f(mid))
        hi = mid;
      else
        lo = mid;
    }
    return hi;
  };
  // g(i): the rightmost collision of left vertex i crosses the junction.
  auto g = [&](int i, int* jout) -> bool {
    const int li = L.pos(i);
    const double si = L.s(i);
    const int j = tangent(li, si);
    *jout = j;
    return !below(li, si, L.pos(i + 1), L.s(i + 1), R.pos(j), R.s(j));
  };
  // junction survives iff L(p) is strictly below L(p-1) -> R(1)
  if (below(L.pos(p - 1), L.s(p - 1), L.pos(p), L.s(p), R.pos(1), R.s(1))) {
    *istar = p;
    *jstar = 1;
    return;
  }
  int jhi = 1;
  if (!g(p - 1, &jhi)) {  // only reachable through rounding: keep the junction
    *istar = p;
    *jstar = 1;
    return;
  }
  int hi = p - 1, lo = hi - 1, step = 1;
  while (lo >= 0) {
    int j;
    if (!g(lo, &j)) break;
    hi = lo;
    jhi = j;
    step <<= 1;
    lo = hi - step;
  }
  if (lo < 0) lo = -1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    int j;
    if (g(mid, &j)) {
      hi = mid;
      jhi = j;
    } else {
      lo = mid;
    }
  }
  *istar = hi;
  *jstar = jhi;
}

// Chains stored as rank lists in LDS, S read from LDS.
template <typename SI>
struct LdsChain {
  const uint16_t* v;
  const double* S;
  __device__ __forceinline__ int pos(int i) const { return v[i]; }
  __device__ __forceinline__ double s(int i) const { return S[SI::at(v[i])]; }
};

// Lower hull (collinear points dropped) of the points 0..d of S (layout SI), computed by NT
// threads with E ranks per leaf.  vert must hold NT*(E+1) entries, cnt and mres NT counts each
// (CT: a signed type holding -1..NT*E+1).  On return vert[0..cnt[0]) are the hull vertices (0
// and d included).  All threads of the block must call; requires 1 <= d <= NT*E.
template <int NT, int E, typename SI, typename CT>
__device__ void tile_hull(const double* S, int d, uint16_t* vert, CT* cnt, CT* mres) {
  constexpr int CP = E / 2 + 1;  // copy entries per thread per level
  const int t = threadIdx.x;
  const int nleaf = (d + E - 1) / E;
  if (t < nleaf) {
    const int a = t * E;
    const int b = min(a + E, d);
    cnt[t] = (CT)leaf_hull<SI>(S, a, b, vert + t * (E + 1));
  }
  __syncthreads();
  for (int lvl = 1; (1 << (lvl - 1)) < nleaf; ++lvl) {
    const int half = 1 << (lvl - 1);
    const int nmerge = (nleaf + (1 << lvl) - 1) >> lvl;
    if (t < nmerge) {
      const int lleaf = t << lvl;
      const int rleaf = lleaf + half;
      int istar = -1, jstar = -1;
      if (rleaf < nleaf) {
        LdsChain<SI> L{vert + lleaf * (E + 1), S};
        LdsChain<SI> R{vert + rleaf * (E + 1), S};
        bridge(L, cnt[lleaf] - 1, R, cnt[rleaf] - 1, &istar, &jstar);
      }
      mres[2 * t] = (CT)istar;
      mres[2 * t + 1] = (CT)jstar;
    }
    __syncthreads();
    // move the surviving right part next to the surviving left part (read all, then write)
    const int m = t >> lvl;
    const int s = t & ((1 << lvl) - 1);
    int istar = -1, jstar = 0, len = 0;
    if (m < nmerge) {
      istar = mres[2 * m];
      jstar = mres[2 * m + 1];
      if (istar >= 0) len = cnt[(m << lvl) + half] - jstar;
    }
    const int lbase = (m << lvl) * (E + 1);
    const int rbase = lbase + half * (E + 1);
    uint16_t tmp[CP];
#pragma unroll
    for (int r = 0; r < CP; ++r) {
      const int e = s + (r << lvl);
      if (e < len) tmp[r] = vert[rbase + jstar + e];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < CP; ++r) {
      const int e = s + (r << lvl);
      if (e < len) vert[lbase + istar + 1 + e] = tmp[r];
    }
    if (s == 0 && istar >= 0) cnt[m << lvl] = (CT)(istar + 1 + len);
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------- ImminentCollisions
// (kIcaRounds, the default number of rounds tried before the hull merge, is in wsr_kernels.h.)

// A candidate vertex: rank position and its S value; pos < 0 means "none".
struct Cand {
  int pos;
  double s;
};

// Per thread, the last candidate held by lower threads (lc) and the first candidate held by
// higher threads (rc, default dflt), and the OR of `flag` over the block (returned).  mineL /
// mineR are the thread's own last / first candidate (pos < 0: none; both or neither).  Inside a
// wave the nearest lanes holding one are found from a ballot and read directly; across waves
// through shL / shR / shF (NT/64 entries each).  One barrier; the caller alternates between two
// sets of exchange slots on consecutive calls (a wave may write the next call's slots while
// others still read this call's).  All threads must call.
template <int NT>
__device__ __forceinline__ bool carry_exchange(Cand mineL, Cand mineR, bool flag, Cand dflt, Cand* shL, Cand* shR,
                                               int* shF, Cand* lc, Cand* rc) {
  constexpr int NW = NT / kWave;
  const int lane = lane_id();
  const int wv = threadIdx.x / kWave;
  const uint64_t has = __ballot(mineL.pos >= 0);
  const uint64_t lower = has & lanemask_lt();
  const uint64_t upper = lane == kWave - 1 ? 0ull : has & (~0ull << (lane + 1));
  const int src_l = lower ? 63 - __clzll((long long)lower) : lane;
  const int src_r = upper ? __ffsll((unsigned long long)upper) - 1 : lane;
  Cand l, r;
  l.pos = __shfl(mineL.pos, src_l, kWave);
  l.s = __shfl(mineL.s, src_l, kWave);
  r.pos = __shfl(mineR.pos, src_r, kWave);
  r.s = __shfl(mineR.s, src_r, kWave);
  if (!lower) l.pos = -1;
  if (!upper) r.pos = -1;
  // the wave's last and first candidates and its flag, for the other waves
  const bool wflag = __ballot(flag) != 0ull;
  if (has) {
    if (lane == 63 - __clzll((long long)has)) shL[wv] = mineL;
    if (lane == __ffsll((unsigned long long)has) - 1) shR[wv] = mineR;
  } else if (lane == 0) {
    shL[wv] = Cand{-1, 0.0};
    shR[wv] = Cand{-1, 0.0};
  }
  if (lane == 0) shF[wv] = wflag ? 1 : 0;
  __syncthreads();
  if (l.pos < 0)
    for (int w = wv - 1; w >= 0; --w)
      if (shL[w].pos >= 0) {
        l = shL[w];
        break;
      }
  if (r.pos < 0)
    for (int w = wv + 1; w < NW; ++w)
      if (shR[w].pos >= 0) {
        r = shR[w];
        break;
      }
  if (r.pos < 0) r = dflt;
  int any = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) any |= shF[w];
  *lc = l;
  *rc = r;
  return any != 0;
}

// Candidates of b next to the removed points rem (within the thread; b and rem disjoint): for
// each removed point, the nearest surviving candidate on either side.  A candidate's collision
// test can only change when one of its neighbouring candidates changed.  No loop: adding rem to
// ~b starts a carry at every removed bit that runs through the non-candidate bits and enters
// the next candidate above (the carry-in bits are sum ^ a ^ b); the same on the bit-reversed
// masks gives the next candidate below.
__device__ __forceinline__ uint32_t ica_neighbours(uint32_t b, uint32_t rem) {
  const uint32_t m = ~b;
  const uint32_t up = ((m + rem) ^ m ^ rem) & b;
  const uint32_t rb = __builtin_bitreverse32(b), rr = __builtin_bitreverse32(rem);
  const uint32_t mr = ~rb;
  const uint32_t dn = __builtin_bitreverse32(((mr + rr) ^ mr ^ rr) & rb);
  return up | dn;
}

// One wave's boundary in the collision exchange: its first and last candidates, the neighbours
// outside the wave its last sweeps assumed, and whether its sweeps overflowed.
struct WaveBound {
  Cand first, last;
  int lassume, rassume;
  int overflow;
};

// ImminentCollisions (Sec. 4.1; Alg. imminent_collisions_v2) on hull candidates: thread t owns
// points k0 = t*E .. k0+E-1 (bit i of *bm = point k0+i is a candidate), point d is the fixed
// right end.  A candidate is removed when it is not strictly below the segment joining its
// neighbouring candidates (the blocks on either side collide: avg y left >= avg y right).
//
// The order of removals does not change the result: a point that is not strictly below the
// segment joining any point on its left and any point on its right is no vertex of the lower
// hull, so it may be removed whatever the other candidates are, and the process stops at the
// hull (collinear points dropped) whatever the order.  Only the final check needs the exact
// neighbours.  Hence:
//   1. a first round with every point a candidate (neighbours = adjacent ranks, the test is
//      y_{k-1} >= y_k), in registers;
//   2. sweeps inside each wave, without barriers, with the neighbours outside the wave taken as
//      last known; a removal re-tests the thread's neighbouring candidates at once, a changed
//      carry re-tests the thread's first / last candidate, until a sweep removes no thread's
//      first or last candidate (then no carry changes);
//   3. one block exchange of the waves' first and last candidates: when no wave assumed wrong
//      outside neighbours, every candidate was tested against its exact neighbours and the
//      candidates are the hull; otherwise the waves sweep again with the exact neighbours.
// Returns true on convergence within max_rounds exchanges (*lc / *rc = the thread's carries:
// last candidate before k0, first candidate after its ranks or the end point d), false when the
// rounds or the sweeps run out (the caller merges hulls instead).  sv[0..E] are this thread's S
// values; S is the LDS copy (layout SI); xs holds 2*NT/64 entries.  All threads must call.
template <int NT, int E, typename SI>
__device__ bool ica_rounds(const double* S, const double (&sv)[E + 1], int d, int max_rounds, uint32_t* bm,
                           Cand* lc, Cand* rc, WaveBound* xs) {
  constexpr int NW = NT / kWave;
  constexpr int kSweepMax = 32;
  const int lane = lane_id();
  const int wv = threadIdx.x / kWave;
  const int k0 = threadIdx.x * E;
  const int wk0 = wv * kWave * E;
  const Cand dflt{d, S[SI::at(d)]};
  uint32_t valid = 0;
#pragma unroll
  for (int i = 0; i < E; ++i) valid |= (k0 + i < d ? 1u : 0u) << i;
  // 1. adjacent neighbours
  uint32_t rem = 0;
  {
    double dl = sv[0] - S[SI::at(max(k0 - 1, 0))];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const double dr = sv[i + 1] - sv[i];
      if (((valid >> i) & 1u) && (k0 + i > 0) && !(dl < dr)) rem |= 1u << i;
      dl = dr;
    }
  }
  uint32_t b = valid & ~rem;
  uint32_t todo = rem ? ica_neighbours(b, rem) : 0u;
  int lprev = k0 - 1;  // neighbours the first round used outside the thread
  int rprev = min(k0 + E, d);
  // outside neighbours of the wave: the adjacent ranks to begin with (any point is a valid
  // test point for removals)
  Cand wl{-1, 0.0}, wr = dflt;
  if (wk0 > 0 && wk0 <= d) wl = Cand{wk0 - 1, S[SI::at(wk0 - 1)]};
  if (wk0 + kWave * E < d) wr = Cand{wk0 + kWave * E, S[SI::at(wk0 + kWave * E)]};
  Cand l{-1, 0.0}, r = dflt, mineL{-1, 0.0}, mineR{-1, 0.0};
  bool lout = true, rout = true;  // the lane's l / r came from outside the wave in the last sweep
  for (int round = 0; round < max_rounds; ++round) {
    // 2. sweeps inside the wave
    int overflow = 0;
    for (int sweep = 0;; ++sweep) {
      mineL = Cand{-1, 0.0};
      mineR = Cand{-1, 0.0};
      if (b) {
        const int hi = 31 - __clz(b);
        const int lo = __ffs(b) - 1;
        mineL = Cand{k0 + hi, S[SI::at(k0 + hi)]};
        mineR = Cand{k0 + lo, S[SI::at(k0 + lo)]};
      }
      const uint64_t has = __ballot(mineL.pos >= 0);
      const uint64_t lower = has & lanemask_lt();
      const uint64_t upper = lane == kWave - 1 ? 0ull : has & (~0ull << (lane + 1));
      const int src_l = lower ? 63 - __clzll((long long)lower) : lane;
      const int src_r = upper ? __ffsll((unsigned long long)upper) - 1 : lane;
      l.pos = __shfl(mineL.pos, src_l, kWave);
      l.s = __shfl(mineL.s, src_l, kWave);
      r.pos = __shfl(mineR.pos, src_r, kWave);
      r.s = __shfl(mineR.s, src_r, kWave);
      lout = !lower;
      rout = !upper;
      if (lout) l = wl;
      if (rout) r = wr;
      if (b) {
        if (l.pos != lprev) todo |= b & (0u - b);
        if (r.pos != rprev) todo |= 1u << (31 - __clz(b));
      }
      lprev = l.pos;
      rprev = r.pos;
      todo &= b;
      rem = 0;
      const uint32_t edges = b ? ((b & (0u - b)) | (1u << (31 - __clz(b)))) : 0u;
      while (todo) {
        const int i = __ffs(todo) - 1;
        todo &= todo - 1u;
        const uint32_t below_i = b & ((1u << i) - 1u);
        const uint32_t above_i = b & ~((2u << i) - 1u);
        const int pp = below_i ? k0 + 31 - __clz(below_i) : l.pos;
        const int np = above_i ? k0 + __ffs(above_i) - 1 : r.pos;
        const double sp = below_i ? S[SI::at(pp)] : l.s;
        const double sn = above_i ? S[SI::at(np)] : r.s;
        if (pp >= 0 && !below(pp, sp, k0 + i, S[SI::at(k0 + i)], np, sn)) {
          b &= ~(1u << i);
          rem |= 1u << i;
          todo |= ica_neighbours(b, 1u << i);  // cascade inside the thread at once
        }
      }
      // no thread lost its first or last candidate: no carry changed, nothing left to test
      if (__ballot((rem & edges) != 0) == 0ull) break;
      if (sweep >= kSweepMax) {
        overflow = 1;
        break;
      }
    }
    // 3. exchange of wave boundaries (mineL / mineR are those of the final candidates)
    WaveBound* x = xs + (round & 1) * NW;
    const uint64_t has = __ballot(mineL.pos >= 0);
    if (has) {
      if (lane == 63 - __clzll((long long)has)) x[wv].last = mineL;
      if (lane == __ffsll((unsigned long long)has) - 1) x[wv].first = mineR;
    } else if (lane == 0) {
      x[wv].last = Cand{-1, 0.0};
      x[wv].first = Cand{-1, 0.0};
    }
    if (lane == 0) {
      x[wv].lassume = wl.pos;
      x[wv].rassume = wr.pos;
      x[wv].overflow = overflow;
    }
    __syncthreads();
    // lane j < NW takes wave j: its exact outside neighbours are the last candidate of the
    // nearest lower wave holding any and the first of the nearest higher one (else d)
    const bool in = lane < NW;
    const WaveBound e = x[in ? lane : 0];
    const bool holds = in && e.last.pos >= 0;
    const uint64_t hm = __ballot(holds);
    const uint64_t lw = hm & lanemask_lt();
    const uint64_t uw = lane == kWave - 1 ? 0ull : hm & (~0ull << (lane + 1));
    const int sl = lw ? 63 - __clzll((long long)lw) : lane;
    const int sr = uw ? __ffsll((unsigned long long)uw) - 1 : lane;
    Cand exl{__shfl(e.last.pos, sl, kWave), __shfl(e.last.s, sl, kWave)};
    Cand exr{__shfl(e.first.pos, sr, kWave), __shfl(e.first.s, sr, kWave)};
    if (!lw) exl = Cand{-1, 0.0};
    if (!uw) exr = dflt;
    const bool wrong = __ballot(holds && (e.lassume != exl.pos || e.rassume != exr.pos)) != 0ull;
    const bool ovf = __ballot(in && e.overflow != 0) != 0ull;
    wl = Cand{__shfl(exl.pos, wv, kWave), __shfl(exl.s, wv, kWave)};
    wr = Cand{__shfl(exr.pos, wv, kWave), __shfl(exr.s, wv, kWave)};
    if (ovf) break;
    if (!wrong) {
      // the check above covers the waves holding candidates; a wave holding none may have swept
      // with stale outside neighbours (a lower wave's last candidate removed in this round), and
      // its lanes' values use them: every lane whose neighbour lies outside its wave takes the
      // exact one just exchanged
      if (lout) l = wl;
      if (rout) r = wr;
      *bm = b;
      *lc = l;
      *rc = r;
      return true;
    }
  }
  *bm = b;
  return false;
}

// The E entries a[k0 .. k0+E) of a flat u16 array (k0 a multiple of 8), read as 16-byte words.
template <int E>
__device__ __forceinline__ void load_u16_block(const uint16_t* a, int k0, uint16_t (&v)[E]) {
  static_assert(E % 8 == 0, "E must be a multiple of 8");
#pragma unroll
  for (int q = 0; q < E / 8; ++q) {
    const uint4 w = *reinterpret_cast<const uint4*>(a + k0 + 8 * q);
    const uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      v[8 * q + 2 * j] = (uint16_t)(u[j] & 0xFFFFu);
      v[8 * q + 2 * j + 1] = (uint16_t)(u[j] >> 16);
    }
  }
}

// num / n for a rank count 1 <= n <= 2^26: the hardware FP64 reciprocal refined by one
// Newton-Raphson step (relative error ~1e-16, far below the FP32 rounding of the results).
__device__ __forceinline__ double div_count(double num, int n) {
  const double dn = (double)n;
  double r = __builtin_amdgcn_rcp(dn);
  r = r * __builtin_fma(-dn, r, 2.0);
  return num * r;
}

// The E entries a[k0 .. k0+E) of a flat u32 array (k0 a multiple of 4), read as 16-byte words.
template <int E>
__device__ __forceinline__ void load_u32_block(const uint32_t* a, int k0, uint32_t (&v)[E]) {
  static_assert(E % 4 == 0, "E must be a multiple of 4");
#pragma unroll
  for (int q = 0; q < E / 4; ++q) {
    const uint4 w = *reinterpret_cast<const uint4*>(a + k0 + 4 * q);
    v[4 * q] = w.x;
    v[4 * q + 1] = w.y;
    v[4 * q + 2] = w.z;
    v[4 * q + 3] = w.w;
  }
}

// Output of a cluster: its FP64 value rounded to FP32 (prox_{lam R}).
struct PlainValue {
  __device__ __forceinline__ float operator()(double u, int, int) const { return (float)u; }
};

// Output of a cluster of ranks [a, b) under Alg. prox's l1 and rewinding lines (prox of
// lam*R + beta*l1, rewinding rho, rewinding line scaled by kappa): u is the cluster's
// prox_{lam R} value, its mean velocity is v = lam (d - a - b)/(d - 1) and its mean weight
// x = u - v.  The cluster is zeroed when |u| < beta, else it gets
//   x + kappa (1 - rho)(v - beta sign(u)) = u - q v - kappa (1 - rho) beta sign(u),
// q = 1 - kappa (1 - rho), evaluated in the second form (at u == 0 the sign term matters only
// when beta == 0, where it vanishes).  kappa = 1 is Alg. prox; kappa = eta is the variant with
// the learning rate on the rewinding line.  FP64, one rounding.
struct L1Rewind {
  double beta, q, omb;
  __host__ __device__ L1Rewind(float b, float r, float k)
      : beta(b), q(1.0 - (double)k * (1.0 - (double)r)), omb((double)k * (1.0 - (double)r) * (double)b) {}
  __device__ __forceinline__ float operator()(double u, double v) const {
    const double r = fma(-q, v, u) - (u > 0.0 ? omb : -omb);
    return fabs(u) < beta ? 0.0f : (float)r;
  }
};
struct L1Value {
  L1Rewind f;
  double lamd;  // lam / (d - 1)
  int d;
  __device__ __forceinline__ float operator()(double u, int a, int b) const {
    return f(u, lamd * (double)(d - a - b));
  }
};

// Cluster value of every rank owned by this thread from its final cluster starts: bm (bit i =
// rank k0+i starts a cluster), sv[0..E] (S at k0..k0+E), carries lc (last start before k0) and
// rc (first start after the thread's ranks, or the end point d).  Rank k0+i gets
// fin(offset + (S_b - S_a) / (b - a), a, b) for its cluster [a, b); res[ix[i]] receives it (ix:
// the original indices of the thread's ranks).  The next cluster start is carried down a register
// sweep, so no S value is read from LDS.
template <int E, typename Fin = PlainValue>
__device__ __forceinline__ void walk_values(uint32_t bm, const double (&sv)[E + 1], Cand lc, Cand rc, int d,
                                            double offset, const uint16_t (&ix)[E], float* res,
                                            Fin fin = Fin()) {
  const int k0 = threadIdx.x * E;
  if (k0 >= d) return;
  float val[E];
  int np = rc.pos;
  double sn = rc.s;
#pragma unroll
  for (int i = E - 1; i >= 0; --i) {
    val[i] = fin(offset + div_count(sn - sv[i], np - (k0 + i)), k0 + i, np);
    if ((bm >> i) & 1u) {
      np = k0 + i;
      sn = sv[i];
    }
  }
  // (np, sn) is now the first start in the thread's ranks (or rc): it closes the entering cluster
  float cur = lc.pos >= 0 ? fin(offset + div_count(sn - lc.s, np - lc.pos), lc.pos, np) : 0.0f;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    if ((bm >> i) & 1u) cur = val[i];
    if (k0 + i < d) res[ix[i]] = cur;
  }
}

// Write the local cluster-start bits of one segment (or tile) to the global bit mask.
// lmask bit j <-> flat position (base & ~31) + j.  Words shared with a neighbour are OR-ed
// atomically (the global mask is zeroed before the forward pass); owned words are stored.
template <int NT>
__device__ __forceinline__ void store_mask_words(uint32_t* mask, int64_t base, int n,
                                                 const uint32_t* lmask) {
  const int off = (int)(base & 31);
  const int nwords = (off + n + 31) >> 5;
  const int64_t g0 = base >> 5;
  const bool first_partial = off != 0;
  const bool last_partial = ((off + n) & 31) != 0;
  for (int j = threadIdx.x; j < nwords; j += NT) {
    const uint32_t v = lmask[j];
    if ((j == 0 && first_partial) || (j == nwords - 1 && last_partial))
      atomicOr(&mask[g0 + j], v);
    else
      mask[g0 + j] = v;
  }
}

}  // namespace wsr
