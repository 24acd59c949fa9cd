// wsr_big.hip -- prox_{lam R} of one segment longer than a workgroup can hold (d > 8192).
//
// Pipeline (every step a kernel on the caller's stream, no host round trip):
//   1. device-wide stable LSD radix sort of (u32 key, i32 index), 4 passes of 8 bits:
//      per-tile digit histograms, per-digit scan over tiles, stable in-tile ranking + scatter
//      (Alg. prox "sort"; the paper notes that sorting bounds the whole prox, Sec. 4);
//   2. per tile of T ranks: centred FP64 prefix sums and the tile's lower hull in LDS
//      (the same leaf + bridge machinery as the short-segment kernel);
//   3. scan of tile sums (global S offsets);
//   4. cross-tile merges: a binary tree over tiles; merging two solved neighbours changes only
//      the chain at their junction, found with the Sec. 4.3 search (theorem search_collision,
//      Alg. search_collisions Merge), so the tree has log2(#tiles) levels of O(log) searches.
//      Each tile keeps the contiguous range ("own range") of its hull vertices that survives;
//      a node's chain is its left end point followed by the own ranges of its tiles;
//   5. per tile: previous / next surviving vertex, then values c + (S_b - S_a)/(b - a),
//      scattered to the original order, plus cluster-start bits.
// The backward pass gathers the upstream gradient in rank order, forms FP64 prefix sums and
// averages over each saved cluster (clusters may span tiles).
#include "wsr_device.h"
#include "wsr_big.h"

namespace wsr {

// ------------------------------------------------------------------------------- radix sort

// Persistent radix kernels walk their tiles in XCD-contiguous order.  Workgroup b runs on XCD
// b % 8 (the dispatcher deals workgroups to the eight XCDs in turn); the workgroups of one XCD
// share one contiguous eighth of the tiles, so the tiles in flight on an XCD are neighbours and
// the partial cache lines where their output runs meet are completed in that XCD's L2 rather than
// written back in pieces from several XCDs.  The grid is a multiple of 8 (chosen by the host).
__device__ __forceinline__ void xcd_tiles(int ntiles, int* first, int* end, int* step) {
  const int x = (int)(blockIdx.x & 7u), j = (int)(blockIdx.x >> 3), gx = (int)(gridDim.x >> 3);
  *first = (int)((int64_t)x * ntiles / 8) + j;
  *end = (int)((int64_t)(x + 1) * ntiles / 8);
  *step = gx;
}

// Buffers of sort pass `pass`.  The first pass's row scan stores in flags[1] the key bits that
// vary over the segment; a later pass whose 8-bit digit is the same for every key would move
// nothing and is skipped.  Of the passes that run, the last writes the final keys (kA) and the
// permutation (vfinal); the others alternate so that each reads what the previous one wrote.
struct RadixBufs {
  const uint32_t* ksrc;  // null: the first pass reads the FP32 weights
  const int32_t* vsrc;
  uint32_t* kdst;
  int32_t* vdst;
  bool run;
};
__device__ __forceinline__ bool radix_pass_runs(int pass, uint32_t varying) {
  return pass == 0 || ((varying >> (8 * pass)) & 255u) != 0u;
}
__device__ __forceinline__ RadixBufs radix_bufs(int pass, uint32_t varying, uint32_t* kA, uint32_t* kB, int32_t* vA,
                                                int32_t* vB, int32_t* vfinal) {
  int n = 0, j = 0;
  for (int p = 0; p < 4; ++p) {
    if (!radix_pass_runs(p, varying)) continue;
    if (p == pass) j = n;
    ++n;
  }
  RadixBufs b{nullptr, nullptr, nullptr, nullptr, radix_pass_runs(pass, varying)};
  if (!b.run) return b;
  // the i-th pass that runs writes the A buffers when n - 1 - i is even (so the last one writes A)
  auto writes_a = [&](int i) { return ((n - 1 - i) & 1) == 0; };
  if (j > 0) {
    const bool a = writes_a(j - 1);
    b.ksrc = a ? kA : kB;
    b.vsrc = a ? vA : vB;
  }
  const bool a = writes_a(j);
  b.kdst = a ? kA : kB;
  b.vdst = j == n - 1 ? vfinal : (a ? vA : vB);
  return b;
}

// Sort buffers of segment sg for pass `pass` (the segment's slices of the workspace arrays; the
// final permutation goes to the caller's saved perm when there is one).
__device__ __forceinline__ RadixBufs seg_radix_bufs(int pass, const LongSeg& sg, uint32_t varying, uint32_t* kA,
                                                    uint32_t* kB, int32_t* vA, int32_t* vB, int32_t* saved_perm) {
  int32_t* vfinal = saved_perm ? saved_perm + sg.start : vA + sg.ebase;
  return radix_bufs(pass, varying, kA + sg.ebase, kB + sg.ebase, vA + sg.ebase, vB + sg.ebase, vfinal);
}

// First-pass input word of element i of a segment: the FP32 weight's bits, or (GRAD) those of
// the proximal-gradient step fmaf(-eta, grad, w) (one rounding).
template <bool GRAD>
__device__ __forceinline__ uint32_t input_bits(const float* w, const float* grad, float eta, uint32_t i) {
  const float x = *at_u32(w, i);
  if constexpr (GRAD) return __float_as_uint(__builtin_fmaf(-eta, *at_u32(grad, i), x));
  return __float_as_uint(x);
}

// Per-tile histogram of one 8-bit digit, written digit-major (hist[digit * nrt + tile], over the
// radix tiles of the whole set; the tiles in flight on one XCD are neighbours, so their counts of
// a digit fill whole cache lines).  Source: the FP32 weights or step inputs (first pass: keys made
// on the fly, non-finite values flagged, and the OR and AND of the tile's keys kept for the
// varying-bits mask) or the keys the previous pass wrote.  Persistent: each workgroup has its
// next tile's words in flight while it counts the current one, so the loads of one tile overlap
// the LDS atomics of another.
template <bool GRAD>
__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(int pass, LongSet set, const float* w,
                                                             const float* grad, float eta, uint32_t* kA,
                                                             uint32_t* kB, int32_t* vA, int32_t* vB,
                                                             int32_t* saved_perm, uint32_t* hist, uint32_t* tbad,
                                                             uint32_t* tor, uint32_t* tand, const uint32_t* flags) {
  constexpr int IPT = kRadixTile / kRadixThreads;
  constexpr int NW = kRadixThreads / kWave;
  constexpr int kHistLanes = 16;
  constexpr int kSub = kWave / kHistLanes;  // sub-histograms per wave
  const int shift = 8 * pass;
  const bool first = pass == 0;
  // one pad word per sub-histogram: the same digit in different lane groups falls on different
  // LDS banks
  __shared__ uint32_t h[NW * kSub][257];
  __shared__ uint32_t red[2][NW];
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wv = tid / kWave;
  for (int j = lane; j < 256 * kSub; j += kWave) h[wv * kSub + j / 256][j % 256] = 0u;
  // the tile's segment, its element count and whether this pass runs for it
  auto tile_info = [&](int tile, const uint32_t** src, uint32_t* nt) -> bool {
    const LongSeg& sg = set.seg(set.seg_of_rtile(tile));
    const int64_t base = (int64_t)(tile - sg.rbase) * kRadixTile;
    *nt = (uint32_t)min((int64_t)kRadixTile, sg.d - base);
    if (first) {
      *src = nullptr;
      return true;
    }
    const RadixBufs b = seg_radix_bufs(pass, sg, flags[kSegFlagWords * set.seg_of_rtile(tile) + 1], kA, kB, vA,
                                       vB, saved_perm);
    *src = b.ksrc + base;
    return b.run;
  };
  // raw 32-bit words of a tile (input bits or keys), all in flight at once: uniform tile base,
  // 32-bit offsets; words past the end of the segment are never counted
  auto load = [&](int tile, uint32_t (&wd)[IPT]) {
    const uint32_t* st;
    uint32_t nt;
    if (!tile_info(tile, &st, &nt)) return;
    if (first) {
      const LongSeg& sg = set.seg(set.seg_of_rtile(tile));
      const uint32_t b0 = (uint32_t)((tile - sg.rbase) * kRadixTile);
      const float* ws = w + sg.start;
      const float* gs = GRAD ? grad + sg.start : nullptr;
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const uint32_t p = (uint32_t)(r * kRadixThreads + tid);
        wd[r] = p < nt ? input_bits<GRAD>(ws, gs, eta, b0 + p) : 0u;
      }
      return;
    }
    if (nt == (uint32_t)kRadixTile) {  // full tile: no bounds checks
#pragma unroll
      for (int r = 0; r < IPT; ++r) wd[r] = st[r * kRadixThreads + tid];
    } else {
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const uint32_t p = (uint32_t)(r * kRadixThreads + tid);
        wd[r] = p < nt ? st[p] : 0u;
      }
    }
  };
  int tile, tend, tstep;
  xcd_tiles(set.nrt, &tile, &tend, &tstep);
  uint32_t word[IPT];
  if (tile < tend) load(tile, word);
  for (; tile < tend; tile += tstep) {
    const uint32_t* unused;
    uint32_t nt;
    const bool run = tile_info(tile, &unused, &nt);
    uint32_t wn[IPT];
    const int next = tile + tstep;
    if (next < tend) load(next, wn);
    if (run) {  // uniform over the workgroup
      int bad = 0;
      uint32_t kor = 0u, kand = 0xFFFFFFFFu;
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const uint32_t p = (uint32_t)(r * kRadixThreads + tid);
        const bool in = p < nt;
        uint32_t key = word[r];
        if (first) {
          const float f = __uint_as_float(key);
          bad |= in && !isfinite(f);
          key = float_to_key(f);
          kor |= in ? key : 0u;
          kand &= in ? key : 0xFFFFFFFFu;
        }
        // each group of kHistLanes lanes counts into its own sub-histogram, so a skewed digit
        // (the top byte of most inputs, long runs in sorted data) puts at most kHistLanes lanes
        // on one address; keys past the end of the segment count into the pad word (never read).
        // No branch per key.
        const uint32_t dg = in ? (key >> shift) & 255u : 256u;
        atomicAdd(&h[wv * kSub + lane / kHistLanes][dg], 1u);
      }
      if (first) {
        // first pass: every tile's non-finite flag and key OR / AND are written each call (no
        // clearing launch)
        kor = wave_or_u32(kor);
        kand = wave_and_u32(kand);
        if (lane == 0) {
          red[0][wv] = kor;
          red[1][wv] = kand;
        }
        const int any = __syncthreads_or(bad);
        if (tid == 0) {
          uint32_t o = 0u, a = 0xFFFFFFFFu;
          for (int q = 0; q < NW; ++q) {
            o |= red[0][q];
            a &= red[1][q];
          }
          tbad[tile] = any ? 1u : 0u;
          tor[tile] = o;
          tand[tile] = a;
        }
      } else {
        __syncthreads();
      }
      for (int j = tid; j < 256; j += kRadixThreads) {
        uint32_t c = 0;
#pragma unroll
        for (int q = 0; q < NW * kSub; ++q) {
          c += h[q][j];
          h[q][j] = 0u;
        }
        hist[(int64_t)j * set.nrt + tile] = c;
      }
      __syncthreads();  // the sub-histograms are clear (and red is free) for the next tile
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r) word[r] = wn[r];
  }
}

// Exclusive scan of one digit's row of tile counts over one segment's tiles (workgroup (digit,
// segment)); row total out.  The row goes through LDS so global reads and writes are coalesced.
// For the first pass (pass == 0) the digit-0 workgroup of each segment also folds the tiles'
// non-finite flags into the segment's flags[0] and their key OR / AND into its varying-bits mask
// flags[1] (plain stores: every call writes them); a later pass whose digit does not vary over
// the segment returns at once.
__global__ __launch_bounds__(256) void k_radix_rowscan(int pass, LongSet set, uint32_t* hist, uint32_t* totals,
                                                       const uint32_t* tbad, const uint32_t* tor,
                                                       const uint32_t* tand, uint32_t* flags) {
  __shared__ uint32_t row_s[kMaxRadixTiles];
  __shared__ int sh[256 / kWave + 1];
  __shared__ uint32_t ored[2][256 / kWave];
  const int digit = blockIdx.x;
  const int si = blockIdx.y;
  const LongSeg& sg = set.seg(si);
  uint32_t* sflags = flags + kSegFlagWords * si;
  if (pass > 0 && !radix_pass_runs(pass, sflags[1])) return;
  const int ntiles = sg.nrt;
  // global reads in batches of U per thread, all in flight together (a plain strided loop waits
  // for each load before the next); indexes past the row end read its last entry again, so every
  // load is unconditional and in bounds
  constexpr int U = 8;
  if (pass == 0 && digit == 0) {
    uint32_t any = 0u, o = 0u, a = 0xFFFFFFFFu;
    for (int i0 = threadIdx.x; i0 < ntiles; i0 += 256 * U) {
      uint32_t fb[U], fo[U], fa[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = sg.rbase + min(i0 + u * 256, ntiles - 1);  // OR / AND: a repeat changes nothing
        fb[u] = tbad[i];
        fo[u] = tor[i];
        fa[u] = tand[i];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        any |= fb[u];
        o |= fo[u];
        a &= fa[u];
      }
    }
    o = wave_or_u32(o);
    a = wave_and_u32(a);
    if (lane_id() == 0) {
      ored[0][threadIdx.x / kWave] = o;
      ored[1][threadIdx.x / kWave] = a;
    }
    any = __syncthreads_or(any != 0u);
    if (threadIdx.x == 0) {
      uint32_t wo = 0u, wa = 0xFFFFFFFFu;
      for (int q = 0; q < 256 / kWave; ++q) {
        wo |= ored[0][q];
        wa &= ored[1][q];
      }
      sflags[0] = any ? 1u : 0u;
      sflags[1] = wo ^ wa;
    }
  }
  uint32_t* row = hist + (int64_t)digit * set.nrt + sg.rbase;
  for (int i0 = threadIdx.x; i0 < ntiles; i0 += 256 * U) {
    uint32_t v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = row[min(i0 + u * 256, ntiles - 1)];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * 256;
      if (i < ntiles) row_s[i] = v[u];
    }
  }
  __syncthreads();
  const int chunk = (ntiles + 255) / 256;
  const int lo = threadIdx.x * chunk;
  const int hi = min(lo + chunk, ntiles);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += (int)row_s[i];
  int total;
  int run = block_excl_scan<256, int>(s, sh, &total);
  for (int i = lo; i < hi; ++i) {
    const int c = (int)row_s[i];
    row_s[i] = (uint32_t)run;
    run += c;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ntiles; i += 256) row[i] = row_s[i];
  if (threadIdx.x == 0) totals[256 * si + digit] = (uint32_t)total;
}

// Items of one tile in wave-striped order (p = wave*64*IPT + r*64 + lane); keys past the end
// of the segment are 0xFFFFFFFF (they sort last and are never written).  In the first pass the
// input bits are loaded (past the end: 0x7FFFFFFF, whose key is 0xFFFFFFFF) and made keys by
// radix_raw_to_key when the tile is used, so a prefetch does not wait for its loads.
template <int IPT, bool GRAD>
__device__ __forceinline__ void radix_load_tile(const float* wsrc, const float* gsrc, float eta,
                                                const uint32_t* ksrc, const int32_t* vsrc, int64_t n, int ltile,
                                                uint32_t (&k)[IPT], int32_t (&v)[IPT]) {
  const uint32_t p0 = (threadIdx.x / kWave) * kWave * IPT + lane_id();
  const int64_t base = (int64_t)ltile * kRadixTile;
  const uint32_t nt = (uint32_t)min((int64_t)kRadixTile, n - base);
  const bool full = nt == (uint32_t)kRadixTile;
  // tile base pointers are uniform; per-item offsets are 32-bit
  if (wsrc) {
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      const uint32_t p = p0 + r * kWave;
      k[r] = (full || p < nt) ? input_bits<GRAD>(wsrc, gsrc, eta, (uint32_t)base + p) : 0x7FFFFFFFu;
      v[r] = (int32_t)(base + p);
    }
  } else {
    const uint32_t* kt = ksrc + base;
    const int32_t* vt = vsrc + base;
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      const uint32_t p = p0 + r * kWave;
      k[r] = (full || p < nt) ? kt[p] : 0xFFFFFFFFu;
      v[r] = (full || p < nt) ? vt[p] : 0;
    }
  }
}

template <int IPT>
__device__ __forceinline__ void radix_raw_to_key(bool raw, uint32_t (&k)[IPT]) {
  if (raw) {
#pragma unroll
    for (int r = 0; r < IPT; ++r) k[r] = float_to_key(__uint_as_float(k[r]));
  }
}

// Stable scatter by one digit, persistent over XCD-contiguous tiles of the set; each workgroup
// loads its next tile's items while it ranks and writes the current one.  Items are ranked in
// wave-striped order, which is the tile's current order, so equal digits keep their relative
// order.  Writes go out digit-run by digit-run, inside the tile's segment.
template <bool GRAD>
__global__ __launch_bounds__(kScatterThreads, 4) void k_radix_scatter(int pass, LongSet set, const float* w,
                                                                const float* grad, float eta, uint32_t* kA,
                                                                uint32_t* kB, int32_t* vA, int32_t* vB,
                                                                int32_t* saved_perm, const uint32_t* hist,
                                                                const uint32_t* totals, const uint32_t* flags) {
  constexpr int IPT = kRadixTile / kScatterThreads;
  constexpr int NW = kScatterThreads / kWave;
  const int shift = 8 * pass;
  const bool first = pass == 0;
  __shared__ uint32_t skey[kRadixTile];
  __shared__ int32_t sval[kRadixTile];
  __shared__ uint32_t wcnt[NW][256];
  __shared__ int delta[256];  // per digit: position of the tile's first key of the digit in the
                              // segment minus its position in the tile
  __shared__ int ish[NW + 1];
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wv = tid / kWave;
  const int wbase = wv * kWave * IPT;
  // thread tid < 256 owns digit tid
  const bool owner = tid < 256;
  struct TileSrc {
    RadixBufs b;
    const float* ws;
    const float* gs;
    int64_t d;
    int ltile;
    int seg;
  };
  auto tile_src = [&](int tile) -> TileSrc {
    TileSrc t;
    t.seg = set.seg_of_rtile(tile);
    const LongSeg& sg = set.seg(t.seg);
    t.b = seg_radix_bufs(pass, sg, flags[kSegFlagWords * t.seg + 1], kA, kB, vA, vB, saved_perm);
    t.ws = first ? w + sg.start : nullptr;
    t.gs = first && GRAD ? grad + sg.start : nullptr;
    t.d = sg.d;
    t.ltile = tile - sg.rbase;
    return t;
  };
  uint32_t k[IPT];
  int32_t v[IPT];
  int tile, tend, tstep;
  xcd_tiles(set.nrt, &tile, &tend, &tstep);
  int cur_seg = -1;
  int rowbase = 0;  // digit base of the owner's digit in the segment: keys of all smaller digits
  if (tile < tend) {
    const TileSrc t = tile_src(tile);
    if (t.b.run) {
      radix_load_tile<IPT, GRAD>(t.ws, t.gs, eta, t.b.ksrc, t.b.vsrc, t.d, t.ltile, k, v);
      radix_raw_to_key<IPT>(first, k);
    }
  }
  for (; tile < tend; tile += tstep) {
    const TileSrc t = tile_src(tile);
    uint32_t kn[IPT];
    int32_t vn[IPT];
    const int next = tile + tstep;
    if (next < tend) {  // the next tile's items are in flight while this one is ranked and written
      const TileSrc tn = tile_src(next);
      if (tn.b.run) radix_load_tile<IPT, GRAD>(tn.ws, tn.gs, eta, tn.b.ksrc, tn.b.vsrc, tn.d, tn.ltile, kn, vn);
    }
    if (t.b.run) {  // uniform over the workgroup
      if (t.seg != cur_seg) {  // digit bases of the segment (the same for all its tiles)
        int gt;
        rowbase = block_excl_scan<kScatterThreads, int>(owner ? (int)totals[256 * t.seg + tid] : 0, ish, &gt);
        cur_seg = t.seg;
      }
      const int64_t base = (int64_t)t.ltile * kRadixTile;
      const int nt = (int)min((int64_t)kRadixTile, t.d - base);
      const int nr = min(IPT, max(0, (nt - wbase + kWave - 1) / kWave));
      const uint32_t tile_pre = owner ? hist[(int64_t)tid * set.nrt + tile] : 0u;
      uint32_t* const kdst = t.b.kdst;
      int32_t* const vdst = t.b.vdst;
      const uint32_t n = (uint32_t)t.d;
      for (int j = lane; j < 256; j += kWave) wcnt[wv][j] = 0u;
      uint16_t rk[IPT];
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        if (r < nr) {
          const uint32_t dg = (k[r] >> shift) & 255u;
          const uint64_t peers = match_digit8(dg);
          const uint32_t b = wcnt[wv][dg];
          const int nbelow = popc_below(peers);
          if (nbelow == 0) wcnt[wv][dg] = b + (uint32_t)__popcll(peers);
          rk[r] = (uint16_t)(b + nbelow);
        }
      }
      __syncthreads();
      // digit offsets inside the tile (thread tid < 256 owns digit tid)
      uint32_t run = 0;
      if (owner) {
        for (int w = 0; w < NW; ++w) {
          const uint32_t c = wcnt[w][tid];
          wcnt[w][tid] = run;
          run += c;
        }
      }
      int tot;
      const int dstart = block_excl_scan<kScatterThreads, int>((int)run, ish, &tot);
      if (owner) {
        for (int w = 0; w < NW; ++w) wcnt[w][tid] += (uint32_t)dstart;
        // global base of this digit = all smaller digits + this digit in the tiles before this one
        delta[tid] = rowbase + (int)tile_pre - dstart;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        if (r < nr) {
          const uint32_t dg = (k[r] >> shift) & 255u;
          const int np = (int)wcnt[wv][dg] + rk[r];
          skey[np] = k[r];
          sval[np] = v[r];
        }
      }
      __syncthreads();
      // write-out by digit runs, four ranks of the thread at a time (their LDS reads issued
      // together); 32-bit byte offsets (n <= 2^27) from the uniform array bases
      constexpr int WB = 4;
      static_assert(IPT % WB == 0, "write-out batches");
#pragma unroll 1
      for (int h = 0; h < IPT; h += WB) {
        uint32_t ko[WB], dso[WB];
        int32_t vo[WB];
#pragma unroll
        for (int q = 0; q < WB; ++q) {
          const int sp = tid + (h + q) * kScatterThreads;
          ko[q] = skey[sp];
          vo[q] = sval[sp];
        }
#pragma unroll
        for (int q = 0; q < WB; ++q)
          dso[q] = (uint32_t)(delta[(ko[q] >> shift) & 255u] + tid + (h + q) * kScatterThreads);
#pragma unroll
        for (int q = 0; q < WB; ++q) {
          // dso < n always holds for consistent histograms; it guards the scatter
          if (tid + (h + q) * kScatterThreads < nt && dso[q] < (uint32_t)n) {
            *at_u32(kdst, dso[q]) = ko[q];
            *at_u32(vdst, dso[q]) = vo[q];
          }
        }
      }
      __syncthreads();  // LDS is reused by the next tile
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      k[r] = kn[r];
      v[r] = vn[r];
    }
    radix_raw_to_key<IPT>(first, k);
  }
}

template __global__ void k_radix_hist<false>(int, LongSet, const float*, const float*, float, uint32_t*, uint32_t*,
                                              int32_t*, int32_t*, int32_t*, uint32_t*, uint32_t*, uint32_t*,
                                              uint32_t*, const uint32_t*);
template __global__ void k_radix_hist<true>(int, LongSet, const float*, const float*, float, uint32_t*, uint32_t*,
                                             int32_t*, int32_t*, int32_t*, uint32_t*, uint32_t*, uint32_t*,
                                             uint32_t*, const uint32_t*);
template __global__ void k_radix_scatter<false>(int, LongSet, const float*, const float*, float, uint32_t*,
                                                 uint32_t*, int32_t*, int32_t*, int32_t*, const uint32_t*,
                                                 const uint32_t*, const uint32_t*);
template __global__ void k_radix_scatter<true>(int, LongSet, const float*, const float*, float, uint32_t*, uint32_t*,
                                                int32_t*, int32_t*, int32_t*, const uint32_t*, const uint32_t*,
                                                const uint32_t*);

// ------------------------------------------------------------------------------- tile hulls

struct TileSmem {
  double S[rpad_size(kBigTile + 1)];  // tile-relative prefix sums (rank-padded), then hull S'
  uint16_t vert[kBigThreads * (kBigE + 1)];  // hull scratch, or the hull's tile-local ranks
  int cnt[kBigThreads];
  int mres[kBigThreads];
  double dred[kBigThreads / kWave + 1];
  int ired[kBigThreads / kWave + 1];
  WaveBound wb[2 * (kBigThreads / kWave)];
  uint32_t hb[kBigThreads];  // fallback path: hull-vertex bits of each thread's ranks
  double xtot;
};
static_assert(kBigTile - 1 + ((kBigTile - 1) >> 4) < kBigThreads * (kBigE + 1),
              "the hull's tile-local ranks (rank-padded) fit the hull scratch");


// Local hull of tile t: points k0..k0+np (np = elements in the tile) with tile-relative sums
//   S'_j = sum_{k0 <= i < k0+j} (x_i - c) + lam/(d-1) * [(k0+j)(d-k0-j) - k0(d-k0)]
//        = X'_j + lam/(d-1) * j (d - 2 k0 - j),
// i.e. S_{k0+j} minus the tile's offset S_{k0}.  Adding that offset back does not change the
// hull; keeping it out keeps S' small (|S'| ~ tile size) so cluster values inside a tile are
// differences of small numbers even when the segment's global prefix sums are ~1e7.
__global__ __launch_bounds__(kBigThreads) void k_big_tile_hull(LongSet set, const uint32_t* keys, LamArgs lamargs,
                                                               int32_t* vpos, double* vS, int32_t* hcnt,
                                                               double* tsum, uint16_t* hbits, int rounds) {
  __shared__ TileSmem sm;
  const int tid = threadIdx.x;
  const int t = blockIdx.x;  // hull tile of the set
  const LongSeg& sg = set.seg(set.seg_of_htile(t));
  const int64_t d = sg.d;
  const uint32_t* skeys = keys + sg.ebase;
  const int64_t k0 = (int64_t)(t - sg.tbase) * kBigTile;  // segment rank of the tile's first rank
  const int np = (int)min((int64_t)kBigTile, d - k0);
  const double c = (double)key_to_float(skeys[d >> 1]);
  const float lam = lamargs.of(sg.seg_id);
  const double lamd = lam > 0.0f ? (double)lam / (double)(d - 1) : 0.0;
  const int j0 = tid * kBigE;
  // the thread's kBigE consecutive sorted keys, straight from global memory as 16-byte words
  // (64-byte aligned: tiles and thread blocks are multiples of 16 keys)
  uint32_t kv[kBigE];
  const uint32_t* kt = skeys + k0;
  if (j0 + kBigE <= np) {
#pragma unroll
    for (int q = 0; q < kBigE / 4; ++q) {
      const uint4 w = *reinterpret_cast<const uint4*>(kt + j0 + 4 * q);
      kv[4 * q] = w.x;
      kv[4 * q + 1] = w.y;
      kv[4 * q + 2] = w.z;
      kv[4 * q + 3] = w.w;
    }
  } else {  // last, partial tile
#pragma unroll
    for (int i = 0; i < kBigE; ++i) kv[i] = j0 + i < np ? kt[j0 + i] : 0u;
  }
  double xs[kBigE];
  double lsum = 0.0;
#pragma unroll
  for (int i = 0; i < kBigE; ++i) {
    xs[i] = j0 + i < np ? (double)key_to_float(kv[i]) - c : 0.0;
    lsum += xs[i];
  }
  double X = block_excl_scan<kBigThreads, double>(lsum, sm.dred, (double*)nullptr);
  double sv[kBigE + 1];
#pragma unroll
  for (int i = 0; i <= kBigE; ++i) {
    const int j = j0 + i;
    sv[i] = X + lamd * (double)j * ((double)(d - 2 * k0) - (double)j);
    if (i < kBigE) {
      if (j <= np) sm.S[rpad(j)] = sv[i];
      if (j == np) sm.xtot = X;
      X += xs[i];
    }
  }
  if (tid == kBigThreads - 1 && np == kBigTile) {
    sm.S[rpad(kBigTile)] = sv[kBigE];
    sm.xtot = X;
  }
  __syncthreads();
  const int64_t vb = (int64_t)t * (kBigTile + 1);
  uint32_t bm;
  Cand lc, rc;
  if (ica_rounds<kBigThreads, kBigE, RankPadded>(sm.S, sv, np, rounds < 0 ? kIcaRounds : rounds, &bm, &lc, &rc,
                                                  sm.wb)) {
    // hull vertices = surviving candidates in rank order, then the tile's end point.  The
    // records go through LDS (S' over the dead prefix sums, tile-local ranks in the hull scratch,
    // both rank-padded) so that the global stores are lane-consecutive.
    const double endS = sm.S[rpad(np)];  // read before the scan's barrier: S is overwritten below
    int nv;
    int at = block_excl_scan<kBigThreads, int>(__popc(bm), sm.ired, &nv);
    hbits[(int64_t)t * kBigThreads + tid] = (uint16_t)bm;
#pragma unroll
    for (int i = 0; i < kBigE; ++i) {
      if ((bm >> i) & 1u) {
        sm.S[rpad(at)] = sv[i];
        sm.vert[rpad(at)] = (uint16_t)(j0 + i);
        ++at;
      }
    }
    __syncthreads();
    for (int i = tid; i < nv; i += kBigThreads) {
      vpos[vb + i] = (int32_t)(k0 + sm.vert[rpad(i)]);
      vS[vb + i] = sm.S[rpad(i)];
    }
    if (tid == 0) {
      vpos[vb + nv] = (int32_t)(k0 + np);
      vS[vb + nv] = endS;
      hcnt[t] = nv + 1;
      tsum[t] = sm.xtot;
    }
    return;
  }
  sm.hb[tid] = 0u;
  tile_hull<kBigThreads, kBigE, RankPadded, int>(sm.S, np, sm.vert, sm.cnt, sm.mres);
  const int nv = sm.cnt[0];
  for (int i = tid; i < nv; i += kBigThreads) {
    const int r = sm.vert[i];
    vpos[vb + i] = (int32_t)(k0 + r);
    vS[vb + i] = sm.S[rpad(r)];
    if (r < np) atomicOr(&sm.hb[r / kBigE], 1u << (r % kBigE));
  }
  __syncthreads();
  hbits[(int64_t)t * kBigThreads + tid] = (uint16_t)sm.hb[tid];
  if (tid == 0) {
    hcnt[t] = nv;
    tsum[t] = sm.xtot;
  }
}

// Tile offsets S_{k0} = (exclusive scan of tile sums of x - c) + lam k0 (d-k0)/(d-1), and the
// initial own ranges [1, hcnt-1]; one workgroup per segment of the set.
template <int CM>
__global__ __launch_bounds__(1024) void k_big_tile_scan(LongSet set, const double* __restrict__ tsum,
                                                        double* __restrict__ tileoff,
                                                        const int32_t* __restrict__ hcnt,
                                                        int32_t* __restrict__ lo, int32_t* __restrict__ hi,
                                                        LamArgs lamargs) {
  // CM >= tiles per thread (ceil(nt / 1024)), chosen by the host
  const LongSeg& sg = set.seg(blockIdx.x);
  const int64_t d = sg.d;
  const int ntiles = sg.nt;
  const int tb = sg.tbase;
  const float lam = lamargs.of(sg.seg_id);
  const double lamd = lam > 0.0f ? (double)lam / (double)(d - 1) : 0.0;
  __shared__ double sh[1024 / kWave + 1];
  const int chunk = (ntiles + 1023) / 1024;
  const int a = threadIdx.x * chunk;
  // every load of the thread's chunk first (one round trip), then the scan
  double ts[CM];
  int hc[CM];
#pragma unroll
  for (int c = 0; c < CM; ++c) {
    const int i = a + c;
    const bool ok = c < chunk && i < ntiles;
    ts[c] = ok ? tsum[tb + i] : 0.0;
    hc[c] = ok ? hcnt[tb + i] : 0;
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < CM; ++c) s += ts[c];
  double run = block_excl_scan<1024, double>(s, sh, (double*)nullptr);
#pragma unroll
  for (int c = 0; c < CM; ++c) {
    const int i = a + c;
    if (c < chunk && i < ntiles) {
      const double k0 = (double)i * (double)kBigTile;
      tileoff[tb + i] = run + lamd * k0 * ((double)d - k0);
      run += ts[c];
      lo[tb + i] = 1;
      hi[tb + i] = hc[c] - 1;
    }
  }
}

// ------------------------------------------------------------------------------- cross-tile merges

// Chain of a node = its left end point, then the own ranges of its tiles.  State in LDS:
// lo16[t] (own range start) and the exclusive prefix pre[t] of the own-range lengths, for the
// tiles of this workgroup's group; vertex data in global memory.  The prefix is either one int
// per tile (pre) or, for the top level's 2^15 tiles, split into an int per 8 tiles plus a 16-bit
// offset per tile (base[t / 8] + off16[t]; 8 own ranges hold at most 8 * 4097 vertices).
struct MergeCtx {
  const uint16_t* lo16;
  const int* pre;
  int gbase;  // first tile of the group
  const int32_t* vpos;
  const double* vS;
  const double* tileoff;
  const int* base = nullptr;
  const uint16_t* off16 = nullptr;
  __device__ __forceinline__ int pre_at(int t) const { return pre ? pre[t] : base[t >> 3] + (int)off16[t]; }
};

// m-th vertex of the node covering group-relative tiles [t0, t1): tile and index in that tile.
__device__ __forceinline__ void node_vertex(const MergeCtx& C, int t0, int t1, int m, int* tile, int* idx) {
  if (m == 0) {
    *tile = t0;
    *idx = 0;
    return;
  }
  const int mm = m - 1 + C.pre_at(t0);
  int lo = t0, hi = t1;  // pre[lo] <= mm < pre[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (C.pre_at(mid) <= mm)
      lo = mid;
    else
      hi = mid;
  }
  *tile = lo;
  *idx = C.lo16[lo] + (mm - C.pre_at(lo));
}

// Wave-cooperative access to a node's chain: any lane may fetch any vertex.  Chain indices
// [wlo, whi] are also held in an LDS window (loaded once per merge, the vertices next to the
// junction, where most bridge probes land); other indices come from global memory.
// LDS-qualified pointers: window reads compile to LDS instructions, which a wave executes in
// order with its own window writes (a generic pointer would read through the flat path, which is
// not ordered with pending LDS writes).
typedef __attribute__((address_space(3))) int lds_int;
typedef __attribute__((address_space(3))) double lds_double;

struct WaveNode {
  const MergeCtx* C;
  int t0, t1;
  const lds_int* wp = nullptr;
  const lds_double* ws = nullptr;
  int wlo = 0, whi = -1;
  __device__ __forceinline__ void load(int tile, int idx, int* p, double* s) const {
    const int g = C->gbase + tile;
    const int64_t at = (int64_t)g * (kBigTile + 1) + idx;
    *p = C->vpos[at];
    *s = C->vS[at] + C->tileoff[g];
  }
  __device__ __forceinline__ void fetch_global(int m, int* p, double* s) const {
    int tile, idx;
    node_vertex(*C, t0, t1, m, &tile, &idx);
    load(tile, idx, p, s);
  }
  __device__ __forceinline__ void fetch(int m, int* p, double* s) const {
    if (m >= wlo && m <= whi) {
      *p = wp[m - wlo];
      *s = ws[m - wlo];
    } else {
      fetch_global(m, p, s);
    }
  }
  // vertices m and m+1 (window, or one search when m+1 is the next vertex of the same tile)
  __device__ __forceinline__ void fetch2(int m, int* p0, double* s0, int* p1, double* s1) const {
    if (m >= wlo && m + 1 <= whi) {
      *p0 = wp[m - wlo];
      *s0 = ws[m - wlo];
      *p1 = wp[m + 1 - wlo];
      *s1 = ws[m + 1 - wlo];
      return;
    }
    int tile, idx;
    node_vertex(*C, t0, t1, m, &tile, &idx);
    const bool same = m > 0 && idx + 1 < (int)C->lo16[tile] + (C->pre_at(tile + 1) - C->pre_at(tile));
    int tile1 = tile, idx1 = idx + 1;
    if (!same) node_vertex(*C, t0, t1, m + 1, &tile1, &idx1);
    load(tile, idx, p0, s0);
    load(tile1, idx1, p1, s1);
  }
};

// First j in [1, q] with R(j) strictly below the segment Q -> R(j+1) (q when none): the
// rightmost collision of the point Q inside R.  Called by all 64 lanes with uniform arguments;
// probes run 64 at a time: one exponential round (lane l probes 2^l), then 64-way refinement.
// The point R(j) comes back in (*rp, *rs): the lane whose probe decided j has already read it.
__device__ int wave_tangent(const WaveNode& R, int q, int qa, double qs, int* rp, double* rs) {
  const int lane = lane_id();
  int pj = 0;
  double sj = 0.0;
  auto f = [&](int j) -> bool {
    if (j >= q) {
      R.fetch(q, &pj, &sj);
      return true;
    }
    int pj1;
    double sj1;
    R.fetch2(j, &pj, &sj, &pj1, &sj1);
    return below(qa, qs, pj, sj, pj1, sj1);
  };
  int lo = 0;
  // the probes R's window can answer first: j = 1 + lane for j <= J (f(j) reads R(j) and
  // R(j+1), f(q) only R(q)); one LDS round instead of a global one when the tangent is near
  const int J = q <= R.whi ? q : R.whi - 1;
  if (R.wlo == 0 && J >= 1) {
    const int jw = 1 + lane;
    const bool tw = jw <= J && f(jw);
    const uint64_t bw = __ballot(tw);
    if (bw) {
      const int fw = __ffsll((unsigned long long)bw) - 1;
      *rp = __shfl(pj, fw, kWave);
      *rs = __shfl(sj, fw, kWave);
      return __shfl(jw, fw, kWave);
    }
    lo = min(J, kWave);  // every j <= J is false (J < q here)
  }
  const int j = lane < 30 ? min(lo + (1 << lane), q) : q;
  const uint64_t b = __ballot(f(j));  // lane 63 probes q, so b != 0
  const int ft = __ffsll((unsigned long long)b) - 1;
  int hi = __shfl(j, ft, kWave);
  lo = ft == 0 ? lo : __shfl(j, ft - 1, kWave);
  int hp = __shfl(pj, ft, kWave);
  double hs = __shfl(sj, ft, kWave);
  while (hi - lo > 1) {
    const int span = hi - lo - 1;  // candidates lo+1 .. hi-1
    const int stride = (span + kWave - 1) / kWave;
    const int jj = lo + 1 + lane * stride;
    const bool valid = jj < hi;
    const uint64_t bb = __ballot(valid && f(jj));
    if (bb == 0) {
      const int nvalid = (span + stride - 1) / stride;
      lo = lo + 1 + (nvalid - 1) * stride;
    } else {
      const int f2 = __ffsll((unsigned long long)bb) - 1;
      const int nhi = __shfl(jj, f2, kWave);
      hp = __shfl(pj, f2, kWave);
      hs = __shfl(sj, f2, kWave);
      lo = f2 == 0 ? lo : __shfl(jj, f2 - 1, kWave);
      hi = nhi;
    }
  }
  *rp = hp;
  *rs = hs;
  return hi;
}

// Bridge between the chains L (0..p) and R (0..q) sharing the junction L(p) == R(0); same
// contract as bridge() but executed by one wave: vertex fetches and tangent probes in parallel.
__device__ void wave_bridge(const WaveNode& L, int p, const WaveNode& R, int q, int* istar, int* jstar) {
  if (q <= 0) {
    *istar = p;
    *jstar = 1;
    return;
  }
  if (p <= 0) {
    *istar = 0;
    *jstar = 1;
    return;
  }
  const int lane = lane_id();
  // L(i) and L(i+1), one fetch round (lanes 0 and 1)
  auto fetch_left = [&](int i, int* li, double* si, int* ln, double* sn) {
    int pv = 0;
    double sv = 0.0;
    if (lane == 0)
      L.fetch(i, &pv, &sv);
    else if (lane == 1)
      L.fetch(i + 1, &pv, &sv);
    *li = __shfl(pv, 0, kWave);
    *ln = __shfl(pv, 1, kWave);
    *si = __shfl(sv, 0, kWave);
    *sn = __shfl(sv, 1, kWave);
  };
  // does L(i) collide inside R (L(i+1) not below L(i) -> its tangent point in R)?
  auto g_at = [&](int li, double si, int ln, double sn, int* jout) -> bool {
    int rp;
    double rs;
    const int j = wave_tangent(R, q, li, si, &rp, &rs);
    *jout = j;
    return !below(li, si, ln, sn, rp, rs);
  };
  auto g = [&](int i, int* jout) -> bool {
    int li, ln;
    double si, sn;
    fetch_left(i, &li, &si, &ln, &sn);
    return g_at(li, si, ln, sn, jout);
  };
  int lp1, lp;
  double sp1, sp;
  {
    int pv = 0;
    double sv = 0.0;
    if (lane == 0)
      L.fetch(p - 1, &pv, &sv);
    else if (lane == 1)
      L.fetch(p, &pv, &sv);
    else if (lane == 2)
      R.fetch(1, &pv, &sv);
    lp1 = __shfl(pv, 0, kWave);
    lp = __shfl(pv, 1, kWave);
    const int a2 = __shfl(pv, 2, kWave);
    sp1 = __shfl(sv, 0, kWave);
    sp = __shfl(sv, 1, kWave);
    const double b2 = __shfl(sv, 2, kWave);
    if (below(lp1, sp1, lp, sp, a2, b2)) {  // junction survives
      *istar = p;
      *jstar = 1;
      return;
    }
  }
  int jhi = 1;
  if (!g_at(lp1, sp1, lp, sp, &jhi)) {  // only reachable through rounding: keep the junction
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

#ifdef WSR_PHASE_CLOCKS
__device__ unsigned long long* g_merge_clocks = nullptr;
int set_merge_clock_buffer(void* clocks) {
  return hipMemcpyToSymbol(HIP_SYMBOL(g_merge_clocks), &clocks, sizeof(clocks)) == hipSuccess ? 0 : -1;
}
#endif

// Levels [lvl_lo, lvl_hi] of the tile merge tree; workgroup g owns tiles [g*2^lvl_hi, ...).
// LDS (static, sized for the largest group GMAX): pre[G+1], rec[5 * (G >> lvl_lo)], lo16[G],
// cnt16[G] with G = 2^lvl_hi <= GMAX and G >> lvl_lo <= RMAX.  One wave per merge.
// A merge record is {bridged, last left tile keeping vertices (t0-1: none), its last kept
// index, first right tile keeping vertices, its first kept index}.
// When finalize != 0 (single group holding every tile, last launch), also writes references to
// the previous and next surviving vertex of every tile.
template <int GMAX, int RMAX>
__global__ __launch_bounds__(kMergeThreads) void k_big_merge(int lvl_lo, int lvl_hi_launch, LongSet set,
                                                             const MergeGroup* groups, const int32_t* vpos,
                                                             const double* vS, const double* tileoff,
                                                             int32_t* lo_g, int32_t* hi_g, int64_t* prev_ref,
                                                             int64_t* next_ref) {
  constexpr int NWV = kMergeThreads / kWave;
  __shared__ int pre[GMAX + 1];
  __shared__ int rec[5 * RMAX];
  __shared__ uint16_t lo16[GMAX];
  __shared__ uint16_t cnt16[GMAX];
  __shared__ int ish[NWV + 1];
  __shared__ int win_p[NWV][2][kWave];  // per wave: the junction windows of L and R
  __shared__ double win_s[NWV][2][kWave];
  // this workgroup's group: from the launch's table, or, for a single segment, group blockIdx.x
  // of 2^lvl_hi tiles with lvl_hi the launch's top level capped at the segment's
  MergeGroup gr;
  if (groups) {
    gr = groups[blockIdx.x];
  } else {
    const LongSeg& sg = set.seg(0);
    const int lh = min(lvl_hi_launch, sg.nlev);
    const int G = 1 << lh;
    gr = MergeGroup{0, sg.tbase + (int)blockIdx.x * G, min(G, sg.nt - (int)blockIdx.x * G), lh, lh == sg.nlev ? 1 : 0};
  }
  const int lvl_hi = gr.lvl_hi;
  const int gbase = gr.gbase;
  const int gn = gr.gn;
  const int finalize = gr.fin;
  const int tid = threadIdx.x;
  const int wv = tid / kWave;
  const int lane = lane_id();
#ifdef WSR_PHASE_CLOCKS
  __shared__ unsigned long long mclk[2][kMergeLevelsPerLaunch];  // longest and summed bridge search
  const int mlaunch = (lvl_lo - 1) / kMergeLevelsPerLaunch;
  unsigned long long* const mc =
      g_merge_clocks && mlaunch < kMergeClockLaunches && blockIdx.x < kMergeClockGroups
          ? g_merge_clocks + ((int64_t)mlaunch * kMergeClockGroups + blockIdx.x) * kMergeClockSlots
          : nullptr;
  if (tid < 2 * kMergeLevelsPerLaunch) mclk[tid / kMergeLevelsPerLaunch][tid % kMergeLevelsPerLaunch] = 0ull;
#endif

  // the exclusive prefix pre[] of the own-range lengths: thread t sums a chunk of consecutive
  // tiles held in registers (all its LDS reads issued at once), one block scan, then writes
  constexpr int kChunkMax = (GMAX + kMergeThreads - 1) / kMergeThreads;
  auto rebuild_prefix = [&]() {
    const int chunk = (gn + kMergeThreads - 1) / kMergeThreads;
    const int a = tid * chunk;
    int c[kChunkMax];
    int s = 0;
#pragma unroll
    for (int j = 0; j < kChunkMax; ++j) {
      c[j] = j < chunk && a + j < gn ? (int)cnt16[a + j] : 0;
      s += c[j];
    }
    int total;
    int run = block_excl_scan<kMergeThreads, int>(s, ish, &total);
#pragma unroll
    for (int j = 0; j < kChunkMax; ++j) {
      if (j < chunk && a + j < gn) pre[a + j] = run;
      run += c[j];
    }
    if (tid == 0) pre[gn] = total;
    __syncthreads();
  };

  // the group's own ranges, up to 8 tiles per thread with all their loads in flight (indexes
  // past the group's end read its last tile again and store nothing)
  constexpr int UL = kChunkMax < 8 ? kChunkMax : 8;
  for (int i0 = tid; i0 < gn; i0 += kMergeThreads * UL) {
    int l[UL], h[UL];
#pragma unroll
    for (int u = 0; u < UL; ++u) {
      const int i = gbase + min(i0 + u * kMergeThreads, gn - 1);
      l[u] = lo_g[i];
      h[u] = hi_g[i];
    }
#pragma unroll
    for (int u = 0; u < UL; ++u) {
      const int i = i0 + u * kMergeThreads;
      if (i < gn) {
        lo16[i] = (uint16_t)l[u];
        cnt16[i] = (uint16_t)max(0, h[u] - l[u] + 1);
      }
    }
  }
  __syncthreads();
  rebuild_prefix();
  MergeCtx C{lo16, pre, gbase, vpos, vS, tileoff};
#ifdef WSR_PHASE_CLOCKS
  if (mc && tid == 0) mc[0] = wall_clock64();
#endif

#ifdef WSR_PHASE_CLOCKS
  unsigned long long t_books = 0ull, t_pre = 0ull;  // bookkeeping (thread 0), pre-bridge (wave 0)
#endif
  for (int lvl = lvl_lo; lvl <= lvl_hi; ++lvl) {
    const int size = 1 << lvl;
    const int half = size >> 1;
    const int nm = min((gn + size - 1) >> lvl, RMAX);
#ifdef WSR_PHASE_CLOCKS
    const unsigned long long tl0 = wall_clock64();
#endif
    for (int m = wv; m < nm; m += NWV) {
      const int t0 = m << lvl;
      const int tm = t0 + half;
      const int t1 = min(t0 + size, gn);
      int r0 = 0, r1 = 0, r2 = 0, r3 = 0, r4 = 0;
      if (tm < gn) {
        const int p = pre[tm] - pre[t0];  // left chain: end point + own vertices; last index p
        const int q = pre[t1] - pre[tm];
        // the 64 vertices of each chain nearest the junction, one fetch round for the wave
        const int wlo = max(0, p - (kWave - 1));
        const int rhi = min(q, kWave - 1);
        {
          WaveNode Lg{&C, t0, tm};
          WaveNode Rg{&C, tm, t1};
          int vp;
          double vs;
          if (wlo + lane <= p) {
            Lg.fetch_global(wlo + lane, &vp, &vs);
            win_p[wv][0][lane] = vp;
            win_s[wv][0][lane] = vs;
          }
          if (lane <= rhi) {
            Rg.fetch_global(lane, &vp, &vs);
            win_p[wv][1][lane] = vp;
            win_s[wv][1][lane] = vs;
          }
        }
        // the wave reads its own window writes (LDS is in order within a wave; this keeps the
        // compiler from moving the reads above the writes)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        WaveNode L{&C, t0, tm, (const lds_int*)win_p[wv][0], (const lds_double*)win_s[wv][0], wlo, p};
        WaveNode R{&C, tm, t1, (const lds_int*)win_p[wv][1], (const lds_double*)win_s[wv][1], 0, rhi};
        int istar, jstar;
#ifdef WSR_PHASE_CLOCKS
        const unsigned long long tb0 = wall_clock64();
        if (m == wv && wv == 0) t_pre += tb0 - tl0;
#endif
        wave_bridge(L, p, R, q, &istar, &jstar);
#ifdef WSR_PHASE_CLOCKS
        if (mc && lane == 0 && lvl - lvl_lo < kMergeLevelsPerLaunch) {
          const unsigned long long tb = wall_clock64() - tb0;
          atomicMax(&mclk[0][lvl - lvl_lo], tb);
          atomicAdd(&mclk[1][lvl - lvl_lo], tb);
        }
#endif
        if (!(istar == p && jstar == 1)) {
          int ti = t0 - 1, ii = 0, tj, jj;
          if (istar > 0) node_vertex(C, t0, tm, istar, &ti, &ii);
          node_vertex(C, tm, t1, jstar, &tj, &jj);
          r0 = 1;
          r1 = ti;
          r2 = ii;
          r3 = tj;
          r4 = jj;
        }
      }
      if (lane == 0) {
        int* r = rec + 5 * m;
        r[0] = r0;
        r[1] = r1;
        r[2] = r2;
        r[3] = r3;
        r[4] = r4;
      }
    }
    __syncthreads();
#ifdef WSR_PHASE_CLOCKS
    const unsigned long long tk0 = wall_clock64();
#endif
#pragma unroll
    for (int k = 0; k < kChunkMax; ++k) {  // tiles tid, tid + NT, ...: their LDS reads overlap
      const int i = tid + k * kMergeThreads;
      const int m = i >> lvl;
      if (i >= gn || m >= nm) continue;
      const int* r = rec + 5 * m;
      if (!r[0]) continue;
      const int tm = (m << lvl) + half;
      if (i < tm) {
        if (i > r[1])
          cnt16[i] = 0;
        else if (i == r[1])
          cnt16[i] = (uint16_t)(r[2] - (int)lo16[i] + 1);
      } else {
        if (i < r[3]) {
          cnt16[i] = 0;
        } else if (i == r[3]) {
          const int oldend = (int)lo16[i] + (int)cnt16[i];
          lo16[i] = (uint16_t)r[4];
          cnt16[i] = (uint16_t)(oldend - r[4]);
        }
      }
    }
    __syncthreads();
    rebuild_prefix();
#ifdef WSR_PHASE_CLOCKS
    if (tid == 0) t_books += wall_clock64() - tk0;
    if (mc && tid == 0 && lvl - lvl_lo < kMergeLevelsPerLaunch) {
      mc[1 + lvl - lvl_lo] = wall_clock64();
      mc[5 + lvl - lvl_lo] = mclk[0][lvl - lvl_lo];
      mc[9 + lvl - lvl_lo] = mclk[1][lvl - lvl_lo];
    }
#endif
  }
  for (int i = tid; i < gn; i += kMergeThreads) {
    lo_g[gbase + i] = lo16[i];
    hi_g[gbase + i] = (int)lo16[i] + (int)cnt16[i] - 1;
  }
#ifdef WSR_PHASE_CLOCKS
  if (mc && tid == 0) {
    mc[14] = t_books;
    mc[15] = t_pre;
  }
  if (mc && !finalize && tid == 0) mc[13] = wall_clock64();
#endif
  if (!finalize) return;
  // Every tile's previous and next surviving vertex on the group's chain (P_0 = tile 0, index 0,
  // then the tiles' own ranges in order): the last own vertex of the last tile before it that
  // keeps any (else P_0) and the first own vertex of the first tile after it that keeps any (else
  // none).  Those tiles come from a max-scan and a reversed min-scan over the threads' chunks of
  // consecutive tiles, packed per tile into pre[] (no longer needed); then the references to the
  // two vertices are stored, tile by tile, lane-consecutive (the apply's workgroups load the
  // vertices themselves, spread over the device).
  __shared__ int fin_w[NWV];
  __shared__ int fin_r[kMergeThreads];
  {
    constexpr int kNone = 0x7FFFFFFF;
    const int chunk = (gn + kMergeThreads - 1) / kMergeThreads;
    const int a0 = tid * chunk;
    int myl = -1, myf = kNone;  // last / first tile of the chunk keeping vertices
#pragma unroll
    for (int j = 0; j < kChunkMax; ++j) {
      const int i = a0 + j;
      if (j < chunk && i < gn && cnt16[i] > 0) {
        myl = i;
        myf = min(myf, i);
      }
    }
    auto imax = [](int x, int y) { return x > y ? x : y; };
    auto imin = [](int x, int y) { return x < y ? x : y; };
    // last keeping tile before the chunk: exclusive max-scan in thread order
    int lbefore;
    {
      const int inc = wave_incl_scan_op(myl, -1, imax);
      const int exc = wave_shift_up(inc, -1);
      if (lane == kWave - 1) fin_w[wv] = inc;
      __syncthreads();
      int b = -1;
      for (int w = 0; w < wv; ++w) b = max(b, fin_w[w]);
      lbefore = max(b, exc);
      __syncthreads();
    }
    // first keeping tile after the chunk: the same scan with min over the reversed thread order
    int fafter;
    {
      fin_r[kMergeThreads - 1 - tid] = myf;
      __syncthreads();
      const int inc = wave_incl_scan_op(fin_r[tid], kNone, imin);
      const int exc = wave_shift_up(inc, kNone);
      if (lane == kWave - 1) fin_w[wv] = inc;
      __syncthreads();
      int b = kNone;
      for (int w = 0; w < wv; ++w) b = min(b, fin_w[w]);
      const int res = min(b, exc);
      __syncthreads();
      fin_r[kMergeThreads - 1 - tid] = res;
      __syncthreads();
      fafter = fin_r[tid];
    }
    // walk the chunk both ways; pre[i] = (previous keeping tile + 1) | (next keeping tile + 1) << 16
    int nexts[kChunkMax];
    {
      int nx = fafter;
#pragma unroll
      for (int j = kChunkMax - 1; j >= 0; --j) {
        const int i = a0 + j;
        nexts[j] = nx;
        if (j < chunk && i < gn && cnt16[i] > 0) nx = i;
      }
      int pv = lbefore;
#pragma unroll
      for (int j = 0; j < kChunkMax; ++j) {
        const int i = a0 + j;
        if (j < chunk && i < gn) {
          pre[i] = (pv + 1) | ((nexts[j] == kNone ? 0 : nexts[j] + 1) << 16);
          if (cnt16[i] > 0) pv = i;
        }
      }
    }
  }
  __syncthreads();
  // the records: each vertex's flat index in the hull arrays (the apply reads the vertex itself)
#pragma unroll
  for (int k = 0; k < kChunkMax; ++k) {
    const int t = tid + k * kMergeThreads;
    if (t >= gn) continue;
    const int pk = pre[t];
    const int pt = (pk & 0xFFFF) - 1, nt = (pk >> 16) - 1;
    const int ptile = pt < 0 ? 0 : pt;
    const int pidx = pt < 0 ? 0 : (int)lo16[pt] + (int)cnt16[pt] - 1;
    prev_ref[gbase + t] = (int64_t)(gbase + ptile) * (kBigTile + 1) + pidx;
    next_ref[gbase + t] = nt >= 0 ? (int64_t)(gbase + nt) * (kBigTile + 1) + (int)lo16[nt] : (int64_t)-1;
  }
#ifdef WSR_PHASE_CLOCKS
  __syncthreads();
  if (mc && tid == 0) mc[13] = wall_clock64();
#endif
}

#define WSR_INSTANTIATE_MERGE(GM)                                                                           \
  template __global__ void k_big_merge<GM, kMergeRecMax>(int, int, LongSet, const MergeGroup*, const int32_t*, \
                                                         const double*, const double*, int32_t*, int32_t*,     \
                                                         int64_t*, int64_t*);
WSR_INSTANTIATE_MERGE(16)
WSR_INSTANTIATE_MERGE(256)
WSR_INSTANTIATE_MERGE(4096)
WSR_INSTANTIATE_MERGE(16384)

// The top merge level of a segment of 2^14 < nt <= 2^15 hull tiles (2^26 < d <= 2^27): the two
// halves (tiles [0, 2^14) and [2^14, nt)), each solved by k_big_merge, are bridged by one wave
// exactly as one merge of k_big_merge, then every tile gets its previous / next surviving vertex.
// One workgroup per such segment (top_segs: their indices in the set; null for a single
// segment).  The prefix of own-range lengths is kept split (an int per 8 tiles, a 16-bit offset
// per tile) so that it and the tiles' own-range starts fit in LDS; each thread holds 32 tiles'
// lengths in registers.
__global__ __launch_bounds__(kTopThreads) void k_big_merge_top(LongSet set, const int32_t* top_segs,
                                                               const int32_t* vpos, const double* vS,
                                                               const double* tileoff, int32_t* lo_g,
                                                               int32_t* hi_g, int64_t* prev_ref, int64_t* next_ref) {
  constexpr int TPT = kMaxHullTiles / kTopThreads;  // tiles per thread
  constexpr int HALF = kMergeGroupMax;
  __shared__ int base[kMaxHullTiles / 8 + 1];
  __shared__ uint16_t off16[kMaxHullTiles + 1];
  __shared__ uint16_t lo16[kMaxHullTiles];
  __shared__ int ish[kTopThreads / kWave + 1];
  __shared__ int rec[5];
  __shared__ int win_p[2][kWave];
  __shared__ double win_s[2][kWave];
  const LongSeg& sg = set.seg(top_segs ? top_segs[blockIdx.x] : 0);
  const int gbase = sg.tbase;
  const int gn = sg.nt;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int t0 = tid * TPT;
  int cnt[TPT];
#pragma unroll
  for (int i = 0; i < TPT; ++i) {
    const int t = t0 + i;
    int l = 0, h = -1;
    if (t < gn) {
      l = lo_g[gbase + t];
      h = hi_g[gbase + t];
      lo16[t] = (uint16_t)l;
    }
    cnt[i] = max(0, h - l + 1);
  }
  // split prefix of the lengths: base at every 8th tile, 16-bit offsets inside
  auto build_prefix = [&]() {
    int sum = 0;
#pragma unroll
    for (int i = 0; i < TPT; ++i) sum += cnt[i];
    int total;
    int run = block_excl_scan<kTopThreads, int>(sum, ish, &total);
    int b = run;
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
      const int t = t0 + i;
      if ((t & 7) == 0) {
        b = run;
        base[t >> 3] = run;
      }
      if (t <= gn) off16[t] = (uint16_t)(run - b);
      run += cnt[i];
    }
    // pre(gn) for gn below kMaxHullTiles was written above (tiles past gn add nothing)
    if (tid == 0 && gn == kMaxHullTiles) {
      base[kMaxHullTiles / 8] = total;
      off16[kMaxHullTiles] = 0;
    }
    __syncthreads();
  };
  build_prefix();
  MergeCtx C{lo16, nullptr, gbase, vpos, vS, tileoff};
  C.base = base;
  C.off16 = off16;
  if (tid < kWave) {  // one wave bridges the halves
    const int tm = HALF, t1 = gn;
    const int p = C.pre_at(tm) - C.pre_at(0);
    const int q = C.pre_at(t1) - C.pre_at(tm);
    const int wlo = max(0, p - (kWave - 1));
    const int rhi = min(q, kWave - 1);
    {
      WaveNode Lg{&C, 0, tm};
      WaveNode Rg{&C, tm, t1};
      int vp;
      double vs;
      if (wlo + lane <= p) {
        Lg.fetch_global(wlo + lane, &vp, &vs);
        win_p[0][lane] = vp;
        win_s[0][lane] = vs;
      }
      if (lane <= rhi) {
        Rg.fetch_global(lane, &vp, &vs);
        win_p[1][lane] = vp;
        win_s[1][lane] = vs;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    WaveNode L{&C, 0, tm, (const lds_int*)win_p[0], (const lds_double*)win_s[0], wlo, p};
    WaveNode R{&C, tm, t1, (const lds_int*)win_p[1], (const lds_double*)win_s[1], 0, rhi};
    int istar, jstar;
    wave_bridge(L, p, R, q, &istar, &jstar);
    int r0 = 0, r1 = 0, r2 = 0, r3 = 0, r4 = 0;
    if (!(istar == p && jstar == 1)) {
      int ti = -1, ii = 0, tj, jj;
      if (istar > 0) node_vertex(C, 0, tm, istar, &ti, &ii);
      node_vertex(C, tm, t1, jstar, &tj, &jj);
      r0 = 1;
      r1 = ti;
      r2 = ii;
      r3 = tj;
      r4 = jj;
    }
    if (lane == 0) {
      rec[0] = r0;
      rec[1] = r1;
      rec[2] = r2;
      rec[3] = r3;
      rec[4] = r4;
    }
  }
  __syncthreads();
  if (rec[0]) {  // cut the own ranges at the bridge (uniform branch)
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
      const int t = t0 + i;
      if (t >= gn) continue;
      if (t < HALF) {
        if (t > rec[1])
          cnt[i] = 0;
        else if (t == rec[1])
          cnt[i] = rec[2] - (int)lo16[t] + 1;
      } else {
        if (t < rec[3]) {
          cnt[i] = 0;
        } else if (t == rec[3]) {
          const int oldend = (int)lo16[t] + cnt[i];
          cnt[i] = oldend - rec[4];
          lo16[t] = (uint16_t)rec[4];
        }
      }
    }
  }
  __syncthreads();  // every prefix read of the merge is done before the rebuild
  build_prefix();
#pragma unroll
  for (int i = 0; i < TPT; ++i) {
    const int t = t0 + i;
    if (t < gn) {
      lo_g[gbase + t] = lo16[t];
      hi_g[gbase + t] = (int)lo16[t] + cnt[i] - 1;
    }
  }
  // global chain: gv[0] = P_0 (tile 0, index 0); gv[1 + pre[t] + i] = own vertex i of tile t;
  // each tile's previous and next surviving vertex, as references into the hull arrays
  const int nglob = 1 + C.pre_at(gn);
  auto gref = [&](int m) -> int64_t {
    int tile, idx;
    node_vertex(C, 0, gn, m, &tile, &idx);
    return (int64_t)(gbase + tile) * (kBigTile + 1) + idx;
  };
  for (int t = tid; t < gn; t += kTopThreads) {
    prev_ref[gbase + t] = gref(C.pre_at(t));
    const int nx = C.pre_at(t + 1) + 1;
    next_ref[gbase + t] = nx < nglob ? gref(nx) : (int64_t)-1;
  }
}

// ------------------------------------------------------------------------------- apply

struct ApplySmem {
  uint32_t kv[rpad_size(kBigTile)];  // sorted keys in rank order, then the values (rank-padded)
  uint32_t lmask[kBigTile / 32 + 2];
  double dred[kBigThreads / kWave + 1];
  int ired[kBigThreads / kWave + 1];
  Cand shL[kBigThreads / kWave], shR[kBigThreads / kWave];
  int shF[kBigThreads / kWave];
};

// Values for the ranks of tile t, scattered to the original order; cluster-start bits.  The
// starts inside the tile are its surviving hull vertices: the tile's hull-vertex bits whose
// vertex index lies in the own range [lo, hi], plus rank k0 when the previous tile's end point
// survives.  S' at a start is the hull's stored value (tiles with few surviving vertices) or is
// recomputed from the sorted keys by the tile kernel's own operations (dense tiles); each thread
// then sweeps its ranks with the neighbouring starts from the other threads (carry exchange) or
// from the merge (tile ends).  l1 != 0: each cluster's output goes through Alg. prox's l1 and
// rewinding lines (beta, rho, rewinding-line scale kappa).  Held to eight waves per SIMD (eight
// workgroups per CU): on unsorted weights its scattered stores through the permutation want as
// many tiles in flight as possible.
__global__ __launch_bounds__(kBigThreads, 8) void k_big_apply(LongSet set, const uint32_t* keys, const int32_t* saved_perm,
                                                           const int32_t* perm_ws, LamArgs lamargs,
                                                           const uint32_t* flags, const uint16_t* hbits,
                                                           const int32_t* hcnt, const double* vS,
                                                           const double* tileoff, const int32_t* lo_g,
                                                           const int32_t* hi_g, const int32_t* vpos,
                                                           const int64_t* prev_ref, const int64_t* next_ref,
                                                           float* out, uint32_t* mask_out,
                                                           float beta, float rho, float kappa, int l1,
                                                           uint32_t* status) {
  constexpr int R = kBigTile / kBigThreads;
  __shared__ ApplySmem sm;
  const int tid = threadIdx.x;
  const int t = blockIdx.x;  // hull tile of the set
  const int si = set.seg_of_htile(t);
  const LongSeg& sg = set.seg(si);
  const int64_t d = sg.d;
  const int64_t seg_start = sg.start;
  const uint32_t* skeys = keys + sg.ebase;
  const int64_t k0 = (int64_t)(t - sg.tbase) * kBigTile;  // segment rank of the tile's first rank
  const int np = (int)min((int64_t)kBigTile, d - k0);
  const int off = (int)((seg_start + k0) & 31);
  const int j0 = tid * kBigE;
  const int nmine = max(0, min(kBigE, np - j0));
  const float lam = lamargs.of(sg.seg_id);
  const bool nonfinite = (flags[kSegFlagWords * si] & 1u) != 0;
  const bool identity = nonfinite || !(lam > 0.0f);
  if (nonfinite && t == sg.tbase && tid == 0 && status) atomicOr(status, kStatusNonFinite);
  // segment-relative 32-bit offsets (d <= 2^27) from a uniform base
  float* const og = out + seg_start;
  const int32_t* const pt = (saved_perm ? saved_perm + seg_start : perm_ws + sg.ebase) + k0;
  const uint32_t* const kt = skeys + k0;
  // the permutation entries are needed only for the final scatter: loaded late (their latency
  // overlaps the last barrier), so they do not hold registers through the scans and passes
  int32_t pl[R];
  auto load_perm = [&]() {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = tid + r * kBigThreads;
      pl[r] = j < np ? min(max(pt[j], 0), (int32_t)(d - 1)) : 0;
    }
  };
  for (int j = tid; j < kBigTile / 32 + 2; j += kBigThreads) sm.lmask[j] = 0u;
  // the thread's cluster-start bits go to the tile's mask words (at most two words per thread)
  auto mark = [&](uint32_t bits) {
    if (bits == 0u) return;
    const int q = j0 + off;
    const uint64_t b = (uint64_t)bits << (q & 31);
    atomicOr(&sm.lmask[q >> 5], (uint32_t)b);
    if (b >> 32) atomicOr(&sm.lmask[(q >> 5) + 1], (uint32_t)(b >> 32));
  };
  if (identity) {
    load_perm();
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = tid + r * kBigThreads;
      if (j < np) {
        const float x = key_to_float(kt[j]);
        *at_u32(og, (uint32_t)pl[r]) =
            nonfinite ? __builtin_nanf("") : (l1 ? L1Rewind(beta, rho, kappa)((double)x, 0.0) : x);
      }
    }
    mark(nmine > 0 ? (1u << nmine) - 1u : 0u);
    __syncthreads();
    if (mask_out) store_mask_words<kBigThreads>(mask_out, seg_start + k0, np, sm.lmask);
    return;
  }
  const uint32_t hb = hbits[(int64_t)t * kBigThreads + tid];
  const int lo = lo_g[t], hi = hi_g[t], hc = hcnt[t];
  const int64_t vb = (int64_t)t * (kBigTile + 1);
  // S' at a start: read from the tile's hull vertices while the tile has few surviving ones, else
  // recomputed for the whole tile from its sorted keys (lane-consecutive reads), by the same
  // operations as the tile kernel, which make the same S'
  const bool dense = hi - lo + 1 > kApplySparseMax;
  if (dense) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = tid + r * kBigThreads;
      if (j < np) sm.kv[rpad(j)] = kt[j];
    }
  }
  const double c = (double)key_to_float(skeys[d >> 1]);
  const double lamd = (double)lam / (double)(d - 1);
  const L1Rewind l1f(beta, rho, kappa);
  const double toff = tileoff[t];
  // the previous / next surviving vertex on the segment's chain, from the references the merge
  // left: its position, its global S (S' + its tile's offset, as every tile forms it) and its S'
  // in its own tile
  const int64_t pref = prev_ref[t], nref = next_ref[t];
  const int ppos = vpos[pref];
  const double ps_loc = vS[pref];
  const double ps = ps_loc + tileoff[pref / (kBigTile + 1)];
  const int npn = nref >= 0 ? vpos[nref] : -1;
  const double ns_loc = nref >= 0 ? vS[nref] : 0.0;
  const double nsn = nref >= 0 ? ns_loc + tileoff[nref / (kBigTile + 1)] : 0.0;
  const double endS = vS[vb + hc - 1];  // the tile's end point, as the tile kernel stored it
  // the previous tile's end point (a cluster entering this tile from it)
  const double endS_prev = t > sg.tbase ? vS[(int64_t)(t - 1) * (kBigTile + 1) + hcnt[t - 1] - 1] : 0.0;
  // surviving starts among the thread's ranks: hull-vertex bits whose vertex index is own (the
  // scan's barriers also order the key writes above before the reads below)
  const int vbase = block_excl_scan<kBigThreads, int>(__popc(hb), sm.ired, (int*)nullptr);
  uint32_t bm = 0u;
  {
    int vi = vbase;
#pragma unroll
    for (int i = 0; i < kBigE; ++i) {
      if ((hb >> i) & 1u) {
        if (vi >= lo && vi <= hi) bm |= 1u << i;
        ++vi;
      }
    }
  }
  const bool k0start = tid == 0 && ppos == k0;  // the previous tile's end point survives
  if (k0start) bm |= 1u;
  auto xc = [&](int i) -> double {
    return j0 + i < np ? (double)key_to_float(sm.kv[rpad(j0 + i)]) - c : 0.0;
  };
  auto sprime = [&](int i, double Xi) -> double {
    const int j = j0 + i;
    return Xi + lamd * (double)j * ((double)(d - 2 * k0) - (double)j);
  };
  double X0 = 0.0;
  if (dense) {
    double lsum = 0.0;
#pragma unroll
    for (int i = 0; i < kBigE; ++i) lsum += xc(i);
    X0 = block_excl_scan<kBigThreads, double>(lsum, sm.dred, (double*)nullptr);
  }
  // S' of rank j0 + i, a start; X is the prefix before it (dense), vi its vertex index (sparse)
  auto start_s = [&](int i, double X, int vi) -> double {
    if (dense) return sprime(i, X);
    return (k0start && i == 0) ? 0.0 : vS[vb + vi];
  };
  // first pass: the thread's first and last start
  Cand mineL{-1, 0.0}, mineR{-1, 0.0};
  {
    double X = X0;
    int vi = vbase;
#pragma unroll 1
    for (int i = 0; i < kBigE; ++i) {
      if ((bm >> i) & 1u) {
        const Cand cd{(int)(k0 + j0 + i), start_s(i, X, vi)};
        if (mineR.pos < 0) mineR = cd;
        mineL = cd;
      }
      if (dense) X += xc(i);
      vi += (hb >> i) & 1u;
    }
  }
  Cand lc, rc;
  carry_exchange<kBigThreads>(mineL, mineR, false, Cand{-1, 0.0}, sm.shL, sm.shR, sm.shF, &lc, &rc);
  if (lc.pos < 0) lc = Cand{ppos, ps};
  // after the tile's last start: its end point when that survives (S'), else the merge's next
  // surviving vertex (global S)
  if (rc.pos < 0) rc = hi == hc - 1 ? Cand{(int)(k0 + np), endS} : Cand{npn, nsn};
  // A cluster inside the tile uses S' (small numbers).  A cluster spanning this tile and one
  // neighbour uses the two tiles' S' with the first tile's end point, (E - S'(pa)) + S'(pb): no
  // global sums, and both tiles read the same stored values.  A longer cluster uses global S formed
  // exactly as the merge kernel forms it (S' + tile offset).  So every tile a cluster touches
  // computes the identical value.  Candidates inside [k0, k0 + np] carry S', others S.
  auto cval = [&](int pa, double sa, int pb, double sb) -> float {
    const bool ina = pa >= k0 && pa <= k0 + np;
    const bool inb = pb >= k0 && pb <= k0 + np;
    double dS;
    if (ina && inb) {
      dS = sb - sa;
    } else if ((pb - 1) / kBigTile == pa / kBigTile + 1) {
      const double sa_l = ina ? sa : (pa % kBigTile == 0 ? 0.0 : ps_loc);  // S'(pa) in its tile
      const double e_a = ina ? endS : endS_prev;                          // that tile's end point
      const double sb_l = inb ? sb : ns_loc;                               // S'(pb) in its tile
      dS = (e_a - sa_l) + sb_l;
    } else {
      const double ga = ina ? (pa == k0 ? ps : sa + toff) : sa;
      const double gb = inb ? sb + toff : sb;
      dS = gb - ga;
    }
    const double u = c + dS / (double)(pb - pa);
    return l1 ? l1f(u, lamd * (double)(d - pa - pb)) : (float)u;
  };
  // second pass, left to right: each start closes the open cluster, whose value then goes to its
  // ranks in this thread.  Rank i's key is read before any value lands on it; the exchange
  // barrier passed after every other thread's reads of these keys.  (The sparse path uses the
  // array only for the values.)
  int pa = lc.pos, a = 0;
  double sa = lc.s;
  {
    double X = X0;
    int vi = vbase;
#pragma unroll 1
    for (int i = 0; i < kBigE; ++i) {
      if ((bm >> i) & 1u) {
        const int p = (int)(k0 + j0 + i);
        const double si = start_s(i, X, vi);
        if (i > a) {
          const uint32_t v = __float_as_uint(cval(pa, sa, p, si));
          for (int m = a; m < i; ++m) sm.kv[rpad(j0 + m)] = v;
        }
        pa = p;
        sa = si;
        a = i;
      }
      if (dense) X += xc(i);
      vi += (hb >> i) & 1u;
    }
  }
  if (a < nmine) {
    const uint32_t v = __float_as_uint(cval(pa, sa, rc.pos, rc.s));
    for (int m = a; m < nmine; ++m) sm.kv[rpad(j0 + m)] = v;
  }
  load_perm();
  mark(bm);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = tid + r * kBigThreads;
    if (j < np) *at_u32(og, (uint32_t)pl[r]) = __uint_as_float(sm.kv[rpad(j)]);
  }
  if (mask_out) store_mask_words<kBigThreads>(mask_out, seg_start + k0, np, sm.lmask);
}

// ------------------------------------------------------------------------------- backward

// Cluster-start bits of one thread's n (1..kBigE) ranks starting at tile-relative rank j0 of a
// tile starting at segment rank k0 (bit i <-> rank k0 + j0 + i); rank 0 of the segment always
// starts a cluster.  At most two mask words are read.
__device__ __forceinline__ uint32_t thread_start_bits(const uint32_t* mask, int64_t seg_start, int64_t kk0,
                                                      int n) {
  const int64_t pf0 = seg_start + kk0;
  const int64_t pfl = pf0 + n - 1;
  uint64_t w = mask[pf0 >> 5];
  if ((pfl >> 5) != (pf0 >> 5)) w |= (uint64_t)mask[pfl >> 5] << 32;
  uint32_t b = (uint32_t)(w >> (pf0 & 31)) & ((1u << n) - 1u);
  if (kk0 == 0) b |= 1u;
  return b;
}

// Cotangent i of one thread's kBigE consecutive ranks (rank order) from the rank-padded LDS copy.
// The tile and apply kernels read it the same way and add in the same order, so the prefix G at a
// cluster start is formed by the same additions in both.
__device__ __forceinline__ double thread_cotangent(const float* lds, int j0, int nmine, int i) {
  return i < nmine ? (double)lds[rpad(j0 + i)] : 0.0;
}
__device__ __forceinline__ double thread_cotangent_sum(const float* lds, int j0, int nmine) {
  double lsum = 0.0;
#pragma unroll
  for (int i = 0; i < kBigE; ++i) lsum += thread_cotangent(lds, j0, nmine, i);
  return lsum;
}

struct BwdTileSmem {
  float g[rpad_size(kBigTile)];  // gathered cotangent in rank order (rank-padded)
  double dred[kBigThreads / kWave + 1];
  int wf[kBigThreads / kWave], wl[kBigThreads / kWave];
  double wfG[kBigThreads / kWave], wlG[kBigThreads / kWave];
};

// Gather the cotangent in rank order (kept for the apply pass), tile sums, first / last cluster
// start of the tile with the local prefix at it.
__global__ __launch_bounds__(kBigThreads) void k_big_bwd_tile(LongSet set, const float* g, const int32_t* perm,
                                                              const uint32_t* mask, float* gsorted_ws, double* tsum,
                                                              int32_t* fpos, double* fG, int32_t* lpos, double* lG) {
  constexpr int R = kBigTile / kBigThreads;
  constexpr int NW = kBigThreads / kWave;
  __shared__ BwdTileSmem sm;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wv = tid / kWave;
  const int t = blockIdx.x;  // hull tile of the set
  const LongSeg& sg = set.seg(set.seg_of_htile(t));
  const int64_t d = sg.d;
  const int64_t seg_start = sg.start;
  float* const gsorted = gsorted_ws + sg.ebase;
  perm += seg_start;  // the segment's saved permutation (segment ranks)
  const int64_t k0 = (int64_t)(t - sg.tbase) * kBigTile;  // segment rank of the tile's first rank
  const int np = (int)min((int64_t)kBigTile, d - k0);
  const int j0 = tid * kBigE;
  const int nmine = max(0, min(kBigE, np - j0));
  // lane-consecutive perm reads and gsorted writes; the gather itself follows the permutation.
  // All perm loads, the thread's start bits, then all gathers, are in flight at once.
  const int32_t* const pt = perm + k0;
  const float* const gs = g + seg_start;
  float* const go = gsorted + k0;
  int32_t pl[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = tid + r * kBigThreads;
    pl[r] = j < np ? min(max(pt[j], 0), (int32_t)(d - 1)) : 0;
  }
  const uint32_t bm = nmine > 0 ? thread_start_bits(mask, seg_start, k0 + j0, nmine) : 0u;
  float gv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) gv[r] = *at_u32(gs, (uint32_t)pl[r]);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = tid + r * kBigThreads;
    if (j < np) {
      sm.g[rpad(j)] = gv[r];
      go[j] = gv[r];
    }
  }
  __syncthreads();
  const double lsum = thread_cotangent_sum(sm.g, j0, nmine);
  double total;
  const double P = block_excl_scan<kBigThreads, double>(lsum, sm.dred, &total);
  // local prefix at the thread's first and last start
  double run = P, Gf = 0.0, Gl = 0.0;
  int f = -1, l = -1;
#pragma unroll
  for (int i = 0; i < kBigE; ++i) {
    if ((bm >> i) & 1u) {
      if (f < 0) {
        f = i;
        Gf = run;
      }
      l = i;
      Gl = run;
    }
    run += thread_cotangent(sm.g, j0, nmine, i);
  }
  // the wave's first and last start, then the block's (no shared-address atomics)
  const uint64_t has = __ballot(bm != 0u);
  if (has) {
    if (lane == __ffsll((unsigned long long)has) - 1) {
      sm.wf[wv] = (int)(k0 + j0 + f);
      sm.wfG[wv] = Gf;
    }
    if (lane == 63 - __clzll((long long)has)) {
      sm.wl[wv] = (int)(k0 + j0 + l);
      sm.wlG[wv] = Gl;
    }
  } else if (lane == 0) {
    sm.wf[wv] = -1;
    sm.wl[wv] = -1;
  }
  __syncthreads();
  if (tid == 0) {
    int fp = -1, lp = -1;
    double fg = 0.0, lg = 0.0;
    for (int w = 0; w < NW; ++w)
      if (sm.wf[w] >= 0) {
        fp = sm.wf[w];
        fg = sm.wfG[w];
        break;
      }
    for (int w = NW - 1; w >= 0; --w)
      if (sm.wl[w] >= 0) {
        lp = sm.wl[w];
        lg = sm.wlG[w];
        break;
      }
    tsum[t] = total;
    fpos[t] = fp;
    fG[t] = fg;
    lpos[t] = lp;
    lG[t] = lg;
  }
}

// One workgroup per segment: tile offsets of G, and for every tile the last cluster start before it
// and the first cluster start after its last local start (with global G values).  The carries are
// "last valid" / "first valid" scans over per-thread chunk summaries (wave shuffles + LDS).
template <int CM>
__global__ __launch_bounds__(1024) void k_big_bwd_scan(LongSet set, const double* __restrict__ tsum,
                                                       const int32_t* __restrict__ fpos,
                                                       const double* __restrict__ fG,
                                                       const int32_t* __restrict__ lpos,
                                                       const double* __restrict__ lG, double* __restrict__ tileoff,
                                                       int32_t* __restrict__ prevp, double* __restrict__ prevG,
                                                       int32_t* __restrict__ nextp, double* __restrict__ nextG) {
  // CM >= tiles per thread (ceil(nt / 1024)), chosen by the host
  __shared__ double sh[1024 / kWave + 1];
  __shared__ Cand shL[1024 / kWave], shR[1024 / kWave];
  __shared__ int shF[1024 / kWave];
  const LongSeg& sg = set.seg(blockIdx.x);
  const int64_t d = sg.d;
  const int ntiles = sg.nt;
  const int tb = sg.tbase;
  const int tid = threadIdx.x;
  const int chunk = (ntiles + 1023) / 1024;
  const int a = tid * chunk;
  // every load of the thread's chunk first (one round trip), then scan and walks
  double ts[CM], lg[CM], fg[CM];
  int lp[CM], fp[CM];
#pragma unroll
  for (int c = 0; c < CM; ++c) {
    const int i = a + c;
    const bool ok = c < chunk && i < ntiles;
    ts[c] = ok ? tsum[tb + i] : 0.0;
    lp[c] = ok ? lpos[tb + i] : -1;
    fp[c] = ok ? fpos[tb + i] : -1;
    lg[c] = ok ? lG[tb + i] : 0.0;
    fg[c] = ok ? fG[tb + i] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < CM; ++c) s += ts[c];
  double total;
  double run = block_excl_scan<1024, double>(s, sh, &total);
  Cand mineL{-1, 0.0}, mineR{-1, 0.0};
  const double run0 = run;
#pragma unroll
  for (int c = 0; c < CM; ++c) {
    if (c < chunk && a + c < ntiles) tileoff[tb + a + c] = run;
    if (lp[c] >= 0) mineL = Cand{lp[c], run + lg[c]};
    if (fp[c] >= 0 && mineR.pos < 0) mineR = Cand{fp[c], run + fg[c]};
    run += ts[c];
  }
  Cand lc, rc;
  carry_exchange<1024>(mineL, mineR, false, Cand{(int)d, total}, shL, shR, shF, &lc, &rc);
  if (lc.pos < 0) lc = Cand{0, 0.0};  // rank 0 always starts a cluster
  // walk the chunk: previous start before each tile, next start after each tile (the tile
  // offsets are formed again by the same additions, not held)
  run = run0;
  Cand firsts[CM];
#pragma unroll
  for (int c = 0; c < CM; ++c) {
    if (c < chunk && a + c < ntiles) {
      prevp[tb + a + c] = lc.pos;
      prevG[tb + a + c] = lc.s;
    }
    if (lp[c] >= 0) lc = Cand{lp[c], run + lg[c]};
    firsts[c] = Cand{fp[c], run + fg[c]};
    run += ts[c];
  }
#pragma unroll
  for (int c = CM - 1; c >= 0; --c) {
    if (c < chunk && a + c < ntiles) {
      nextp[tb + a + c] = rc.pos;
      nextG[tb + a + c] = rc.s;
    }
    if (firsts[c].pos >= 0) rc = firsts[c];
  }
}

#define WSR_INSTANTIATE_SCANS(CM)                                                                         \
  template __global__ void k_big_tile_scan<CM>(LongSet, const double*, double*, const int32_t*, int32_t*,    \
                                               int32_t*, LamArgs);                                             \
  template __global__ void k_big_bwd_scan<CM>(LongSet, const double*, const int32_t*, const double*,           \
                                              const int32_t*, const double*, double*, int32_t*, double*,       \
                                              int32_t*, double*);
WSR_INSTANTIATE_SCANS(4)
WSR_INSTANTIATE_SCANS(8)
WSR_INSTANTIATE_SCANS(16)
WSR_INSTANTIATE_SCANS(32)

struct BwdApplySmem {
  float v[rpad_size(kBigTile)];  // cotangent in rank order, then the results (rank-padded)
  double dred[kBigThreads / kWave + 1];
  Cand shL[kBigThreads / kWave], shR[kBigThreads / kWave];
  int shF[kBigThreads / kWave];
};

// Per rank: the mean cotangent of its cluster, scattered to the original order.  Each thread
// holds G (global prefix) at its kBigE ranks; the start before its first start and after its last
// one come from the other threads (carry exchange) or, at the tile ends, from the tile scan.
__global__ __launch_bounds__(kBigThreads) void k_big_bwd_apply(LongSet set, const float* gsorted_ws,
                                                               const int32_t* perm, const uint32_t* mask,
                                                               const double* tileoff, const int32_t* prevp,
                                                               const double* prevG, const int32_t* nextp,
                                                               const double* nextG, float* gout) {
  constexpr int R = kBigTile / kBigThreads;
  __shared__ BwdApplySmem sm;
  const int tid = threadIdx.x;
  const int t = blockIdx.x;  // hull tile of the set
  const LongSeg& sg = set.seg(set.seg_of_htile(t));
  const int64_t d = sg.d;
  const int64_t seg_start = sg.start;
  const float* const gsorted = gsorted_ws + sg.ebase;
  perm += seg_start;  // the segment's saved permutation (segment ranks)
  const int64_t k0 = (int64_t)(t - sg.tbase) * kBigTile;  // segment rank of the tile's first rank
  const int np = (int)min((int64_t)kBigTile, d - k0);
  const int j0 = tid * kBigE;
  const int nmine = max(0, min(kBigE, np - j0));
  // segment-relative 32-bit offsets (d <= 2^27) from a uniform base; every load is issued first
  float* const og = gout + seg_start;
  const int32_t* const pt = perm + k0;
  const float* const gt = gsorted + k0;
  float gl[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = tid + r * kBigThreads;
    gl[r] = j < np ? gt[j] : 0.0f;
  }
  const uint32_t bm = nmine > 0 ? thread_start_bits(mask, seg_start, k0 + j0, nmine) : 0u;
  const double toff = tileoff[t];
  const Cand after{nextp[t], nextG[t]};
  const Cand before{prevp[t], prevG[t]};
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = tid + r * kBigThreads;
    if (j < np) sm.v[rpad(j)] = gl[r];
  }
  __syncthreads();
  const double lsum = thread_cotangent_sum(sm.v, j0, nmine);
  const double P = block_excl_scan<kBigThreads, double>(lsum, sm.dred, (double*)nullptr);
  // G at a rank = tile offset + local prefix, formed as the tile kernel forms it for the tile
  // scan; first pass: the thread's first and last start
  Cand mineL{-1, 0.0}, mineR{-1, 0.0};
  double run = P;
#pragma unroll
  for (int i = 0; i < kBigE; ++i) {
    if ((bm >> i) & 1u) {
      const Cand c{(int)(k0 + j0 + i), toff + run};
      if (mineR.pos < 0) mineR = c;
      mineL = c;
    }
    run += thread_cotangent(sm.v, j0, nmine, i);
  }
  Cand lc, rc;
  carry_exchange<kBigThreads>(mineL, mineR, false, after, sm.shL, sm.shR, sm.shF, &lc, &rc);
  if (lc.pos < 0) lc = before;
  // second pass, left to right: each start closes the open cluster, whose mean then goes to its
  // ranks in this thread (rank i's cotangent is read before any result lands on it; the exchange
  // barrier passed after every other thread's reads).  Every tile a cluster touches forms its
  // mean from the same two G values and the same division.
  int pa = lc.pos, a = 0;
  double sa = lc.s;
  run = P;
#pragma unroll
  for (int i = 0; i < kBigE; ++i) {
    if ((bm >> i) & 1u) {
      const int p = (int)(k0 + j0 + i);
      const double gi = toff + run;
      if (i > a) {
        const float v = (float)div_count(gi - sa, p - pa);
        for (int m = a; m < i; ++m) sm.v[rpad(j0 + m)] = v;
      }
      pa = p;
      sa = gi;
      a = i;
    }
    run += thread_cotangent(sm.v, j0, nmine, i);
  }
  if (a < nmine) {
    const float v = (float)div_count(rc.s - sa, max(1, rc.pos - pa));
    for (int m = a; m < nmine; ++m) sm.v[rpad(j0 + m)] = v;
  }
  // the permutation entries are needed only for the final scatter: loaded late (their latency
  // overlaps the last barrier), so they do not hold registers through the scan and passes
  int32_t pl[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = tid + r * kBigThreads;
    pl[r] = j < np ? min(max(pt[j], 0), (int32_t)(d - 1)) : 0;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = tid + r * kBigThreads;
    if (j < np) *at_u32(og, (uint32_t)pl[r]) = sm.v[rpad(j)];
  }
}

// Statistics of a long segment from its sorted keys (App. B: R(w) from the sorted order).
// k_big_stats_tile: per rank tile, the centred weighted sum sum_k (2k-d+1)(x_k - c) in FP64 and
// the counts of non-zero weights and of distinct non-zero values (a rank counts when its value
// differs from the previous rank's, read across the tile edge); k_big_stats_final adds the
// tiles in a fixed order.  Deterministic.
__global__ __launch_bounds__(kBigThreads) void k_big_stats_tile(LongSet set, const uint32_t* keys, double* tsum,
                                                                int32_t* tnz, int32_t* tnd) {
  __shared__ double dred[kBigThreads / kWave + 1];
  __shared__ long long lred[kBigThreads / kWave + 1];
  const int tid = threadIdx.x;
  const LongSeg& sg = set.seg(set.seg_of_htile(blockIdx.x));
  const int64_t d = sg.d;
  const uint32_t* skeys = keys + sg.ebase;
  const int64_t k0 = (int64_t)(blockIdx.x - sg.tbase) * kBigTile;
  const int np = (int)min((int64_t)kBigTile, d - k0);
  const double c = (double)key_to_float(skeys[d >> 1]);
  double lsum = 0.0;
  long long cnt = 0;  // non-zero weights in the high half, distinct non-zero values in the low
#pragma unroll 4
  for (int r = 0; r < kBigE; ++r) {
    const int j = tid + r * kBigThreads;
    if (j < np) {
      const int64_t kk = k0 + j;
      const float x = key_to_float(skeys[kk]);
      const float xp = kk > 0 ? key_to_float(skeys[kk - 1]) : 0.0f;
      lsum += (double)(2 * kk - d + 1) * ((double)x - c);
      if (x != 0.0f) cnt += (1ll << 32) + ((kk == 0 || x != xp) ? 1 : 0);
    }
  }
  double total;
  long long ctot;
  (void)block_excl_scan<kBigThreads, double, false>(lsum, dred, &total);
  (void)block_excl_scan<kBigThreads, long long, false>(cnt, lred, &ctot);
  if (tid == 0) {
    tsum[blockIdx.x] = total;
    tnz[blockIdx.x] = (int32_t)(ctot >> 32);
    tnd[blockIdx.x] = (int32_t)(ctot & 0xFFFFFFFFll);
  }
}

__global__ __launch_bounds__(1024) void k_big_stats_final(LongSet set, const double* tsum, const int32_t* tnz,
                                                          const int32_t* tnd, const uint32_t* flags, SegStats* out) {
  __shared__ double dred[1024 / kWave + 1];
  __shared__ long long zred[1024 / kWave + 1], nred[1024 / kWave + 1];
  const int tid = threadIdx.x;
  const LongSeg& sg = set.seg(blockIdx.x);  // one workgroup per segment
  const int64_t d = sg.d;
  double s = 0.0;
  long long nz = 0, nd = 0;
  for (int t = sg.tbase + tid; t < sg.tbase + sg.nt; t += 1024) {
    s += tsum[t];
    nz += tnz[t];
    nd += tnd[t];
  }
  double total;
  long long ztot, ntot;
  (void)block_excl_scan<1024, double, false>(s, dred, &total);
  (void)block_excl_scan<1024, long long, false>(nz, zred, &ztot);
  (void)block_excl_scan<1024, long long, false>(nd, nred, &ntot);
  if (tid == 0) {
    if (flags[kSegFlagWords * blockIdx.x] & 1u)
      out[sg.seg_id] = SegStats{__builtin_nan(""), -1, -1};
    else
      out[sg.seg_id] = SegStats{total / (double)(d - 1), ntot, ztot};
  }
}

}  // namespace wsr
