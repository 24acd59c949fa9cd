// wsr_api.hip -- host side of the C ABI declared in include/wsr.h: argument validation,
// workspace layout, size-class routing, plans and launch sequences.  Nothing here allocates or
// synchronises inside a compute call; plans allocate once at creation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/wsr.h"
#include "wsr_big.h"
#include "wsr_kernels.h"

namespace wsr {
namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

constexpr int kMaxMergeRounds = 64;  // largest collision-round cap a plan accepts

enum SizeClass { kSkip = -1, kC2048 = 0, kC4096 = 1, kC8192 = 2, kBig = 3 };
constexpr int kNumSmall = 3;
constexpr int kClassMax[kNumSmall] = {2048, 4096, 8192};

inline int size_class(int64_t d) {
  if (d <= 0) return kSkip;
  for (int c = 0; c < kNumSmall; ++c)
    if (d <= kClassMax[c]) return c;
  return kBig;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// True when every segment starts at a multiple of 32: then no cluster-start mask word is shared
// by two segments and every word is written with a plain store, so no zero fill is needed.
bool offsets_word_aligned(const int64_t* h_offsets, int64_t n_seg) {
  for (int64_t s = 0; s <= n_seg; ++s)
    if (h_offsets[s] & 31) return false;
  return true;
}

int validate_offsets(const int64_t* h_offsets, int64_t n_seg, int64_t* max_big) {
  if (!h_offsets || n_seg < 0) return WSR_ERR_INVALID;
  if (h_offsets[0] != 0) return WSR_ERR_INVALID;
  int64_t mb = 0;
  for (int64_t s = 0; s < n_seg; ++s) {
    const int64_t d = h_offsets[s + 1] - h_offsets[s];
    if (d < 0) return WSR_ERR_INVALID;
    if (d > WSR_MAX_SEGMENT) return WSR_ERR_UNSUPPORTED;
    if (size_class(d) == kBig) mb = std::max(mb, d);
  }
  if (max_big) *max_big = mb;
  return WSR_OK;
}

// Host description of a set of long segments solved by one launch sequence: the per-segment
// records (element, radix-tile and hull-tile bases) and the set's totals.
struct LongSetHost {
  std::vector<LongSeg> segs;
  int64_t elems = 0;  // workspace elements (each segment's base aligned to 64 elements)
  int nrt = 0, nt = 0;
  int max_nt = 0;
  int max_nlev = 0;
};

int levels_of(int nt) {
  int nlev = 0;
  while ((1 << nlev) < nt) ++nlev;
  return nlev;
}

// The set of the long segments `ids` of these offsets (ids in order).
LongSetHost make_set(const int64_t* h_offsets, const std::vector<int32_t>& ids) {
  LongSetHost hs;
  for (int32_t id : ids) {
    LongSeg g{};
    g.start = h_offsets[id];
    g.d = h_offsets[id + 1] - g.start;
    g.ebase = hs.elems;
    g.rbase = hs.nrt;
    g.nrt = (int)ceil_div(g.d, kRadixTile);
    g.tbase = hs.nt;
    g.nt = (int)ceil_div(g.d, kBigTile);
    g.seg_id = id;
    g.nlev = levels_of(g.nt);
    hs.elems += (g.d + 63) / 64 * 64;
    hs.nrt += g.nrt;
    hs.nt += g.nt;
    hs.max_nt = std::max(hs.max_nt, g.nt);
    hs.max_nlev = std::max(hs.max_nlev, g.nlev);
    hs.segs.push_back(g);
  }
  return hs;
}

// A set passed by value: one segment, no device tables.
LongSet single_set(const LongSetHost& hs) {
  LongSet set{};
  set.one = hs.segs[0];
  set.nsegs = 1;
  set.nrt = hs.nrt;
  set.nt = hs.nt;
  return set;
}

// Workspace of the long-segment path for one set: element arrays over all its segments,
// radix-tile and hull-tile arrays over all its tiles, per-segment records.
struct BigWs {
  uint32_t* flags;       // kSegFlagWords per segment: [0] non-finite weight seen, [1] varying key bits
  uint32_t* tbad;        // per radix tile: non-finite weight seen (first pass)
  uint32_t *tor, *tand;  // per radix tile: OR and AND of its keys (first pass)
  uint32_t *keysA, *keysB;
  int32_t *valsA, *valsB;
  uint32_t *hist, *totals;
  int32_t* vpos;
  double* vS;
  uint16_t* hbits;  // per tile and thread: hull-vertex bits of the thread's ranks
  int32_t *hcnt, *lo, *hi;
  int64_t *prev_ref, *next_ref;  // per tile: its previous / next surviving vertex (index into vpos, vS)
  double *tsum, *tileoff;
  // backward
  int32_t *fpos, *lpos, *prev_pos, *next_pos;
  double *fG, *lG, *prevG, *nextG;
  size_t bytes;
};

BigWs big_layout(int64_t elems, int64_t nrt, int64_t nt, int64_t nsegs, void* base) {
  BigWs w{};
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? (void*)((char*)base + off) : nullptr;
    off += align_up(bytes);
    return p;
  };
  w.flags = (uint32_t*)take(sizeof(uint32_t) * kSegFlagWords * nsegs);
  w.tbad = (uint32_t*)take(sizeof(uint32_t) * nrt);
  w.tor = (uint32_t*)take(sizeof(uint32_t) * nrt);
  w.tand = (uint32_t*)take(sizeof(uint32_t) * nrt);
  w.keysA = (uint32_t*)take(sizeof(uint32_t) * elems);
  w.keysB = (uint32_t*)take(sizeof(uint32_t) * elems);
  w.valsA = (int32_t*)take(sizeof(int32_t) * elems);
  w.valsB = (int32_t*)take(sizeof(int32_t) * elems);
  w.hist = (uint32_t*)take(sizeof(uint32_t) * 256 * nrt);
  w.totals = (uint32_t*)take(sizeof(uint32_t) * 256 * nsegs);
  w.vpos = (int32_t*)take(sizeof(int32_t) * nt * (kBigTile + 1));
  w.vS = (double*)take(sizeof(double) * nt * (kBigTile + 1));
  w.hbits = (uint16_t*)take(sizeof(uint16_t) * nt * kBigThreads);
  w.hcnt = (int32_t*)take(sizeof(int32_t) * nt);
  w.lo = (int32_t*)take(sizeof(int32_t) * nt);
  w.hi = (int32_t*)take(sizeof(int32_t) * nt);
  w.prev_ref = (int64_t*)take(sizeof(int64_t) * nt);
  w.next_ref = (int64_t*)take(sizeof(int64_t) * nt);
  w.tsum = (double*)take(sizeof(double) * nt);
  w.tileoff = (double*)take(sizeof(double) * nt);
  w.fpos = (int32_t*)take(sizeof(int32_t) * nt);
  w.lpos = (int32_t*)take(sizeof(int32_t) * nt);
  w.prev_pos = (int32_t*)take(sizeof(int32_t) * nt);
  w.next_pos = (int32_t*)take(sizeof(int32_t) * nt);
  w.fG = (double*)take(sizeof(double) * nt);
  w.lG = (double*)take(sizeof(double) * nt);
  w.prevG = (double*)take(sizeof(double) * nt);
  w.nextG = (double*)take(sizeof(double) * nt);
  w.bytes = off;
  return w;
}
BigWs big_layout(const LongSetHost& hs, void* base) {
  return big_layout(hs.elems, hs.nrt, hs.nt, (int64_t)hs.segs.size(), base);
}

// Workspace of one segment of length d (the segments of a plain call are solved one after another).
size_t big_bytes(int64_t max_big) {
  if (max_big <= 0) return 0;
  return big_layout((max_big + 63) / 64 * 64, ceil_div(max_big, kRadixTile), ceil_div(max_big, kBigTile), 1,
                    nullptr).bytes;
}
size_t set_bytes(const LongSetHost& hs) { return hs.segs.empty() ? 0 : big_layout(hs, nullptr).bytes; }

// Launches of the merge levels done in LDS (k_big_merge): levels [lvl_lo, lvl_hi] with groups of
// up to 2^lvl_hi tiles; the merge groups of each launch over the segments of a set (a segment
// takes part while it has levels left, and a segment of one tile takes part in the first launch
// only, to write its previous / next vertices).  Levels above kMergeLevelsInLds (segments of more
// than 2^14 tiles) are done by k_big_merge_top.
struct MergeLaunch {
  int lvl_lo, lvl_hi, gmax;
  std::vector<MergeGroup> groups;
};
std::vector<MergeLaunch> merge_launches(const LongSetHost& hs) {
  std::vector<MergeLaunch> out;
  const int top = std::min(std::max(hs.max_nlev, 1), kMergeLevelsInLds);
  for (int lo = 1; lo <= top; lo += kMergeLevelsPerLaunch) {
    MergeLaunch L;
    L.lvl_lo = lo;
    L.lvl_hi = std::min(lo + kMergeLevelsPerLaunch - 1, kMergeLevelsInLds);
    int gmax = 1;
    for (size_t si = 0; si < hs.segs.size(); ++si) {
      const LongSeg& g = hs.segs[si];
      if (lo > std::max(g.nlev, 1) || (g.nlev == 0 && lo > 1)) continue;
      const int lh = std::min(L.lvl_hi, g.nlev);
      const int G = 1 << lh;
      gmax = std::max(gmax, G);
      const int fin = lh == g.nlev ? 1 : 0;
      for (int gb = 0; gb < g.nt; gb += G)
        L.groups.push_back(MergeGroup{(int)si, g.tbase + gb, std::min(G, g.nt - gb), lh, fin});
    }
    L.gmax = gmax;
    if (!L.groups.empty()) out.push_back(L);
  }
  return out;
}

int last_error() { return hipGetLastError() == hipSuccess ? WSR_OK : WSR_ERR_HIP; }

// ---- optional per-launch HIP-event trace (wsr_trace_enable / wsr_trace_collect)
constexpr int kTracePool = 4096;
struct TraceRec {
  const char* name;
  int ev;
};
struct Trace {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> ev;  // 2 * kTracePool
  std::vector<TraceRec> recs;
} g_trace;

// WSR_DEBUG=1 in the environment: report the first failing launch on stderr.
bool debug_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("WSR_DEBUG");
    return e && e[0] == '1';
  }();
  return on;
}

struct TraceScope {
  hipStream_t s;
  const char* name;
  int slot = -1;
  TraceScope(const char* nm, hipStream_t st) : s(st), name(nm) {
    std::lock_guard<std::mutex> lk(g_trace.mu);
    if (!g_trace.on || (int)g_trace.recs.size() >= kTracePool) return;
    slot = (int)g_trace.recs.size();
    g_trace.recs.push_back({nm, slot});
    (void)hipEventRecord(g_trace.ev[2 * slot], s);
  }
  ~TraceScope() {
    if (slot >= 0) (void)hipEventRecord(g_trace.ev[2 * slot + 1], s);
    if (debug_enabled()) {
      const hipError_t e = hipPeekAtLastError();
      if (e != hipSuccess) std::fprintf(stderr, "wsr: launch of %s failed: %s\n", name, hipGetErrorString(e));
    }
  }
};
#define WSR_TRACE(name, stream) TraceScope wsr_trace_scope_(name, stream)

template <int TMAX, int NT>
void launch_small_fwd(int nblocks, const SegArgs& a, const float* w, float* out, int32_t* perm,
                      uint32_t* mask, hipStream_t s) {
  if (a.merge_rounds == kRouteEnd)
    hipLaunchKernelGGL((k_prox_fwd_small<TMAX, NT, true>), dim3(nblocks), dim3(NT), 0, s, a, w, out, perm, mask);
  else
    hipLaunchKernelGGL((k_prox_fwd_small<TMAX, NT, false>), dim3(nblocks), dim3(NT), 0, s, a, w, out, perm, mask);
}
template <int TMAX, int NT>
void launch_small_bwd(int nblocks, const SegArgs& a, const float* g, float* gw, const int32_t* perm,
                      const uint32_t* mask, hipStream_t s) {
  hipLaunchKernelGGL((k_prox_bwd_small<TMAX, NT>), dim3(nblocks), dim3(NT), 0, s, a, g, gw, perm, mask);
}

void small_fwd(int cls, int nblocks, const SegArgs& a, const float* w, float* out, int32_t* perm,
               uint32_t* mask, hipStream_t s) {
  switch (cls) {
    case kC2048: { WSR_TRACE("prox_fwd_small_2048", s); launch_small_fwd<2048, 256>(nblocks, a, w, out, perm, mask, s); } break;
    case kC4096: { WSR_TRACE("prox_fwd_small_4096", s); launch_small_fwd<4096, 512>(nblocks, a, w, out, perm, mask, s); } break;
    default: { WSR_TRACE("prox_fwd_small_8192", s); launch_small_fwd<8192, 1024>(nblocks, a, w, out, perm, mask, s); } break;
  }
}
void small_bwd(int cls, int nblocks, const SegArgs& a, const float* g, float* gw, const int32_t* perm,
               const uint32_t* mask, hipStream_t s) {
  switch (cls) {
    case kC2048: { WSR_TRACE("prox_bwd_small_2048", s); launch_small_bwd<2048, 256>(nblocks, a, g, gw, perm, mask, s); } break;
    case kC4096: { WSR_TRACE("prox_bwd_small_4096", s); launch_small_bwd<4096, 512>(nblocks, a, g, gw, perm, mask, s); } break;
    default: { WSR_TRACE("prox_bwd_small_8192", s); launch_small_bwd<8192, 1024>(nblocks, a, g, gw, perm, mask, s); } break;
  }
}

void zero_words(uint32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>(ceil_div(n, 256), 2048);
  WSR_TRACE("zero_words", s);
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
}

int cu_count() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, c = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
      c = 256;
    cus = c;
  }
  return cus;
}

// Workgroups of the persistent radix scatter: as many as are resident at once (2 per CU).
int scatter_grid() { return 2 * cu_count(); }
// Workgroups of the persistent radix histogram.
int hist_grid() { return kHistPerCu * cu_count(); }

// Alg. prox's l1 and rewinding lines, applied to every cluster when on != 0.
struct L1Opt {
  float beta = 0.0f;
  float rho = 0.0f;
  int on = 0;
  float kappa = 1.0f;  // scale of the rewinding line
};

bool l1_args_ok(float beta, float rho) {
  return std::isfinite(beta) && beta >= 0.0f && rho >= 0.0f && rho <= 1.0f;
}

// Grid of a persistent radix kernel: at most `maxg` workgroups, a multiple of 8 (every XCD gets a
// contiguous share of the tiles).
int radix_grid(int ntiles, int maxg) { return (std::min(ntiles, maxg) + 7) / 8 * 8; }

// Device tables of a set built once with a plan (segment records, tile -> segment maps, merge
// groups per launch, the segments that need the top merge level).
struct SetTables {
  LongSet set{};
  std::vector<MergeLaunch> launches;  // host copies; groups_dev[i] holds launches[i].groups
  std::vector<MergeGroup*> groups_dev;
  int32_t* top_dev = nullptr;
  int ntop = 0;
};

// Launch context of one set: the set, its host description and (plans) its device tables.
struct SetRun {
  LongSet set;
  const LongSetHost* hs;
  const SetTables* tab;  // null: a single segment, groups computed in the kernels
};

// Stable LSD radix sort of every segment of the set (up to 4 passes of 8 bits; a later pass whose
// digit is the same for every key of a segment is skipped for it on the device): sorted keys end
// in b.keysA (at each segment's element base), the permutation in saved_perm (flat, segment
// ranks) or in b.valsA; b.flags gets each segment's non-finite bit and varying key bits.  In the
// first pass the input is w, or fmaf(-eta, grad, w) when grad is given.
void big_sort(const SetRun& r, const float* w, const float* grad, float eta, const BigWs& b, int32_t* saved_perm,
              hipStream_t s) {
  const int nrt = r.set.nrt;
  const int nsegs = r.set.nsegs;
  for (int pass = 0; pass < 4; ++pass) {
    const dim3 hgrid(radix_grid(nrt, hist_grid())), sgrid(radix_grid(nrt, scatter_grid()));
    { WSR_TRACE("radix_hist", s);
    if (grad)
      hipLaunchKernelGGL(k_radix_hist<true>, hgrid, dim3(kRadixThreads), 0, s, pass, r.set, w, grad, eta, b.keysA,
                         b.keysB, b.valsA, b.valsB, saved_perm, b.hist, b.tbad, b.tor, b.tand, b.flags);
    else
      hipLaunchKernelGGL(k_radix_hist<false>, hgrid, dim3(kRadixThreads), 0, s, pass, r.set, w, grad, eta, b.keysA,
                         b.keysB, b.valsA, b.valsB, saved_perm, b.hist, b.tbad, b.tor, b.tand, b.flags); }
    { WSR_TRACE("radix_rowscan", s);
    hipLaunchKernelGGL(k_radix_rowscan, dim3(256, nsegs), dim3(256), 0, s, pass, r.set, b.hist, b.totals, b.tbad,
                       b.tor, b.tand, b.flags); }
    { WSR_TRACE("radix_scatter", s);
    if (grad)
      hipLaunchKernelGGL(k_radix_scatter<true>, sgrid, dim3(kScatterThreads), 0, s, pass, r.set, w, grad, eta,
                         b.keysA, b.keysB, b.valsA, b.valsB, saved_perm, b.hist, b.totals, b.flags);
    else
      hipLaunchKernelGGL(k_radix_scatter<false>, sgrid, dim3(kScatterThreads), 0, s, pass, r.set, w, grad, eta,
                         b.keysA, b.keysB, b.valsA, b.valsB, saved_perm, b.hist, b.totals, b.flags); }
  }
}

// Tile scans hold CM tiles per thread.
int scan_cm(int max_nt) { return max_nt <= 4 * 1024 ? 4 : max_nt <= 8 * 1024 ? 8 : max_nt <= 16 * 1024 ? 16 : 32; }

// Merge levels of every segment of the set: the LDS levels, then the top level for segments of
// more than 2^14 tiles.
void big_merges(const SetRun& r, const BigWs& b, hipStream_t s) {
  std::vector<MergeLaunch> local;
  const std::vector<MergeLaunch>* launches = r.tab ? &r.tab->launches : &local;
  if (!r.tab) local = merge_launches(*r.hs);
  for (size_t i = 0; i < launches->size(); ++i) {
    const MergeLaunch& L = (*launches)[i];
    const MergeGroup* groups = r.tab ? r.tab->groups_dev[i] : nullptr;
    const int grid = (int)L.groups.size();
    WSR_TRACE("big_merge", s);
#define WSR_LAUNCH_MERGE(GM)                                                                                \
  hipLaunchKernelGGL((k_big_merge<GM, kMergeRecMax>), dim3(grid), dim3(kMergeThreads), 0, s, L.lvl_lo, L.lvl_hi, \
                     r.set, groups, b.vpos, b.vS, b.tileoff, b.lo, b.hi, b.prev_ref, b.next_ref)
    if (L.gmax <= 16)
      WSR_LAUNCH_MERGE(16);
    else if (L.gmax <= 256)
      WSR_LAUNCH_MERGE(256);
    else if (L.gmax <= 4096)
      WSR_LAUNCH_MERGE(4096);
    else
      WSR_LAUNCH_MERGE(16384);
#undef WSR_LAUNCH_MERGE
  }
  int ntop = 0;
  const int32_t* top = nullptr;
  if (r.tab) {
    ntop = r.tab->ntop;
    top = r.tab->top_dev;
  } else {
    ntop = r.hs->segs[0].nlev > kMergeLevelsInLds ? 1 : 0;
  }
  if (ntop > 0) {
    WSR_TRACE("big_merge_top", s);
    hipLaunchKernelGGL(k_big_merge_top, dim3(ntop), dim3(kTopThreads), 0, s, r.set, top, b.vpos, b.vS, b.tileoff,
                       b.lo, b.hi, b.prev_ref, b.next_ref);
  }
}

// Forward of every segment of the set (in place allowed: every read of w and grad happens in the
// sort's first pass, before any output is written).
int big_forward(const SetRun& r, const float* w, const float* grad, float eta, float* out, LamArgs lam,
                int32_t* saved_perm, uint32_t* saved_mask, void* ws, hipStream_t s, const L1Opt& l1,
                int rounds = -1, uint32_t* status = nullptr) {
  BigWs b = big_layout(*r.hs, ws);
  big_sort(r, w, grad, eta, b, saved_perm, s);
  const int nt = r.set.nt;
  const int nsegs = r.set.nsegs;
  { WSR_TRACE("big_tile_hull", s);
  hipLaunchKernelGGL(k_big_tile_hull, dim3(nt), dim3(kBigThreads), 0, s, r.set, b.keysA, lam, b.vpos, b.vS, b.hcnt,
                     b.tsum, b.hbits, rounds); }
  { WSR_TRACE("big_tile_scan", s);
#define WSR_LAUNCH_TILE_SCAN(CM)                                                                          \
  hipLaunchKernelGGL(k_big_tile_scan<CM>, dim3(nsegs), dim3(1024), 0, s, r.set, b.tsum, b.tileoff, b.hcnt, b.lo, \
                     b.hi, lam)
  switch (scan_cm(r.hs->max_nt)) {
    case 4: WSR_LAUNCH_TILE_SCAN(4); break;
    case 8: WSR_LAUNCH_TILE_SCAN(8); break;
    case 16: WSR_LAUNCH_TILE_SCAN(16); break;
    default: WSR_LAUNCH_TILE_SCAN(32); break;
  }
#undef WSR_LAUNCH_TILE_SCAN
  }
  big_merges(r, b, s);
  { WSR_TRACE("big_apply", s);
  hipLaunchKernelGGL(k_big_apply, dim3(nt), dim3(kBigThreads), 0, s, r.set, b.keysA, saved_perm, b.valsA, lam,
                     b.flags, b.hbits, b.hcnt, b.vS, b.tileoff, b.lo, b.hi, b.vpos, b.prev_ref, b.next_ref, out,
                     saved_mask, l1.beta, l1.rho, l1.kappa, l1.on, status); }
  return last_error();
}

int big_backward(const SetRun& r, const float* g, float* gw, const int32_t* perm, const uint32_t* mask, void* ws,
                 hipStream_t s) {
  BigWs b = big_layout(*r.hs, ws);
  const int nt = r.set.nt;
  float* gsorted = (float*)b.keysA;
  { WSR_TRACE("big_bwd_tile", s);
  hipLaunchKernelGGL(k_big_bwd_tile, dim3(nt), dim3(kBigThreads), 0, s, r.set, g, perm, mask, gsorted, b.tsum,
                     b.fpos, b.fG, b.lpos, b.lG); }
  { WSR_TRACE("big_bwd_scan", s);
#define WSR_LAUNCH_BWD_SCAN(CM)                                                                           \
  hipLaunchKernelGGL(k_big_bwd_scan<CM>, dim3(r.set.nsegs), dim3(1024), 0, s, r.set, b.tsum, b.fpos, b.fG, b.lpos, \
                     b.lG, b.tileoff, b.prev_pos, b.prevG, b.next_pos, b.nextG)
  switch (scan_cm(r.hs->max_nt)) {
    case 4: WSR_LAUNCH_BWD_SCAN(4); break;
    case 8: WSR_LAUNCH_BWD_SCAN(8); break;
    case 16: WSR_LAUNCH_BWD_SCAN(16); break;
    default: WSR_LAUNCH_BWD_SCAN(32); break;
  }
#undef WSR_LAUNCH_BWD_SCAN
  }
  { WSR_TRACE("big_bwd_apply", s);
  hipLaunchKernelGGL(k_big_bwd_apply, dim3(nt), dim3(kBigThreads), 0, s, r.set, gsorted, perm, mask, b.tileoff,
                     b.prev_pos, b.prevG, b.next_pos, b.nextG, gw); }
  return last_error();
}

// Statistics of every segment of the set: the sort, then the tile partials and their fixed-order
// sum per segment (records at the segments' ids).
int big_stats(const SetRun& r, const float* w, SegStats* out, void* ws, hipStream_t s) {
  BigWs b = big_layout(*r.hs, ws);
  big_sort(r, w, nullptr, 0.0f, b, nullptr, s);
  { WSR_TRACE("big_stats_tile", s);
  hipLaunchKernelGGL(k_big_stats_tile, dim3(r.set.nt), dim3(kBigThreads), 0, s, r.set, b.keysA, b.tsum, b.hcnt,
                     b.lo); }
  { WSR_TRACE("big_stats_final", s);
  hipLaunchKernelGGL(k_big_stats_final, dim3(r.set.nsegs), dim3(1024), 0, s, r.set, b.tsum, b.hcnt, b.lo, b.flags,
                     out); }
  return last_error();
}

// One long segment of a plain call, solved on its own.
struct OneSeg {
  LongSetHost hs;
  SetRun run;
  OneSeg(const int64_t* h_offsets, int32_t id) : hs(make_set(h_offsets, {id})) {
    run = SetRun{single_set(hs), &hs, nullptr};
  }
  OneSeg(const OneSeg&) = delete;
};

void small_stats(int cls, int nblocks, const SegArgs& a, const float* w, SegStats* st, hipStream_t s) {
  switch (cls) {
    case kC2048: { WSR_TRACE("seg_stats_small_2048", s);
      hipLaunchKernelGGL((k_seg_stats_small<2048, 256>), dim3(nblocks), dim3(256), 0, s, a, w, st); } break;
    case kC4096: { WSR_TRACE("seg_stats_small_4096", s);
      hipLaunchKernelGGL((k_seg_stats_small<4096, 512>), dim3(nblocks), dim3(512), 0, s, a, w, st); } break;
    default: { WSR_TRACE("seg_stats_small_8192", s);
      hipLaunchKernelGGL((k_seg_stats_small<8192, 1024>), dim3(nblocks), dim3(1024), 0, s, a, w, st); } break;
  }
}

}  // namespace
}  // namespace wsr

using namespace wsr;
static_assert(sizeof(SegStats) == sizeof(wsr_segment_stats_t), "stats layout");

struct wsr_plan {
  int64_t n_seg = 0;
  int64_t total = 0;
  int device = 0;
  int64_t* d_offsets = nullptr;
  int32_t* d_sched = nullptr;                // all small schedules back to back
  int64_t sched_off[kNumSmall] = {0, 0, 0};  // start of class c in d_sched
  int64_t sched_cnt[kNumSmall] = {0, 0, 0};
  std::vector<int64_t> h_offsets;
  std::vector<int32_t> big_segs;  // long segments, in order
  bool word_aligned = false;      // every offset a multiple of 32 (no mask zero fill needed)
  // merge route per size class (short classes, then long segments): cap on ImminentCollisions
  // rounds before the bounded-depth hull merge (0 = hull merge only), or -1: EndCollisions
  // (short classes only)
  int rounds[kNumSmall + 1] = {kIcaRounds, kIcaRounds, kIcaRounds, kIcaRounds};
  int small_route(int c) const { return rounds[c] >= 0 ? rounds[c] : kRouteEnd; }
  // sort route per short size class (kSortBucket or kSortRadix)
  int sort[kNumSmall] = {kSortBucket, kSortBucket, kSortBucket};
  uint32_t* d_status = nullptr;  // sticky status word (kStatusNonFinite), read by wsr_read_status
  // the long segments as one set, solved by one launch sequence; its device tables live in d_tables
  LongSetHost longs;
  SetTables tab;
  void* d_tables = nullptr;
  SetRun long_run() const { return SetRun{tab.set, &longs, &tab}; }
};

namespace {

// Device tables of the plan's long segments (one allocation, at plan creation): the segment
// records, the radix-tile and hull-tile -> segment maps, the merge groups of every launch and the
// segments that need the top merge level.
int build_set_tables(wsr_plan* p) {
  const LongSetHost& hs = p->longs;
  if (hs.segs.empty()) return WSR_OK;
  SetTables& t = p->tab;
  t.launches = merge_launches(hs);
  std::vector<int32_t> rseg(hs.nrt), hseg(hs.nt), top;
  for (size_t si = 0; si < hs.segs.size(); ++si) {
    const LongSeg& g = hs.segs[si];
    for (int i = 0; i < g.nrt; ++i) rseg[g.rbase + i] = (int32_t)si;
    for (int i = 0; i < g.nt; ++i) hseg[g.tbase + i] = (int32_t)si;
    if (g.nlev > kMergeLevelsInLds) top.push_back((int32_t)si);
  }
  // one buffer: segments, rseg, hseg, top list, then each launch's groups (256-byte aligned parts)
  std::vector<size_t> parts = {sizeof(LongSeg) * hs.segs.size(), sizeof(int32_t) * rseg.size(),
                               sizeof(int32_t) * hseg.size(), sizeof(int32_t) * std::max<size_t>(top.size(), 1)};
  for (const MergeLaunch& L : t.launches) parts.push_back(sizeof(MergeGroup) * L.groups.size());
  size_t total = 0;
  std::vector<size_t> at;
  for (size_t b : parts) {
    at.push_back(total);
    total += align_up(b);
  }
  std::vector<char> host(total, 0);
  auto put = [&](int i, const void* src, size_t n) { if (n) std::memcpy(host.data() + at[i], src, n); };
  put(0, hs.segs.data(), parts[0]);
  put(1, rseg.data(), parts[1]);
  put(2, hseg.data(), parts[2]);
  put(3, top.data(), sizeof(int32_t) * top.size());
  for (size_t i = 0; i < t.launches.size(); ++i) put(4 + (int)i, t.launches[i].groups.data(), parts[4 + i]);
  if (hipMalloc(&p->d_tables, total) != hipSuccess) return WSR_ERR_HIP;
  if (hipMemcpy(p->d_tables, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) return WSR_ERR_HIP;
  char* base = (char*)p->d_tables;
  t.set = LongSet{};
  t.set.segs = (const LongSeg*)(base + at[0]);
  t.set.rseg = (const int32_t*)(base + at[1]);
  t.set.hseg = (const int32_t*)(base + at[2]);
  t.set.nsegs = (int)hs.segs.size();
  t.set.nrt = hs.nrt;
  t.set.nt = hs.nt;
  t.top_dev = (int32_t*)(base + at[3]);
  t.ntop = (int)top.size();
  for (size_t i = 0; i < t.launches.size(); ++i) t.groups_dev.push_back((MergeGroup*)(base + at[4 + i]));
  return WSR_OK;
}

}  // namespace

extern "C" {

int wsr_version(void) { return 200; }

const char* wsr_status_string(int status) {
  switch (status) {
    case WSR_OK: return "ok";
    case WSR_ERR_INVALID: return "invalid argument";
    case WSR_ERR_WORKSPACE: return "workspace too small";
    case WSR_ERR_HIP: return "HIP launch error";
    case WSR_ERR_UNSUPPORTED: return "segment longer than WSR_MAX_SEGMENT";
    default: return "unknown status";
  }
}

int wsr_workspace_bytes(const int64_t* h_offsets, int64_t n_seg, size_t* bytes) {
  if (!bytes) return WSR_ERR_INVALID;
  int64_t mb = 0;
  const int rc = validate_offsets(h_offsets, n_seg, &mb);
  if (rc) return rc;
  *bytes = big_bytes(mb);
  return WSR_OK;
}

}  // extern "C"

namespace {

int forward_impl(const float* w, float* out, const int64_t* h_offsets, int64_t n_seg, float lambda,
                 int32_t* saved_perm, uint32_t* saved_mask, void* ws, size_t ws_bytes, void* stream,
                 const L1Opt& l1) {
  (void)hipGetLastError();  // report only errors of this call
  if (!w || !out) return WSR_ERR_INVALID;
  if ((saved_perm == nullptr) != (saved_mask == nullptr)) return WSR_ERR_INVALID;
  if (!std::isfinite(lambda) || lambda < 0.0f) return WSR_ERR_INVALID;
  int64_t mb = 0;
  int rc = validate_offsets(h_offsets, n_seg, &mb);
  if (rc) return rc;
  const size_t need = big_bytes(mb);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) return WSR_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const int64_t total = h_offsets[n_seg];
  if (saved_mask && !offsets_word_aligned(h_offsets, n_seg)) zero_words(saved_mask, ceil_div(total, 32), s);
  for (int64_t seg = 0; seg < n_seg; ++seg) {
    const int64_t start = h_offsets[seg];
    const int64_t d = h_offsets[seg + 1] - start;
    const int cls = size_class(d);
    if (cls == kSkip) continue;
    if (cls == kBig) {
      const OneSeg one(h_offsets, (int32_t)seg);
      rc = big_forward(one.run, w, nullptr, 0.0f, out, LamArgs{nullptr, lambda, 1.0f}, saved_perm, saved_mask, ws, s,
                       l1);
      if (rc) return rc;
      continue;
    }
    SegArgs a{nullptr, nullptr, nullptr, lambda, start, (int)d, 0, l1.beta, l1.rho, l1.on, l1.kappa};
    small_fwd(cls, 1, a, w, out, saved_perm, saved_mask, s);
  }
  return last_error();
}

#ifdef WSR_PHASE_CLOCKS
// Measurement build: where the short-segment forward writes its phase timestamps (kPhaseSlots per
// workgroup, the size classes of one call one after another), and for how many workgroups.
unsigned long long* g_phase_clocks = nullptr;
int64_t g_phase_blocks = 0;
#endif

int forward_batched_impl(const wsr_plan* plan, const float* w, float* out, const float* d_lambda,
                         float lambda_scalar, int32_t* saved_perm, uint32_t* saved_mask, void* ws,
                         size_t ws_bytes, void* stream, const L1Opt& l1) {
  (void)hipGetLastError();  // report only errors of this call
  if (!plan || !w || !out) return WSR_ERR_INVALID;
  if ((saved_perm == nullptr) != (saved_mask == nullptr)) return WSR_ERR_INVALID;
  if (!d_lambda && (!std::isfinite(lambda_scalar) || lambda_scalar < 0.0f)) return WSR_ERR_INVALID;
  const size_t need = set_bytes(plan->longs);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) return WSR_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (saved_mask && !plan->word_aligned) zero_words(saved_mask, ceil_div(plan->total, 32), s);
#ifdef WSR_PHASE_CLOCKS
  int64_t clock_base = 0;
#endif
  for (int c = 0; c < kNumSmall; ++c) {
    if (plan->sched_cnt[c] == 0) continue;
    SegArgs a{plan->d_offsets, plan->d_sched + plan->sched_off[c], d_lambda, lambda_scalar, 0, 0, 0,
              l1.beta, l1.rho, l1.on, l1.kappa};
    a.merge_rounds = plan->small_route(c);
    a.status = plan->d_status;
    a.sort_route = plan->sort[c];
#ifdef WSR_PHASE_CLOCKS
    if (g_phase_clocks && clock_base + plan->sched_cnt[c] <= g_phase_blocks)
      a.clocks = g_phase_clocks + clock_base * kPhaseSlots;
    clock_base += plan->sched_cnt[c];
#endif
    small_fwd(c, (int)plan->sched_cnt[c], a, w, out, saved_perm, saved_mask, s);
  }
  if (!plan->longs.segs.empty()) {
    const int rc = big_forward(plan->long_run(), w, nullptr, 0.0f, out, LamArgs{d_lambda, lambda_scalar, 1.0f},
                               saved_perm, saved_mask, ws, s, l1, plan->rounds[kNumSmall], plan->d_status);
    if (rc) return rc;
  }
  return last_error();
}

// The step's form: lambda multiplier of the short-segment kernels and the l1 / rewinding options.
struct StepForm {
  float lam_mul;
  L1Opt l1;
};
StepForm step_form(float eta, float beta, float rho, int flags) {
  const bool variant = (flags & WSR_STEP_ETA_IN_DISPLACEMENT) != 0;
  // standard: the prox of eta*(alpha R + beta l1): lambda = eta*alpha, beta' = eta*beta (FP32);
  // variant: alpha and beta unscaled, eta on the rewinding line
  return StepForm{variant ? 1.0f : eta, L1Opt{variant ? beta : eta * beta, rho, 1, variant ? eta : 1.0f}};
}

int step_args_ok(const wsr_plan* plan, const float* w, const float* grad, float eta, const float* out,
                 const float* d_alpha, float alpha_scalar, float beta, float rho, int flags, const void* ws,
                 size_t ws_bytes) {
  if (!plan || !w || !grad || !out) return WSR_ERR_INVALID;
  if (flags & ~WSR_STEP_ETA_IN_DISPLACEMENT) return WSR_ERR_INVALID;
  if (!std::isfinite(eta) || eta < 0.0f || !l1_args_ok(beta, rho)) return WSR_ERR_INVALID;
  if (!d_alpha && (!std::isfinite(alpha_scalar) || alpha_scalar < 0.0f)) return WSR_ERR_INVALID;
  const size_t need = set_bytes(plan->longs);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) return WSR_ERR_WORKSPACE;
  return WSR_OK;
}

// The fused launch of size class c over its first nblocks segments with merge route `route` and
// sort route `sort`.
void step_small(const wsr_plan* plan, int c, int nblocks, int route, int sort, const float* w, const float* grad,
                float eta, float* out, const float* d_alpha, float alpha_scalar, const StepForm& f, hipStream_t s) {
  SegArgs a{plan->d_offsets, plan->d_sched + plan->sched_off[c], d_alpha, alpha_scalar, 0, 0, 0,
            f.l1.beta, f.l1.rho, f.l1.on, f.l1.kappa, grad, eta, f.lam_mul, route, plan->d_status, sort};
  small_fwd(c, nblocks, a, w, out, nullptr, nullptr, s);
}

// The long segments of the step, as one set: the sort's first pass reads fmaf(-eta, grad, w), so
// the gradient step costs no pass of its own; lambda = alpha_s * lam_mul on the device.
int step_big(const wsr_plan* plan, int rounds, const float* w, const float* grad, float eta, float* out,
             const float* d_alpha, float alpha_scalar, const StepForm& f, void* ws, hipStream_t s) {
  return big_forward(plan->long_run(), w, grad, eta, out, LamArgs{d_alpha, alpha_scalar, f.lam_mul}, nullptr, nullptr,
                     ws, s, f.l1, rounds, plan->d_status);
}

int step_batched_impl(const wsr_plan* plan, const float* w, const float* grad, float eta, float* out,
                      const float* d_alpha, float alpha_scalar, float beta, float rho, int flags, void* ws,
                      size_t ws_bytes, void* stream) {
  (void)hipGetLastError();  // report only errors of this call
  int rc = step_args_ok(plan, w, grad, eta, out, d_alpha, alpha_scalar, beta, rho, flags, ws, ws_bytes);
  if (rc) return rc;
  const StepForm f = step_form(eta, beta, rho, flags);
  hipStream_t s = (hipStream_t)stream;
  for (int c = 0; c < kNumSmall; ++c) {
    if (plan->sched_cnt[c] == 0) continue;
    step_small(plan, c, (int)plan->sched_cnt[c], plan->small_route(c), plan->sort[c], w, grad, eta, out, d_alpha,
               alpha_scalar, f, s);
  }
  if (!plan->longs.segs.empty()) {
    rc = step_big(plan, plan->rounds[kNumSmall], w, grad, eta, out, d_alpha, alpha_scalar, f, ws, s);
    if (rc) return rc;
  }
  return last_error();
}

// Autotuner core: for every short size class, times the batched launch of the class alone under
// each candidate merge route and keeps the fastest; EndCollisions is a candidate only when a probe
// over the class's first segments (one workgroup per CU pair) shows it no slower than 1.5x the
// default route there.  Then, with that merge route, the radix-only sort route against the
// bucket-rank sort (the radix sort wins on rows with many equal weights, where the bucket sort
// takes its tie path or overflows).  Long segments: the caps {0, kIcaRounds, 16}, timed on all of
// them together.
//   small(c, nblocks, route, sort): launches class c over its first nblocks segments
//   big(rounds): runs the plan's long segments (one set), returns a status
template <class SmallFn, class BigFn>
int autotune_impl(wsr_plan* plan, SmallFn&& small, BigFn&& big, hipStream_t s) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return WSR_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return WSR_ERR_HIP;
  }
  constexpr int kReps = 3;
  int rc = WSR_OK;
  // a warm-up launch, then `reps` timed launches
  auto time_it = [&](auto&& launch, int reps, float* ms) -> int {
    launch();
    if (hipEventRecord(e0, s) != hipSuccess) return WSR_ERR_HIP;
    for (int r = 0; r < reps; ++r) launch();
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return WSR_ERR_HIP;
    if (hipEventElapsedTime(ms, e0, e1) != hipSuccess) return WSR_ERR_HIP;
    return last_error();
  };
  for (int c = 0; c < kNumSmall && rc == WSR_OK; ++c) {
    const int cnt = (int)plan->sched_cnt[c];
    if (cnt == 0) continue;
    std::vector<int> cand = {0, 2, kIcaRounds, 16, 64};  // 0: hull merge only
    {
      const int np = std::min(cnt, 2 * cu_count());
      float t_def = 0.0f, t_end = 0.0f;
      rc = time_it([&] { small(c, np, kIcaRounds, kSortBucket); }, 1, &t_def);
      if (rc) break;
      rc = time_it([&] { small(c, np, kRouteEnd, kSortBucket); }, 1, &t_end);
      if (rc) break;
      if (t_end <= 1.5f * t_def) cand.push_back(kRouteEnd);
    }
    float best = 0.0f;
    int best_route = kIcaRounds;
    for (size_t i = 0; i < cand.size(); ++i) {
      float ms = 0.0f;
      rc = time_it([&] { small(c, cnt, cand[i], kSortBucket); }, kReps, &ms);
      if (rc) break;
      if (i == 0 || ms < best) {
        best = ms;
        best_route = cand[i];
      }
    }
    if (rc) break;
    plan->rounds[c] = best_route == kRouteEnd ? -1 : best_route;
    float t_radix = 0.0f;
    rc = time_it([&] { small(c, cnt, best_route, kSortRadix); }, kReps, &t_radix);
    if (rc) break;
    plan->sort[c] = t_radix < best ? kSortRadix : kSortBucket;
  }
  if (rc == WSR_OK && !plan->longs.segs.empty()) {
    float best = 0.0f;
    bool first = true;
    for (int r : {0, kIcaRounds, 16}) {
      float ms = 0.0f;
      int lrc = WSR_OK;
      rc = time_it([&] {
        const int e = big(r);
        if (e) lrc = e;
      }, kReps, &ms);
      if (!rc) rc = lrc;
      if (rc) break;
      if (first || ms < best) {
        best = ms;
        first = false;
        plan->rounds[kNumSmall] = r;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // namespace

// ---- fixed device scratch of the allocation-free forward (wsr_prox_forward_noalloc)
// One copy per GPU, created with the code object and held until the process ends.  In host code
// the array's name is not a device address: the kernels get the address that
// hipGetSymbolAddress returns for the current device, looked up once per device.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static_assert(kNoAllocScratchBytes == WSR_NOALLOC_SCRATCH_BYTES, "scratch size as declared in the header");
static_assert(kSortBucket == WSR_SORT_BUCKET && kSortRadix == WSR_SORT_RADIX, "sort routes as declared in the header");
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

int noalloc_scratch(void** out) {
  static std::mutex mu;
  static std::vector<void*> per_device;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return WSR_ERR_HIP;
  std::lock_guard<std::mutex> lk(mu);
  if ((size_t)dev >= per_device.size()) per_device.resize((size_t)dev + 1, nullptr);
  if (per_device[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return WSR_ERR_HIP;
    per_device[dev] = p;
  }
  *out = per_device[dev];
  return WSR_OK;
}

extern "C" {

int wsr_prox_forward(const float* w, float* out, const int64_t* h_offsets, int64_t n_seg, float lambda,
                     int32_t* saved_perm, uint32_t* saved_mask, void* ws, size_t ws_bytes, void* stream) {
  return forward_impl(w, out, h_offsets, n_seg, lambda, saved_perm, saved_mask, ws, ws_bytes, stream, L1Opt{});
}

int wsr_prox_forward_noalloc(const float* w, float* out, const int64_t* h_offsets, int64_t n_seg, float lambda,
                             int32_t* saved_perm, uint32_t* saved_mask, void* stream) {
  int64_t mb = 0;
  int rc = validate_offsets(h_offsets, n_seg, &mb);
  if (rc) return rc;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  if (mb > 0) {
    if (big_bytes(mb) > kNoAllocScratchBytes) return WSR_ERR_WORKSPACE;  // beyond the fixed scratch
    rc = noalloc_scratch(&ws);
    if (rc) return rc;
    ws_bytes = kNoAllocScratchBytes;
  }
  return forward_impl(w, out, h_offsets, n_seg, lambda, saved_perm, saved_mask, ws, ws_bytes, stream, L1Opt{});
}

int wsr_prox_l1_forward(const float* w, float* out, const int64_t* h_offsets, int64_t n_seg, float lambda,
                        float beta, float rho, void* ws, size_t ws_bytes, void* stream) {
  if (!l1_args_ok(beta, rho)) return WSR_ERR_INVALID;
  return forward_impl(w, out, h_offsets, n_seg, lambda, nullptr, nullptr, ws, ws_bytes, stream,
                      L1Opt{beta, rho, 1});
}

int wsr_segment_stats(const float* w, const int64_t* h_offsets, int64_t n_seg, wsr_segment_stats_t* d_stats,
                      void* ws, size_t ws_bytes, void* stream) {
  (void)hipGetLastError();  // report only errors of this call
  if (!w || !d_stats) return WSR_ERR_INVALID;
  int64_t mb = 0;
  int rc = validate_offsets(h_offsets, n_seg, &mb);
  if (rc) return rc;
  if (n_seg > INT32_MAX) return WSR_ERR_UNSUPPORTED;
  const size_t need = big_bytes(mb);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) return WSR_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  SegStats* st = reinterpret_cast<SegStats*>(d_stats);
  zero_words(reinterpret_cast<uint32_t*>(st), n_seg * (int64_t)(sizeof(SegStats) / 4), s);  // empty segments
  for (int64_t seg = 0; seg < n_seg; ++seg) {
    const int64_t start = h_offsets[seg];
    const int64_t d = h_offsets[seg + 1] - start;
    const int cls = size_class(d);
    if (cls == kSkip) continue;
    if (cls == kBig) {
      const OneSeg one(h_offsets, (int32_t)seg);
      rc = big_stats(one.run, w, st, ws, s);
      if (rc) return rc;
      continue;
    }
    SegArgs a{nullptr, nullptr, nullptr, 0.0f, start, (int)d, (int)seg};
    small_stats(cls, 1, a, w, st, s);
  }
  return last_error();
}

int wsr_prox_backward(const float* grad_out, float* grad_w, const int64_t* h_offsets, int64_t n_seg,
                      const int32_t* saved_perm, const uint32_t* saved_mask, void* ws, size_t ws_bytes,
                      void* stream) {
  (void)hipGetLastError();  // report only errors of this call
  if (!grad_out || !grad_w || !saved_perm || !saved_mask || grad_out == grad_w) return WSR_ERR_INVALID;
  int64_t mb = 0;
  int rc = validate_offsets(h_offsets, n_seg, &mb);
  if (rc) return rc;
  const size_t need = big_bytes(mb);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) return WSR_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  for (int64_t seg = 0; seg < n_seg; ++seg) {
    const int64_t start = h_offsets[seg];
    const int64_t d = h_offsets[seg + 1] - start;
    const int cls = size_class(d);
    if (cls == kSkip) continue;
    if (cls == kBig) {
      const OneSeg one(h_offsets, (int32_t)seg);
      rc = big_backward(one.run, grad_out, grad_w, saved_perm, saved_mask, ws, s);
      if (rc) return rc;
      continue;
    }
    SegArgs a{nullptr, nullptr, nullptr, 0.0f, start, (int)d, 0};
    small_bwd(cls, 1, a, grad_out, grad_w, saved_perm, saved_mask, s);
  }
  return last_error();
}

int wsr_plan_create(const int64_t* h_offsets, int64_t n_seg, int flags, wsr_plan** plan) {
  if (!plan || (flags & ~(WSR_PLAN_MERGE_HULL | WSR_PLAN_MERGE_END))) return WSR_ERR_INVALID;
  if ((flags & WSR_PLAN_MERGE_HULL) && (flags & WSR_PLAN_MERGE_END)) return WSR_ERR_INVALID;
  *plan = nullptr;
  int64_t mb = 0;
  int rc = validate_offsets(h_offsets, n_seg, &mb);
  if (rc) return rc;
  if (n_seg > INT32_MAX) return WSR_ERR_UNSUPPORTED;
  wsr_plan* p = new wsr_plan();
  p->n_seg = n_seg;
  p->total = h_offsets[n_seg];
  p->h_offsets.assign(h_offsets, h_offsets + n_seg + 1);
  p->word_aligned = offsets_word_aligned(h_offsets, n_seg);
  if (flags & WSR_PLAN_MERGE_HULL)
    for (int c = 0; c <= kNumSmall; ++c) p->rounds[c] = 0;
  if (flags & WSR_PLAN_MERGE_END)
    for (int c = 0; c < kNumSmall; ++c) p->rounds[c] = -1;
  (void)hipGetDevice(&p->device);
  // schedules: segments of each class, longest first (short tail of the launch)
  std::vector<int32_t> cls_list[kNumSmall];
  for (int64_t s = 0; s < n_seg; ++s) {
    const int64_t d = h_offsets[s + 1] - h_offsets[s];
    const int c = size_class(d);
    if (c == kSkip) continue;
    if (c == kBig)
      p->big_segs.push_back((int32_t)s);
    else
      cls_list[c].push_back((int32_t)s);
  }
  std::vector<int32_t> sched;
  for (int c = 0; c < kNumSmall; ++c) {
    std::stable_sort(cls_list[c].begin(), cls_list[c].end(), [&](int32_t a, int32_t b) {
      return (h_offsets[a + 1] - h_offsets[a]) > (h_offsets[b + 1] - h_offsets[b]);
    });
    p->sched_off[c] = (int64_t)sched.size();
    p->sched_cnt[c] = (int64_t)cls_list[c].size();
    sched.insert(sched.end(), cls_list[c].begin(), cls_list[c].end());
  }
  if (hipMalloc(&p->d_offsets, sizeof(int64_t) * (n_seg + 1)) != hipSuccess) {
    delete p;
    return WSR_ERR_HIP;
  }
  if (hipMemcpy(p->d_offsets, h_offsets, sizeof(int64_t) * (n_seg + 1), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p->d_offsets);
    delete p;
    return WSR_ERR_HIP;
  }
  if (hipMalloc(&p->d_status, sizeof(uint32_t)) != hipSuccess ||
      hipMemset(p->d_status, 0, sizeof(uint32_t)) != hipSuccess) {
    (void)hipFree(p->d_offsets);
    if (p->d_status) (void)hipFree(p->d_status);
    delete p;
    return WSR_ERR_HIP;
  }
  if (!sched.empty()) {
    if (hipMalloc(&p->d_sched, sizeof(int32_t) * sched.size()) != hipSuccess ||
        hipMemcpy(p->d_sched, sched.data(), sizeof(int32_t) * sched.size(), hipMemcpyHostToDevice) !=
            hipSuccess) {
      (void)wsr_plan_destroy(p);
      return WSR_ERR_HIP;
    }
  }
  p->longs = make_set(h_offsets, p->big_segs);
  if (build_set_tables(p) != WSR_OK) {
    (void)wsr_plan_destroy(p);
    return WSR_ERR_HIP;
  }
  *plan = p;
  return WSR_OK;
}

int wsr_plan_destroy(wsr_plan* plan) {
  if (!plan) return WSR_ERR_INVALID;
  if (plan->d_offsets) (void)hipFree(plan->d_offsets);
  if (plan->d_sched) (void)hipFree(plan->d_sched);
  if (plan->d_status) (void)hipFree(plan->d_status);
  if (plan->d_tables) (void)hipFree(plan->d_tables);
  delete plan;
  return WSR_OK;
}

int wsr_read_status(const wsr_plan* plan, uint32_t* flags, int clear, void* stream) {
  if (!plan || !flags) return WSR_ERR_INVALID;
  (void)hipGetLastError();  // report only errors of this call
  hipStream_t s = (hipStream_t)stream;
  uint32_t v = 0;
  if (hipMemcpyAsync(&v, plan->d_status, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
    return WSR_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return WSR_ERR_HIP;
  if (clear) {
    zero_words(plan->d_status, 1, s);
    if (hipStreamSynchronize(s) != hipSuccess) return WSR_ERR_HIP;
  }
  *flags = v;
  return last_error();
}

int wsr_plan_workspace_bytes(const wsr_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return WSR_ERR_INVALID;
  *bytes = set_bytes(plan->longs);
  return WSR_OK;
}

int wsr_plan_merge_rounds(const wsr_plan* plan, int32_t* rounds) {
  if (!plan || !rounds) return WSR_ERR_INVALID;
  for (int c = 0; c <= kNumSmall; ++c) rounds[c] = plan->rounds[c];
  return WSR_OK;
}

int wsr_plan_set_merge_rounds(wsr_plan* plan, const int32_t* rounds) {
  if (!plan || !rounds) return WSR_ERR_INVALID;
  for (int c = 0; c <= kNumSmall; ++c)
    if (rounds[c] < (c < kNumSmall ? -1 : 0) || rounds[c] > kMaxMergeRounds) return WSR_ERR_INVALID;
  for (int c = 0; c <= kNumSmall; ++c) plan->rounds[c] = rounds[c];
  return WSR_OK;
}

int wsr_plan_sort_routes(const wsr_plan* plan, int32_t* routes) {
  if (!plan || !routes) return WSR_ERR_INVALID;
  for (int c = 0; c < kNumSmall; ++c) routes[c] = plan->sort[c];
  return WSR_OK;
}

int wsr_plan_set_sort_routes(wsr_plan* plan, const int32_t* routes) {
  if (!plan || !routes) return WSR_ERR_INVALID;
  for (int c = 0; c < kNumSmall; ++c)
    if (routes[c] != kSortBucket && routes[c] != kSortRadix) return WSR_ERR_INVALID;
  for (int c = 0; c < kNumSmall; ++c) plan->sort[c] = routes[c];
  return WSR_OK;
}

int wsr_plan_autotune(wsr_plan* plan, const float* w, float* out, const float* d_lambda, float lambda_scalar,
                      void* ws, size_t ws_bytes, void* stream) {
  (void)hipGetLastError();  // report only errors of this call
  if (!plan || !w || !out || out == w) return WSR_ERR_INVALID;
  if (!d_lambda && (!std::isfinite(lambda_scalar) || lambda_scalar < 0.0f)) return WSR_ERR_INVALID;
  const size_t need = set_bytes(plan->longs);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) return WSR_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  return autotune_impl(
      plan,
      [&](int c, int nblocks, int route, int sort) {
        SegArgs a{plan->d_offsets, plan->d_sched + plan->sched_off[c], d_lambda, lambda_scalar, 0, 0, 0};
        a.merge_rounds = route;
        a.sort_route = sort;
        small_fwd(c, nblocks, a, w, out, nullptr, nullptr, s);
      },
      [&](int rounds) {
        return big_forward(plan->long_run(), w, nullptr, 0.0f, out, LamArgs{d_lambda, lambda_scalar, 1.0f}, nullptr,
                           nullptr, ws, s, L1Opt{}, rounds);
      },
      s);
}

int wsr_plan_autotune_step(wsr_plan* plan, const float* w, const float* grad, float eta, float* scratch,
                           const float* d_alpha, float alpha_scalar, float beta, float rho, int flags, void* ws,
                           size_t ws_bytes, void* stream) {
  (void)hipGetLastError();  // report only errors of this call
  int rc = step_args_ok(plan, w, grad, eta, scratch, d_alpha, alpha_scalar, beta, rho, flags, ws, ws_bytes);
  if (rc) return rc;
  if (scratch == w || scratch == grad) return WSR_ERR_INVALID;
  const StepForm f = step_form(eta, beta, rho, flags);
  hipStream_t s = (hipStream_t)stream;
  return autotune_impl(
      plan,
      [&](int c, int nblocks, int route, int sort) {
        step_small(plan, c, nblocks, route, sort, w, grad, eta, scratch, d_alpha, alpha_scalar, f, s);
      },
      [&](int rounds) { return step_big(plan, rounds, w, grad, eta, scratch, d_alpha, alpha_scalar, f, ws, s); },
      s);
}

int wsr_prox_forward_batched(const wsr_plan* plan, const float* w, float* out, const float* d_lambda,
                             float lambda_scalar, int32_t* saved_perm, uint32_t* saved_mask, void* ws,
                             size_t ws_bytes, void* stream) {
  return forward_batched_impl(plan, w, out, d_lambda, lambda_scalar, saved_perm, saved_mask, ws, ws_bytes,
                              stream, L1Opt{});
}

int wsr_prox_l1_forward_batched(const wsr_plan* plan, const float* w, float* out, const float* d_lambda,
                                float lambda_scalar, float beta, float rho, void* ws, size_t ws_bytes,
                                void* stream) {
  if (!l1_args_ok(beta, rho)) return WSR_ERR_INVALID;
  return forward_batched_impl(plan, w, out, d_lambda, lambda_scalar, nullptr, nullptr, ws, ws_bytes, stream,
                              L1Opt{beta, rho, 1});
}

int wsr_prox_step_batched(const wsr_plan* plan, const float* w, const float* grad, float eta, float* out,
                          const float* d_alpha, float alpha_scalar, float beta, float rho, int flags, void* ws,
                          size_t ws_bytes, void* stream) {
  return step_batched_impl(plan, w, grad, eta, out, d_alpha, alpha_scalar, beta, rho, flags, ws, ws_bytes,
                           stream);
}

int wsr_segment_stats_batched(const wsr_plan* plan, const float* w, wsr_segment_stats_t* d_stats, void* ws,
                              size_t ws_bytes, void* stream) {
  (void)hipGetLastError();  // report only errors of this call
  if (!plan || !w || !d_stats) return WSR_ERR_INVALID;
  const size_t need = set_bytes(plan->longs);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) return WSR_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  SegStats* st = reinterpret_cast<SegStats*>(d_stats);
  zero_words(reinterpret_cast<uint32_t*>(st), plan->n_seg * (int64_t)(sizeof(SegStats) / 4), s);
  for (int c = 0; c < kNumSmall; ++c) {
    if (plan->sched_cnt[c] == 0) continue;
    SegArgs a{plan->d_offsets, plan->d_sched + plan->sched_off[c], nullptr, 0.0f, 0, 0, 0};
    a.sort_route = plan->sort[c];
    small_stats(c, (int)plan->sched_cnt[c], a, w, st, s);
  }
  if (!plan->longs.segs.empty()) {
    const int rc = big_stats(plan->long_run(), w, st, ws, s);
    if (rc) return rc;
  }
  return last_error();
}

int wsr_prox_backward_batched(const wsr_plan* plan, const float* grad_out, float* grad_w,
                              const int32_t* saved_perm, const uint32_t* saved_mask, void* ws, size_t ws_bytes,
                              void* stream) {
  (void)hipGetLastError();  // report only errors of this call
  if (!plan || !grad_out || !grad_w || !saved_perm || !saved_mask || grad_out == grad_w) return WSR_ERR_INVALID;
  const size_t need = set_bytes(plan->longs);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) return WSR_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
#ifdef WSR_PHASE_CLOCKS
  int64_t clock_base = 0;
#endif
  for (int c = 0; c < kNumSmall; ++c) {
    if (plan->sched_cnt[c] == 0) continue;
    SegArgs a{plan->d_offsets, plan->d_sched + plan->sched_off[c], nullptr, 0.0f, 0, 0, 0};
#ifdef WSR_PHASE_CLOCKS
    if (g_phase_clocks && clock_base + plan->sched_cnt[c] <= g_phase_blocks)
      a.clocks = g_phase_clocks + clock_base * kPhaseSlots;
    clock_base += plan->sched_cnt[c];
#endif
    small_bwd(c, (int)plan->sched_cnt[c], a, grad_out, grad_w, saved_perm, saved_mask, s);
  }
  if (!plan->longs.segs.empty()) {
    const int rc = big_backward(plan->long_run(), grad_out, grad_w, saved_perm, saved_mask, ws, s);
    if (rc) return rc;
  }
  return last_error();
}

int wsr_trace_enable(int on) {
  std::lock_guard<std::mutex> lk(g_trace.mu);
  if (on && g_trace.ev.empty()) {
    g_trace.ev.resize(2 * kTracePool);
    for (auto& e : g_trace.ev)
      if (hipEventCreate(&e) != hipSuccess) return WSR_ERR_HIP;
  }
  g_trace.on = on != 0;
  return WSR_OK;
}

int wsr_trace_collect(int max_entries, char* names, int64_t* counts, double* total_ms, int* n_out) {
  if (max_entries < 0 || (max_entries > 0 && (!names || !counts || !total_ms)) || !n_out) return WSR_ERR_INVALID;
  std::lock_guard<std::mutex> lk(g_trace.mu);
  std::vector<std::pair<const char*, std::pair<int64_t, double>>> agg;
  int rc = WSR_OK;
  for (const TraceRec& r : g_trace.recs) {
    if (hipEventSynchronize(g_trace.ev[2 * r.ev + 1]) != hipSuccess) {
      rc = WSR_ERR_HIP;
      continue;
    }
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, g_trace.ev[2 * r.ev], g_trace.ev[2 * r.ev + 1]) != hipSuccess) {
      rc = WSR_ERR_HIP;
      continue;
    }
    auto it = std::find_if(agg.begin(), agg.end(), [&](const auto& a) { return std::strcmp(a.first, r.name) == 0; });
    if (it == agg.end()) {
      agg.push_back({r.name, {1, (double)ms}});
    } else {
      it->second.first += 1;
      it->second.second += ms;
    }
  }
  g_trace.recs.clear();
  int n = 0;
  for (const auto& a : agg) {
    if (n >= max_entries) break;
    std::strncpy(names + 64 * n, a.first, 63);
    names[64 * n + 63] = 0;
    counts[n] = a.second.first;
    total_ms[n] = a.second.second;
    ++n;
  }
  *n_out = n;
  return rc;
}

#ifdef WSR_PHASE_CLOCKS
// Measurement build only (not declared in the public header): the buffer of kPhaseSlots
// timestamps per workgroup that later batched forwards and backwards of short segments fill
// (null: none), and the device's wall-clock rate in kHz.
__attribute__((visibility("default"))) int wsr_phase_clock_buffer(void* clocks, int64_t n_blocks) {
  if (n_blocks < 0 || (clocks == nullptr) != (n_blocks == 0)) return WSR_ERR_INVALID;
  g_phase_clocks = (unsigned long long*)clocks;
  g_phase_blocks = n_blocks;
  return WSR_OK;
}
__attribute__((visibility("default"))) int wsr_phase_clock_rate_khz(int* khz) {
  int dev = 0;
  if (!khz || hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
    return WSR_ERR_HIP;
  return WSR_OK;
}
__attribute__((visibility("default"))) int wsr_phase_clock_slots(void) { return kPhaseSlots; }
// The buffer of the tile merge launches' timestamps (kMergeClockLaunches x kMergeClockGroups x
// kMergeClockSlots words; null: none).
__attribute__((visibility("default"))) int wsr_phase_merge_clock_buffer(void* clocks) {
  return set_merge_clock_buffer(clocks) == 0 ? WSR_OK : WSR_ERR_HIP;
}
// Resident workgroups per CU of the short-segment forward of size class cls (default merge route)
// by the runtime's occupancy calculator.
__attribute__((visibility("default"))) int wsr_phase_occupancy(int cls, int* blocks_per_cu) {
  if (!blocks_per_cu || cls < 0 || cls >= kNumSmall) return WSR_ERR_INVALID;
  hipError_t e;
  switch (cls) {
    case kC2048: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_prox_fwd_small<2048, 256, false>, 256, 0); break;
    case kC4096: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_prox_fwd_small<4096, 512, false>, 512, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_prox_fwd_small<8192, 1024, false>, 1024, 0); break;
  }
  return e == hipSuccess ? WSR_OK : WSR_ERR_HIP;
}
#endif

}  // extern "C"
