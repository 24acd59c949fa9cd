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

// Workspace of the long-segment path for segments of length <= d.
struct BigWs {
  uint32_t* flags;
  float* lamtmp;   // a segment's lambda formed on the device (proximal-gradient step)
  uint32_t* tbad;  // per radix tile: non-finite weight seen (first pass)
  uint32_t *tor, *tand;  // per radix tile: OR and AND of its keys (first pass)
  uint32_t *keysA, *keysB;
  int32_t *valsA, *valsB;
  uint32_t *hist, *totals;
  int32_t* vpos;
  double* vS;
  uint16_t* hbits;  // per tile and thread: hull-vertex bits of the thread's ranks
  int32_t *hcnt, *lo, *hi, *prev_pos, *next_pos;
  double *tsum, *tileoff, *prev_s, *next_s;
  // backward
  int32_t *fpos, *lpos;
  double *fG, *lG, *prevG, *nextG;
  size_t bytes;
};

BigWs big_layout(int64_t d, void* base) {
  BigWs w{};
  const int64_t nrt = ceil_div(d, kRadixTile);
  const int64_t nt = ceil_div(d, kBigTile);
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? (void*)((char*)base + off) : nullptr;
    off += align_up(bytes);
    return p;
  };
  w.flags = (uint32_t*)take(256);  // [0] non-finite weight seen, [1] key bits that vary
  w.lamtmp = (float*)take(256);
  w.tbad = (uint32_t*)take(sizeof(uint32_t) * nrt);
  w.tor = (uint32_t*)take(sizeof(uint32_t) * nrt);
  w.tand = (uint32_t*)take(sizeof(uint32_t) * nrt);
  w.keysA = (uint32_t*)take(sizeof(uint32_t) * d);
  w.keysB = (uint32_t*)take(sizeof(uint32_t) * d);
  w.valsA = (int32_t*)take(sizeof(int32_t) * d);
  w.valsB = (int32_t*)take(sizeof(int32_t) * d);
  w.hist = (uint32_t*)take(sizeof(uint32_t) * 256 * nrt);
  w.totals = (uint32_t*)take(sizeof(uint32_t) * 256);
  w.vpos = (int32_t*)take(sizeof(int32_t) * nt * (kBigTile + 1));
  w.vS = (double*)take(sizeof(double) * nt * (kBigTile + 1));
  w.hbits = (uint16_t*)take(sizeof(uint16_t) * nt * kBigThreads);
  w.hcnt = (int32_t*)take(sizeof(int32_t) * nt);
  w.lo = (int32_t*)take(sizeof(int32_t) * nt);
  w.hi = (int32_t*)take(sizeof(int32_t) * nt);
  w.prev_pos = (int32_t*)take(sizeof(int32_t) * nt);
  w.next_pos = (int32_t*)take(sizeof(int32_t) * nt);
  w.tsum = (double*)take(sizeof(double) * nt);
  w.tileoff = (double*)take(sizeof(double) * nt);
  w.prev_s = (double*)take(sizeof(double) * nt);
  w.next_s = (double*)take(sizeof(double) * nt);
  w.fpos = (int32_t*)take(sizeof(int32_t) * nt);
  w.lpos = (int32_t*)take(sizeof(int32_t) * nt);
  w.fG = (double*)take(sizeof(double) * nt);
  w.lG = (double*)take(sizeof(double) * nt);
  w.prevG = (double*)take(sizeof(double) * nt);
  w.nextG = (double*)take(sizeof(double) * nt);
  w.bytes = off;
  return w;
}

size_t big_bytes(int64_t max_big) { return max_big > 0 ? big_layout(max_big, nullptr).bytes : 0; }

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

// Stable LSD radix sort of one long segment (up to 4 passes of 8 bits; a later pass whose digit
// is the same for every key is skipped on the device): sorted keys end in b.keysA, the
// permutation in perm_final; b.flags[0] gets the non-finite bit, b.flags[1] the varying key bits.
void big_sort(const float* wseg, int64_t d, const BigWs& b, int32_t* perm_final, hipStream_t s) {
  const int nrt = (int)ceil_div(d, kRadixTile);
  for (int pass = 0; pass < 4; ++pass) {
    { WSR_TRACE("radix_hist", s);
    hipLaunchKernelGGL(k_radix_hist, dim3(radix_grid(nrt, hist_grid())), dim3(kRadixThreads), 0, s, pass, wseg,
                       b.keysA, b.keysB, b.valsA, b.valsB, perm_final, d, b.hist, nrt, b.tbad, b.tor, b.tand,
                       b.flags); }
    { WSR_TRACE("radix_rowscan", s);
    hipLaunchKernelGGL(k_radix_rowscan, dim3(256), dim3(256), 0, s, pass, b.hist, nrt, b.totals, b.tbad, b.tor,
                       b.tand, b.flags); }
    { WSR_TRACE("radix_scatter", s);
    hipLaunchKernelGGL(k_radix_scatter, dim3(radix_grid(nrt, scatter_grid())), dim3(kScatterThreads), 0, s, pass,
                       wseg, b.keysA, b.keysB, b.valsA, b.valsB, perm_final, d, b.hist, b.totals, nrt, b.flags); }
  }
}

// Forward of one long segment [start, start + d).
int big_forward(const float* w, float* out, int64_t start, int64_t d, const float* lam_arr, int seg_id,
                float lam_scalar, int32_t* saved_perm, uint32_t* saved_mask, void* ws, hipStream_t s,
                const L1Opt& l1, int rounds = -1, uint32_t* status = nullptr) {
  BigWs b = big_layout(d, ws);
  const int nt = (int)ceil_div(d, kBigTile);
  int32_t* perm_final = saved_perm ? saved_perm + start : b.valsA;
  big_sort(w + start, d, b, perm_final, s);
  { WSR_TRACE("big_tile_hull", s);
  hipLaunchKernelGGL(k_big_tile_hull, dim3(nt), dim3(kBigThreads), 0, s, b.keysA, d, lam_arr, seg_id,
                     lam_scalar, b.vpos, b.vS, b.hcnt, b.tsum, b.hbits, rounds); }
  { WSR_TRACE("big_tile_scan", s);
#define WSR_LAUNCH_TILE_SCAN(CM)                                                                         \
  hipLaunchKernelGGL(k_big_tile_scan<CM>, dim3(1), dim3(1024), 0, s, b.tsum, b.tileoff, b.hcnt, b.lo, b.hi, nt, \
                     d, lam_arr, seg_id, lam_scalar)
  if (nt <= 4 * 1024)
    WSR_LAUNCH_TILE_SCAN(4);
  else if (nt <= 8 * 1024)
    WSR_LAUNCH_TILE_SCAN(8);
  else
    WSR_LAUNCH_TILE_SCAN(16);
#undef WSR_LAUNCH_TILE_SCAN
  }
  int nlev = 0;
  while ((1 << nlev) < nt) ++nlev;
  int lvl_lo = 1;
  do {
    const int lvl_hi = std::min(lvl_lo + kMergeLevelsPerLaunch - 1, nlev);
    const int G = 1 << lvl_hi;
    const int groups = (int)ceil_div(nt, G);
    const int fin = lvl_hi == nlev ? 1 : 0;
    if (G > kMergeGroupMax) return WSR_ERR_UNSUPPORTED;
    WSR_TRACE("big_merge", s);
#define WSR_LAUNCH_MERGE(GM)                                                                             \
  hipLaunchKernelGGL((k_big_merge<GM, kMergeRecMax>), dim3(groups), dim3(kMergeThreads), 0, s, lvl_lo, lvl_hi, \
                     nt, b.vpos, b.vS, b.tileoff, b.lo, b.hi, fin, b.prev_pos, b.prev_s, b.next_pos, b.next_s)
    if (G <= 16)
      WSR_LAUNCH_MERGE(16);
    else if (G <= 256)
      WSR_LAUNCH_MERGE(256);
    else if (G <= 4096)
      WSR_LAUNCH_MERGE(4096);
    else
      WSR_LAUNCH_MERGE(16384);
#undef WSR_LAUNCH_MERGE
    lvl_lo = lvl_hi + 1;
  } while (lvl_lo <= nlev);
  { WSR_TRACE("big_apply", s);
  hipLaunchKernelGGL(k_big_apply, dim3(nt), dim3(kBigThreads), 0, s, b.keysA, perm_final, d, lam_arr, seg_id,
                     lam_scalar, b.flags, b.hbits, b.hcnt, b.vS, b.tileoff, b.lo, b.hi, b.prev_pos, b.prev_s,
                     b.next_pos, b.next_s, out, saved_mask, start, l1.beta, l1.rho, l1.kappa, l1.on, status); }
  return last_error();
}

int big_backward(const float* g, float* gw, int64_t start, int64_t d, const int32_t* perm,
                 const uint32_t* mask, void* ws, hipStream_t s) {
  BigWs b = big_layout(d, ws);
  const int nt = (int)ceil_div(d, kBigTile);
  float* gsorted = (float*)b.keysA;
  { WSR_TRACE("big_bwd_tile", s);
  hipLaunchKernelGGL(k_big_bwd_tile, dim3(nt), dim3(kBigThreads), 0, s, g, perm + start, mask, d, start,
                     gsorted, b.tsum, b.fpos, b.fG, b.lpos, b.lG); }
  { WSR_TRACE("big_bwd_scan", s);
#define WSR_LAUNCH_BWD_SCAN(CM)                                                                          \
  hipLaunchKernelGGL(k_big_bwd_scan<CM>, dim3(1), dim3(1024), 0, s, b.tsum, b.fpos, b.fG, b.lpos, b.lG, nt, d, \
                     b.tileoff, b.prev_pos, b.prevG, b.next_pos, b.nextG)
  if (nt <= 4 * 1024)
    WSR_LAUNCH_BWD_SCAN(4);
  else if (nt <= 8 * 1024)
    WSR_LAUNCH_BWD_SCAN(8);
  else
    WSR_LAUNCH_BWD_SCAN(16);
#undef WSR_LAUNCH_BWD_SCAN
  }
  { WSR_TRACE("big_bwd_apply", s);
  hipLaunchKernelGGL(k_big_bwd_apply, dim3(nt), dim3(kBigThreads), 0, s, gsorted, perm + start, mask, d,
                     start, b.tileoff, b.prev_pos, b.prevG, b.next_pos, b.nextG, gw); }
  return last_error();
}

// Statistics of one long segment: the sort, then the tile partials and their fixed-order sum.
int big_stats(const float* w, int64_t start, int64_t d, SegStats* out, void* ws, hipStream_t s) {
  BigWs b = big_layout(d, ws);
  const int nt = (int)ceil_div(d, kBigTile);
  big_sort(w + start, d, b, b.valsA, s);
  { WSR_TRACE("big_stats_tile", s);
  hipLaunchKernelGGL(k_big_stats_tile, dim3(nt), dim3(kBigThreads), 0, s, b.keysA, d, b.tsum, b.hcnt, b.lo); }
  { WSR_TRACE("big_stats_final", s);
  hipLaunchKernelGGL(k_big_stats_final, dim3(1), dim3(1024), 0, s, b.tsum, b.hcnt, b.lo, nt, d, b.flags, out); }
  return last_error();
}

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
  int64_t max_big = 0;
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
  uint32_t* d_status = nullptr;  // sticky status word (kStatusNonFinite), read by wsr_read_status
};

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
      rc = big_forward(w, out, start, d, nullptr, 0, lambda, saved_perm, saved_mask, ws, s, l1);
      if (rc) return rc;
      continue;
    }
    SegArgs a{nullptr, nullptr, nullptr, lambda, start, (int)d, 0, l1.beta, l1.rho, l1.on, l1.kappa};
    small_fwd(cls, 1, a, w, out, saved_perm, saved_mask, s);
  }
  return last_error();
}

int forward_batched_impl(const wsr_plan* plan, const float* w, float* out, const float* d_lambda,
                         float lambda_scalar, int32_t* saved_perm, uint32_t* saved_mask, void* ws,
                         size_t ws_bytes, void* stream, const L1Opt& l1) {
  (void)hipGetLastError();  // report only errors of this call
  if (!plan || !w || !out) return WSR_ERR_INVALID;
  if ((saved_perm == nullptr) != (saved_mask == nullptr)) return WSR_ERR_INVALID;
  if (!d_lambda && (!std::isfinite(lambda_scalar) || lambda_scalar < 0.0f)) return WSR_ERR_INVALID;
  const size_t need = big_bytes(plan->max_big);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) return WSR_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (saved_mask && !plan->word_aligned) zero_words(saved_mask, ceil_div(plan->total, 32), s);
  for (int c = 0; c < kNumSmall; ++c) {
    if (plan->sched_cnt[c] == 0) continue;
    SegArgs a{plan->d_offsets, plan->d_sched + plan->sched_off[c], d_lambda, lambda_scalar, 0, 0, 0,
              l1.beta, l1.rho, l1.on, l1.kappa};
    a.merge_rounds = plan->small_route(c);
    a.status = plan->d_status;
    small_fwd(c, (int)plan->sched_cnt[c], a, w, out, saved_perm, saved_mask, s);
  }
  for (int32_t seg : plan->big_segs) {
    const int64_t start = plan->h_offsets[seg];
    const int64_t d = plan->h_offsets[seg + 1] - start;
    const int rc = big_forward(w, out, start, d, d_lambda, seg, lambda_scalar, saved_perm, saved_mask, ws, s, l1,
                               plan->rounds[kNumSmall], plan->d_status);
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
  const size_t need = big_bytes(plan->max_big);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) return WSR_ERR_WORKSPACE;
  return WSR_OK;
}

// The fused launch of size class c over its first nblocks segments with merge route `route`.
void step_small(const wsr_plan* plan, int c, int nblocks, int route, const float* w, const float* grad, float eta,
                float* out, const float* d_alpha, float alpha_scalar, const StepForm& f, hipStream_t s) {
  SegArgs a{plan->d_offsets, plan->d_sched + plan->sched_off[c], d_alpha, alpha_scalar, 0, 0, 0,
            f.l1.beta, f.l1.rho, f.l1.on, f.l1.kappa, grad, eta, f.lam_mul, route, plan->d_status};
  small_fwd(c, nblocks, a, w, out, nullptr, nullptr, s);
}

// One long segment of the step: z = fmaf(-eta, grad, w) into out, then the device-wide path in place.
int step_big(const wsr_plan* plan, int32_t seg, int rounds, const float* w, const float* grad, float eta, float* out,
             const float* d_alpha, float alpha_scalar, const StepForm& f, void* ws, hipStream_t s) {
  const int64_t start = plan->h_offsets[seg];
  const int64_t d = plan->h_offsets[seg + 1] - start;
  {
    WSR_TRACE("grad_step", s);
    const int64_t blocks = std::min<int64_t>(ceil_div(d, 256), 4 * (int64_t)cu_count());
    hipLaunchKernelGGL(k_grad_step, dim3((unsigned)blocks), dim3(256), 0, s, out + start, w + start,
                       grad + start, eta, d);
  }
  const float* lam_arr = d_alpha;
  int lam_seg = seg;
  const float lam_scalar = alpha_scalar * f.lam_mul;
  if (d_alpha && f.lam_mul != 1.0f) {
    BigWs b = big_layout(d, ws);
    WSR_TRACE("scale_lambda", s);
    hipLaunchKernelGGL(k_scale_lambda, dim3(1), dim3(64), 0, s, b.lamtmp, d_alpha, seg, alpha_scalar, f.lam_mul);
    lam_arr = b.lamtmp;
    lam_seg = 0;
  }
  return big_forward(out, out, start, d, lam_arr, lam_seg, lam_scalar, nullptr, nullptr, ws, s, f.l1, rounds,
                     plan->d_status);
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
    step_small(plan, c, (int)plan->sched_cnt[c], plan->small_route(c), w, grad, eta, out, d_alpha, alpha_scalar, f,
               s);
  }
  for (int32_t seg : plan->big_segs) {
    rc = step_big(plan, seg, plan->rounds[kNumSmall], w, grad, eta, out, d_alpha, alpha_scalar, f, ws, s);
    if (rc) return rc;
  }
  return last_error();
}

// Autotuner core: for every short size class, times the batched launch of the class alone under
// each candidate route and keeps the fastest; EndCollisions is a candidate only when a probe over
// the class's first segments (one workgroup per CU pair) shows it no slower than 1.5x the default
// route there.  Long segments: the caps {0, kIcaRounds, 16}, timed on the longest one.
//   small(c, nblocks, route): launches class c over its first nblocks segments
//   big(seg, rounds): runs long segment seg, returns a status
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
      rc = time_it([&] { small(c, np, kIcaRounds); }, 1, &t_def);
      if (rc) break;
      rc = time_it([&] { small(c, np, kRouteEnd); }, 1, &t_end);
      if (rc) break;
      if (t_end <= 1.5f * t_def) cand.push_back(kRouteEnd);
    }
    float best = 0.0f;
    for (size_t i = 0; i < cand.size(); ++i) {
      float ms = 0.0f;
      rc = time_it([&] { small(c, cnt, cand[i]); }, kReps, &ms);
      if (rc) break;
      if (i == 0 || ms < best) {
        best = ms;
        plan->rounds[c] = cand[i] == kRouteEnd ? -1 : cand[i];
      }
    }
  }
  if (rc == WSR_OK && !plan->big_segs.empty()) {
    int32_t seg = plan->big_segs[0];
    for (int32_t q : plan->big_segs)
      if (plan->h_offsets[q + 1] - plan->h_offsets[q] > plan->h_offsets[seg + 1] - plan->h_offsets[seg]) seg = q;
    float best = 0.0f;
    bool first = true;
    for (int r : {0, kIcaRounds, 16}) {
      float ms = 0.0f;
      int lrc = WSR_OK;
      rc = time_it([&] {
        const int e = big(seg, r);
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
      rc = big_stats(w, start, d, st + seg, ws, s);
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
      rc = big_backward(grad_out, grad_w, start, d, saved_perm, saved_mask, ws, s);
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
  p->max_big = mb;
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
      (void)hipFree(p->d_offsets);
      (void)hipFree(p->d_status);
      if (p->d_sched) (void)hipFree(p->d_sched);
      delete p;
      return WSR_ERR_HIP;
    }
  }
  *plan = p;
  return WSR_OK;
}

int wsr_plan_destroy(wsr_plan* plan) {
  if (!plan) return WSR_ERR_INVALID;
  if (plan->d_offsets) (void)hipFree(plan->d_offsets);
  if (plan->d_sched) (void)hipFree(plan->d_sched);
  if (plan->d_status) (void)hipFree(plan->d_status);
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
  *bytes = big_bytes(plan->max_big);
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

int wsr_plan_autotune(wsr_plan* plan, const float* w, float* out, const float* d_lambda, float lambda_scalar,
                      void* ws, size_t ws_bytes, void* stream) {
  (void)hipGetLastError();  // report only errors of this call
  if (!plan || !w || !out || out == w) return WSR_ERR_INVALID;
  if (!d_lambda && (!std::isfinite(lambda_scalar) || lambda_scalar < 0.0f)) return WSR_ERR_INVALID;
  const size_t need = big_bytes(plan->max_big);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) return WSR_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  return autotune_impl(
      plan,
      [&](int c, int nblocks, int route) {
        SegArgs a{plan->d_offsets, plan->d_sched + plan->sched_off[c], d_lambda, lambda_scalar, 0, 0, 0};
        a.merge_rounds = route;
        small_fwd(c, nblocks, a, w, out, nullptr, nullptr, s);
      },
      [&](int32_t seg, int rounds) {
        const int64_t start = plan->h_offsets[seg];
        const int64_t d = plan->h_offsets[seg + 1] - start;
        return big_forward(w, out, start, d, d_lambda, seg, lambda_scalar, nullptr, nullptr, ws, s, L1Opt{}, rounds);
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
      [&](int c, int nblocks, int route) {
        step_small(plan, c, nblocks, route, w, grad, eta, scratch, d_alpha, alpha_scalar, f, s);
      },
      [&](int32_t seg, int rounds) {
        return step_big(plan, seg, rounds, w, grad, eta, scratch, d_alpha, alpha_scalar, f, ws, s);
      },
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
  const size_t need = big_bytes(plan->max_big);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) return WSR_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  SegStats* st = reinterpret_cast<SegStats*>(d_stats);
  zero_words(reinterpret_cast<uint32_t*>(st), plan->n_seg * (int64_t)(sizeof(SegStats) / 4), s);
  for (int c = 0; c < kNumSmall; ++c) {
    if (plan->sched_cnt[c] == 0) continue;
    SegArgs a{plan->d_offsets, plan->d_sched + plan->sched_off[c], nullptr, 0.0f, 0, 0, 0};
    small_stats(c, (int)plan->sched_cnt[c], a, w, st, s);
  }
  for (int32_t seg : plan->big_segs) {
    const int64_t start = plan->h_offsets[seg];
    const int64_t d = plan->h_offsets[seg + 1] - start;
    const int rc = big_stats(w, start, d, st + seg, ws, s);
    if (rc) return rc;
  }
  return last_error();
}

int wsr_prox_backward_batched(const wsr_plan* plan, const float* grad_out, float* grad_w,
                              const int32_t* saved_perm, const uint32_t* saved_mask, void* ws, size_t ws_bytes,
                              void* stream) {
  (void)hipGetLastError();  // report only errors of this call
  if (!plan || !grad_out || !grad_w || !saved_perm || !saved_mask || grad_out == grad_w) return WSR_ERR_INVALID;
  const size_t need = big_bytes(plan->max_big);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) return WSR_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  for (int c = 0; c < kNumSmall; ++c) {
    if (plan->sched_cnt[c] == 0) continue;
    SegArgs a{plan->d_offsets, plan->d_sched + plan->sched_off[c], nullptr, 0.0f, 0, 0, 0};
    small_bwd(c, (int)plan->sched_cnt[c], a, grad_out, grad_w, saved_perm, saved_mask, s);
  }
  for (int32_t seg : plan->big_segs) {
    const int64_t start = plan->h_offsets[seg];
    const int64_t d = plan->h_offsets[seg + 1] - start;
    const int rc = big_backward(grad_out, grad_w, start, d, saved_perm, saved_mask, ws, s);
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

}  // extern "C"
