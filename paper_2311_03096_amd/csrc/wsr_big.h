// wsr_big.h -- geometry and kernels of the long-segment (device-wide) path.
//
// The long segments of a call form a set that one launch sequence solves: every kernel covers
// the tiles of all segments of the set, each tile knowing its segment from a tile -> segment
// table (a single segment is passed by value, without tables).  Workspace arrays hold the
// segments back to back: element arrays at the segment's element base, radix-tile and hull-tile
// arrays at its tile bases, small per-segment records at its index.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wsr_kernels.h"

namespace wsr {

constexpr int kRadixThreads = 256;   // histogram workgroup; the scatter's digit scan uses
                                     // one thread per digit
constexpr int kRadixTile = 8192;     // keys per radix tile (digit runs average 32 keys)
constexpr int64_t kMaxLong = (int64_t)1 << 27;            // longest segment
constexpr int kMaxRadixTiles = (int)(kMaxLong / kRadixTile);  // radix tiles of the longest segment
constexpr int kHistPerCu = 3;         // resident workgroups per CU of the persistent histogram
constexpr int kScatterThreads = 512;  // scatter workgroup (16 keys per thread)
constexpr int kBigThreads = 256;
constexpr int kBigE = 16;
constexpr int kBigTile = kBigThreads * kBigE;  // ranks per hull tile
constexpr int kApplySparseMax = 256;  // surviving hull vertices up to which a tile's S' values
                                      // are read from the hull rather than recomputed
constexpr int kMergeThreads = 512;  // one wave per merge
constexpr int kMergeLevelsPerLaunch = 4;
constexpr int kMergeGroupMax = 1 << 14;                         // tiles of one merge group in LDS
constexpr int kMergeRecMax = 1 << (kMergeLevelsPerLaunch - 1);  // merges at a launch's first level
constexpr int kMergeLevelsInLds = 14;                           // levels done by k_big_merge
constexpr int kMaxHullTiles = (int)(kMaxLong / kBigTile);       // hull tiles of the longest segment
constexpr int kTopThreads = 1024;                               // top merge level (k_big_merge_top)
static_assert(kMergeGroupMax == 1 << kMergeLevelsInLds, "merge group of the LDS levels");
static_assert(kMaxHullTiles == 2 * kMergeGroupMax, "one top level above the LDS merge groups");
static_assert(kRadixThreads == 256, "one histogram bin per thread");
static_assert(kMaxHullTiles / 1024 <= 32, "tile scans hold at most 32 tiles per thread");
static_assert(kScatterThreads >= 256, "digit scan assumes one digit per thread");

// One long segment of a set.
struct LongSeg {
  int64_t start;   // flat offset of the segment in w / out / grad / saved perm
  int64_t d;       // length
  int64_t ebase;   // offset of its elements in the workspace element arrays
  int rbase, nrt;  // its radix tiles [rbase, rbase + nrt) of the set
  int tbase, nt;   // its hull tiles [tbase, tbase + nt) of the set
  int seg_id;      // index of the segment in per-segment lambda / statistics arrays
  int nlev;        // merge levels: ceil(log2(nt))
};

// The long segments of one launch sequence.  One segment travels by value (segs == nullptr);
// several come from device tables built with a plan.
struct LongSet {
  const LongSeg* segs;
  const int32_t* rseg;  // radix tile -> segment
  const int32_t* hseg;  // hull tile -> segment
  LongSeg one;
  int nsegs;
  int nrt, nt;  // radix / hull tiles of the whole set
  __device__ __forceinline__ const LongSeg& seg(int s) const { return segs ? segs[s] : one; }
  __device__ __forceinline__ int seg_of_rtile(int t) const { return rseg ? rseg[t] : 0; }
  __device__ __forceinline__ int seg_of_htile(int t) const { return hseg ? hseg[t] : 0; }
};

// Lambda of a segment: (arr ? arr[seg_id] : scalar) * mul in FP32 (mul = eta for the
// proximal-gradient step's standard form, else 1).
struct LamArgs {
  const float* arr;
  float scalar;
  float mul;
  __device__ __forceinline__ float of(int seg_id) const { return (arr ? arr[seg_id] : scalar) * mul; }
};

// One merge group of a launch of k_big_merge: tiles [gbase, gbase + gn) of segment s, levels up to
// lvl_hi; fin: the launch holds the segment's last level (write the previous / next surviving
// vertex of every tile).
struct MergeGroup {
  int s, gbase, gn, lvl_hi, fin;
};

// Per-segment records in the workspace (flags): [0] a non-finite input, [1] the key bits that
// vary over the segment.
constexpr int kSegFlagWords = 4;

template <bool GRAD>
__global__ void k_radix_hist(int pass, LongSet set, const float* w, const float* grad, float eta, uint32_t* kA,
                             uint32_t* kB, int32_t* vA, int32_t* vB, int32_t* saved_perm, uint32_t* hist,
                             uint32_t* tbad, uint32_t* tor, uint32_t* tand, const uint32_t* flags);
__global__ void k_radix_rowscan(int pass, LongSet set, uint32_t* hist, uint32_t* totals, const uint32_t* tbad,
                                const uint32_t* tor, const uint32_t* tand, uint32_t* flags);
template <bool GRAD>
__global__ void k_radix_scatter(int pass, LongSet set, const float* w, const float* grad, float eta, uint32_t* kA,
                                uint32_t* kB, int32_t* vA, int32_t* vB, int32_t* saved_perm, const uint32_t* hist,
                                const uint32_t* totals, const uint32_t* flags);
__global__ void k_big_tile_hull(LongSet set, const uint32_t* keys, LamArgs lam, int32_t* vpos, double* vS,
                                int32_t* hcnt, double* tsum, uint16_t* hbits, int rounds);
template <int CM>
__global__ void k_big_tile_scan(LongSet set, const double* tsum, double* tileoff, const int32_t* hcnt,
                                int32_t* lo, int32_t* hi, LamArgs lam);
template <int GMAX, int RMAX>
__global__ void k_big_merge(int lvl_lo, int lvl_hi, LongSet set, const MergeGroup* groups, const int32_t* vpos,
                            const double* vS, const double* tileoff, int32_t* lo_g, int32_t* hi_g,
                            int64_t* prev_ref, int64_t* next_ref);
__global__ void k_big_merge_top(LongSet set, const int32_t* top_segs, const int32_t* vpos, const double* vS,
                                const double* tileoff, int32_t* lo_g, int32_t* hi_g, int64_t* prev_ref,
                                int64_t* next_ref);
__global__ void k_big_apply(LongSet set, const uint32_t* keys, const int32_t* saved_perm, const int32_t* perm_ws,
                            LamArgs lam, const uint32_t* flags, const uint16_t* hbits, const int32_t* hcnt,
                            const double* vS, const double* tileoff, const int32_t* lo_g, const int32_t* hi_g,
                            const int32_t* vpos, const int64_t* prev_ref, const int64_t* next_ref, float* out,
                            uint32_t* mask_out, float beta, float rho, float kappa, int l1, uint32_t* status);
__global__ void k_big_bwd_tile(LongSet set, const float* g, const int32_t* perm, const uint32_t* mask, float* gsorted,
                               double* tsum, int32_t* fpos, double* fG, int32_t* lpos, double* lG);
template <int CM>
__global__ void k_big_bwd_scan(LongSet set, const double* tsum, const int32_t* fpos, const double* fG,
                               const int32_t* lpos, const double* lG, double* tileoff, int32_t* prevp, double* prevG,
                               int32_t* nextp, double* nextG);
__global__ void k_big_bwd_apply(LongSet set, const float* gsorted, const int32_t* perm, const uint32_t* mask,
                                const double* tileoff, const int32_t* prevp, const double* prevG,
                                const int32_t* nextp, const double* nextG, float* gout);

#ifdef WSR_PHASE_CLOCKS
// Measurement build: where the tile merge launches record their timestamps (null: nowhere).
// Per launch (slot (lvl_lo - 1) / kMergeLevelsPerLaunch, below kMergeClockLaunches) and
// workgroup (below kMergeClockGroups), kMergeClockSlots words: 0 the start of the first level,
// 1 + l the end of level l of the launch, 5 + l the longest and 9 + l the summed bridge search
// of the level's merges, 13 the end of the launch's work, 14 the summed bookkeeping after the
// levels' searches (thread 0), 15 the summed time from each level's start to wave 0's bridge
// search (wall-clock ticks).
constexpr int kMergeClockLaunches = 4;
constexpr int kMergeClockGroups = 4096;
constexpr int kMergeClockSlots = 16;
int set_merge_clock_buffer(void* clocks);
#endif

__global__ void k_big_stats_tile(LongSet set, const uint32_t* keys, double* tsum, int32_t* tnz, int32_t* tnd);
__global__ void k_big_stats_final(LongSet set, const double* tsum, const int32_t* tnz, const int32_t* tnd,
                                  const uint32_t* flags, SegStats* out);

}  // namespace wsr
