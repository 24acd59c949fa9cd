// wsr_big.h -- geometry and kernels of the long-segment (device-wide) path.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wsr_kernels.h"

namespace wsr {

constexpr int kRadixThreads = 256;   // histogram workgroup; the scatter's digit scan uses
                                     // one thread per digit
constexpr int kRadixTile = 8192;     // keys per radix tile (digit runs average 32 keys)
constexpr int kMaxRadixTiles = (1 << 26) / kRadixTile;  // radix tiles of the longest segment
constexpr int kHistPerCu = 4;         // resident workgroups per CU of the persistent histogram
constexpr int kScatterThreads = 512;  // scatter workgroup (16 keys per thread)
constexpr int kBigThreads = 256;
constexpr int kBigE = 16;
constexpr int kBigTile = kBigThreads * kBigE;  // ranks per hull tile
constexpr int kApplySparseMax = 256;  // surviving hull vertices up to which a tile's S' values
                                      // are read from the hull rather than recomputed
constexpr int kMergeThreads = 512;  // one wave per merge
constexpr int kMergeLevelsPerLaunch = 4;
constexpr int kMergeGroupMax = 1 << 14;                         // tiles of the longest segment
constexpr int kMergeRecMax = 1 << (kMergeLevelsPerLaunch - 1);  // merges at a launch's first level
static_assert((int64_t)kMergeGroupMax * kBigTile >= ((int64_t)1 << 26), "top merge group too small");
static_assert(kRadixThreads == 256, "one histogram bin per thread");
static_assert(kMergeGroupMax / 1024 <= 16, "tile scans hold at most 16 tiles per thread");
static_assert(kScatterThreads >= 256, "digit scan assumes one digit per thread");

__global__ void k_radix_hist(int pass, const float* wsrc, uint32_t* kA, uint32_t* kB, int32_t* vA, int32_t* vB,
                             int32_t* vfinal, int64_t n, uint32_t* hist, int ntiles, uint32_t* tbad, uint32_t* tor,
                             uint32_t* tand, const uint32_t* flags);
__global__ void k_radix_rowscan(int pass, uint32_t* hist, int ntiles, uint32_t* totals, const uint32_t* tbad,
                                const uint32_t* tor, const uint32_t* tand, uint32_t* flags);
__global__ void k_radix_scatter(int pass, const float* w, uint32_t* kA, uint32_t* kB, int32_t* vA, int32_t* vB,
                                int32_t* vfinal, int64_t n, const uint32_t* hist, const uint32_t* totals,
                                int ntiles, const uint32_t* flags);
__global__ void k_big_tile_hull(const uint32_t* skeys, int64_t d, const float* lam_arr, int seg_id,
                                float lam_scalar, int32_t* vpos, double* vS, int32_t* hcnt,
                                double* tsum, uint16_t* hbits, int rounds);
template <int CM>
__global__ void k_big_tile_scan(const double* tsum, double* tileoff, const int32_t* hcnt,
                                int32_t* lo, int32_t* hi, int ntiles, int64_t d,
                                const float* lam_arr, int seg_id, float lam_scalar);
template <int GMAX, int RMAX>
__global__ void k_big_merge(int lvl_lo, int lvl_hi, int ntiles, const int32_t* vpos,
                            const double* vS, const double* tileoff, int32_t* lo_g, int32_t* hi_g,
                            int finalize, int32_t* prev_pos, double* prev_s, int32_t* next_pos,
                            double* next_s);
__global__ void k_big_apply(const uint32_t* skeys, const int32_t* perm, int64_t d,
                            const float* lam_arr, int seg_id, float lam_scalar,
                            const uint32_t* flags, const uint16_t* hbits, const int32_t* hcnt,
                            const double* vS, const double* tileoff, const int32_t* lo_g,
                            const int32_t* hi_g,
                            const int32_t* prev_pos, const double* prev_s, const int32_t* next_pos,
                            const double* next_s, float* out, uint32_t* mask_out,
                            int64_t seg_start, float beta, float rho, float kappa, int l1,
                            uint32_t* status);
__global__ void k_big_bwd_tile(const float* g, const int32_t* perm, const uint32_t* mask,
                               int64_t d, int64_t seg_start, float* gsorted, double* tsum,
                               int32_t* fpos, double* fG, int32_t* lpos, double* lG);
template <int CM>
__global__ void k_big_bwd_scan(const double* tsum, const int32_t* fpos, const double* fG,
                               const int32_t* lpos, const double* lG, int ntiles, int64_t d,
                               double* tileoff, int32_t* prevp, double* prevG, int32_t* nextp,
                               double* nextG);
__global__ void k_big_bwd_apply(const float* gsorted, const int32_t* perm, const uint32_t* mask,
                                int64_t d, int64_t seg_start, const double* tileoff,
                                const int32_t* prevp, const double* prevG, const int32_t* nextp,
                                const double* nextG, float* gout);

__global__ void k_big_stats_tile(const uint32_t* skeys, int64_t d, double* tsum, int32_t* tnz, int32_t* tnd);
__global__ void k_big_stats_final(const double* tsum, const int32_t* tnz, const int32_t* tnd, int ntiles,
                                  int64_t d, const uint32_t* flags, SegStats* out);

}  // namespace wsr
