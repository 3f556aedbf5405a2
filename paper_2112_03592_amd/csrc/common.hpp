// Shared definitions of the aprconv HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "aprconv.h"

namespace apr {

constexpr int kMaxL = APR_MAX_LEVELS;
constexpr uint32_t kNoY = 0x7fffffffu;   // "no further element" marker for y searches
// child-map entry of a child cell outside the image; else (1 << 31 if a tree
// node) | index
constexpr uint32_t kChildPad = 0xffffffffu;

// Per-level geometry, passed by value to kernels.
struct Meta {
  int32_t l_min, l_max, t_lo, t_hi;      // particle levels, tree levels (t_hi < t_lo: no tree)
  int32_t dz[kMaxL], dx[kMaxL], dy[kMaxL];
  uint32_t prow[kMaxL];                  // first particle row of level l
  uint32_t trow[kMaxL];                  // first tree row of level l
};

// Tile descriptor of the convolution work list: level, tile z, tile x.
// tile list entry: level (8 bits) | first y of the tile's particles (16) |
// tile z (20) | tile x (20)
__host__ __device__ inline uint64_t tile_pack(int l, int tz, int tx, int y0) {
  return (uint64_t(l) << 56) | (uint64_t(uint32_t(y0) & 0xffffu) << 40) | (uint64_t(uint32_t(tz)) << 20) |
         uint64_t(uint32_t(tx));
}
__host__ __device__ inline void tile_unpack(uint64_t t, int& l, int& tz, int& tx, int& y0) {
  l = int(t >> 56);
  y0 = int((t >> 40) & 0xffffu);
  tz = int((t >> 20) & 0xfffffu);
  tx = int(t & 0xfffffu);
}

constexpr int kTileZ = 8;   // output rows per tile along z
constexpr int kTileX = 8;   // output rows per tile along x
// The convolution sweeps a tile along y in windows: runs of output y (over the
// tile's rows) spanning at most kWinY cells, a new window starting after a
// stretch of more than kWinGap cells without outputs.
constexpr int kWinY = 64;
constexpr int kWinGap = 64;
// Work-item cost model of the conv launch, in output cells: a window costs its
// span + 16, starting an item (row lookups, first batches) kItemCost; items
// are cut to at most half the ideal share of one of kConvSlots resident
// workgroups (two 5^3 workgroups per CU on 256 CUs).
constexpr uint64_t kItemCost = 32;
constexpr uint64_t kConvSlots = 512;

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
__device__ inline uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// number of set bits of m below this lane
__device__ inline uint32_t mask_rank(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
}
__device__ inline uint64_t ballot(bool p) { return __ballot(p); }

// LDS writes by some lanes of a wave become visible to the other lanes.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroup barrier that orders LDS only: global loads and stores still in
// flight stay in flight (a plain __syncthreads() also waits for every
// outstanding store).  For kernels whose threads exchange data through LDS
// alone and never read global memory written by another thread.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ inline void row_range(const uint32_t* __restrict__ ends, uint32_t row, uint32_t& b,
                                 uint32_t& e) {
  e = ends[row];
  b = row ? ends[row - 1] : 0u;
}

// Storage conversions (FP32 arithmetic everywhere).
template <typename T> __device__ inline float to_f32(T v);
template <> __device__ inline float to_f32<float>(float v) { return v; }
template <> __device__ inline float to_f32<__hip_bfloat16>(__hip_bfloat16 v) {
  return __bfloat162float(v);
}
template <typename T> __device__ inline T from_f32(float v);
template <> __device__ inline float from_f32<float>(float v) { return v; }
template <> __device__ inline __hip_bfloat16 from_f32<__hip_bfloat16>(float v) {
  return __float2bfloat16(v);   // round to nearest even
}

// CH values of a row at p (16-byte aligned when CH * sizeof(T) is a multiple
// of 16: vector loads/stores), converted to/from FP32
template <typename T, int CH>
__device__ inline void load_vec(const T* p, float* v) {
  constexpr int kB = CH * int(sizeof(T));
  if constexpr (kB % 16 == 0) {
    uint4 raw[kB / 16];
#pragma unroll
    for (int i = 0; i < kB / 16; ++i) raw[i] = reinterpret_cast<const uint4*>(p)[i];
    T t[CH];
    __builtin_memcpy(t, raw, kB);
#pragma unroll
    for (int c = 0; c < CH; ++c) v[c] = to_f32<T>(t[c]);
  } else {
#pragma unroll
    for (int c = 0; c < CH; ++c) v[c] = to_f32<T>(p[c]);
  }
}

template <typename T, int CH>
__device__ inline void store_vec(T* p, const T* t) {
  constexpr int kB = CH * int(sizeof(T));
  if constexpr (kB % 16 == 0) {
    uint4 raw[kB / 16];
    __builtin_memcpy(raw, t, kB);
#pragma unroll
    for (int i = 0; i < kB / 16; ++i) reinterpret_cast<uint4*>(p)[i] = raw[i];
  } else {
#pragma unroll
    for (int c = 0; c < CH; ++c) p[c] = t[c];
  }
}

// ---------------------------------------------------------------------------
// Host-side state and error reporting
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);

#define APR_HIP(call)                                                              \
  do {                                                                             \
    hipError_t _e = (call);                                                        \
    if (_e != hipSuccess) {                                                        \
      ::apr::set_error(std::string(#call) + ": " + hipGetErrorString(_e));         \
      return APR_EDEVICE;                                                          \
    }                                                                              \
  } while (0)

#define APR_FAIL(code, msg)    \
  do {                         \
    ::apr::set_error(msg);     \
    return (code);             \
  } while (0)

// Exclusive scan of n uint32 values in place on `stream`; returns the total in
// *total_dev (device uint32, may be nullptr).
apr_status scan_u32(uint32_t* data, int64_t n, uint32_t* total_dev, hipStream_t stream);

}  // namespace apr

struct apr_handle {
  int device = 0;
  apr::Meta meta{};
  int64_t n_p = 0, n_t = 0, n_rows = 0, n_trows = 0;
  int64_t per_level_p[apr::kMaxL] = {0};
  int64_t per_level_t[apr::kMaxL] = {0};
  uint16_t* py = nullptr;     // particle y [n_p]
  uint32_t* pend = nullptr;   // particle row ends [n_rows]
  uint16_t* ty = nullptr;     // tree y [n_t]
  uint32_t* tend = nullptr;   // tree row ends [n_trows]
  uint64_t* tiles = nullptr;  // conv tiles [n_tiles]: level, tile z, tile x, first y
  int64_t n_tiles = 0;
  uint32_t* wins = nullptr;     // sweep windows of the tiles, in tile order: y0 | (y1 << 16)
  int64_t n_wins = 0;
  uint32_t* items = nullptr;    // conv work items [n_items][4]: tile code (2 words), first window, end window
  int64_t n_items = 0;
  int64_t xcd_off[9] = {0};   // items of XCD x: [xcd_off[x], xcd_off[x + 1]), heaviest first
  int32_t* gmap[2] = {nullptr, nullptr};   // gather maps for k = 3, 5: [k^3][n_p]
  uint32_t* cmap = nullptr;                 // child map of the tree nodes [8][n_t] (kChildPad outside the image)
  // inverse of the gather maps for the coarse and tree taps: for source s
  // (particle s as a coarser source, or tree node t at n_p + t) the readers
  // p * k^3 + q with gmap[q][p] naming s, sorted, at inv_ent[inv_off[s] ..
  // inv_off[s + 1])
  uint32_t* inv_off[2] = {nullptr, nullptr};
  uint32_t* inv_ent[2] = {nullptr, nullptr};
  // particles that have readers in the inverse map, ascending (so level by
  // level): level l's are inv_act[inv_act_lvl[l] .. inv_act_lvl[l + 1])
  uint32_t* inv_act[2] = {nullptr, nullptr};
  int64_t inv_act_lvl[2][apr::kMaxL + 2] = {};
  int64_t device_bytes = 0;
  std::vector<void*> allocs;
};
