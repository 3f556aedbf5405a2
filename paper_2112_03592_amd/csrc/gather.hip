// Multichannel APR convolution and the adjoint of APR convolution, built on
// the per-APR gather map (for every particle and tap: which element supplies
// V_l(c_p + o) -- written once by the convolution's own patch builder).
//
//   forward      Y[p, co] = b[co] + sum_o sum_ci W_l[co, ci, o] Xcat[src(p, o), ci]
//   data grad    the transpose of the forward, evaluated as gathers:
//                  * same-level readers of a particle s: the particle at
//                    c_s - o reads s with tap o  (s's own gather map, flipped);
//                  * finer readers: level-(l+1) particles with s as their
//                    coarser source, from the inverse of the gather map;
//                  * tree readers: level-L particles whose taps land on a tree
//                    node t (inverse map), then the adjoint of the child mean
//                    pushed from the coarsest tree level down to the particles.
//   weight grad  dW_l[co, ci, o] = sum_{p at level l} dY[p, co] Xcat[src(p, o), ci],
//                per-block FP32 sums, FP64 partials, fixed-order FP64 reduce.
// Every output has a single writer and a fixed summation order: results are
// deterministic.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "common.hpp"
#include "fp8.hpp"

namespace apr {

constexpr int kGWaves = 4;   // waves per block in the row-based kernels
constexpr uint32_t kIdxMask = (1u << 30) - 1;
constexpr uint32_t kPad = 0xffffffffu;   // gather-map entry of a tap outside the image

using cfloat = const __attribute__((address_space(4))) float;
__device__ inline cfloat* as_const(const float* p) { return (cfloat*)(uintptr_t)p; }

// first index in [b, e) with ys[i] >= y (rows are sorted)
__device__ inline uint32_t lower_bound_y(const uint16_t* ys, uint32_t b, uint32_t e, int y) {
  while (b < e) {
    const uint32_t mid = (b + e) >> 1;
    if (int(ys[mid]) < y) b = mid + 1; else e = mid;
  }
  return b;
}

template <typename T>
__device__ inline void load_row(const T* base, int C, float* v) {
  for (int c = 0; c < C; ++c) v[c] = to_f32<T>(base[c]);
}

// ---------------------------------------------------------------------------
// Multichannel forward on the vector ALUs: one lane per particle of level l
// (flat over the level's particles, blocks mapped so that each XCD takes a
// contiguous run).  The gather-map entries of a chunk of taps are all loaded
// before the first row load (independent loads in flight); the level's
// weights sit in LDS as [tap][c_in][c_out] (same address in every lane:
// broadcast reads).
// ---------------------------------------------------------------------------
constexpr int kFlatThreads = 256;

template <int K, int CIN, int COUT>
struct FlatCfg {
  static constexpr int K3 = K * K * K;
  static constexpr int NW = K3 * CIN * COUT;
  static constexpr int CHUNK = K3 <= 27 ? K3 : 25;   // taps whose map entries are loaded together
};

// first block of the contiguous run given to XCD blockIdx % 8
__device__ inline uint32_t xcd_block(uint32_t n_blocks) {
  const uint32_t per_xcd = gridDim.x / 8;
  const uint32_t blk = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  return blk < n_blocks ? blk : 0xffffffffu;
}

template <int K, int CIN, int COUT, typename TX, typename TY>
__global__ __launch_bounds__(kFlatThreads) void mc_fwd_kernel(
    const uint32_t* __restrict__ gmap, int64_t n_p, uint32_t p_begin, uint32_t p_end, const TX* __restrict__ x,
    const TX* __restrict__ tree, const float* __restrict__ w_level, const float* __restrict__ bias, int relu,
    const TY* __restrict__ residual, TY* __restrict__ y, uint32_t n_blocks) {
  using Cfg = FlatCfg<K, CIN, COUT>;
  constexpr int K3 = Cfg::K3, CHUNK = Cfg::CHUNK;
  __shared__ float sw[Cfg::NW];
  for (int i = threadIdx.x; i < Cfg::NW; i += kFlatThreads) {
    const int q = i % K3, ci = (i / K3) % CIN, co = i / (K3 * CIN);   // source layout [co][ci][q]
    sw[(q * CIN + ci) * COUT + co] = w_level[i];
  }
  __syncthreads();
  const uint32_t blk = xcd_block(n_blocks);
  if (blk == 0xffffffffu) return;
  const uint32_t p = p_begin + blk * kFlatThreads + threadIdx.x;
  if (p >= p_end) return;
  float acc[COUT];
#pragma unroll
  for (int co = 0; co < COUT; ++co) acc[co] = bias ? bias[co] : 0.f;
  for (int q0 = 0; q0 < K3; q0 += CHUNK) {
    uint32_t g[CHUNK];
#pragma unroll
    for (int j = 0; j < CHUNK; ++j) g[j] = (q0 + j < K3) ? gmap[size_t(q0 + j) * size_t(n_p) + p] : kPad;
#pragma unroll
    for (int j = 0; j < CHUNK; ++j) {
      if (g[j] == kPad) continue;
      const TX* src = (((g[j] >> 30) == 3) ? tree : x) + size_t(g[j] & kIdxMask) * CIN;
      float v[CIN];
      load_vec<TX, CIN>(src, v);
      const float* wq = sw + (q0 + j) * CIN * COUT;
#pragma unroll
      for (int ci = 0; ci < CIN; ++ci)
#pragma unroll
        for (int co = 0; co < COUT; ++co) acc[co] = fmaf(wq[ci * COUT + co], v[ci], acc[co]);
    }
  }
  TY out[COUT];
#pragma unroll
  for (int co = 0; co < COUT; ++co) {
    float o = acc[co];
    if (residual) o += to_f32<TY>(residual[size_t(p) * COUT + co]);
    if (relu) o = fmaxf(o, 0.f);
    out[co] = from_f32<TY>(o);
  }
  store_vec<TY, COUT>(y + size_t(p) * COUT, out);
}

// number of children of a level-L cell that lie in the image
__device__ inline int n_children(const Meta& m, int L, int z, int x, int y) {
  const int C = L + 1;
  return (2 * z + 1 < m.dz[C] ? 2 : 1) * (2 * x + 1 < m.dx[C] ? 2 : 1) * (2 * y + 1 < m.dy[C] ? 2 : 1);
}

// ---------------------------------------------------------------------------
// Data gradient, last step: adjoint of the child mean.  For every element at
// level L (tree node, or particle when `to_particles`), add its parent's
// accumulated gradient divided by the parent's child count.  Launched level
// by level from the coarsest, so the parent's value is final.
// ---------------------------------------------------------------------------
template <int CIN>
__global__ __launch_bounds__(64 * kGWaves) void push_down_kernel(
    Meta m, int L, const uint16_t* __restrict__ ys, const uint32_t* __restrict__ ends, uint32_t row0,
    const uint16_t* __restrict__ ty, const uint32_t* __restrict__ tend, const float* __restrict__ dt,
    float* __restrict__ out) {
  const int64_t row = int64_t(blockIdx.x) * kGWaves + threadIdx.x / 64;
  if (row >= int64_t(m.dz[L]) * m.dx[L]) return;
  const int z = int(row / m.dx[L]), xr = int(row % m.dx[L]);
  uint32_t b, e;
  row_range(ends, row0 + uint32_t(row), b, e);
  if (b == e) return;
  const int P = L - 1;
  uint32_t pb, pe;
  row_range(tend, m.trow[P] + uint32_t(z >> 1) * m.dx[P] + (xr >> 1), pb, pe);
  for (uint32_t i = b + lane_id(); i < e; i += 64) {
    const int yv = ys[i];
    const uint32_t par = lower_bound_y(ty, pb, pe, yv >> 1);   // the parent exists by construction
    const float inv = 1.f / float(n_children(m, P, z >> 1, xr >> 1, yv >> 1));
#pragma unroll
    for (int ci = 0; ci < CIN; ++ci) out[size_t(i) * CIN + ci] += dt[size_t(par) * CIN + ci] * inv;
  }
}

// The same step parent-major, on the child map: one lane per tree node of
// level P adds its gradient divided by its child count to each child (tree
// nodes and particles of level P + 1).  Every child has one parent, so no two
// lanes write one row, and each child gets the same single addition as above.
template <int CIN>
__global__ __launch_bounds__(256) void push_down_parent_kernel(const uint32_t* __restrict__ cmap, int64_t n_t,
                                                               uint32_t t_begin, uint32_t t_end,
                                                               float* __restrict__ dt, float* __restrict__ dx) {
  const uint32_t i = t_begin + blockIdx.x * 256u + threadIdx.x;
  if (i >= t_end) return;
  uint32_t code[8];
  int n = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    code[j] = cmap[size_t(j) * size_t(n_t) + i];
    n += code[j] != kChildPad;
  }
  const float inv = 1.f / float(n);
  float v[CIN];
  load_vec<float, CIN>(dt + size_t(i) * CIN, v);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (code[j] == kChildPad) continue;
    float* o = ((code[j] >> 31) ? dt : dx) + size_t(code[j] & 0x7fffffffu) * CIN;
    float u[CIN];
    load_vec<float, CIN>(o, u);
#pragma unroll
    for (int c = 0; c < CIN; ++c) u[c] += v[c] * inv;
    store_vec<float, CIN>(o, u);
  }
}

// ---------------------------------------------------------------------------
// Weight gradient: block j of level l sums dY[p, co] * Xcat[src(p, o), ci]
// over its particles (staged PCH at a time in LDS) for every (co, ci, o), in
// FP32, and writes an FP64 partial.
// ---------------------------------------------------------------------------
constexpr int kWgtThreads = 256;
constexpr int kWgtParticles = 2048;   // particles per block

template <int K, int CIN, int COUT, typename TX>
__global__ __launch_bounds__(kWgtThreads) void bwd_weight_partial_kernel(
    int64_t p_begin, int64_t p_end, const int32_t* __restrict__ gmap, int64_t n_p,
    const TX* __restrict__ x, const TX* __restrict__ tree, const float* __restrict__ dy,
    double* __restrict__ partial) {
  constexpr int K3 = K * K * K;
  constexpr int NOUT = COUT * CIN * K3;
  constexpr int PCH = (K3 * CIN >= 2000) ? 8 : ((K3 * CIN >= 500) ? 16 : 32);
  constexpr int NPT = (NOUT + kWgtThreads - 1) / kWgtThreads;   // outputs per thread
  __shared__ float sv[PCH][K3 * CIN];
  __shared__ float sg[PCH][COUT];
  const int tid = threadIdx.x;
  const int64_t blk_b = p_begin + int64_t(blockIdx.x) * kWgtParticles;
  const int64_t blk_e = min(p_end, blk_b + kWgtParticles);
  float acc[NPT];
#pragma unroll
  for (int j = 0; j < NPT; ++j) acc[j] = 0.f;
  for (int64_t c0 = blk_b; c0 < blk_e; c0 += PCH) {
    const int np = int(min<int64_t>(PCH, blk_e - c0));
    __syncthreads();
    for (int j = tid; j < PCH * K3; j += kWgtThreads) {
      const int pp = j / K3, q = j % K3;
      float v[CIN];
#pragma unroll
      for (int ci = 0; ci < CIN; ++ci) v[ci] = 0.f;
      if (pp < np) {
        const uint32_t g = gmap[size_t(q) * size_t(n_p) + size_t(c0 + pp)];
        if (g != kPad) {
          const uint32_t idx = g & kIdxMask;
          load_row<TX>(((g >> 30) == 3) ? tree + size_t(idx) * CIN : x + size_t(idx) * CIN, CIN, v);
        }
      }
#pragma unroll
      for (int ci = 0; ci < CIN; ++ci) sv[pp][q * CIN + ci] = v[ci];
    }
    for (int j = tid; j < PCH * COUT; j += kWgtThreads) {
      const int pp = j / COUT, co = j % COUT;
      sg[pp][co] = (pp < np) ? dy[size_t(c0 + pp) * COUT + co] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < NPT; ++jj) {
      const int o = tid + jj * kWgtThreads;   // o = (co * CIN + ci) * K3 + q
      if (o >= NOUT) break;
      const int q = o % K3, ci = (o / K3) % CIN, co = o / (K3 * CIN);
      float s = acc[jj];
      for (int pp = 0; pp < np; ++pp) s = fmaf(sg[pp][co], sv[pp][q * CIN + ci], s);
      acc[jj] = s;
    }
  }
#pragma unroll
  for (int jj = 0; jj < NPT; ++jj) {
    const int o = tid + jj * kWgtThreads;
    if (o < NOUT) partial[size_t(blockIdx.x) * NOUT + o] = double(acc[jj]);
  }
}

// dw[lo][o] = sum over the blocks [blk_b, blk_e) of partial[blk][o], in order
// Fixed-order FP64 reduction of the block partials [blk_b, blk_e) in two
// stages: chunks of kRedChunk partials are summed in place into the chunk's
// first row (blockIdx.y = chunk), then the chunk sums in order.
constexpr int kRedChunk = 64;

__global__ void bwd_weight_chunk_kernel(double* __restrict__ partial, int64_t blk_b, int64_t blk_e, int nout) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j0 = blk_b + int64_t(blockIdx.y) * kRedChunk;
  if (o >= nout || j0 >= blk_e) return;
  const int64_t j1 = min(blk_e, j0 + kRedChunk);
  double s = 0.0;
  for (int64_t j = j0; j < j1; ++j) s += partial[size_t(j) * nout + o];
  partial[size_t(j0) * nout + o] = s;
}

__global__ void bwd_weight_reduce_kernel(const double* __restrict__ partial, int64_t blk_b, int64_t blk_e,
                                         int nout, float* __restrict__ dw) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nout) return;
  double s = 0.0;
  for (int64_t j = blk_b; j < blk_e; j += kRedChunk) s += partial[size_t(j) * nout + o];
  dw[o] = float(s);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int level_blocks(const apr_handle* h, int l) {
  return int((h->per_level_p[l] + kWgtParticles - 1) / kWgtParticles);
}

static int64_t level_first(const apr_handle* h, int l) {
  int64_t b = 0;
  for (int q = h->meta.l_min; q < l; ++q) b += h->per_level_p[q];
  return b;
}

static const int32_t* gather_map(const apr_handle* h, int k) { return h->gmap[k == 3 ? 0 : 1]; }

#define APR_CH_DISPATCH(CIN_, COUT_, ...)                                            \
  if (cin == CIN_ && cout == COUT_) {                                                \
    constexpr int CI = CIN_, CO = COUT_;                                             \
    __VA_ARGS__;                                                                     \
  }

// ---------------------------------------------------------------------------
// Multichannel forward, 16 -> 16 channels, BF16 activations, on MFMA
// (v_mfma_f32_16x16x16_bf16: 16 particles x 16 input channels times 16 input
// x 16 output channels per tap, 27 taps accumulated in FP32).  Lane l holds
// A[m = l % 16][k = 4 (l / 16) + i], B[k = 4 (l / 16) + i][n = l % 16] and
// D[m = 4 (l / 16) + i][n = l % 16], i = 0..3.  The per-level weights of
// every tap stay in registers as BF16 (B operands); a wave walks 16-particle
// tiles of one level, the blocks mapped so that each XCD takes a contiguous
// run of tiles (neighbouring tiles share gathered rows in that XCD's L2).
// ---------------------------------------------------------------------------
typedef short mfma_s4 __attribute__((ext_vector_type(4)));
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

__device__ inline short bf16_bits(float v) {
  const __hip_bfloat16 b = from_f32<__hip_bfloat16>(v);
  short r;
  __builtin_memcpy(&r, &b, 2);
  return r;
}

constexpr int kMfmaWaves = 4;
constexpr int kMfmaBlocksPerXcd = 96;   // 32 CUs x 12 waves / 4 waves per block

// four FP8 codes of a row word widened to the A operand on the conversion
// unit (exact: every E4M3 value is a BF16 value, so the BF16 bits are the
// high half of the FP32 bits)
__device__ inline mfma_s4 fp8x4_to_bf16(uint32_t c) {
  float f[4];
  fp8x4_to_f32(c, f);
  return mfma_s4{short(__float_as_uint(f[0]) >> 16), short(__float_as_uint(f[1]) >> 16),
                 short(__float_as_uint(f[2]) >> 16), short(__float_as_uint(f[3]) >> 16)};
}

typedef __bf16 mfma_b8 __attribute__((ext_vector_type(8)));

// 16 -> 16 channels, 3^3, BF16 rows on v_mfma_f32_16x16x32_bf16 (gfx950).  The reduction axis of instruction m (m = 0..13)
// is two taps x 16 input channels: lane l (r16 = l % 16, kg = l / 16) holds
// A[particle r16][k = 8 kg + i] = row(tap 2m + kg / 2)[8 (kg % 2) + i], one
// 16-byte load, and B[k][n = r16] = W[r16][8 (kg % 2) + i][2m
// + kg / 2] staged in LDS; tap 27 is zero.  D: lane l holds outputs 4 kg + i
// of channel r16.  Persistent waves over an XCD-contiguous tile range.  Half
// the row loads and MFMA instructions of the 16x16x16 form below.
template <typename TX, typename TY>
__global__ __launch_bounds__(64 * kMfmaWaves) void mc16_mfma32_kernel(
    const uint32_t* __restrict__ gmap, int64_t n_p, uint32_t p_begin, uint32_t p_end,
    const TX* __restrict__ x, const TX* __restrict__ tree, const float* __restrict__ w_level,
    const float* __restrict__ bias, int relu, const TY* __restrict__ residual, TY* __restrict__ y) {
  constexpr int K3 = 27, NM = 14;
  static_assert(std::is_same<TX, __hip_bfloat16>::value, "BF16 rows");
  // B operands of the level, [instruction][lane], staged once per block
  __shared__ uint4 sb[NM][64];
  for (int j = threadIdx.x; j < NM * 64; j += 64 * kMfmaWaves) {
    const int m = j / 64, ln = j % 64, n = ln & 15, q = 2 * m + (ln >> 5), c = 8 * ((ln >> 4) & 1);
    uint32_t v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t lo = q < K3 ? uint16_t(bf16_bits(w_level[(n * 16 + c + 2 * i) * K3 + q])) : 0u;
      const uint32_t hi = q < K3 ? uint16_t(bf16_bits(w_level[(n * 16 + c + 2 * i + 1) * K3 + q])) : 0u;
      v[i] = lo | (hi << 16);
    }
    sb[m][ln] = make_uint4(v[0], v[1], v[2], v[3]);
  }
  __syncthreads();
  // XCD blockIdx % 8 takes the contiguous tile range [tb, te); its waves
  // stride through it
  const uint32_t n_tiles = (p_end - p_begin + 15) / 16;
  const uint32_t per = (n_tiles + 7) / 8;
  const uint32_t tb = (blockIdx.x % 8) * per;
  const uint32_t te = min(n_tiles, tb + per);
  const uint32_t waves_per_xcd = (gridDim.x / 8) * kMfmaWaves;
  uint32_t tile = tb + (blockIdx.x / 8) * kMfmaWaves + threadIdx.x / 64;
  if (tile >= te) return;
  const int lane = int(threadIdx.x & 63);
  const int r16 = lane & 15, kg = lane >> 4, half = kg & 1, qo = kg >> 1;
  const float bco = bias ? bias[r16] : 0.f;
  // map entries of this lane's taps for particle r16 of a tile (kPad past the end)
  auto load_map = [&](uint32_t tl, uint32_t (&g)[NM]) {
    const uint32_t p = p_begin + tl * 16 + uint32_t(r16);
    const bool valid = tl < te && p < p_end;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      const int q = 2 * m + qo;
      g[m] = (valid && q < K3) ? gmap[size_t(q) * size_t(n_p) + p] : kPad;
    }
  };
  uint32_t g[NM];
  load_map(tile, g);
  for (; tile < te; tile += waves_per_xcd) {
    uint4 a[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      a[m] = make_uint4(0u, 0u, 0u, 0u);
      if (g[m] != kPad) {
        const TX* row = ((g[m] >> 30) == 3 ? tree : x) + size_t(g[m] & kIdxMask) * 16;
        a[m] = *reinterpret_cast<const uint4*>(row + 8 * half);
      }
    }
    mfma_f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int m = 0; m < NM; ++m)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(mfma_b8, a[m]),
                                                    __builtin_bit_cast(mfma_b8, sb[m][lane]), acc, 0, 0, 0);
    const uint32_t t0 = p_begin + tile * 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t pm = t0 + 4 * kg + i;
      if (pm >= p_end) continue;
      float o = acc[i] + bco;
      if (residual) o += to_f32<TY>(residual[size_t(pm) * 16 + r16]);
      if (relu) o = fmaxf(o, 0.f);
      y[size_t(pm) * 16 + r16] = from_f32<TY>(o);
    }
    load_map(tile + waves_per_xcd, g);
  }
}

// 16 -> 16 channels, 3^3, on v_mfma_f32_16x16x16_bf16 (FP8 rows, widened
// exactly): lane l (r16 = l % 16, kg = l / 16) holds A[particle r16][input
// channel 4 kg + i] of a tap and B[4 kg + i][output channel r16].
template <typename TX, typename TY>
__global__ __launch_bounds__(64 * kMfmaWaves) void mc16_mfma_kernel(
    const uint32_t* __restrict__ gmap, int64_t n_p, uint32_t p_begin, uint32_t p_end,
    const TX* __restrict__ x, const TX* __restrict__ tree, const float* __restrict__ w_level,
    const float* __restrict__ bias, int relu, const TY* __restrict__ residual, TY* __restrict__ y) {
  constexpr int K3 = 27;
  // XCD blockIdx % 8 takes the contiguous tile range [tb, te); its waves
  // stride through it
  const uint32_t n_tiles = (p_end - p_begin + 15) / 16;
  const uint32_t per = (n_tiles + 7) / 8;
  const uint32_t tb = (blockIdx.x % 8) * per;
  const uint32_t te = min(n_tiles, tb + per);
  const uint32_t waves_per_xcd = (gridDim.x / 8) * kMfmaWaves;
  uint32_t tile = tb + (blockIdx.x / 8) * kMfmaWaves + threadIdx.x / 64;
  if (tile >= te) return;
  const int lane = int(threadIdx.x & 63);
  const int r16 = lane & 15, kg = lane >> 4;
  mfma_s4 bw[K3];
#pragma unroll
  for (int q = 0; q < K3; ++q)
#pragma unroll
    for (int i = 0; i < 4; ++i) bw[q][i] = bf16_bits(w_level[(r16 * 16 + 4 * kg + i) * K3 + q]);
  const float bco = bias ? bias[r16] : 0.f;
  for (; tile < te; tile += waves_per_xcd) {
    const uint32_t t0 = p_begin + tile * 16;
    const uint32_t p = t0 + r16;
    const bool valid = p < p_end;
    uint32_t g[K3];
#pragma unroll
    for (int q = 0; q < K3; ++q) g[q] = valid ? gmap[size_t(q) * size_t(n_p) + p] : kPad;
    mfma_f4 acc = {0.f, 0.f, 0.f, 0.f};
    if constexpr (std::is_same<TX, fp8e4m3>::value) {
      // every row word in flight first, then widen and multiply tap by tap
      uint32_t raw[K3];
#pragma unroll
      for (int q = 0; q < K3; ++q)
        raw[q] = (g[q] != kPad) ? *reinterpret_cast<const uint32_t*>(((g[q] >> 30) == 3 ? tree : x) +
                                                                     size_t(g[q] & kIdxMask) * 16 + 4 * kg)
                                : 0u;
#pragma unroll
      for (int q = 0; q < K3; ++q)
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fp8x4_to_bf16(raw[q]), bw[q], acc, 0, 0, 0);
    } else {
      mfma_s4 a[K3];
#pragma unroll
      for (int q = 0; q < K3; ++q) {
        a[q] = mfma_s4{0, 0, 0, 0};
        if (g[q] != kPad)
          a[q] = *reinterpret_cast<const mfma_s4*>(((g[q] >> 30) == 3 ? tree : x) + size_t(g[q] & kIdxMask) * 16 +
                                                   4 * kg);
      }
#pragma unroll
      for (int q = 0; q < K3; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[q], bw[q], acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t pm = t0 + 4 * kg + i;
      if (pm >= p_end) continue;
      float o = acc[i] + bco;
      if (residual) o += to_f32<TY>(residual[size_t(pm) * 16 + r16]);
      if (relu) o = fmaxf(o, 0.f);
      y[size_t(pm) * 16 + r16] = from_f32<TY>(o);
    }
  }
}

template <typename TX, typename TY>
static void launch_mc16_mfma(const apr_handle* h, const apr_conv_desc* d, const void* x, const void* tree,
                             const float* w, void* y, hipStream_t s) {
  const Meta& m = h->meta;
  uint32_t begin = 0;
  for (int l = m.l_min; l <= m.l_max; ++l) {
    const uint32_t np_l = uint32_t(h->per_level_p[l]);
    if (np_l) {
      const float* wl = w + size_t(d->n_wlevels == 1 ? 0 : l - m.l_min) * 16 * 16 * 27;
      const uint32_t tiles = (np_l + 15) / 16;
      // enough waves to fill every CU (3 per SIMD), no more than one per tile
      const uint32_t blocks_per_xcd = std::min<uint32_t>(kMfmaBlocksPerXcd, (tiles / 8 + kMfmaWaves) / kMfmaWaves);
      void (*kern)(const uint32_t*, int64_t, uint32_t, uint32_t, const TX*, const TX*, const float*, const float*,
                   int, const TY*, TY*) = mc16_mfma_kernel<TX, TY>;
      if constexpr (std::is_same<TX, __hip_bfloat16>::value) kern = mc16_mfma32_kernel<TX, TY>;
      hipLaunchKernelGGL(kern, dim3(8 * std::max<uint32_t>(1, blocks_per_xcd)), dim3(64 * kMfmaWaves), 0, s,
                         reinterpret_cast<const uint32_t*>(gather_map(h, 3)), h->n_p, begin, begin + np_l,
                         static_cast<const TX*>(x), static_cast<const TX*>(tree), wl, d->bias, d->relu,
                         static_cast<const TY*>(d->residual), static_cast<TY*>(y));
    }
    begin += np_l;
  }
}

// APR_WIDE_OFFSETS=1 in the environment selects the 64-bit addressing forms of
// the 16 -> 16 weight gradient and data-gradient kernels at every size (they
// are otherwise taken only above the buffer limit), so that both forms can be
// compared on small inputs.
// (APR_WIDE_OFFSETS=2: the weight gradient's two-buffer 32-bit form instead.)
static int wide_offsets_mode() {
  const char* e = std::getenv("APR_WIDE_OFFSETS");
  return (e && e[0] == '2') ? 2 : (e && e[0] && e[0] != '0') ? 1 : 0;
}
static bool wide_offsets_forced() { return wide_offsets_mode() == 1; }

// Sixteen channels of zeros (FP32 or BF16): the row a padded tap reads.
__device__ __align__(64) uint32_t kZeroRow[16] = {};

// Byte offsets at and above kBufOob are outside every buffer the BUF forms
// read (the host takes those forms only when the gathered arrays are
// smaller), and a raw buffer load outside its buffer's size returns zero.
constexpr uint32_t kBufOob = 0xF0000000u;
constexpr int kBufDword3 = 0x00020000;   // buffer resource word 3 on gfx9 parts (raw, 32-bit data)

template <typename TX>
__device__ inline TX buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ inline float buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, int(off), 0, 0));
}
template <>
__device__ inline __hip_bfloat16 buf_load<__hip_bfloat16>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  const unsigned short u = __builtin_amdgcn_raw_buffer_load_b16(r, int(off), 0, 0);
  return __builtin_bit_cast(__hip_bfloat16, u);
}
__device__ inline mfma_f4 buf_load_row4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(mfma_f4, __builtin_amdgcn_raw_buffer_load_b128(r, int(off), 0, 0));
}
template <typename TX>
__device__ inline TX bits_or(TX a, TX b) {
  using U = typename std::conditional<sizeof(TX) == 4, uint32_t, unsigned short>::type;
  return __builtin_bit_cast(TX, U(__builtin_bit_cast(U, a) | __builtin_bit_cast(U, b)));
}

// ---------------------------------------------------------------------------
// 16 -> 16 channels with FP32 rows on MFMA (v_mfma_f32_16x16x4_f32), for the
// FP32 forward and for the same-level part of the data gradient (BWD: rows
// are dY, taps flipped, only same-level entries, weights transposed).  The
// reduction axis (16 input channels) is split as c = 4 kg + j over the lane
// group kg = l / 16 and the four instructions j of a tap: lane l loads the
// contiguous float4 R[src][4 kg .. 4 kg + 3] and holds A_j[m = l % 16][k = kg]
// = R[src(p_m)][4 kg + j] and B_j[k = kg][n = l % 16] = Wt[4 kg + j][n]; D
// lane layout as in the BF16 kernel.  B operands staged per block in LDS in
// lane order; persistent waves over an XCD-contiguous tile range.
// ---------------------------------------------------------------------------
template <bool BWD, typename TY, bool BUF>
__global__ __launch_bounds__(64 * kMfmaWaves) __attribute__((amdgpu_waves_per_eu(1, 4))) void mc16_f32_mfma_kernel(
    const uint32_t* __restrict__ gmap, int64_t n_p, uint32_t p_begin, uint32_t p_end, const float* __restrict__ rows,
    uint32_t rows_bytes, const float* __restrict__ tree, const float* __restrict__ w_level,
    const float* __restrict__ bias, int relu, const TY* __restrict__ residual, TY* __restrict__ out) {
  constexpr int K3 = 27;
  // (unused, and dropped by the compiler, when BUF is false)
  const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(rows), 0, int(rows_bytes), kBufDword3);
  __shared__ mfma_f4 sb[K3][64];
  for (int j = threadIdx.x; j < K3 * 64; j += 64 * kMfmaWaves) {
    const int q = j / 64, ln = j % 64, n = ln & 15, k = ln >> 4;
    mfma_f4 v;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int c = 4 * k + jj;
      v[jj] = BWD ? w_level[(c * 16 + n) * K3 + q] : w_level[(n * 16 + c) * K3 + q];
    }
    sb[q][ln] = v;
  }
  __syncthreads();
  const uint32_t n_tiles = (p_end - p_begin + 15) / 16;
  const uint32_t per = (n_tiles + 7) / 8;
  const uint32_t tb = (blockIdx.x % 8) * per;
  const uint32_t te = min(n_tiles, tb + per);
  const uint32_t waves_per_xcd = (gridDim.x / 8) * kMfmaWaves;
  const int lane = int(threadIdx.x & 63);
  const int r16 = lane & 15, kg = lane >> 4;
  const float bco = (!BWD && bias) ? bias[r16] : 0.f;
  for (uint32_t tile = tb + (blockIdx.x / 8) * kMfmaWaves + threadIdx.x / 64; tile < te; tile += waves_per_xcd) {
    asm volatile("" ::: "memory");   // keep the B operands in LDS (read per tile)
    const uint32_t t0 = p_begin + tile * 16;
    const uint32_t p = t0 + r16;
    const bool valid = p < p_end;
    uint32_t g[K3];
#pragma unroll
    for (int q = 0; q < K3; ++q) {   // unconditional loads (a row past the end reads the first)
      const uint32_t gv = gmap[size_t(BWD ? K3 - 1 - q : q) * size_t(n_p) + (valid ? p : p_begin)];
      g[q] = valid ? gv : kPad;
    }
    // every gathered row of the tile in flight before the first product, no
    // branch per tap: a padded tap (in the adjoint, every tap whose source is
    // not a same-level particle) reads zeros
    mfma_f4 a[K3];
#pragma unroll
    for (int q = 0; q < K3; ++q) {
      const uint32_t gg = g[q];
      if constexpr (BWD) {
        const bool use = (gg >> 30) == 1;
        if constexpr (BUF)
          a[q] = buf_load_row4(rr, use ? ((gg & kIdxMask) << 6) | uint32_t(kg << 4) : kBufOob);
        else
          a[q] = *reinterpret_cast<const mfma_f4*>((use ? rows : reinterpret_cast<const float*>(kZeroRow)) +
                                                   size_t(use ? gg & kIdxMask : 0u) * 16 + 4 * kg);
      } else {
        const float* src = gg == kPad ? reinterpret_cast<const float*>(kZeroRow) : ((gg >> 30) == 3 ? tree : rows);
        a[q] = *reinterpret_cast<const mfma_f4*>(src + size_t(gg == kPad ? 0u : gg & kIdxMask) * 16 + 4 * kg);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    mfma_f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < K3; ++q) {
      const mfma_f4 b = sb[q][lane];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q][j], b[j], acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t pm = t0 + 4 * kg + i;
      if (pm >= p_end) continue;
      float o = acc[i] + bco;
      if (!BWD && residual) o += to_f32<TY>(residual[size_t(pm) * 16 + r16]);
      if (!BWD && relu) o = fmaxf(o, 0.f);
      out[size_t(pm) * 16 + r16] = from_f32<TY>(o);
    }
  }
}

template <bool BWD, typename TY>
static void launch_mc16_f32_mfma(const apr_handle* h, uint32_t begin, uint32_t np_l, const float* rows,
                                 const float* tree, const float* wl, const float* bias, int relu, const TY* residual,
                                 TY* out, hipStream_t s) {
  const uint32_t tiles = (np_l + 15) / 16;
  const uint32_t blocks_per_xcd = std::min<uint32_t>(kMfmaBlocksPerXcd, (tiles / 8 + kMfmaWaves) / kMfmaWaves);
  // the adjoint reads dY rows through 32-bit buffer offsets below kBufOob bytes
  const uint64_t rb = uint64_t(h->n_p) * 64;
  const bool buf = BWD && rb <= kBufOob && !wide_offsets_forced();
  auto kern = buf ? mc16_f32_mfma_kernel<BWD, TY, true> : mc16_f32_mfma_kernel<BWD, TY, false>;
  hipLaunchKernelGGL(kern, dim3(8 * std::max<uint32_t>(1, blocks_per_xcd)), dim3(64 * kMfmaWaves), 0, s,
                     reinterpret_cast<const uint32_t*>(gather_map(h, 3)), h->n_p, begin, begin + np_l, rows,
                     uint32_t(buf ? rb : 0), tree, wl, bias, relu, residual, out);
}

template <int K, int CI, int CO, typename TX, typename TY>
static void launch_mc_fwd(const apr_handle* h, const apr_conv_desc* d, const void* x, const void* tree,
                          const float* w, void* y, hipStream_t s) {
  const Meta& m = h->meta;
  uint32_t begin = 0;
  for (int l = m.l_min; l <= m.l_max; ++l) {
    const uint32_t np_l = uint32_t(h->per_level_p[l]);
    if (np_l) {
      const float* wl = w + size_t(d->n_wlevels == 1 ? 0 : l - m.l_min) * CO * CI * K * K * K;
      const uint32_t nb = (np_l + kFlatThreads - 1) / kFlatThreads;
      hipLaunchKernelGGL((mc_fwd_kernel<K, CI, CO, TX, TY>), dim3((nb + 7) / 8 * 8), dim3(kFlatThreads), 0, s,
                         reinterpret_cast<const uint32_t*>(gather_map(h, K)), h->n_p, begin, begin + np_l,
                         static_cast<const TX*>(x), static_cast<const TX*>(tree), wl, d->bias, d->relu,
                         static_cast<const TY*>(d->residual), static_cast<TY*>(y), nb);
    }
    begin += np_l;
  }
}

template <int K, int CI, int CO>
static apr_status mc_fwd_dtypes(const apr_handle* h, const apr_conv_desc* d, const void* x, const void* tree,
                                const float* w, void* y, hipStream_t s) {
  if (d->x_dtype == APR_F32 && d->y_dtype == APR_F32)
    launch_mc_fwd<K, CI, CO, float, float>(h, d, x, tree, w, y, s);
  else if (d->x_dtype == APR_BF16 && d->y_dtype == APR_BF16)
    launch_mc_fwd<K, CI, CO, __hip_bfloat16, __hip_bfloat16>(h, d, x, tree, w, y, s);
  else if (d->x_dtype == APR_BF16 && d->y_dtype == APR_F32)
    launch_mc_fwd<K, CI, CO, __hip_bfloat16, float>(h, d, x, tree, w, y, s);
  else if (d->x_dtype == APR_F32 && d->y_dtype == APR_BF16)
    launch_mc_fwd<K, CI, CO, float, __hip_bfloat16>(h, d, x, tree, w, y, s);
  else
    APR_FAIL(APR_EUNSUPPORTED, "apr_conv: unsupported dtype combination");
  APR_HIP(hipGetLastError());
  return APR_OK;
}

// FP8 activations (network shapes, k = 3): FP8 x into 16 -> 16 on matrix
// cores or 16 -> 1 on the vector ALUs; FP32 / BF16 x into FP8 y.
template <typename TY>
static apr_status mc_fp8_in(const apr_handle* h, const apr_conv_desc* d, const void* x, const void* tree,
                            const float* w, void* y, hipStream_t s) {
  if (d->c_in == 16 && d->c_out == 16) {
    if (((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(tree)) & 3) != 0)
      APR_FAIL(APR_EINVAL, "apr_conv: FP8 rows must be 4-byte aligned");
    launch_mc16_mfma<fp8e4m3, TY>(h, d, x, tree, w, y, s);
  } else {
    launch_mc_fwd<3, 16, 1, fp8e4m3, TY>(h, d, x, tree, w, y, s);
  }
  APR_HIP(hipGetLastError());
  return APR_OK;
}

template <typename TX>
static apr_status mc_fp8_out(const apr_handle* h, const apr_conv_desc* d, const void* x, const void* tree,
                             const float* w, void* y, hipStream_t s) {
  if (d->c_in == 1)
    launch_mc_fwd<3, 1, 16, TX, fp8e4m3>(h, d, x, tree, w, y, s);
  else
    launch_mc_fwd<3, 16, 16, TX, fp8e4m3>(h, d, x, tree, w, y, s);
  APR_HIP(hipGetLastError());
  return APR_OK;
}

static apr_status mc_conv_fp8(const apr_handle* h, const apr_conv_desc* d, const void* x, const void* tree,
                              const float* w, void* y, hipStream_t s) {
  const int cin = d->c_in, cout = d->c_out;
  if (d->k != 3) APR_FAIL(APR_EUNSUPPORTED, "apr_conv: FP8 storage needs k = 3");
  if (d->x_dtype == APR_FP8) {
    if (!((cin == 16 && cout == 16) || (cin == 16 && cout == 1)))
      APR_FAIL(APR_EUNSUPPORTED, "apr_conv: FP8 x supports (c_in, c_out) = (16,16) and (16,1)");
    if (d->y_dtype == APR_FP8) return mc_fp8_in<fp8e4m3>(h, d, x, tree, w, y, s);
    if (d->y_dtype == APR_BF16) return mc_fp8_in<__hip_bfloat16>(h, d, x, tree, w, y, s);
    if (d->y_dtype == APR_F32) return mc_fp8_in<float>(h, d, x, tree, w, y, s);
    APR_FAIL(APR_EUNSUPPORTED, "apr_conv: unsupported dtype combination");
  }
  if (!((cin == 1 && cout == 16) || (cin == 16 && cout == 16)))
    APR_FAIL(APR_EUNSUPPORTED, "apr_conv: FP8 y supports (c_in, c_out) = (1,16) and (16,16)");
  if (d->x_dtype == APR_F32) return mc_fp8_out<float>(h, d, x, tree, w, y, s);
  if (d->x_dtype == APR_BF16) return mc_fp8_out<__hip_bfloat16>(h, d, x, tree, w, y, s);
  APR_FAIL(APR_EUNSUPPORTED, "apr_conv: unsupported dtype combination");
}

apr_status mc_conv(const apr_handle* h, const apr_conv_desc* d, const void* x, const void* tree,
                   const float* w, void* y, hipStream_t s) {
  if (!gather_map(h, d->k))
    APR_FAIL(APR_EINVAL, "apr_conv: this path needs the gather map; build the access with "
                         "APR_BUILD_GATHER3 / APR_BUILD_GATHER5");
  const int cin = d->c_in, cout = d->c_out;
  if (d->x_dtype == APR_FP8 || d->y_dtype == APR_FP8) return mc_conv_fp8(h, d, x, tree, w, y, s);
  if (d->k == 3 && cin == 16 && cout == 16 && d->x_dtype == APR_BF16 &&
      ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(tree)) & 15) == 0) {
    if (d->y_dtype == APR_BF16)
      launch_mc16_mfma<__hip_bfloat16, __hip_bfloat16>(h, d, x, tree, w, y, s);
    else
      launch_mc16_mfma<__hip_bfloat16, float>(h, d, x, tree, w, y, s);
    APR_HIP(hipGetLastError());
    return APR_OK;
  }
  if (d->k == 3 && cin == 16 && cout == 16 && d->x_dtype == APR_F32 &&
      ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(tree)) & 15) == 0) {
    const Meta& m = h->meta;
    uint32_t begin = 0;
    for (int l = m.l_min; l <= m.l_max; ++l) {
      const uint32_t np_l = uint32_t(h->per_level_p[l]);
      const float* wl = w + size_t(d->n_wlevels == 1 ? 0 : l - m.l_min) * 16 * 16 * 27;
      if (np_l) {
        if (d->y_dtype == APR_F32)
          launch_mc16_f32_mfma<false, float>(h, begin, np_l, static_cast<const float*>(x),
                                             static_cast<const float*>(tree), wl, d->bias, d->relu,
                                             static_cast<const float*>(d->residual), static_cast<float*>(y), s);
        else
          launch_mc16_f32_mfma<false, __hip_bfloat16>(h, begin, np_l, static_cast<const float*>(x),
                                                      static_cast<const float*>(tree), wl, d->bias, d->relu,
                                                      static_cast<const __hip_bfloat16*>(d->residual),
                                                      static_cast<__hip_bfloat16*>(y), s);
      }
      begin += np_l;
    }
    APR_HIP(hipGetLastError());
    return APR_OK;
  }
  if (d->k == 3) {
    APR_CH_DISPATCH(1, 1, return mc_fwd_dtypes<3, CI, CO>(h, d, x, tree, w, y, s))
    APR_CH_DISPATCH(1, 16, return mc_fwd_dtypes<3, CI, CO>(h, d, x, tree, w, y, s))
    APR_CH_DISPATCH(16, 16, return mc_fwd_dtypes<3, CI, CO>(h, d, x, tree, w, y, s))
    APR_CH_DISPATCH(16, 1, return mc_fwd_dtypes<3, CI, CO>(h, d, x, tree, w, y, s))
    APR_CH_DISPATCH(2, 3, return mc_fwd_dtypes<3, CI, CO>(h, d, x, tree, w, y, s))
  } else {
    APR_CH_DISPATCH(1, 1, return mc_fwd_dtypes<5, CI, CO>(h, d, x, tree, w, y, s))
    APR_CH_DISPATCH(2, 3, return mc_fwd_dtypes<5, CI, CO>(h, d, x, tree, w, y, s))
  }
  APR_FAIL(APR_EUNSUPPORTED, "apr_conv: unsupported (k, c_in, c_out); supported: k=3 (1,1) (1,16) "
                             "(16,16) (16,1) (2,3); k=5 (1,1) (2,3)");
}

// ---------------------------------------------------------------------------
// Inverse map of the coarse and tree taps (built once with the gather map):
// counts per source, exclusive scan, fill, then each source's readers sorted
// (the fill order of the atomics is arbitrary; the sort makes it fixed).
// ---------------------------------------------------------------------------
__device__ inline int64_t inv_target(uint32_t g, int64_t n_p) {
  const uint32_t t = g >> 30;
  if (g == kPad || t == 1) return -1;
  return t == 2 ? int64_t(g & kIdxMask) : n_p + int64_t(g & kIdxMask);
}

__global__ void inv_count_kernel(const uint32_t* __restrict__ gmap, int64_t n_p, int64_t n_pairs,
                                 uint32_t* __restrict__ count) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_pairs) return;
  const int64_t t = inv_target(gmap[i], n_p);
  if (t >= 0) atomicAdd(&count[t], 1u);
}

__global__ void inv_fill_kernel(const uint32_t* __restrict__ gmap, int64_t n_p, int64_t n_pairs, int k3,
                                const uint32_t* __restrict__ off, uint32_t* __restrict__ cursor,
                                uint32_t* __restrict__ ent) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;   // i = q * n_p + p
  if (i >= n_pairs) return;
  const int64_t t = inv_target(gmap[i], n_p);
  if (t < 0) return;
  const uint32_t q = uint32_t(i / n_p), p = uint32_t(i % n_p);
  ent[off[t] + atomicAdd(&cursor[t], 1u)] = p * uint32_t(k3) + q;
}

// readers of one source ordered by (tap, reader)
__global__ void inv_sort_kernel(const uint32_t* __restrict__ off, int64_t n_targets, int k3,
                                uint32_t* __restrict__ ent) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_targets) return;
  const uint32_t b = off[t], e = off[t + 1];
  auto key = [&](uint32_t c) { return (uint64_t(c % uint32_t(k3)) << 32) | (c / uint32_t(k3)); };
  for (uint32_t i = b + 1; i < e; ++i) {
    const uint32_t v = ent[i];
    const uint64_t kv = key(v);
    uint32_t j = i;
    while (j > b && key(ent[j - 1]) > kv) {
      ent[j] = ent[j - 1];
      --j;
    }
    ent[j] = v;
  }
}

// ---------------------------------------------------------------------------
// Data gradient on the gather map and its inverse, one lane per element:
//   particles of level l: same-level readers (own map, flipped taps) with
//   W_l, then the level-(l+1) readers that use the particle as their coarser
//   source (inverse map) with W_(l+1); one write per particle;
//   tree nodes of level L: the level-L readers landing on the node (inverse
//   map) with W_L.  Weights are staged in LDS as [tap][c_out][c_in].
// ---------------------------------------------------------------------------
constexpr int kInvThreads = 256;

template <int K, int CIN, int COUT>
__device__ inline void stage_wt(const float* __restrict__ w, float* sw) {
  constexpr int K3 = K * K * K, NW = K3 * CIN * COUT;
  for (int i = threadIdx.x; i < NW; i += kInvThreads) {
    const int q = i % K3, ci = (i / K3) % CIN, co = i / (K3 * CIN);   // source layout [co][ci][q]
    sw[(q * COUT + co) * CIN + ci] = w[i];
  }
}

template <int CIN, int COUT>
__device__ inline void acc_tap(const float* __restrict__ sw_q, const float* __restrict__ dyrow, float* acc) {
  float g[COUT];
  load_vec<float, COUT>(dyrow, g);
#pragma unroll
  for (int co = 0; co < COUT; ++co)
#pragma unroll
    for (int ci = 0; ci < CIN; ++ci) acc[ci] = fmaf(sw_q[co * CIN + ci], g[co], acc[ci]);
}

// readers of one source from the inverse map, taps in the same order in
// every lane: the dY rows of the lane's readers through tap q are summed,
// then one product with W_q^T whose weights every lane reads at the same LDS
// address; taps no lane of the wave reads are skipped
template <int K, int CIN, int COUT>
__device__ inline void acc_inverse(const uint32_t* __restrict__ inv_ent, uint32_t b, uint32_t e,
                                   const float* __restrict__ dy, const float* __restrict__ sw, float* acc) {
  constexpr int K3 = K * K * K;
  uint32_t i = b;
  uint32_t c = i < e ? inv_ent[i] : 0xffffffffu;
  for (int q = 0; q < K3; ++q) {
    float g[COUT];
#pragma unroll
    for (int co = 0; co < COUT; ++co) g[co] = 0.f;
    bool any = false;
    while (i < e && int(c % K3) == q) {
      // the next entry is read before this row (unconditionally: e - 1 is an entry of this source)
      const uint32_t cn = inv_ent[min(i + 1, e - 1)];
      float v[COUT];
      load_vec<float, COUT>(dy + size_t(c / K3) * COUT, v);
#pragma unroll
      for (int co = 0; co < COUT; ++co) g[co] += v[co];
      any = true;
      ++i;
      c = i < e ? cn : 0xffffffffu;
    }
    if (!__any(any)) continue;
    const float* w = sw + q * COUT * CIN;
#pragma unroll
    for (int co = 0; co < COUT; ++co)
#pragma unroll
      for (int ci = 0; ci < CIN; ++ci) acc[ci] = fmaf(w[co * CIN + ci], g[co], acc[ci]);
  }
}

// SAME = false: only the readers from the inverse map, added to dx (the
// same-level part was written by the MFMA kernel)
// act (SAME = false only): the lanes take the particles act[p_begin ..
// p_end) instead of p_begin .. p_end - 1
template <int K, int CIN, int COUT, bool SAME>
__global__ __launch_bounds__(kInvThreads) void bwd_dx_kernel(const uint32_t* __restrict__ gmap, int64_t n_p,
                                                             uint32_t p_begin, uint32_t p_end,
                                                             const uint32_t* __restrict__ act,
                                                             const uint32_t* __restrict__ inv_off,
                                                             const uint32_t* __restrict__ inv_ent,
                                                             const float* __restrict__ dy, const float* w_l,
                                                             const float* w_fine, float* __restrict__ dx) {
  constexpr int K3 = K * K * K, NW = K3 * CIN * COUT;
  __shared__ float sw[SAME ? NW : 1], swf[NW];
  if (SAME) stage_wt<K, CIN, COUT>(w_l, sw);
  if (w_fine) stage_wt<K, CIN, COUT>(w_fine, swf);
  __syncthreads();
  const uint32_t j = p_begin + blockIdx.x * uint32_t(kInvThreads) + threadIdx.x;
  if (j >= p_end) return;
  const uint32_t s = (!SAME && act) ? act[j] : j;
  if (!SAME && !(w_fine && inv_off[s + 1] > inv_off[s])) return;
  float acc[CIN];
  if (SAME) {
#pragma unroll
    for (int ci = 0; ci < CIN; ++ci) acc[ci] = 0.f;
  } else {
    load_vec<float, CIN>(dx + size_t(s) * CIN, acc);
  }
  // the same-level reader of s through tap q sits at c_s - o: entry k^3-1-q of s's map
  constexpr int CH = K3 <= 27 ? K3 : 25;
  for (int q0 = 0; SAME && q0 < K3; q0 += CH) {
    uint32_t g[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) g[j] = (q0 + j < K3) ? gmap[size_t(K3 - 1 - (q0 + j)) * size_t(n_p) + s] : kPad;
#pragma unroll
    for (int j = 0; j < CH; ++j)
      if (g[j] != kPad && (g[j] >> 30) == 1) acc_tap<CIN, COUT>(sw + (q0 + j) * COUT * CIN, dy + size_t(g[j] & kIdxMask) * COUT, acc);
  }
  if (w_fine) acc_inverse<K, CIN, COUT>(inv_ent, inv_off[s], inv_off[s + 1], dy, swf, acc);
  store_vec<float, CIN>(dx + size_t(s) * CIN, acc);
}

template <int K, int CIN, int COUT>
__global__ __launch_bounds__(kInvThreads) void bwd_dt_kernel(int64_t n_p, uint32_t t_begin, uint32_t t_end,
                                                             const uint32_t* __restrict__ inv_off,
                                                             const uint32_t* __restrict__ inv_ent,
                                                             const float* __restrict__ dy, const float* w_L,
                                                             float* __restrict__ dt) {
  constexpr int K3 = K * K * K, NW = K3 * CIN * COUT;
  __shared__ float sw[NW];
  if (w_L) stage_wt<K, CIN, COUT>(w_L, sw);
  __syncthreads();
  const uint32_t t = t_begin + blockIdx.x * uint32_t(kInvThreads) + threadIdx.x;
  if (t >= t_end) return;
  float acc[CIN];
#pragma unroll
  for (int ci = 0; ci < CIN; ++ci) acc[ci] = 0.f;
  if (w_L) acc_inverse<K, CIN, COUT>(inv_ent, inv_off[n_p + t], inv_off[n_p + t + 1], dy, sw, acc);
  store_vec<float, CIN>(dt + size_t(t) * CIN, acc);
}

// particles s with readers in the inverse map: flag, then (after an exclusive
// scan of the flags) scatter s to its rank
__global__ void inv_act_flag_kernel(const uint32_t* __restrict__ off, int64_t n_p, uint32_t* __restrict__ flag) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s < n_p) flag[s] = off[s + 1] > off[s] ? 1u : 0u;
}

__global__ void inv_act_scatter_kernel(const uint32_t* __restrict__ off, int64_t n_p,
                                       const uint32_t* __restrict__ rank, uint32_t* __restrict__ act) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s < n_p && off[s + 1] > off[s]) act[rank[s]] = uint32_t(s);
}

apr_status build_inverse_map(apr_handle* h, int k, hipStream_t s,
                             apr_status (*alloc_u32)(apr_handle*, uint32_t**, int64_t),
                             apr_status (*scan)(uint32_t*, int64_t, uint32_t*, hipStream_t), uint32_t* total_dev) {
  const int gi = k == 3 ? 0 : 1;
  const int k3 = k * k * k;
  const int64_t n_pairs = h->n_p * k3, n_targets = h->n_p + h->n_t;
  if (n_pairs >= (int64_t(1) << 32)) APR_FAIL(APR_EUNSUPPORTED, "apr_access_build: n_particles * k^3 must be < 2^32");
  apr_status st = alloc_u32(h, &h->inv_off[gi], n_targets + 1);
  if (st != APR_OK) return st;
  uint32_t* cursor = nullptr;
  if (hipMalloc(&cursor, size_t(n_targets + 1) * 4) != hipSuccess) {
    (void)hipGetLastError();
    APR_FAIL(APR_ENOMEM, "hipMalloc failed (inverse map cursor)");
  }
  const uint32_t* gm = reinterpret_cast<const uint32_t*>(h->gmap[gi]);
  const unsigned gp = unsigned((n_pairs + 255) / 256), gt = unsigned((n_targets + 255) / 256);
  APR_HIP(hipMemsetAsync(h->inv_off[gi], 0, size_t(n_targets + 1) * 4, s));
  hipLaunchKernelGGL(inv_count_kernel, dim3(gp), dim3(256), 0, s, gm, h->n_p, n_pairs, h->inv_off[gi]);
  APR_HIP(hipGetLastError());
  st = scan(h->inv_off[gi], n_targets + 1, total_dev, s);
  if (st != APR_OK) {
    (void)hipFree(cursor);
    return st;
  }
  uint32_t n_ent = 0;
  APR_HIP(hipMemcpyAsync(&n_ent, total_dev, 4, hipMemcpyDeviceToHost, s));
  APR_HIP(hipStreamSynchronize(s));
  st = alloc_u32(h, &h->inv_ent[gi], std::max<int64_t>(n_ent, 1));
  if (st != APR_OK) {
    (void)hipFree(cursor);
    return st;
  }
  APR_HIP(hipMemsetAsync(cursor, 0, size_t(n_targets + 1) * 4, s));
  hipLaunchKernelGGL(inv_fill_kernel, dim3(gp), dim3(256), 0, s, gm, h->n_p, n_pairs, k3, h->inv_off[gi], cursor,
                     h->inv_ent[gi]);
  hipLaunchKernelGGL(inv_sort_kernel, dim3(gt), dim3(256), 0, s, h->inv_off[gi], n_targets, k3, h->inv_ent[gi]);
  APR_HIP(hipGetLastError());
  // the particles with readers, compacted (the cursor array is reused for the
  // flags and their exclusive scan), and where each level's run starts
  const unsigned gpn = unsigned((h->n_p + 255) / 256);
  hipLaunchKernelGGL(inv_act_flag_kernel, dim3(gpn), dim3(256), 0, s, h->inv_off[gi], h->n_p, cursor);
  APR_HIP(hipGetLastError());
  st = scan(cursor, h->n_p, total_dev, s);
  if (st != APR_OK) {
    (void)hipFree(cursor);
    return st;
  }
  uint32_t n_act = 0;
  APR_HIP(hipMemcpyAsync(&n_act, total_dev, 4, hipMemcpyDeviceToHost, s));
  APR_HIP(hipStreamSynchronize(s));
  st = alloc_u32(h, &h->inv_act[gi], std::max<int64_t>(n_act, 1));
  if (st != APR_OK) {
    (void)hipFree(cursor);
    return st;
  }
  hipLaunchKernelGGL(inv_act_scatter_kernel, dim3(gpn), dim3(256), 0, s, h->inv_off[gi], h->n_p, cursor,
                     h->inv_act[gi]);
  APR_HIP(hipGetLastError());
  const Meta& m = h->meta;
  int64_t first = 0;
  for (int l = m.l_min; l <= m.l_max + 1; ++l) {
    uint32_t r = n_act;
    if (first < h->n_p) APR_HIP(hipMemcpyAsync(&r, cursor + first, 4, hipMemcpyDeviceToHost, s));
    APR_HIP(hipStreamSynchronize(s));
    h->inv_act_lvl[gi][l] = r;
    if (l <= m.l_max) first += h->per_level_p[l];
  }
  APR_HIP(hipStreamSynchronize(s));
  (void)hipFree(cursor);
  return APR_OK;
}

template <int K, int CI, int CO>
static apr_status bwd_data_impl(const apr_handle* h, const apr_conv_desc* d, const float* dy, const float* w,
                                float* dx, float* dt, hipStream_t s) {
  const Meta& m = h->meta;
  constexpr int K3 = K * K * K;
  auto wlev = [&](int l) { return w + size_t(d->n_wlevels == 1 ? 0 : l - m.l_min) * CO * CI * K3; };
  const int gi = K == 3 ? 0 : 1;
  const uint32_t* gm = reinterpret_cast<const uint32_t*>(gather_map(h, K));
  uint32_t begin = 0;
  for (int l = m.l_min; l <= m.l_max; ++l) {
    const uint32_t np_l = uint32_t(h->per_level_p[l]);
    const float* wf = (l + 1 <= m.l_max && h->per_level_p[l + 1]) ? wlev(l + 1) : nullptr;
    if (np_l) {
      if constexpr (K == 3 && CI == 16 && CO == 16) {
        launch_mc16_f32_mfma<true, float>(h, begin, np_l, dy, nullptr, wlev(l), nullptr, 0, nullptr, dx, s);
        // only the level's particles that have readers at level l + 1
        const uint32_t ab = uint32_t(h->inv_act_lvl[gi][l]), ae = uint32_t(h->inv_act_lvl[gi][l + 1]);
        if (wf && ae > ab)
          hipLaunchKernelGGL((bwd_dx_kernel<K, CI, CO, false>), dim3((ae - ab + kInvThreads - 1) / kInvThreads),
                             dim3(kInvThreads), 0, s, gm, h->n_p, ab, ae, h->inv_act[gi], h->inv_off[gi],
                             h->inv_ent[gi], dy, wlev(l), wf, dx);
      } else {
        hipLaunchKernelGGL((bwd_dx_kernel<K, CI, CO, true>), dim3((np_l + kInvThreads - 1) / kInvThreads),
                           dim3(kInvThreads), 0, s, gm, h->n_p, begin, begin + np_l, nullptr, h->inv_off[gi],
                           h->inv_ent[gi], dy, wlev(l), wf, dx);
      }
    }
    begin += np_l;
  }
  uint32_t tb = 0;
  for (int L = m.t_lo; L <= m.t_hi; ++L) {
    const uint32_t nt_l = uint32_t(h->per_level_t[L]);
    const float* wL = (L >= m.l_min && h->per_level_p[L]) ? wlev(L) : nullptr;
    if (nt_l)
      hipLaunchKernelGGL((bwd_dt_kernel<K, CI, CO>), dim3((nt_l + kInvThreads - 1) / kInvThreads), dim3(kInvThreads),
                         0, s, h->n_p, tb, tb + nt_l, h->inv_off[gi], h->inv_ent[gi], dy, wL, dt);
    tb += nt_l;
  }
  // adjoint of the child means, coarsest tree level first
  if (h->cmap) {
    uint32_t pb = 0;
    for (int P = m.t_lo; P <= m.t_hi; ++P) {
      const uint32_t np_ = uint32_t(h->per_level_t[P]);
      if (np_)
        hipLaunchKernelGGL((push_down_parent_kernel<CI>), dim3((np_ + 255) / 256), dim3(256), 0, s, h->cmap, h->n_t,
                           pb, pb + np_, dt, dx);
      pb += np_;
    }
  } else {
    for (int L = m.t_lo + 1; L <= m.t_hi; ++L) {
      const int64_t rows = int64_t(m.dz[L]) * m.dx[L];
      hipLaunchKernelGGL((push_down_kernel<CI>), dim3(unsigned((rows + kGWaves - 1) / kGWaves)),
                         dim3(64 * kGWaves), 0, s, m, L, h->ty, h->tend, m.trow[L], h->ty, h->tend, dt, dt);
    }
    for (int l = std::max(m.l_min, m.t_lo + 1); l <= m.l_max; ++l) {
      if (!h->per_level_p[l]) continue;
      const int64_t rows = int64_t(m.dz[l]) * m.dx[l];
      hipLaunchKernelGGL((push_down_kernel<CI>), dim3(unsigned((rows + kGWaves - 1) / kGWaves)),
                         dim3(64 * kGWaves), 0, s, m, l, h->py, h->pend, m.prow[l], h->ty, h->tend, dt, dx);
    }
  }
  APR_HIP(hipGetLastError());
  return APR_OK;
}

// ---------------------------------------------------------------------------
// Weight gradient of a 16 -> 16, 3^3 layer on MFMA (v_mfma_f32_16x16x4_f32):
// dW_l[co][ci][q] = sum_p dY[p][co] X[src(p, q)][ci] is, per tap, a 16 x 16
// product with the particles as the reduction axis.  One block per run of
// kWgtParticles particles of one level (the same units as the generic
// kernel), the 27 taps split over its four waves: four particles per
// instruction, A[m = co][k] = dY[p_k][co], B[k][n = ci] = X[src(p_k, q)][ci];
// lane l holds A[l % 16][l / 16], B[l / 16][l % 16] and D[4 (l / 16) + i]
// [l % 16].  Up to 7 FP32 accumulators per lane; the sums go out as FP64
// partials for the fixed-order reduction.
// ---------------------------------------------------------------------------
// BUF = true: the gathers are raw buffer loads with 32-bit offsets.  A tap
// reads both x and the tree, the source it does not use (and a padded tap,
// both) at an offset past the buffer, which returns zero, so a gather costs a
// handful of 32-bit operations instead of 64-bit pointer selects; the map
// entries of a step come through LDS.
//
// MODE 0: 64-bit addresses; 1: x and the tree as two buffers (above);
// 2: x and the tree lie within kBufOob bytes of each other, and one buffer
// spanning both (based at x, which then is the lower of the two; x_off and
// t_off their byte offsets in it) serves every gather with one load.
template <typename TX, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 4))) void bwd_weight_mfma16_kernel(int64_t p_begin, int64_t p_end,
                                                                const uint32_t* __restrict__ gmap, int64_t n_p,
                                                                const TX* __restrict__ x, const TX* __restrict__ tree,
                                                                uint32_t x_bytes, uint32_t t_bytes,
                                                                uint32_t x_off, uint32_t t_off,
                                                                const float* __restrict__ dy,
                                                                double* __restrict__ partial) {
  constexpr bool BUF = MODE != 0;
  constexpr int K3 = 27, NOUT = 16 * 16 * 27, TQ = 7;   // taps per wave: 7, 7, 7, 6
  constexpr int LOGR = sizeof(TX) == 4 ? 6 : 5;         // log2 of the bytes of a 16-channel row
  const int lane = int(threadIdx.x & 63), wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int r16 = lane & 15, kg = lane >> 4;
  const int q0 = wave * TQ, nq = min(TQ, K3 - q0);
  const int64_t u_b = p_begin + int64_t(blockIdx.x) * kWgtParticles;
  const int64_t u_e = min(p_end, u_b + kWgtParticles);
  // (unused, and dropped by the compiler, when BUF is false)
  const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(const_cast<TX*>(x), 0, int(x_bytes), kBufDword3);
  const __amdgpu_buffer_rsrc_t rt = __builtin_amdgcn_make_buffer_rsrc(const_cast<TX*>(tree), 0, int(t_bytes), kBufDword3);
  mfma_f4 acc[TQ];
#pragma unroll
  for (int t = 0; t < TQ; ++t) acc[t] = mfma_f4{0.f, 0.f, 0.f, 0.f};
  // 24 particles per step: six groups of four, every gather of the step in flight together
  constexpr int NJ = 6, NE = TQ * 4 * NJ, NEP = (NE + 63) / 64;   // map entries of one wave's step
  // BUF form: the wave's map entries of a step are loaded (coalesced, NEP per
  // lane, one step ahead) and staged in LDS, then read back as broadcasts,
  // instead of one load per lane and tap through the texture path.  Entries
  // past NE are padding that nothing reads.
  __shared__ uint32_t s_map[4][64 * NEP];
  __shared__ uint2 s_off2[MODE == 1 ? 4 : 1][MODE == 1 ? 64 * NEP : 1];   // two-buffer form: (x, tree) offsets
  uint32_t nxt[NEP];
  auto load_map = [&](int64_t ps) {
#pragma unroll
    for (int r = 0; r < NEP; ++r) {
      const int i = 64 * r + lane, t = i / (4 * NJ), e = i % (4 * NJ);
      const int64_t p = ps + e;
      nxt[r] = gmap[size_t(min(q0 + t, K3 - 1)) * size_t(n_p) + size_t(p < u_e ? p : u_b)];
    }
  };
  if constexpr (BUF) load_map(u_b);
  for (int64_t p0 = u_b; p0 < u_e; p0 += 4 * NJ) {
    float a[NJ];
    uint32_t g[NJ][TQ];
    if constexpr (BUF) {
      __builtin_amdgcn_wave_barrier();   // the previous step's reads of s_map come first
#pragma unroll
      for (int r = 0; r < NEP; ++r) {   // entries of particles past the block's end read as padded
        const uint32_t gg = p0 + (64 * r + lane) % (4 * NJ) < u_e ? nxt[r] : kPad;
        if constexpr (MODE == 2) {
          // staged as the row's byte offset in the span buffer (past it when
          // padded; the shift drops the source bits), so a gather adds only
          // its lane's channel offset
          s_map[wave][64 * r + lane] =
              gg == kPad ? kBufOob : (gg << LOGR) + (gg >= 0xC0000000u ? t_off : x_off);
        } else if constexpr (MODE == 1) {
          // the offsets in x and in the tree, the unused one (both when
          // padded) past its buffer
          const bool in_tree = gg >= 0xC0000000u, pad = gg == kPad;
          const uint32_t off = gg << LOGR;
          s_off2[wave][64 * r + lane] = make_uint2(in_tree ? kBufOob : off, (in_tree && !pad) ? off : kBufOob);
        } else {
          s_map[wave][64 * r + lane] = gg;
        }
      }
      __builtin_amdgcn_wave_barrier();
      load_map(p0 + 4 * NJ);
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int64_t p = p0 + 4 * j + kg;
      const bool valid = p < u_e;
      const size_t pc = size_t(valid ? p : u_b);   // loads stay unconditional (u_b < u_e)
      a[j] = dy[pc * 16 + r16];   // zero past the block's end: masked at the product
      // the last wave's seventh tap (past 27) re-reads tap 26 into an
      // accumulator that is never stored
#pragma unroll
      for (int t = 0; t < TQ; ++t) {
        if constexpr (MODE == 2) {
          g[j][t] = s_map[wave][t * 4 * NJ + 4 * j + kg];
        } else if constexpr (MODE == 1) {
          g[j][t] = 0u;   // (the offsets are read at the gathers)
        } else {
          const uint32_t gv = gmap[size_t(min(q0 + t, K3 - 1)) * size_t(n_p) + pc];
          g[j][t] = valid ? gv : kPad;
        }
      }
    }
    // Every gather is issued unconditionally, a padded tap reading zeros, and
    // all of them before the first product, so the loads stay in flight
    // together (no branch and no wait per tap).  The scheduling barriers keep
    // the compiler from pulling a use up to its load.
    TX raw[NJ][TQ];
    if constexpr (MODE == 2) {
      __builtin_amdgcn_sched_barrier(0);
      const uint32_t lo_ch = uint32_t(r16 * int(sizeof(TX)));
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int t = 0; t < TQ; ++t) raw[j][t] = buf_load<TX>(rx, g[j][t] + lo_ch);
      __builtin_amdgcn_sched_barrier(0);
    } else if constexpr (BUF) {
      __builtin_amdgcn_sched_barrier(0);
      const uint32_t lo_ch = uint32_t(r16 * int(sizeof(TX)));
      TX vt[NJ][TQ];
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int t = 0; t < TQ; ++t) {
          const uint2 o = s_off2[wave][t * 4 * NJ + 4 * j + kg];
          raw[j][t] = buf_load<TX>(rx, o.x + lo_ch);
          vt[j][t] = buf_load<TX>(rt, o.y + lo_ch);
        }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int t = 0; t < TQ; ++t) raw[j][t] = bits_or(raw[j][t], vt[j][t]);
    } else {
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int t = 0; t < TQ; ++t) {
          const uint32_t gg = g[j][t];
          const TX* src = gg == kPad ? reinterpret_cast<const TX*>(kZeroRow) : ((gg >> 30) == 3 ? tree : x);
          raw[j][t] = src[size_t(gg == kPad ? 0u : (gg & kIdxMask)) * 16 + r16];
        }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const float aj = p0 + 4 * j + kg < u_e ? a[j] : 0.f;
#pragma unroll
      for (int t = 0; t < TQ; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(aj, to_f32<TX>(raw[j][t]), acc[t], 0, 0, 0);
    }
  }
  double* out = partial + size_t(blockIdx.x) * NOUT;
#pragma unroll
  for (int t = 0; t < TQ; ++t) {
    if (t >= nq) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) out[((4 * kg + i) * 16 + r16) * K3 + q0 + t] = double(acc[t][i]);
  }
}

template <int K, int CI, int CO, typename TX>
static apr_status bwd_weight_impl(const apr_handle* h, const apr_conv_desc* d, const void* x, const void* tree,
                                  const float* dy, float* dw, double* ws, hipStream_t s) {
  const Meta& m = h->meta;
  constexpr int NOUT = CO * CI * K * K * K;
  constexpr bool kMfma = K == 3 && CI == 16 && CO == 16;
  int64_t blk = 0;
  for (int l = m.l_min; l <= m.l_max; ++l) {
    const int nb = level_blocks(h, l);
    if (!nb) continue;
    const int64_t b = level_first(h, l);
    if constexpr (kMfma) {
      // 32-bit buffer offsets when x and the tree stay below kBufOob bytes:
      // one buffer over both when they lie close enough, else one each
      const uint64_t xb = uint64_t(h->n_p) * 16 * sizeof(TX), tb = uint64_t(h->n_t) * 16 * sizeof(TX);
      const int forced = wide_offsets_mode();
      const uintptr_t xa = reinterpret_cast<uintptr_t>(x), ta = reinterpret_cast<uintptr_t>(tree);
      const uintptr_t lo = (h->n_t && ta < xa) ? ta : xa;
      const uintptr_t hi = std::max<uintptr_t>(xa + xb, h->n_t ? ta + tb : 0);
      int mode = xb <= kBufOob && tb <= kBufOob && forced != 1 ? 1 : 0;
      if (mode == 1 && forced == 0 && hi - lo <= kBufOob) mode = 2;
      const TX* xp = static_cast<const TX*>(x);
      const TX* tp = static_cast<const TX*>(h->n_t ? tree : nullptr);
      uint32_t xbytes = uint32_t(mode ? xb : 0), tbytes = uint32_t(mode ? tb : 0), xoff = 0, toff = 0;
      if (mode == 2) {
        xp = reinterpret_cast<const TX*>(lo);
        xbytes = uint32_t(hi - lo);
        xoff = uint32_t(xa - lo);
        toff = h->n_t ? uint32_t(ta - lo) : 0u;
      }
      auto kern = mode == 2   ? bwd_weight_mfma16_kernel<TX, 2>
                  : mode == 1 ? bwd_weight_mfma16_kernel<TX, 1>
                              : bwd_weight_mfma16_kernel<TX, 0>;
      hipLaunchKernelGGL(kern, dim3(nb), dim3(256), 0, s, b, b + h->per_level_p[l],
                         reinterpret_cast<const uint32_t*>(gather_map(h, K)), h->n_p, xp, tp, xbytes, tbytes, xoff,
                         toff, dy, ws + size_t(blk) * NOUT);
    } else
      hipLaunchKernelGGL((bwd_weight_partial_kernel<K, CI, CO, TX>), dim3(nb), dim3(kWgtThreads), 0, s, b,
                         b + h->per_level_p[l], gather_map(h, K), h->n_p, static_cast<const TX*>(x),
                         static_cast<const TX*>(tree), dy, ws + size_t(blk) * NOUT);
    blk += nb;
  }
  const unsigned rg = unsigned((NOUT + 255) / 256);
  auto reduce = [&](int64_t bb, int64_t be, float* out) {
    const unsigned nc = unsigned((be - bb + kRedChunk - 1) / kRedChunk);
    if (nc > 0)
      hipLaunchKernelGGL(bwd_weight_chunk_kernel, dim3(rg, nc), dim3(256), 0, s, ws, bb, be, NOUT);
    hipLaunchKernelGGL(bwd_weight_reduce_kernel, dim3(rg), dim3(256), 0, s, ws, bb, be, NOUT, out);
  };
  if (d->n_wlevels == 1) {
    reduce(0, blk, dw);
  } else {
    int64_t bb = 0;
    for (int l = m.l_min; l <= m.l_max; ++l) {
      const int nb = level_blocks(h, l);
      reduce(bb, bb + nb, dw + size_t(l - m.l_min) * NOUT);
      bb += nb;
    }
  }
  APR_HIP(hipGetLastError());
  return APR_OK;
}

static apr_status check_desc(const apr_handle* h, const apr_conv_desc* d, const char* who) {
  if (!h || !d) APR_FAIL(APR_EINVAL, std::string(who) + ": null handle or descriptor");
  if (d->k != 3 && d->k != 5) APR_FAIL(APR_EUNSUPPORTED, std::string(who) + ": k must be 3 or 5");
  const int nl = h->meta.l_max - h->meta.l_min + 1;
  if (d->n_wlevels != 1 && d->n_wlevels != nl)
    APR_FAIL(APR_EINVAL, std::string(who) + ": n_wlevels must be 1 or l_max - l_min + 1");
  if (!gather_map(h, d->k))
    APR_FAIL(APR_EINVAL, std::string(who) + ": build the access with APR_BUILD_GATHER3 / APR_BUILD_GATHER5");
  return APR_OK;
}

}  // namespace apr

using namespace apr;

extern "C" apr_status apr_conv_bwd_data(const apr_handle* h, const apr_conv_desc* d, const float* dy,
                                        const float* w, float* dx, float* dtree, void* stream) {
  apr_status st = check_desc(h, d, "apr_conv_bwd_data");
  if (st != APR_OK) return st;
  if (h->n_p == 0) return APR_OK;
  if (!dy || !w || !dx || (h->n_t && !dtree)) APR_FAIL(APR_EINVAL, "apr_conv_bwd_data: null buffer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int cin = d->c_in, cout = d->c_out;
  if (d->k == 3) {
    APR_CH_DISPATCH(1, 1, return bwd_data_impl<3, CI, CO>(h, d, dy, w, dx, dtree, s))
    APR_CH_DISPATCH(1, 16, return bwd_data_impl<3, CI, CO>(h, d, dy, w, dx, dtree, s))
    APR_CH_DISPATCH(16, 16, return bwd_data_impl<3, CI, CO>(h, d, dy, w, dx, dtree, s))
    APR_CH_DISPATCH(16, 1, return bwd_data_impl<3, CI, CO>(h, d, dy, w, dx, dtree, s))
    APR_CH_DISPATCH(2, 3, return bwd_data_impl<3, CI, CO>(h, d, dy, w, dx, dtree, s))
  } else {
    APR_CH_DISPATCH(1, 1, return bwd_data_impl<5, CI, CO>(h, d, dy, w, dx, dtree, s))
    APR_CH_DISPATCH(2, 3, return bwd_data_impl<5, CI, CO>(h, d, dy, w, dx, dtree, s))
  }
  APR_FAIL(APR_EUNSUPPORTED, "apr_conv_bwd_data: unsupported (k, c_in, c_out)");
}

extern "C" size_t apr_conv_bwd_weight_ws(const apr_handle* h, const apr_conv_desc* d) {
  if (!h || !d || (d->k != 3 && d->k != 5) || d->c_in < 1 || d->c_out < 1) return 0;
  int64_t nb = 0;
  for (int l = h->meta.l_min; l <= h->meta.l_max; ++l) nb += level_blocks(h, l);
  return size_t(nb) * size_t(d->c_in) * size_t(d->c_out) * size_t(d->k * d->k * d->k) * sizeof(double);
}

extern "C" apr_status apr_conv_bwd_weight(const apr_handle* h, const apr_conv_desc* d, const void* x,
                                          const void* tree, const float* dy, float* dw, void* ws,
                                          size_t ws_bytes, void* stream) {
  apr_status st = check_desc(h, d, "apr_conv_bwd_weight");
  if (st != APR_OK) return st;
  if (ws_bytes < apr_conv_bwd_weight_ws(h, d)) APR_FAIL(APR_EINVAL, "apr_conv_bwd_weight: workspace too small");
  if (!x || !dy || !dw || (h->n_t && !tree) || (apr_conv_bwd_weight_ws(h, d) && !ws))
    APR_FAIL(APR_EINVAL, "apr_conv_bwd_weight: null buffer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int cin = d->c_in, cout = d->c_out;
  double* w64 = static_cast<double*>(ws);
  if (h->n_p == 0) {
    const size_t n = size_t(d->n_wlevels) * cin * cout * d->k * d->k * d->k;
    APR_HIP(hipMemsetAsync(dw, 0, n * sizeof(float), s));
    return APR_OK;
  }
#define APR_WGT(KK, XT)                                                                    \
  APR_CH_DISPATCH(1, 1, return (bwd_weight_impl<KK, CI, CO, XT>(h, d, x, tree, dy, dw, w64, s))) \
  APR_CH_DISPATCH(1, 16, return (bwd_weight_impl<KK, CI, CO, XT>(h, d, x, tree, dy, dw, w64, s))) \
  APR_CH_DISPATCH(16, 16, return (bwd_weight_impl<KK, CI, CO, XT>(h, d, x, tree, dy, dw, w64, s))) \
  APR_CH_DISPATCH(16, 1, return (bwd_weight_impl<KK, CI, CO, XT>(h, d, x, tree, dy, dw, w64, s))) \
  APR_CH_DISPATCH(2, 3, return (bwd_weight_impl<KK, CI, CO, XT>(h, d, x, tree, dy, dw, w64, s)))
  if (d->k == 3 && d->x_dtype == APR_F32) { APR_WGT(3, float) }
  if (d->k == 3 && d->x_dtype == APR_BF16) { APR_WGT(3, __hip_bfloat16) }
  if (d->k == 5 && d->x_dtype == APR_F32) {
    APR_CH_DISPATCH(1, 1, return (bwd_weight_impl<5, CI, CO, float>(h, d, x, tree, dy, dw, w64, s)))
    APR_CH_DISPATCH(2, 3, return (bwd_weight_impl<5, CI, CO, float>(h, d, x, tree, dy, dw, w64, s)))
  }
#undef APR_WGT
  APR_FAIL(APR_EUNSUPPORTED, "apr_conv_bwd_weight: unsupported (k, c_in, c_out, dtype)");
}
