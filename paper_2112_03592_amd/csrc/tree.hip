// Tree values (Section 3.4): every interior node takes the mean of its
// children, level by level from the finest.  One wave per tree row; the row
// is swept along y in windows of 64 parent cells.  Children of the window
// (particles and tree nodes of the four child rows, 128 child cells each) are
// scattered into an LDS slot array, then each lane sums the children of one
// parent in a fixed order (deterministic, no atomics).
//
// The same kernel run once in index mode (at access build) writes every
// node's child list (child map, [8][N_t], fixed child order); fills are then
// gathers over that map, one lane per node, with the same summation order as
// the row-window kernel (which remains the path of handles without a child
// map).  The coarse levels, which hold few nodes, are filled by one
// workgroup in a single launch.
#include "common.hpp"
#include "fp8.hpp"

namespace apr {

constexpr int kFillWaves = 4;
constexpr int kWin = 64;   // parent cells per window

// INDEX: write child codes ((1 << 31 if tree node) | index) to cmap [8][n_t]
// instead of the means
template <typename T, bool INDEX>
__global__ __launch_bounds__(64 * kFillWaves) void fill_level_kernel(
    Meta m, int L, const uint16_t* __restrict__ py, const uint32_t* __restrict__ pend,
    const uint16_t* __restrict__ ty, const uint32_t* __restrict__ tend, const T* __restrict__ x,
    T* __restrict__ tree, int ch_stride, uint32_t* __restrict__ cmap, int64_t n_t) {
  __shared__ float slot[kFillWaves][4][2 * kWin];
  const int wave = threadIdx.x / 64;
  const uint32_t lane = lane_id();
  const int64_t nrows = int64_t(m.dz[L]) * m.dx[L];
  const int64_t row = int64_t(blockIdx.x) * kFillWaves + wave;
  if (row >= nrows) return;
  if constexpr (!INDEX) {
    x += blockIdx.y;      // channel handled by this block
    tree += blockIdx.y;
  }
  uint32_t pb, pe;
  row_range(tend, m.trow[L] + uint32_t(row), pb, pe);
  if (pb == pe) return;
  const int z = int(row / m.dx[L]);
  const int xr = int(row % m.dx[L]);
  const int C = L + 1;
  const bool has_p = (C >= m.l_min && C <= m.l_max);
  const bool has_t = (C <= m.t_hi);
  // child lists: j = 2*(2a+b) + src, src 0 = particle row, 1 = tree row
  uint32_t cp[8], ce[8];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int j = 2 * (2 * a + b);
      const int cz = 2 * z + a, cx = 2 * xr + b;
      cp[j] = ce[j] = cp[j + 1] = ce[j + 1] = 0;
      if (cz >= m.dz[C] || cx >= m.dx[C]) continue;
      if (has_p) row_range(pend, m.prow[C] + uint32_t(cz) * m.dx[C] + cx, cp[j], ce[j]);
      if (has_t) row_range(tend, m.trow[C] + uint32_t(cz) * m.dx[C] + cx, cp[j + 1], ce[j + 1]);
    }
  const int nza = (2 * z + 1 < m.dz[C]) ? 2 : 1;
  const int nxb = (2 * xr + 1 < m.dx[C]) ? 2 : 1;
  const int dyc = m.dy[C];
  float* sl = &slot[wave][0][0];
  uint32_t pp = pb;
  while (pp < pe) {
    const uint32_t i = pp + lane;
    const bool valid = i < pe;
    const int yt = valid ? int(ty[i]) : 0x7fffffff;
    const int y0 = __shfl(yt, 0, 64);
    const bool inwin = valid && yt < y0 + kWin;
    const uint32_t npar = __popcll(ballot(inwin));
    const int cy_end = 2 * (y0 + kWin);
    for (int j = 0; j < 8; ++j) {
      if (cp[j] >= ce[j]) continue;
      const uint16_t* ys = (j & 1) ? ty : py;
      const T* vs = (j & 1) ? tree : x;
      float* dst = sl + (j >> 1) * (2 * kWin);
      uint32_t base = cp[j];
      while (true) {
        const uint32_t k = base + lane;
        const bool v = k < ce[j];
        const int cyv = v ? int(ys[k]) : 0x7fffffff;
        const bool in = v && cyv < cy_end;   // every earlier child belongs to an earlier window
        if (in && cyv >= 2 * y0) {
          if constexpr (INDEX)
            dst[cyv - 2 * y0] = __uint_as_float(((j & 1) ? 0x80000000u : 0u) | k);
          else
            dst[cyv - 2 * y0] = to_f32<T>(vs[size_t(k) * ch_stride]);
        }
        const uint32_t cnt = __popcll(ballot(in));
        if (cnt == 64 && base + 64 < ce[j]) {
          base += 64;
          continue;
        }
        cp[j] = base + cnt;
        break;
      }
    }
    wave_lds_sync();
    if (inwin) {
      const int c0 = 2 * yt;
      const int nc = (c0 + 1 < dyc) ? 2 : 1;
      if constexpr (INDEX) {
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) {
              const bool in = a < nza && b < nxb && c < nc;
              cmap[size_t(4 * a + 2 * b + c) * n_t + i] =
                  in ? __float_as_uint(sl[(2 * a + b) * (2 * kWin) + (c0 + c - 2 * y0)]) : kChildPad;
            }
      } else {
        float s = 0.f;
        int n = 0;
        for (int a = 0; a < nza; ++a)
          for (int b = 0; b < nxb; ++b)
            for (int c = 0; c < nc; ++c) {
              s += sl[(2 * a + b) * (2 * kWin) + (c0 + c - 2 * y0)];
              ++n;
            }
        tree[size_t(i) * ch_stride] = from_f32<T>(s / float(n));
      }
    }
    wave_lds_sync();
    pp += npar;
  }
}

// Mean of the children of tree node i over the channels (CH > 0: CH
// channels, vector row access; CH == 0: C channels, scalar loop), children
// in child-map order -- the order of the one-channel kernel, so results are
// bit-identical to it.
template <typename T, int CH>
__device__ inline void fill_node(const uint32_t* __restrict__ cmap, int64_t n_t, uint32_t i,
                                 const T* __restrict__ x, T* __restrict__ tree, int C) {
  uint32_t code[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) code[j] = cmap[size_t(j) * n_t + i];
  if constexpr (CH > 0) {
    float s[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) s[c] = 0.f;
    int n = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (code[j] == kChildPad) continue;
      float v[CH];
      load_vec<T, CH>(((code[j] >> 31) ? tree : x) + size_t(code[j] & 0x7fffffffu) * CH, v);
#pragma unroll
      for (int c = 0; c < CH; ++c) s[c] += v[c];
      ++n;
    }
    T out[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) out[c] = from_f32<T>(s[c] / float(n));
    store_vec<T, CH>(tree + size_t(i) * CH, out);
  } else {
    for (int c = 0; c < C; ++c) {
      float s = 0.f;
      int n = 0;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (code[j] == kChildPad) continue;
        s += to_f32<T>((((code[j] >> 31) ? tree : x) + size_t(code[j] & 0x7fffffffu) * C)[c]);
        ++n;
      }
      tree[size_t(i) * C + c] = from_f32<T>(s / float(n));
    }
  }
}

constexpr int kFillFlat = 256;
constexpr int kFillSmallThreads = 1024;
constexpr int64_t kFillSmall = 1024;    // coarse levels up to this many nodes in all go to one workgroup

// one tree level, one lane per node
template <typename T, int CH>
__global__ __launch_bounds__(kFillFlat) void fill_flat_kernel(const uint32_t* __restrict__ cmap, int64_t n_t,
                                                              uint32_t t_begin, uint32_t t_end,
                                                              const T* __restrict__ x, T* __restrict__ tree, int C) {
  const uint32_t i = t_begin + blockIdx.x * uint32_t(kFillFlat) + threadIdx.x;
  if (i < t_end) fill_node<T, CH>(cmap, n_t, i, x, tree, C);
}

struct LevelSpans {
  uint32_t begin[kMaxL + 1];   // first tree node of level L (nodes of L: [begin[L], begin[L + 1]))
};

// the coarse levels [L_lo, L_hi], finest first, by one workgroup (a barrier
// between levels orders each level after its children)
template <typename T, int CH>
__global__ __launch_bounds__(kFillSmallThreads) void fill_small_kernel(const uint32_t* __restrict__ cmap, int64_t n_t,
                                                                        LevelSpans sp, int L_lo, int L_hi,
                                                                        const T* __restrict__ x,
                                                                        T* __restrict__ tree, int C) {
  for (int L = L_hi; L >= L_lo; --L) {
    for (uint32_t i = sp.begin[L] + threadIdx.x; i < sp.begin[L + 1]; i += kFillSmallThreads)
      fill_node<T, CH>(cmap, n_t, i, x, tree, C);
    __syncthreads();
  }
}

}  // namespace apr

using namespace apr;

namespace apr {
apr_status build_child_map(const apr_handle* h, uint32_t* cmap, hipStream_t s) {
  const Meta& m = h->meta;
  for (int L = m.t_hi; L >= m.t_lo; --L) {
    const int64_t rows = int64_t(m.dz[L]) * m.dx[L];
    const unsigned grid = unsigned((rows + kFillWaves - 1) / kFillWaves);
    hipLaunchKernelGGL((fill_level_kernel<float, true>), dim3(grid), dim3(64 * kFillWaves), 0, s, m, L, h->py,
                       h->pend, h->ty, h->tend, nullptr, nullptr, 1, cmap, h->n_t);
    APR_HIP(hipGetLastError());
  }
  return APR_OK;
}

template <typename T, int CH>
static apr_status fill_by_child_map(const apr_handle* h, const T* x, T* tree, int C, hipStream_t s) {
  const Meta& m = h->meta;
  LevelSpans sp{};
  uint32_t acc = 0;
  for (int L = m.t_lo; L <= m.t_hi; ++L) {
    sp.begin[L] = acc;
    acc += uint32_t(h->per_level_t[L]);
  }
  sp.begin[m.t_hi + 1] = acc;
  // coarse levels whose nodes together fit one workgroup's sweep
  int L_small = m.t_lo - 1;
  int64_t small = 0;
  while (L_small + 1 <= m.t_hi && small + h->per_level_t[L_small + 1] <= kFillSmall) {
    ++L_small;
    small += h->per_level_t[L_small];
  }
  for (int L = m.t_hi; L > L_small; --L) {
    const uint32_t b = sp.begin[L], e = sp.begin[L + 1];
    if (b == e) continue;
    hipLaunchKernelGGL((fill_flat_kernel<T, CH>), dim3((e - b + kFillFlat - 1) / kFillFlat), dim3(kFillFlat), 0, s,
                       h->cmap, h->n_t, b, e, x, tree, C);
  }
  if (L_small >= m.t_lo && small > 0)
    hipLaunchKernelGGL((fill_small_kernel<T, CH>), dim3(1), dim3(kFillSmallThreads), 0, s, h->cmap, h->n_t, sp,
                       m.t_lo, L_small, x, tree, C);
  APR_HIP(hipGetLastError());
  return APR_OK;
}

template <typename T>
static apr_status fill_dispatch(const apr_handle* h, const void* xv, void* tv, int C, hipStream_t s) {
  const T* x = static_cast<const T*>(xv);
  T* tree = static_cast<T*>(tv);
  const bool aligned16 = ((reinterpret_cast<uintptr_t>(xv) | reinterpret_cast<uintptr_t>(tv)) & 15) == 0;
  if (C == 1) return fill_by_child_map<T, 1>(h, x, tree, 1, s);
  if (C == 16 && aligned16) return fill_by_child_map<T, 16>(h, x, tree, 16, s);
  return fill_by_child_map<T, 0>(h, x, tree, C, s);
}
}  // namespace apr

extern "C" apr_status apr_fill_tree(const apr_handle* h, const void* x, void* tree,
                                    int32_t channels, int32_t dtype, void* stream) {
  if (!h) APR_FAIL(APR_EINVAL, "apr_fill_tree: null handle");
  if (channels < 1 || channels > 65535) APR_FAIL(APR_EINVAL, "apr_fill_tree: channels must be in [1, 65535]");
  if (dtype != APR_F32 && dtype != APR_BF16 && dtype != APR_FP8) APR_FAIL(APR_EUNSUPPORTED, "apr_fill_tree: dtype");
  if (dtype == APR_FP8 && (channels != 16 || !h->cmap))
    APR_FAIL(APR_EUNSUPPORTED, "apr_fill_tree: FP8 storage needs 16 channels (and the child map)");
  if (h->n_t == 0) return APR_OK;
  if (!x || !tree) APR_FAIL(APR_EINVAL, "apr_fill_tree: null x or tree");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == APR_FP8) {
    if (((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(tree)) & 15) != 0)
      APR_FAIL(APR_EINVAL, "apr_fill_tree: FP8 rows must be 16-byte aligned");
    return fill_by_child_map<fp8e4m3, 16>(h, static_cast<const fp8e4m3*>(x), static_cast<fp8e4m3*>(tree), 16, s);
  }
  if (h->cmap)
    return dtype == APR_F32 ? fill_dispatch<float>(h, x, tree, channels, s)
                            : fill_dispatch<__hip_bfloat16>(h, x, tree, channels, s);
  // without a child map (more than 2^31 - 1 particles): the row-window kernel
  const Meta& m = h->meta;
  for (int L = m.t_hi; L >= m.t_lo; --L) {
    const int64_t rows = int64_t(m.dz[L]) * m.dx[L];
    const unsigned grid = unsigned((rows + kFillWaves - 1) / kFillWaves);
    const dim3 g(grid, unsigned(channels));
    if (dtype == APR_F32) {
      hipLaunchKernelGGL((fill_level_kernel<float, false>), g, dim3(64 * kFillWaves), 0, s, m, L, h->py,
                         h->pend, h->ty, h->tend, static_cast<const float*>(x),
                         static_cast<float*>(tree), channels, nullptr, h->n_t);
    } else {
      hipLaunchKernelGGL((fill_level_kernel<__hip_bfloat16, false>), g, dim3(64 * kFillWaves), 0, s, m, L,
                         h->py, h->pend, h->ty, h->tend, static_cast<const __hip_bfloat16*>(x),
                         static_cast<__hip_bfloat16*>(tree), channels, nullptr, h->n_t);
    }
    APR_HIP(hipGetLastError());
  }
  return APR_OK;
}
