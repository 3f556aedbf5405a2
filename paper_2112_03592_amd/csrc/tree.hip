// Tree values (Section 3.4): every interior node takes the mean of its
// children, level by level from the finest.  One wave per tree row; the row
// is swept along y in windows of 64 parent cells.  Children of the window
// (particles and tree nodes of the four child rows, 128 child cells each) are
// scattered into an LDS slot array, then each lane sums the children of one
// parent in a fixed order (deterministic, no atomics).
//
// Many channels: the same kernel run once in index mode writes every node's
// child list (child map, [8][N_t], fixed child order); the fill of all
// channels is then a gather over that map, one lane per node, with the same
// summation order as the one-channel kernel.
#include "common.hpp"

namespace apr {

constexpr int kFillWaves = 4;
constexpr int kWin = 64;   // parent cells per window

constexpr uint32_t kChildPad = 0xffffffffu;   // child-map entry of a child cell outside the image

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

// Mean of the children of every tree node of one level over CH channels,
// one lane per node, children in child-map order (the order of the
// one-channel kernel: bit-identical results).
template <typename T, int CH>
__global__ __launch_bounds__(256) void fill_mc_kernel(const uint32_t* __restrict__ cmap, int64_t n_t,
                                                      uint32_t t_begin, uint32_t t_end, const T* __restrict__ x,
                                                      T* __restrict__ tree) {
  const uint32_t i = t_begin + blockIdx.x * 256u + threadIdx.x;
  if (i >= t_end) return;
  float s[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) s[c] = 0.f;
  int n = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const uint32_t code = cmap[size_t(j) * n_t + i];
    if (code == kChildPad) continue;
    const T* src = ((code >> 31) ? tree : x) + size_t(code & 0x7fffffffu) * CH;
    float v[CH];
    load_vec<T, CH>(src, v);
#pragma unroll
    for (int c = 0; c < CH; ++c) s[c] += v[c];
    ++n;
  }
  T out[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) out[c] = from_f32<T>(s[c] / float(n));
  store_vec<T, CH>(tree + size_t(i) * CH, out);
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
static apr_status fill_mc(const apr_handle* h, const T* x, T* tree, hipStream_t s) {
  const Meta& m = h->meta;
  uint32_t lvl_begin[kMaxL + 1];
  uint32_t acc = 0;
  for (int L = m.t_lo; L <= m.t_hi; ++L) {
    lvl_begin[L] = acc;
    acc += uint32_t(h->per_level_t[L]);
  }
  for (int L = m.t_hi; L >= m.t_lo; --L) {
    const uint32_t b = lvl_begin[L], e = b + uint32_t(h->per_level_t[L]);
    if (b == e) continue;
    hipLaunchKernelGGL((fill_mc_kernel<T, CH>), dim3((e - b + 255) / 256), dim3(256), 0, s, h->cmap, h->n_t, b, e,
                       x, tree);
    APR_HIP(hipGetLastError());
  }
  return APR_OK;
}
}  // namespace apr

extern "C" apr_status apr_fill_tree(const apr_handle* h, const void* x, void* tree,
                                    int32_t channels, int32_t dtype, void* stream) {
  if (!h) APR_FAIL(APR_EINVAL, "apr_fill_tree: null handle");
  if (channels < 1 || channels > 65535) APR_FAIL(APR_EINVAL, "apr_fill_tree: channels must be in [1, 65535]");
  if (dtype != APR_F32 && dtype != APR_BF16) APR_FAIL(APR_EUNSUPPORTED, "apr_fill_tree: dtype");
  if (h->n_t == 0) return APR_OK;
  if (!x || !tree) APR_FAIL(APR_EINVAL, "apr_fill_tree: null x or tree");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (channels == 16 && h->cmap && ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(tree)) & 15) == 0) {
    if (dtype == APR_F32)
      return fill_mc<float, 16>(h, static_cast<const float*>(x), static_cast<float*>(tree), s);
    return fill_mc<__hip_bfloat16, 16>(h, static_cast<const __hip_bfloat16*>(x), static_cast<__hip_bfloat16*>(tree),
                                       s);
  }
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
