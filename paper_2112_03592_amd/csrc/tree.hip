// Tree values (Section 3.4): every interior node takes the mean of its
// children, level by level from the finest.  One wave per tree row; the row
// is swept along y in windows of 64 parent cells.  Children of the window
// (particles and tree nodes of the four child rows, 128 child cells each) are
// scattered into an LDS slot array, then each lane sums the children of one
// parent in a fixed order (deterministic, no atomics).
#include "common.hpp"

namespace apr {

constexpr int kFillWaves = 4;
constexpr int kWin = 64;   // parent cells per window

template <typename T>
__global__ __launch_bounds__(64 * kFillWaves) void fill_level_kernel(
    Meta m, int L, const uint16_t* __restrict__ py, const uint32_t* __restrict__ pend,
    const uint16_t* __restrict__ ty, const uint32_t* __restrict__ tend, const T* __restrict__ x,
    T* __restrict__ tree, int ch_stride) {
  __shared__ float slot[kFillWaves][4][2 * kWin];
  const int wave = threadIdx.x / 64;
  const uint32_t lane = lane_id();
  const int64_t nrows = int64_t(m.dz[L]) * m.dx[L];
  const int64_t row = int64_t(blockIdx.x) * kFillWaves + wave;
  if (row >= nrows) return;
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
        if (in && cyv >= 2 * y0) dst[cyv - 2 * y0] = to_f32<T>(vs[size_t(k) * ch_stride]);
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
      float s = 0.f;
      int n = 0;
      const int c0 = 2 * yt;
      const int nc = (c0 + 1 < dyc) ? 2 : 1;
      for (int a = 0; a < nza; ++a)
        for (int b = 0; b < nxb; ++b)
          for (int c = 0; c < nc; ++c) {
            s += sl[(2 * a + b) * (2 * kWin) + (c0 + c - 2 * y0)];
            ++n;
          }
      tree[size_t(i) * ch_stride] = from_f32<T>(s / float(n));
    }
    wave_lds_sync();
    pp += npar;
  }
}

}  // namespace apr

using namespace apr;

extern "C" apr_status apr_fill_tree(const apr_handle* h, const void* x, void* tree,
                                    int32_t channels, int32_t dtype, void* stream) {
  if (!h) APR_FAIL(APR_EINVAL, "apr_fill_tree: null handle");
  if (channels < 1) APR_FAIL(APR_EINVAL, "apr_fill_tree: channels must be >= 1");
  if (dtype != APR_F32 && dtype != APR_BF16) APR_FAIL(APR_EUNSUPPORTED, "apr_fill_tree: dtype");
  if (h->n_t == 0) return APR_OK;
  if (!x || !tree) APR_FAIL(APR_EINVAL, "apr_fill_tree: null x or tree");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Meta& m = h->meta;
  for (int L = m.t_hi; L >= m.t_lo; --L) {
    const int64_t rows = int64_t(m.dz[L]) * m.dx[L];
    const unsigned grid = unsigned((rows + kFillWaves - 1) / kFillWaves);
    for (int c = 0; c < channels; ++c) {
      if (dtype == APR_F32) {
        hipLaunchKernelGGL(fill_level_kernel<float>, dim3(grid), dim3(64 * kFillWaves), 0, s, m, L,
                           h->py, h->pend, h->ty, h->tend, static_cast<const float*>(x) + c,
                           static_cast<float*>(tree) + c, channels);
      } else {
        hipLaunchKernelGGL(fill_level_kernel<__hip_bfloat16>, dim3(grid), dim3(64 * kFillWaves), 0,
                           s, m, L, h->py, h->pend, h->ty, h->tend,
                           static_cast<const __hip_bfloat16*>(x) + c,
                           static_cast<__hip_bfloat16*>(tree) + c, channels);
      }
    }
    APR_HIP(hipGetLastError());
  }
  return APR_OK;
}
