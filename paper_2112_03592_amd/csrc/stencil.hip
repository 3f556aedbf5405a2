// Per-level stencils on the host in FP64 (Section 4.2, Eq. restrict_stenc;
// Section 4.3, Eq. adapt_grad).
//
// Restriction: with R_l the s^3 block average and P_l the piecewise-constant
// prolongation (s = 2^(l_max - l)), K_{w_l} = R_l K_w P_l is again a stencil.
// Both operators factor over the three axes, so w_l = (M x M x M) w with the
// 1-D matrix  M[J][t] = (1/s) * #{a in [0, s) : floor((a + t) / s) = J},
// J, t in [-r, r]; it is applied axis by axis.
#include <cmath>
#include <vector>

#include "common.hpp"

using namespace apr;

static void restrict_matrix(int k, int64_t s, std::vector<double>& M) {
  const int r = k / 2;
  M.assign(size_t(k) * k, 0.0);
  for (int t = -r; t <= r; ++t)
    for (int64_t a = 0; a < s; ++a) {
      const int64_t q = a + t;
      const int64_t J = (q >= 0) ? q / s : -((-q + s - 1) / s);   // floor division
      if (J < -r || J > r) continue;
      M[size_t(J + r) * k + (t + r)] += 1.0 / double(s);
    }
}

// out[j0][j1][j2] = sum_t M[j_axis][t] in[...t on `axis`...]
static void apply_axis(int k, const std::vector<double>& M, int axis, const double* in, double* out) {
  for (int i0 = 0; i0 < k; ++i0)
    for (int i1 = 0; i1 < k; ++i1)
      for (int i2 = 0; i2 < k; ++i2) {
        double acc = 0.0;
        for (int t = 0; t < k; ++t) {
          const int a0 = axis == 0 ? t : i0, a1 = axis == 1 ? t : i1, a2 = axis == 2 ? t : i2;
          const int j = axis == 0 ? i0 : (axis == 1 ? i1 : i2);
          acc += M[size_t(j) * k + t] * in[(a0 * k + a1) * k + a2];
        }
        out[(i0 * k + i1) * k + i2] = acc;
      }
}

extern "C" apr_status apr_stencil_levels(int32_t mode, int32_t k, int32_t n_filters, const double* w,
                                         int32_t l_min, int32_t l_max, int32_t flip, float* out) {
  if (k < 3 || k > 13 || k % 2 == 0) APR_FAIL(APR_EUNSUPPORTED, "apr_stencil_levels: k must be odd, 3 to 13");
  if (n_filters < 1 || !w || !out) APR_FAIL(APR_EINVAL, "apr_stencil_levels: bad arguments");
  if (l_min < 0 || l_max < l_min || l_max >= kMaxL)
    APR_FAIL(APR_EINVAL, "apr_stencil_levels: bad level range");
  if (mode < APR_STENCIL_SAME || mode > APR_STENCIL_ADAPTIVE)
    APR_FAIL(APR_EINVAL, "apr_stencil_levels: unknown mode");
  const int k3 = k * k * k;
  std::vector<double> src(k3), a(k3), b(k3), M;
  for (int l = l_min; l <= l_max; ++l) {
    const int64_t s = int64_t(1) << (l_max - l);
    if (mode == APR_STENCIL_RESTRICT) restrict_matrix(k, s, M);
    for (int f = 0; f < n_filters; ++f) {
      const double* wf = w + size_t(f) * k3;
      for (int i = 0; i < k3; ++i) src[i] = flip ? wf[k3 - 1 - i] : wf[i];
      const double* res = src.data();
      if (mode == APR_STENCIL_RESTRICT && s > 1) {
        apply_axis(k, M, 0, src.data(), a.data());
        apply_axis(k, M, 1, a.data(), b.data());
        apply_axis(k, M, 2, b.data(), a.data());
        res = a.data();
      }
      const double scale = (mode == APR_STENCIL_ADAPTIVE) ? std::ldexp(1.0, -(l_max - l)) : 1.0;
      float* o = out + (size_t(l - l_min) * n_filters + f) * k3;
      for (int i = 0; i < k3; ++i) o[i] = float(res[i] * scale);
    }
  }
  return APR_OK;
}
