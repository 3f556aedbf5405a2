// Elementwise and reduction helpers of the APR surrogate network: input
// statistics, normalisation, ReLU / bias gradient, relative L2 loss and its
// gradient, and the Adam update.  Reductions use a fixed grid of kRedBlocks
// blocks and FP64 partials summed in a fixed order: results are
// deterministic.
#include <cmath>

#include "common.hpp"

namespace apr {

constexpr int kRedBlocks = 256;
constexpr int kRedThreads = 256;

// sum of f(i) over i < n, FP64, block-level tree reduction -> part[blockIdx]
template <typename F>
__device__ inline void block_sum(int64_t n, F f, double* part) {
  __shared__ double red[kRedThreads];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < n; i += int64_t(gridDim.x) * kRedThreads)
    s += f(i);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = kRedThreads / 2; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__device__ inline double log_clamped(float v) { return log(fmax(double(v), 1.0)); }

// op 0: statistics of u; op 1: of log(max(u, 1))
__global__ __launch_bounds__(kRedThreads) void sum_sq_kernel(int op, const float* __restrict__ u, int64_t n,
                                                              double* __restrict__ part) {
  auto val = [&](int64_t i) { return op ? log_clamped(u[i]) : double(u[i]); };
  block_sum(n, [&](int64_t i) { return val(i); }, part);
  block_sum(n, [&](int64_t i) { const double v = val(i); return v * v; }, part + kRedBlocks);
}

// stats = {mean, std} from the partial sums (one thread, fixed order); a
// zero spread gives std 1 so that later divisions stay finite
__global__ void moments_finish_kernel(const double* __restrict__ part, int64_t n, double* __restrict__ stats) {
  double s = 0.0, q = 0.0;
  for (int b = 0; b < kRedBlocks; ++b) {
    s += part[b];
    q += part[kRedBlocks + b];
  }
  const double mean = n ? s / double(n) : 0.0;
  const double var = n ? fmax(q / double(n) - mean * mean, 0.0) : 0.0;
  stats[0] = mean;
  stats[1] = var > 0.0 ? sqrt(var) : 1.0;
}

// Elementwise maps between particle values and network space, FP64
// arithmetic; (mu, sd) = stats.  Linear residual (ops 0-3) and
// multiplicative residual (ops 4-7) parametrisations:
//   0: (a - mu) / sd            4: (log a+ - mu) / sd        (input)
//   1: (a - b) / sd             5: (log a+ - log b+) / sd    (target)
//   2: b + sd * a               6: b * exp(sd * a)           (output s)
//   3: sd * a                   7: sd * a * b                (ds/dnet * a, b = s)
// with a+ = max(a, 1).
__global__ void pointwise_kernel(int op, const float* __restrict__ a, const float* __restrict__ b, int64_t n,
                                 const double* __restrict__ stats, float* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double mu = stats[0], sd = stats[1];
  const double av = a[i];
  double r;
  switch (op) {
    case 0: r = (av - mu) / sd; break;
    case 1: r = (av - double(b[i])) / sd; break;
    case 2: r = double(b[i]) + sd * av; break;
    case 3: r = sd * av; break;
    case 4: r = (log_clamped(a[i]) - mu) / sd; break;
    case 5: r = (log_clamped(a[i]) - log_clamped(b[i])) / sd; break;
    case 6: r = double(b[i]) * exp(sd * av); break;
    default: r = sd * av * double(b[i]); break;
  }
  out[i] = float(r);
}

// Per-level weights from weight sets indexed by the distance to the finest
// level, d = l_max - l, with every level coarser than n_sets - 1 sharing the
// last set.  dir 0: out[l - l_min] = in[set(l)];  dir 1 (gradient):
// out[s] = sum over levels of set s, ascending l.
__global__ void level_weights_kernel(int dir, const float* __restrict__ in, float* __restrict__ out,
                                     int64_t per_set, int n_sets, int l_min, int l_max) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= per_set) return;
  auto set_of = [&](int l) { return min(l_max - l, n_sets - 1); };
  if (dir == 0) {
    for (int l = l_min; l <= l_max; ++l) out[size_t(l - l_min) * per_set + i] = in[size_t(set_of(l)) * per_set + i];
  } else {
    for (int s = 0; s < n_sets; ++s) {
      float acc = 0.f;
      for (int l = l_min; l <= l_max; ++l)
        if (set_of(l) == s) acc += in[size_t(l - l_min) * per_set + i];
      out[size_t(s) * per_set + i] = acc;
    }
  }
}

__global__ void relu_grad_kernel(const float* __restrict__ y, const float* __restrict__ dy, int64_t n,
                                 int relu, float* __restrict__ dy_pre) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  dy_pre[i] = (relu && !(y[i] > 0.f)) ? 0.f : dy[i];
}

// part[c * kRedBlocks + b] = block b's sum of g[p][c]
__global__ __launch_bounds__(kRedThreads) void col_sum_kernel(const float* __restrict__ g, int64_t rows, int c,
                                                              double* __restrict__ part) {
  for (int j = 0; j < c; ++j) {
    block_sum(rows, [&](int64_t p) { return double(g[size_t(p) * c + j]); }, part + size_t(j) * kRedBlocks);
    __syncthreads();
  }
}

__global__ void col_sum_finish_kernel(const double* __restrict__ part, int c, float* __restrict__ out) {
  const int j = threadIdx.x;
  if (j >= c) return;
  double s = 0.0;
  for (int b = 0; b < kRedBlocks; ++b) s += part[size_t(j) * kRedBlocks + b];
  out[j] = float(s);
}

__global__ __launch_bounds__(kRedThreads) void l2_parts_kernel(const float* __restrict__ a, const float* __restrict__ b,
                                                               int64_t n, double* __restrict__ part) {
  block_sum(n, [&](int64_t i) { const double d = double(a[i]) - double(b[i]); return d * d; }, part);
  block_sum(n, [&](int64_t i) { return double(b[i]) * double(b[i]); }, part + kRedBlocks);
}

// out[0] = |a-b|^2 / |b|^2, out[1] = |b|^2 (FP64)
__global__ void l2_finish_kernel(const double* __restrict__ part, double* __restrict__ out) {
  double d = 0.0, q = 0.0;
  for (int b = 0; b < kRedBlocks; ++b) {
    d += part[b];
    q += part[kRedBlocks + b];
  }
  out[0] = q > 0.0 ? d / q : d;
  out[1] = q;
}

__global__ void l2_grad_kernel(const float* __restrict__ a, const float* __restrict__ b, int64_t n,
                               const double* __restrict__ sums, float scale, float* __restrict__ grad) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double q = sums[1] > 0.0 ? sums[1] : 1.0;
  grad[i] = float(double(scale) * 2.0 * (double(a[i]) - double(b[i])) / q);
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static unsigned blocks_for(int64_t n) { return unsigned((n + 255) / 256); }

}  // namespace apr

using namespace apr;

extern "C" size_t apr_nn_workspace(int32_t channels) {
  return size_t(2 * kRedBlocks + 4) * sizeof(double) + size_t(channels < 1 ? 1 : channels) * kRedBlocks * sizeof(double);
}

extern "C" apr_status apr_moments(int32_t op, const float* u, int64_t n, double* stats, void* ws, void* stream) {
  if ((n > 0 && !u) || !stats || !ws || n < 0 || op < 0 || op > 1) APR_FAIL(APR_EINVAL, "apr_moments: bad argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* part = static_cast<double*>(ws);
  hipLaunchKernelGGL(sum_sq_kernel, dim3(kRedBlocks), dim3(kRedThreads), 0, s, op, u, n, part);
  hipLaunchKernelGGL(moments_finish_kernel, dim3(1), dim3(1), 0, s, part, n, stats);
  APR_HIP(hipGetLastError());
  return APR_OK;
}

extern "C" apr_status apr_pointwise(int32_t op, const float* a, const float* b, int64_t n, const double* stats,
                                    float* out, void* stream) {
  const bool needs_b = op == 1 || op == 2 || op == 5 || op == 6 || op == 7;
  if (n < 0 || op < 0 || op > 7) APR_FAIL(APR_EINVAL, "apr_pointwise: bad argument");
  if (n == 0) return APR_OK;
  if (!a || !stats || !out || (needs_b && !b)) APR_FAIL(APR_EINVAL, "apr_pointwise: null buffer");
  hipLaunchKernelGGL(pointwise_kernel, dim3(blocks_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), op, a,
                     b, n, stats, out);
  APR_HIP(hipGetLastError());
  return APR_OK;
}

extern "C" apr_status apr_level_weights(int32_t dir, const float* in, float* out, int64_t per_set, int32_t n_sets,
                                        int32_t l_min, int32_t l_max, void* stream) {
  if (!in || !out || per_set < 0 || n_sets < 1 || l_min < 0 || l_max < l_min || l_max >= APR_MAX_LEVELS ||
      (dir != 0 && dir != 1) || in == out)
    APR_FAIL(APR_EINVAL, "apr_level_weights: bad argument");
  if (per_set == 0) return APR_OK;
  hipLaunchKernelGGL(level_weights_kernel, dim3(blocks_for(per_set)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), dir, in, out, per_set, n_sets, l_min, l_max);
  APR_HIP(hipGetLastError());
  return APR_OK;
}

extern "C" apr_status apr_relu_bias_grad(const float* y, const float* dy, int64_t rows, int32_t c, int32_t relu,
                                         float* dy_pre, float* db, void* ws, void* stream) {
  if (rows < 0 || c < 1 || c > 256 || !ws || (rows > 0 && (!dy || !dy_pre || (relu && !y))))
    APR_FAIL(APR_EINVAL, "apr_relu_bias_grad: bad argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = rows * c;
  if (n) hipLaunchKernelGGL(relu_grad_kernel, dim3(blocks_for(n)), dim3(256), 0, s, y, dy, n, relu, dy_pre);
  if (db) {
    double* part = static_cast<double*>(ws);
    hipLaunchKernelGGL(col_sum_kernel, dim3(kRedBlocks), dim3(kRedThreads), 0, s, dy_pre, rows, c, part);
    hipLaunchKernelGGL(col_sum_finish_kernel, dim3(1), dim3(256), 0, s, part, c, db);
  }
  APR_HIP(hipGetLastError());
  return APR_OK;
}

extern "C" apr_status apr_rel_l2(const float* a, const float* b, int64_t n, double* out, float* grad,
                                 float grad_scale, void* ws, void* stream) {
  if ((n > 0 && (!a || !b)) || !out || !ws || n < 0) APR_FAIL(APR_EINVAL, "apr_rel_l2: bad argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* part = static_cast<double*>(ws);
  hipLaunchKernelGGL(l2_parts_kernel, dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, b, n, part);
  hipLaunchKernelGGL(l2_finish_kernel, dim3(1), dim3(1), 0, s, part, out);
  if (grad && n)
    hipLaunchKernelGGL(l2_grad_kernel, dim3(blocks_for(n)), dim3(256), 0, s, a, b, n, out, grad_scale, grad);
  APR_HIP(hipGetLastError());
  return APR_OK;
}

extern "C" apr_status apr_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float beta1,
                               float beta2, float eps, int32_t step, void* stream) {
  if (n < 0 || step < 1) APR_FAIL(APR_EINVAL, "apr_adam: bad argument");
  if (n == 0) return APR_OK;
  if (!p || !g || !m || !v) APR_FAIL(APR_EINVAL, "apr_adam: null buffer");
  const float c1 = 1.f - std::pow(beta1, float(step)), c2 = 1.f - std::pow(beta2, float(step));
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), p, g, m, v,
                     n, lr, beta1, beta2, eps, c1, c2);
  APR_HIP(hipGetLastError());
  return APR_OK;
}
