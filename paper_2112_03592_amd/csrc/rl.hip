// Richardson-Lucy deconvolution on the APR (Section 6.2): a host loop over
// the tree-fill and convolution kernels, with the quotient and the update
// fused into the convolution epilogues.
#include <algorithm>
#include <mutex>
#include <string>

#include "common.hpp"

namespace apr {

// max |u| over n values: one pass of per-block maxima, then one block
__global__ __launch_bounds__(256) void absmax_kernel(const float* __restrict__ u, int64_t n,
                                                     float* __restrict__ out, int stage) {
  __shared__ float red[4];
  float m = 0.f;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    m = fmaxf(m, fabsf(u[i]));
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if (lane_id() == 0) red[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    out[stage == 0 ? blockIdx.x : 0] = m;
  }
}

__global__ void scale_kernel(float* __restrict__ v, float s) { v[0] *= s; }

__global__ void copy_kernel(const float* __restrict__ a, float* __restrict__ b, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

}  // namespace apr

using namespace apr;

namespace apr {
apr_status conv_impl(const apr_handle* h, const apr_conv_desc* d, const void* x, const void* tree,
                     const float* w, void* y, const float* eps_dev, void* stream);
}

extern "C" size_t apr_richardson_lucy_workspace(const apr_handle* h) {
  if (!h) return 0;
  const size_t np = size_t(h->n_p), nt = size_t(h->n_t);
  return (nt + 3 * np + 1024 + 64) * sizeof(float) + 256;
}

namespace apr {
// The iterations over a workspace whose start `base` is 256-byte aligned and
// holds (N_t + 3 N_p + 1088) floats: tree [N_t] | rho [N_p] | ping [N_p] |
// pong [N_p] | block maxima [1024] | eps.
static apr_status rl_run(const apr_handle* h, int32_t k, int32_t n_wlevels, const float* w, const float* w_flip,
                         const float* u, const float* init, float* out, int32_t n_iter, float eps_rel, float power,
                         char* base, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t np = h->n_p;
  float* tree = reinterpret_cast<float*>(base);
  const float* tree_in = h->n_t ? tree : nullptr;   // no tree levels: nothing to read (and rho starts at base)
  float* rho = tree + h->n_t;
  float* ping = rho + np;
  float* pong = ping + np;
  float* blk = pong + np;
  float* eps = blk + 1024;
  const int nblk = int(std::min<int64_t>(1024, (np + 255) / 256));
  hipLaunchKernelGGL(absmax_kernel, dim3(nblk), dim3(256), 0, s, u, np, blk, 0);
  hipLaunchKernelGGL(absmax_kernel, dim3(1), dim3(256), 0, s, blk, int64_t(nblk), eps, 1);
  hipLaunchKernelGGL(scale_kernel, dim3(1), dim3(1), 0, s, eps, eps_rel);
  APR_HIP(hipGetLastError());

  apr_conv_desc d{};
  d.k = k;
  d.c_in = d.c_out = 1;
  d.n_wlevels = n_wlevels;
  d.x_dtype = d.y_dtype = APR_F32;
  const float* i0 = init ? init : u;
  const float* cur = i0;
  for (int it = 0; it < n_iter; ++it) {
    float* nxt = (it == n_iter - 1) ? out : ((cur == ping) ? pong : ping);
    apr_status st = apr_fill_tree(h, cur, tree, 1, APR_F32, stream);
    if (st != APR_OK) return st;
    // rho = u / max(corr(i, w_flip), eps)
    d.epilogue = APR_EPI_RATIO;
    d.epi_arg = u;
    st = conv_impl(h, &d, cur, tree_in, w_flip, rho, eps, stream);
    if (st != APR_OK) return st;
    st = apr_fill_tree(h, rho, tree, 1, APR_F32, stream);
    if (st != APR_OK) return st;
    // i <- i * corr(rho, w)   (or i * corr(rho, w)^power)
    d.epilogue = power == 1.f ? APR_EPI_MUL : APR_EPI_MULPOW;
    d.power = power;
    d.epi_arg = cur;
    st = conv_impl(h, &d, rho, tree_in, w, nxt, nullptr, stream);
    if (st != APR_OK) return st;
    cur = nxt;
  }
  if (n_iter == 0) {
    hipLaunchKernelGGL(copy_kernel, dim3(unsigned((np + 255) / 256)), dim3(256), 0, s, i0, out, np);
    APR_HIP(hipGetLastError());
  }
  return APR_OK;
}

static apr_status rl_check(const apr_handle* h, const float* w, const float* w_flip, const float* u,
                           const float* init, float* out, int32_t n_iter, float power, const char* who) {
  if (!h || !w || !w_flip || !u || !out) APR_FAIL(APR_EINVAL, std::string(who) + ": null argument");
  if (n_iter < 0) APR_FAIL(APR_EINVAL, std::string(who) + ": n_iter < 0");
  if (!(power > 0.f) || !(power < 16.f)) APR_FAIL(APR_EINVAL, std::string(who) + ": power must be in (0, 16)");
  if (out == u || (init && out == init)) APR_FAIL(APR_EINVAL, std::string(who) + ": out must not alias u or init");
  return APR_OK;
}

// Scratch of the allocation-free variant: one array per device, held until
// the process ends.  Host code never names it directly: the device address
// comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) float scratch[APR_RL_STATIC_FLOATS];
static std::mutex g_scratch_mu;
static float* g_scratch_ptr[64] = {nullptr};

static apr_status scratch_for_current_device(float** out) {
  int dev = 0;
  APR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) APR_FAIL(APR_EUNSUPPORTED, "apr_richardson_lucy_static: device index >= 64");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      APR_FAIL(APR_EDEVICE, std::string("apr_richardson_lucy_static: hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return APR_OK;
}
}  // namespace apr

extern "C" apr_status apr_richardson_lucy(const apr_handle* h, int32_t k, int32_t n_wlevels,
                                          const float* w, const float* w_flip, const float* u,
                                          const float* init, float* out, int32_t n_iter, float eps_rel,
                                          float power, void* work, void* stream) {
  apr_status st = rl_check(h, w, w_flip, u, init, out, n_iter, power, "apr_richardson_lucy");
  if (st != APR_OK) return st;
  if (!work) APR_FAIL(APR_EINVAL, "apr_richardson_lucy: null workspace");
  if (h->n_p == 0) return APR_OK;
  char* base = static_cast<char*>(work);
  base += (256 - (reinterpret_cast<uintptr_t>(base) & 255)) & 255;
  return rl_run(h, k, n_wlevels, w, w_flip, u, init, out, n_iter, eps_rel, power, base, stream);
}

extern "C" apr_status apr_richardson_lucy_static(const apr_handle* h, int32_t k, int32_t n_wlevels,
                                                 const float* w, const float* w_flip, const float* u,
                                                 const float* init, float* out, int32_t n_iter, float eps_rel,
                                                 float power, void* stream) {
  apr_status st = rl_check(h, w, w_flip, u, init, out, n_iter, power, "apr_richardson_lucy_static");
  if (st != APR_OK) return st;
  const uint64_t need = uint64_t(h->n_t) + 3 * uint64_t(h->n_p) + 1024 + 64;
  if (need > uint64_t(APR_RL_STATIC_FLOATS))
    APR_FAIL(APR_EINVAL, "apr_richardson_lucy_static: N_t + 3 N_p + 1088 = " + std::to_string(need) +
                             " floats exceeds the static scratch of " + std::to_string(APR_RL_STATIC_FLOATS) +
                             " floats; use apr_richardson_lucy with a workspace");
  if (h->n_p == 0) return APR_OK;
  float* base = nullptr;
  st = scratch_for_current_device(&base);
  if (st != APR_OK) return st;
  return rl_run(h, k, n_wlevels, w, w_flip, u, init, out, n_iter, eps_rel, power, reinterpret_cast<char*>(base),
                stream);
}
