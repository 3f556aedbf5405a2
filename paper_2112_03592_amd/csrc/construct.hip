// APR construction on the GPU (Section 2.3) for synthetic sphere-field images:
// the level rule decides which cells of the image pyramid are split, the
// splits are closed for 2:1 balance, the unsplit cells under split parents
// are the particles (LinearAccess of Algorithm 1), and each particle takes the
// mean of the image over its cell (average downsampling).
//
// Level rule: a location at distance d from the nearest sphere surface asks
// for level l_max - floor(log2(1 + d/2)), so a cell of side s = 2^(l_max-l)
// is split when some point of the box spanned by its pixel centres lies at
// d < 2 (s - 1).  Balance: from fine to coarse, the parent of every cell that
// touches (26-neighbourhood) a split cell of its level is split.
//
// Image: background b, spheres of intensity f (a pixel is inside when its
// centre is within the radius), the indicator blurred by a normalised
// Gaussian truncated at 4 sigma with zeros outside the image:
// clean = b + (f - b) (G * 1_union).  Noise on the sum S over a cell of n
// pixels: S + sqrt(S) Z, Z the sum of twelve uniforms minus six from
// Philox4x64-10 (Salmon et al., SC'11) keyed by the cell; value = sum / n.
//
// The distance and inside tests are evaluated in FP64 in a fixed order with
// no contraction, so the partition does not depend on the compiler.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"

#pragma clang fp contract(off)

struct apr_field {
  int32_t dims[3] = {0, 0, 0};
  int32_t l_min = 0, l_max = 0;
  int64_t n_p = 0, n_rows = 0;
  uint16_t* y_idx = nullptr;   // device [n_p]
  uint64_t* xz_end = nullptr;  // device [n_rows]
  float* values = nullptr;     // device [n_p]
};

namespace apr {
namespace {

struct Level {
  int32_t dz, dx, dy, w;     // grid and 32-bit words per row
  int64_t word0;             // first word of the level in the word arrays
  int64_t row0;              // first row of the level (particle rows)
};

struct Geo {
  int32_t n[3];
  int32_t l_min, l_max;
  Level lv[kMaxL];
};

__device__ __host__ inline int64_t words_of(const Level& L) { return int64_t(L.dz) * L.dx * L.w; }

// ---------------------------------------------------------------------------
// Split sets
// ---------------------------------------------------------------------------

// cells of level l split by sphere blockIdx.x: box of its reach, cells whose
// pixel-centre box lies within 2 (s - 1) of the sphere surface
__global__ void rule_kernel(Geo g, int l, const double* __restrict__ cen, const double* __restrict__ rad,
                            uint32_t* __restrict__ split) {
  const Level L = g.lv[l];
  const int s = 1 << (g.l_max - l);
  const double thr = 2.0 * double(s - 1);
  const int sp = blockIdx.x;
  const double c[3] = {cen[3 * sp], cen[3 * sp + 1], cen[3 * sp + 2]};
  const double r = rad[sp];
  const double reach = r + thr;
  const int dl[3] = {L.dz, L.dx, L.dy};
  int i0[3], cnt[3];
  for (int a = 0; a < 3; ++a) {
    const int lo = max(0, int(floor((c[a] - reach) / double(s))) - 1);
    const int hi = min(dl[a] - 1, int(floor((c[a] + reach) / double(s))) + 1);
    i0[a] = lo;
    cnt[a] = hi - lo + 1;
    if (cnt[a] <= 0) return;
  }
  const int64_t total = int64_t(cnt[0]) * cnt[1] * cnt[2];
  for (int64_t q = threadIdx.x; q < total; q += blockDim.x) {
    const int iz = i0[0] + int(q / (int64_t(cnt[1]) * cnt[2]));
    const int ix = i0[1] + int((q / cnt[2]) % cnt[1]);
    const int iy = i0[2] + int(q % cnt[2]);
    const int id[3] = {iz, ix, iy};
    double nr[3], fr[3];
    for (int a = 0; a < 3; ++a) {
      const double lo = double(id[a]) * double(s) + 0.5;
      const double hi = double(min((id[a] + 1) * s, g.n[a])) - 0.5;
      nr[a] = fmax(fmax(lo - c[a], c[a] - hi), 0.0);
      fr[a] = fmax(fabs(c[a] - lo), fabs(c[a] - hi));
    }
    const double dmin = sqrt((nr[0] * nr[0] + nr[1] * nr[1]) + nr[2] * nr[2]);
    const double dmax = sqrt((fr[0] * fr[0] + fr[1] * fr[1]) + fr[2] * fr[2]);
    const double dist = r < dmin ? dmin - r : (r > dmax ? r - dmax : 0.0);
    if (dist < thr) {
      const int64_t wd = L.word0 + (int64_t(iz) * L.dx + ix) * L.w + (iy >> 5);
      atomicOr(&split[wd], 1u << (iy & 31));
    }
  }
}

// split[l] |= parents of the cells touching a split cell of level l + 1: a
// level-l cell (Z, X, Y) is marked when a split level-(l+1) cell lies in
// [2Z-1, 2Z+2] x [2X-1, 2X+2] x [2Y-1, 2Y+2]
__global__ void balance_kernel(Geo g, int l, uint32_t* __restrict__ split) {
  const Level L = g.lv[l], F = g.lv[l + 1];
  const int64_t n = words_of(L);
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int w = int(q % L.w);
  const int64_t rowi = q / L.w;
  const int Z = int(rowi / L.dx), X = int(rowi % L.dx);
  // OR of the 4 x 4 finer rows over fine y in [64 w - 1, 64 w + 64]
  uint64_t mid = 0;   // fine bits 64 w .. 64 w + 63
  uint32_t lo_edge = 0, hi_edge = 0;
  for (int zz = 2 * Z - 1; zz <= 2 * Z + 2; ++zz) {
    if (zz < 0 || zz >= F.dz) continue;
    for (int xx = 2 * X - 1; xx <= 2 * X + 2; ++xx) {
      if (xx < 0 || xx >= F.dx) continue;
      const uint32_t* fr = split + F.word0 + (int64_t(zz) * F.dx + xx) * F.w;
      const int fw = 2 * w;
      if (fw < F.w) mid |= uint64_t(fr[fw]);
      if (fw + 1 < F.w) mid |= uint64_t(fr[fw + 1]) << 32;
      if (fw > 0) lo_edge |= fr[fw - 1] >> 31;
      if (fw + 2 < F.w) hi_edge |= fr[fw + 2] & 1u;
    }
  }
  uint32_t add = 0;
  for (int b = 0; b < 32; ++b) {
    const int p = 2 * b;   // fine positions p - 1 .. p + 2
    bool any = ((mid >> p) & 3u) != 0;
    any = any || (p == 0 ? lo_edge != 0 : ((mid >> (p - 1)) & 1u) != 0);
    any = any || (p + 2 == 64 ? hi_edge != 0 : ((mid >> (p + 2)) & 1u) != 0);
    if (any && 32 * w + b < L.dy) add |= 1u << b;
  }
  split[L.word0 + q] |= add;
}

// particle bits of a level-l word: cells that exist (level l_min, or a split
// parent) and are not split themselves (level l_max is never split)
__device__ inline uint32_t particle_bits(const Geo& g, int l, int64_t q, const uint32_t* __restrict__ split) {
  const Level L = g.lv[l];
  const int w = int(q % L.w);
  const int64_t rowi = q / L.w;
  const int Z = int(rowi / L.dx), X = int(rowi % L.dx);
  const int nv = min(32, L.dy - 32 * w);
  uint32_t exists = nv >= 32 ? 0xffffffffu : ((1u << nv) - 1u);
  if (l > g.l_min) {
    const Level P = g.lv[l - 1];
    const uint32_t pw = split[P.word0 + (int64_t(Z >> 1) * P.dx + (X >> 1)) * P.w + (w >> 1)];
    const uint32_t half = (pw >> (16 * (w & 1))) & 0xffffu;
    uint32_t wide = 0;
    for (int b = 0; b < 16; ++b)
      if ((half >> b) & 1u) wide |= 3u << (2 * b);
    exists &= wide;
  }
  if (l < g.l_max) exists &= ~split[L.word0 + q];
  return exists;
}

__global__ void count_kernel(Geo g, int l, const uint32_t* __restrict__ split, uint32_t* __restrict__ cnt) {
  const Level L = g.lv[l];
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= words_of(L)) return;
  cnt[L.word0 + q] = uint32_t(__builtin_popcount(particle_bits(g, l, q, split)));
}

// xz_end[row] = particles in rows <= row: the scanned word offset where the
// next row begins
__global__ void row_end_kernel(Geo g, int l, const uint32_t* __restrict__ off, uint64_t* __restrict__ xz_end) {
  const Level L = g.lv[l];
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= int64_t(L.dz) * L.dx) return;
  xz_end[L.row0 + r] = off[L.word0 + (r + 1) * L.w];
}

// ---------------------------------------------------------------------------
// Image: sphere indicator, separable Gaussian blur, block sums
// ---------------------------------------------------------------------------

__global__ void indicator_kernel(Geo g, const double* __restrict__ cen, const double* __restrict__ rad,
                                 float* __restrict__ img) {
  const int sp = blockIdx.x;
  const double c[3] = {cen[3 * sp], cen[3 * sp + 1], cen[3 * sp + 2]};
  const double r = rad[sp];
  int lo[3], cnt[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = max(0, int(floor(c[a] - r - 1.0)));
    const int hi = min(g.n[a], int(ceil(c[a] + r + 1.0)));
    cnt[a] = hi - lo[a];
    if (cnt[a] <= 0) return;
  }
  const int64_t total = int64_t(cnt[0]) * cnt[1] * cnt[2];
  for (int64_t q = threadIdx.x; q < total; q += blockDim.x) {
    const int z = lo[0] + int(q / (int64_t(cnt[1]) * cnt[2]));
    const int x = lo[1] + int((q / cnt[2]) % cnt[1]);
    const int y = lo[2] + int(q % cnt[2]);
    const double dz = (double(z) + 0.5) - c[0], dx = (double(x) + 0.5) - c[1], dy = (double(y) + 0.5) - c[2];
    if ((dz * dz + dx * dx) + dy * dy <= r * r)
      img[(int64_t(z) * g.n[1] + x) * g.n[2] + y] = 1.0f;
  }
}

// one axis of the separable blur (FP64 accumulation, zeros outside); the
// last axis also maps the blurred indicator to intensities
template <int AX>
__global__ void blur_kernel(Geo g, const float* __restrict__ in, float* __restrict__ out, int radius,
                            const double* __restrict__ taps, int last, double bg, double fg) {
  const int64_t n = int64_t(g.n[0]) * g.n[1] * g.n[2];
  const int64_t stride = AX == 0 ? int64_t(g.n[1]) * g.n[2] : (AX == 1 ? int64_t(g.n[2]) : 1);
  const int len = g.n[AX];
  for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += int64_t(gridDim.x) * blockDim.x) {
    const int pos = int((p / stride) % len);
    double acc = 0.0;
    for (int t = -radius; t <= radius; ++t) {
      const int q = pos + t;
      if (q < 0 || q >= len) continue;
      acc = acc + taps[t + radius] * double(in[p + int64_t(t) * stride]);
    }
    out[p] = last ? float(bg + (fg - bg) * acc) : float(acc);
  }
}

// FP64 sums of the image over the cells of level l_max - 1 (partial cells at
// the edges hold fewer pixels)
__global__ void sum_from_image_kernel(Geo g, const float* __restrict__ img, double* __restrict__ out) {
  const Level L = g.lv[g.l_max - 1];
  const int64_t n = int64_t(L.dz) * L.dx * L.dy;
  for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < n; q += int64_t(gridDim.x) * blockDim.x) {
    const int Y = int(q % L.dy), X = int((q / L.dy) % L.dx), Z = int(q / (int64_t(L.dy) * L.dx));
    double acc = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 2; ++c) {
          const int z = 2 * Z + a, x = 2 * X + b, y = 2 * Y + c;
          if (z < g.n[0] && x < g.n[1] && y < g.n[2]) acc = acc + double(img[(int64_t(z) * g.n[1] + x) * g.n[2] + y]);
        }
    out[q] = acc;
  }
}

__global__ void sum_from_level_kernel(Geo g, int l, const double* __restrict__ fine, double* __restrict__ out) {
  const Level L = g.lv[l], F = g.lv[l + 1];
  const int64_t n = int64_t(L.dz) * L.dx * L.dy;
  for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < n; q += int64_t(gridDim.x) * blockDim.x) {
    const int Y = int(q % L.dy), X = int((q / L.dy) % L.dx), Z = int(q / (int64_t(L.dy) * L.dx));
    double acc = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 2; ++c) {
          const int z = 2 * Z + a, x = 2 * X + b, y = 2 * Y + c;
          if (z < F.dz && x < F.dx && y < F.dy) acc = acc + fine[(int64_t(z) * F.dx + x) * F.dy + y];
        }
    out[q] = acc;
  }
}

// ---------------------------------------------------------------------------
// Particles: y, values (noise from Philox4x64-10)
// ---------------------------------------------------------------------------

__device__ inline void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ inline double cell_normal(uint64_t key, uint64_t seed) {
  double z = 0.0;
  for (int b = 0; b < 3; ++b) {
    uint64_t c[4] = {key, uint64_t(b), 0, 0};
    philox4x64(c, seed, 0);
    for (int i = 0; i < 4; ++i) z = z + double(c[i] >> 11) * 0x1.0p-53;
  }
  return z - 6.0;
}

__global__ void particle_kernel(Geo g, int l, const uint32_t* __restrict__ split, const uint32_t* __restrict__ off,
                                const float* __restrict__ img, const double* __restrict__ sums, int noise,
                                uint64_t seed, uint16_t* __restrict__ y_idx, float* __restrict__ values) {
  const Level L = g.lv[l];
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= words_of(L)) return;
  uint32_t bits = particle_bits(g, l, q, split);
  if (!bits) return;
  const int w = int(q % L.w);
  const int64_t rowi = q / L.w;
  const int Z = int(rowi / L.dx), X = int(rowi % L.dx);
  const int s = 1 << (g.l_max - l);
  const double nzx = double(min((Z + 1) * s, g.n[0]) - Z * s) * double(min((X + 1) * s, g.n[1]) - X * s);
  uint32_t p = off[L.word0 + q];
  while (bits) {
    const int b = __builtin_ctz(bits);
    bits &= bits - 1;
    const int Y = 32 * w + b;
    double S = l == g.l_max ? double(img[(int64_t(Z) * g.n[1] + X) * g.n[2] + Y])
                            : sums[(int64_t(Z) * L.dx + X) * L.dy + Y];
    const double n = nzx * double(min((Y + 1) * s, g.n[2]) - Y * s);
    if (noise) {
      const uint64_t key = (uint64_t(l) << 48) | (uint64_t(Z) << 32) | (uint64_t(X) << 16) | uint64_t(Y);
      S = S + sqrt(S) * cell_normal(key, seed);
    }
    y_idx[p] = uint16_t(Y);
    values[p] = float(S / n);
    ++p;
  }
}

void free_field(apr_field* f) {
  if (!f) return;
  (void)hipFree(f->y_idx);
  (void)hipFree(f->xz_end);
  (void)hipFree(f->values);
  delete f;
}

// device scratch freed on every exit path
struct Scratch {
  std::vector<void*> p;
  template <typename T>
  apr_status alloc(T** out, int64_t count) {
    *out = nullptr;
    if (count <= 0) return APR_OK;
    void* q = nullptr;
    if (hipMalloc(&q, size_t(count) * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      APR_FAIL(APR_ENOMEM, "apr_sphere_field: hipMalloc failed (" + std::to_string(count * int64_t(sizeof(T))) +
                               " bytes)");
    }
    p.push_back(q);
    *out = static_cast<T*>(q);
    return APR_OK;
  }
  ~Scratch() {
    for (void* q : p) (void)hipFree(q);
  }
};

unsigned grid_for(int64_t n, int block = 256) {
  return unsigned(std::max<int64_t>(1, std::min<int64_t>((n + block - 1) / block, int64_t(1) << 20)));
}

#define CF_TRY(expr)                    \
  do {                                  \
    apr_status _s = (expr);             \
    if (_s != APR_OK) {                 \
      free_field(f);                    \
      return _s;                        \
    }                                   \
  } while (0)
#define CF_HIP(call)                                                               \
  do {                                                                             \
    hipError_t _e = (call);                                                        \
    if (_e != hipSuccess) {                                                        \
      set_error(std::string(#call) + ": " + hipGetErrorString(_e));                \
      free_field(f);                                                               \
      return APR_EDEVICE;                                                          \
    }                                                                              \
  } while (0)

apr_status sphere_field_impl(const apr_sphere_field_desc* d, hipStream_t s, apr_field** out) {
  if (!d || !out) APR_FAIL(APR_EINVAL, "apr_sphere_field: null argument");
  *out = nullptr;
  for (int a = 0; a < 3; ++a)
    if (d->dims[a] <= 0) APR_FAIL(APR_EINVAL, "apr_sphere_field: image dims must be positive");
  if (d->dims[2] > 65535) APR_FAIL(APR_EUNSUPPORTED, "apr_sphere_field: y size above 65535");
  if (d->n_spheres < 0 || (d->n_spheres > 0 && (!d->centres || !d->radii)))
    APR_FAIL(APR_EINVAL, "apr_sphere_field: bad sphere list");
  if (d->n_spheres > (int64_t(1) << 31) - 1) APR_FAIL(APR_EUNSUPPORTED, "apr_sphere_field: too many spheres");
  if (d->edge_sigma < 0) APR_FAIL(APR_EINVAL, "apr_sphere_field: negative blur");
  Geo g{};
  int lmax = 0;
  while ((1 << lmax) < std::max({d->dims[0], d->dims[1], d->dims[2]})) ++lmax;
  if (lmax >= kMaxL) APR_FAIL(APR_EUNSUPPORTED, "apr_sphere_field: too many levels");
  if (d->l_min < 0 || d->l_min > lmax) APR_FAIL(APR_EINVAL, "apr_sphere_field: need 0 <= l_min <= l_max");
  for (int a = 0; a < 3; ++a) g.n[a] = d->dims[a];
  g.l_min = d->l_min;
  g.l_max = lmax;
  int64_t words = 0, rows = 0;
  for (int l = d->l_min; l <= lmax; ++l) {
    const int64_t sh = int64_t(1) << (lmax - l);
    Level& L = g.lv[l];
    L.dz = int32_t((d->dims[0] + sh - 1) / sh);
    L.dx = int32_t((d->dims[1] + sh - 1) / sh);
    L.dy = int32_t((d->dims[2] + sh - 1) / sh);
    L.w = (L.dy + 31) / 32;
    L.word0 = words;
    L.row0 = rows;
    words += words_of(L);
    rows += int64_t(L.dz) * L.dx;
  }
  if (words >= int64_t(0xffffffffu)) APR_FAIL(APR_EUNSUPPORTED, "apr_sphere_field: image too large");
  const int64_t npix = int64_t(d->dims[0]) * d->dims[1] * d->dims[2];

  apr_field* f = new apr_field();
  for (int a = 0; a < 3; ++a) f->dims[a] = d->dims[a];
  f->l_min = d->l_min;
  f->l_max = lmax;
  f->n_rows = rows;
  Scratch sc;
  double *cen = nullptr, *rad = nullptr;
  uint32_t *split = nullptr, *off = nullptr, *total = nullptr;
  CF_TRY(sc.alloc(&cen, 3 * d->n_spheres));
  CF_TRY(sc.alloc(&rad, d->n_spheres));
  CF_TRY(sc.alloc(&split, words));
  CF_TRY(sc.alloc(&off, words + 1));
  CF_TRY(sc.alloc(&total, 1));
  if (d->n_spheres) {
    CF_HIP(hipMemcpyAsync(cen, d->centres, size_t(d->n_spheres) * 24, hipMemcpyHostToDevice, s));
    CF_HIP(hipMemcpyAsync(rad, d->radii, size_t(d->n_spheres) * 8, hipMemcpyHostToDevice, s));
  }
  // ---- split sets, balance, particle counts
  CF_HIP(hipMemsetAsync(split, 0, size_t(words) * 4, s));
  for (int l = d->l_min; l < lmax && d->n_spheres; ++l) {
    hipLaunchKernelGGL(rule_kernel, dim3(unsigned(d->n_spheres)), dim3(256), 0, s, g, l, cen, rad, split);
    CF_HIP(hipGetLastError());
  }
  for (int l = lmax - 2; l >= d->l_min; --l) {
    hipLaunchKernelGGL(balance_kernel, dim3(grid_for(words_of(g.lv[l]))), dim3(256), 0, s, g, l, split);
    CF_HIP(hipGetLastError());
  }
  for (int l = d->l_min; l <= lmax; ++l) {
    hipLaunchKernelGGL(count_kernel, dim3(grid_for(words_of(g.lv[l]))), dim3(256), 0, s, g, l, split, off);
    CF_HIP(hipGetLastError());
  }
  CF_HIP(hipMemsetAsync(off + words, 0, 4, s));
  CF_TRY(scan_u32(off, words + 1, total, s));
  uint32_t np = 0;
  CF_HIP(hipMemcpyAsync(&np, off + words, 4, hipMemcpyDeviceToHost, s));
  CF_HIP(hipStreamSynchronize(s));
  f->n_p = np;
  CF_HIP(hipMalloc(&f->xz_end, size_t(std::max<int64_t>(rows, 1)) * 8));
  CF_HIP(hipMalloc(&f->y_idx, size_t(std::max<int64_t>(np, 1)) * 2));
  CF_HIP(hipMalloc(&f->values, size_t(std::max<int64_t>(np, 1)) * 4));
  for (int l = d->l_min; l <= lmax; ++l) {
    hipLaunchKernelGGL(row_end_kernel, dim3(grid_for(int64_t(g.lv[l].dz) * g.lv[l].dx)), dim3(256), 0, s, g, l,
                       off, f->xz_end);
    CF_HIP(hipGetLastError());
  }
  // ---- image and block sums
  float *img = nullptr, *tmp = nullptr;
  CF_TRY(sc.alloc(&img, npix));
  CF_TRY(sc.alloc(&tmp, npix));
  CF_HIP(hipMemsetAsync(img, 0, size_t(npix) * 4, s));
  if (d->n_spheres) {
    hipLaunchKernelGGL(indicator_kernel, dim3(unsigned(d->n_spheres)), dim3(256), 0, s, g, cen, rad, img);
    CF_HIP(hipGetLastError());
  }
  {
    const int radius = d->edge_sigma > 0 ? int(4.0 * d->edge_sigma + 0.5) : 0;
    std::vector<double> taps(size_t(2 * radius + 1));
    double sum = 0.0;
    for (int t = -radius; t <= radius; ++t) {
      const double v = d->edge_sigma > 0 ? std::exp(-0.5 * (double(t) / d->edge_sigma) * (double(t) / d->edge_sigma))
                                         : 1.0;
      taps[size_t(t + radius)] = v;
      sum += v;
    }
    for (double& v : taps) v /= sum;
    double* dtaps = nullptr;
    CF_TRY(sc.alloc(&dtaps, int64_t(taps.size())));
    CF_HIP(hipMemcpyAsync(dtaps, taps.data(), taps.size() * 8, hipMemcpyHostToDevice, s));
    const unsigned gb = grid_for(npix);
    hipLaunchKernelGGL(blur_kernel<0>, dim3(gb), dim3(256), 0, s, g, img, tmp, radius, dtaps, 0, 0.0, 0.0);
    hipLaunchKernelGGL(blur_kernel<1>, dim3(gb), dim3(256), 0, s, g, tmp, img, radius, dtaps, 0, 0.0, 0.0);
    hipLaunchKernelGGL(blur_kernel<2>, dim3(gb), dim3(256), 0, s, g, img, tmp, radius, dtaps, 1, d->background,
                       d->foreground);
    CF_HIP(hipGetLastError());
    std::swap(img, tmp);   // img: the clean image
  }
  std::vector<double*> sums(size_t(lmax + 1), nullptr);
  for (int l = lmax - 1; l >= d->l_min; --l) {
    const Level& L = g.lv[l];
    const int64_t n = int64_t(L.dz) * L.dx * L.dy;
    CF_TRY(sc.alloc(&sums[size_t(l)], n));
    if (l == lmax - 1)
      hipLaunchKernelGGL(sum_from_image_kernel, dim3(grid_for(n)), dim3(256), 0, s, g, img, sums[size_t(l)]);
    else
      hipLaunchKernelGGL(sum_from_level_kernel, dim3(grid_for(n)), dim3(256), 0, s, g, l, sums[size_t(l) + 1],
                         sums[size_t(l)]);
    CF_HIP(hipGetLastError());
  }
  for (int l = d->l_min; l <= lmax; ++l) {
    hipLaunchKernelGGL(particle_kernel, dim3(grid_for(words_of(g.lv[l]))), dim3(256), 0, s, g, l, split, off, img,
                       sums[size_t(l)], d->noise, d->seed, f->y_idx, f->values);
    CF_HIP(hipGetLastError());
  }
  CF_HIP(hipStreamSynchronize(s));
  *out = f;
  return APR_OK;
}

}  // namespace
}  // namespace apr

extern "C" apr_status apr_sphere_field(const apr_sphere_field_desc* desc, void* stream, apr_field** out) {
  try {
    return apr::sphere_field_impl(desc, static_cast<hipStream_t>(stream), out);
  } catch (const std::exception& e) {
    apr::set_error(std::string("apr_sphere_field: ") + e.what());
    return APR_ENOMEM;
  }
}

extern "C" apr_status apr_field_get_info(const apr_field* f, apr_field_info* o) {
  if (!f || !o) APR_FAIL(APR_EINVAL, "apr_field_get_info: null argument");
  for (int a = 0; a < 3; ++a) o->dims[a] = f->dims[a];
  o->l_min = f->l_min;
  o->l_max = f->l_max;
  o->n_particles = f->n_p;
  o->n_rows = f->n_rows;
  o->y_idx = f->y_idx;
  o->xz_end = f->xz_end;
  o->values = f->values;
  return APR_OK;
}

extern "C" apr_status apr_field_destroy(apr_field* f) {
  apr::free_field(f);
  return APR_OK;
}
