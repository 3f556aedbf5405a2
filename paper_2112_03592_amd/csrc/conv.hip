// Single-channel APR convolution (Section 4.1), GPU design after Section 5.2,
// re-shaped for wave64 / CDNA4.
//
// Work item: one tile of kTileZ x kTileX particle rows (z, x) at one level l,
// from the non-empty tile list (the pre-pass of Section 5.2).  A workgroup
// (512 threads for 3^3, 1024 for 5^3) sweeps its tile along y in chunks; each chunk starts at the
// smallest unprocessed y of the tile's output particles (empty stretches are
// skipped) and spans at most kYC cells.  Per chunk:
//   B. list the output particles of the centre rows that fall in
//      [y0, y0 + kYC), and fetch the y at every source-row pointer;
//   C. reconstruct the level-l patch of the halo rows in LDS over
//      [y0 - r, ymax + r] from three sorted sources -- APR level l, tree level
//      l (cells containing finer particles), APR level l-1 (each element covers
//      2 x 2 x 2 level-l cells).  With 26-neighbour 2:1 balance these cover
//      every cell within radius 2 of a level-l particle.  Elements of all
//      source rows are spread flat over the threads (coalesced within a row),
//      y and value fetched in one memory round;
//   D. every listed particle accumulates its k^3 taps from the patch in FP32
//      (weights in scalar registers) and writes its output.
// Per-row bookkeeping uses one writer per row (the last element of a prefix),
// no atomics.  Threads share data through LDS only (outputs are never read
// back), so the barriers order LDS and leave stores in flight.  The blockIdx -> tile map gives each XCD a contiguous run of
// tiles so that halo rows shared by neighbouring tiles hit the same L2.
#include <algorithm>
#include <type_traits>

#include "common.hpp"

namespace apr {

constexpr int kYC = 64;          // output cells per chunk along y
constexpr int kBig = 1 << 28;    // y of an element past the end of its row
// Launch shape per stencil size.  The kernel waits on memory most of the
// time, so resident waves decide its speed: the 3^3 patch lets three
// workgroups share a CU once registers are capped for six waves per SIMD;
// the larger 5^3 patch allows two, so those workgroups are 1024 threads wide
// (eight waves per SIMD).  Elements in flight per thread are set so that
// nothing spills under those caps (spilled registers go through HBM).
template <int K>
struct ConvShape {
  static constexpr int kThreads = K == 3 ? 512 : 1024;
  static constexpr int kBatch = K == 3 ? 2 : 1;        // independent elements per thread in flight
  static constexpr int kWavesPerSimd = K == 3 ? 6 : 8;
};

struct ConvArgs {
  Meta m;
  const uint16_t* py;
  const uint32_t* pend;
  const uint16_t* ty;
  const uint32_t* tend;
  const uint64_t* tiles;
  int64_t n_tiles;
  int64_t xcd_off[9];     // tiles of XCD x: [xcd_off[x], xcd_off[x + 1])
  const void* x;
  const void* tree;
  const float* w;
  int32_t n_wlevels;
  void* y;
  int32_t epi;
  float eps;
  const float* eps_dev;   // when set, the ratio clamp is read from device memory
  float power;            // exponent of APR_EPI_MULPOW
  const void* epi_arg;
  const int64_t* sel;   // neighbour-map mode: sorted particle list
  int64_t n_sel;
  int64_t* map;         // neighbour-map mode output [n_sel][k^3]
  int32_t* map32;       // gather-map mode: every particle, [k^3][N_p] (type << 30 | index, -1 pad;
                        // n_sel holds N_p)
};

// exclusive scan of n LDS entries in place by one wave (E entries per lane,
// n <= 64 * E); data[n] = total.  `fill(k)` yields the value of entry k.
template <int E, typename F>
__device__ inline void wave_scan_into(uint32_t* data, int n, F fill) {
  const uint32_t lane = lane_id();
  uint32_t v[E];
  uint32_t sum = 0;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int k = int(lane) * E + q;
    v[q] = (k < n) ? fill(k) : 0u;
    sum += v[q];
  }
  uint32_t incl = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o, 64);
    if (lane >= uint32_t(o)) incl += t;
  }
  uint32_t run = incl - sum;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int k = int(lane) * E + q;
    if (k < n) data[k] = run;
    run += v[q];
  }
  if (lane == 63) data[n] = incl;
}

// largest r in [0, n) with pre[r] <= v (pre non-decreasing, pre[0] = 0 <= v)
__device__ inline int find_row(const uint32_t* pre, int n, uint32_t v) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

// NF = 3: three stencils per level on the same patch (the three directions of
// a gradient filter), output the magnitude sqrt(sum of squares).
template <int K, typename TX, typename TY, bool INDEX, int NF = 1>
__global__ __launch_bounds__(ConvShape<K>::kThreads)
__attribute__((amdgpu_waves_per_eu(INDEX ? 4 : ConvShape<K>::kWavesPerSimd))) void conv1_kernel(ConvArgs a) {
  constexpr int NT = ConvShape<K>::kThreads, NW = NT / 64;
  constexpr int kBatch = ConvShape<K>::kBatch;
  constexpr int R = K / 2;
  constexpr int TZ = kTileZ, TX_ = kTileX;
  constexpr int HZ = TZ + 2 * R, HX = TX_ + 2 * R;
  constexpr int NH = HZ * HX;                        // halo rows at level l
  constexpr int PZ = ((TZ - 1 + R) >> 1) + 2;        // parent rows (level l-1)
  constexpr int PX = ((TX_ - 1 + R) >> 1) + 2;
  constexpr int NCR = PZ * PX;
  constexpr int NSRC = 2 * NH + NCR;                 // [0,NH) APR l, [NH,2NH) tree l, rest APR l-1
  constexpr int NC = TZ * TX_;                       // centre (output) rows
  constexpr int PY = kYC + 2 * R;
  constexpr int K3 = K * K * K;
  constexpr int OCAP = kYC + 1;                      // centre-row elements examined per chunk
  constexpr int NOUT = NC * OCAP;
  constexpr int ES = (NSRC + 63) / 64;               // scan entries per lane
  constexpr uint16_t kUnlisted = 0xffffu;
  using PT = typename std::conditional<INDEX, long long, float>::type;
  static_assert(NC <= 64 && kYC == 64, "centre rows and offsets pack into 16 bits");
  static_assert(NSRC < 65536 && NT >= NSRC, "one thread per source row");

  __shared__ PT patch[NH * PY];
  __shared__ uint32_t sp[NSRC], se[NSRC], spre[NSRC + 1], scons[NSRC];
  __shared__ int yfirst[NSRC];
  __shared__ uint8_t cmask[NCR];            // coarse row -> valid target halo rows (bit q: dz = q/2, dx = q%2)
  __shared__ int16_t cbase[NCR];            // coarse row -> halo row of target q = 0
  __shared__ uint32_t op[NC], oe[NC], opd[NC], ocnt[NC], opre[2][NC + 1];
  __shared__ int rymax[NC], rnext[NC];      // per centre row: last listed y, next y
  __shared__ uint16_t o_pos[NOUT];          // (centre row << 6) | (y - y0), or kUnlisted
  __shared__ int s_y0;

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const uint32_t lane = lane_id();

  // XCD-aware tile order: block b runs on XCD b % 8, which takes its own
  // contiguous range of the tile list (equal work per XCD, heaviest first).
  const int xcd = int(blockIdx.x % 8);
  const int64_t t = a.xcd_off[xcd] + int64_t(blockIdx.x / 8);
  if (t >= a.xcd_off[xcd + 1]) return;
  int l, tz, tx, ty0;
  tile_unpack(a.tiles[t], l, tz, tx, ty0);
  // workgroup-uniform: keep them in scalar registers
  l = __builtin_amdgcn_readfirstlane(l);
  tz = __builtin_amdgcn_readfirstlane(tz);
  tx = __builtin_amdgcn_readfirstlane(tx);
  const Meta& m = a.m;
  const int z0 = tz * TZ, x0 = tx * TX_;
  const int Dz = m.dz[l], Dx = m.dx[l], Dy = m.dy[l];
  const bool has_c = l > m.l_min;
  const bool has_t = l <= m.t_hi;
  const TX* __restrict__ xv = static_cast<const TX*>(a.x);
  const TX* __restrict__ tv = static_cast<const TX*>(a.tree);
  const uint16_t* __restrict__ py = a.py;
  const uint16_t* __restrict__ ty = a.ty;
  // per-level weights: read-only for the whole launch and uniform across the
  // workgroup, so the tap loop reads them through scalar loads
  using cfloat = const __attribute__((address_space(4))) float;
  cfloat* wl = (cfloat*)(uintptr_t)(INDEX ? a.w : a.w + (a.n_wlevels == 1 ? 0 : (l - m.l_min)) * K3 * NF);

  // ---- setup
  const PT pad = INDEX ? PT(-1) : PT(0);
  for (int i = tid; i < NH * PY; i += NT) patch[i] = pad;
  for (int s = tid; s < NSRC; s += NT) {
    uint32_t b = 0, e = 0;
    if (s < 2 * NH) {
      const int h = s < NH ? s : s - NH;
      const int z = z0 - R + h / HX, x = x0 - R + h % HX;
      const bool in = z >= 0 && x >= 0 && z < Dz && x < Dx;
      if (in && s < NH) row_range(a.pend, m.prow[l] + uint32_t(z) * Dx + x, b, e);
      if (in && s >= NH && has_t) row_range(a.tend, m.trow[l] + uint32_t(z) * Dx + x, b, e);
    } else {
      // the coarse element of parent row j covers halo rows
      // hz = 2 * (j / PX) + R - 2 + {0, 1}, hx likewise; a halo row is a
      // target if it lies in the halo and in the level-l grid (a coarse cell
      // on the far edge of an odd-sized grid covers cells outside the image,
      // which stay zero padding)
      const int j = s - 2 * NH;
      const int pz = z0 / 2 - 1 + j / PX, px = x0 / 2 - 1 + j % PX;
      if (has_c && pz >= 0 && px >= 0 && pz < m.dz[l - 1] && px < m.dx[l - 1])
        row_range(a.pend, m.prow[l - 1] + uint32_t(pz) * m.dx[l - 1] + px, b, e);
      const int hz0 = 2 * (j / PX) + R - 2, hx0 = 2 * (j % PX) + R - 2;
      int msk = 0;
      for (int q = 0; q < 4; ++q) {
        const int hz = hz0 + (q >> 1), hx = hx0 + (q & 1);
        if (hz >= 0 && hx >= 0 && hz < HZ && hx < HX && z0 - R + hz < Dz && x0 - R + hx < Dx)
          msk |= 1 << q;
      }
      cmask[j] = uint8_t(msk);
      cbase[j] = int16_t(hz0 * HX + hx0);
    }
    sp[s] = b;
    se[s] = e;
    scons[s] = 0;
  }
  for (int c = tid; c < NC; c += NT) {
    uint32_t b = 0, e = 0;
    const int z = z0 + c / TX_, x = x0 + c % TX_;
    if (z < Dz && x < Dx) row_range(a.pend, m.prow[l] + uint32_t(z) * Dx + x, b, e);
    op[c] = b;
    oe[c] = e;
    ocnt[c] = 0;
    rymax[c] = -1;
    rnext[c] = int(kNoY);
  }
  lds_barrier();
  if (wave == 0) {
    if (lane == 0) s_y0 = ty0;   // first y of the tile's particles, from the tile list
    wave_scan_into<1>(opre[0], NC, [&](int c) { return min(oe[c] - op[c], uint32_t(OCAP)); });
  }
  lds_barrier();

  int par = 0;
  while (true) {
    const int y0 = s_y0;
    if (y0 == int(kNoY)) break;
    const uint32_t* ocap = opre[par];
    const uint32_t nb = ocap[NC];

    // ---- B (one memory round): the listed elements of a centre row are a
    // prefix of its items; the last of them (or the first item, when none is
    // listed) records the row's count, last y and next y.  Also fetch the y
    // at every source-row pointer.
    int yf = kBig;
    if (tid < NSRC && sp[tid] < se[tid]) yf = (tid >= NH && tid < 2 * NH) ? int(ty[sp[tid]]) : int(py[sp[tid]]);
    for (uint32_t base = tid; base < nb; base += NT * kBatch) {
      int cc[kBatch], yv[kBatch], yn[kBatch];
      uint32_t ii[kBatch], jj[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const uint32_t it = base + u * NT;
        const bool ok = it < nb;
        cc[u] = ok ? find_row(ocap, NC, it) : 0;
        jj[u] = ok ? it - ocap[cc[u]] : 0u;
        ii[u] = op[cc[u]] + jj[u];
        yv[u] = ok ? int(py[ii[u]]) : 0;
        yn[u] = (ok && ii[u] + 1 < oe[cc[u]]) ? int(py[ii[u] + 1]) : int(kNoY);
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const uint32_t it = base + u * NT;
        if (it >= nb) continue;
        const int c = cc[u];
        if (yv[u] < y0 + kYC) {
          o_pos[it] = uint16_t((c << 6) | (yv[u] - y0));
          if (yn[u] >= y0 + kYC) {
            ocnt[c] = jj[u] + 1;
            rymax[c] = yv[u];
            rnext[c] = yn[u];
          }
        } else {
          o_pos[it] = kUnlisted;
          if (jj[u] == 0) rnext[c] = yv[u];
        }
      }
    }
    if (tid < NSRC) yfirst[tid] = yf;
    lds_barrier();
    // every wave reduces the per-row results itself (no extra barrier)
    int ymax_c = (lane < uint32_t(NC)) ? rymax[lane] : -1;
    int ynx = (lane < uint32_t(NC)) ? rnext[lane] : int(kNoY);
    for (int o = 32; o > 0; o >>= 1) {
      ymax_c = max(ymax_c, __shfl_xor(ymax_c, o, 64));
      ynx = min(ynx, __shfl_xor(ynx, o, 64));
    }
    const int wlo = y0 - R, whi = ymax_c + R;
    const int drop = (ynx == int(kNoY)) ? whi + 1 : ynx - R;   // cells below `drop` are never needed again

    // ---- C0 (no memory round): wave 1 advances the centre pointers and sizes
    // the next chunk's centre items; wave 0 sizes every source row's share
    // of this window (y grows by >= 1 per element; a coarse element covers
    // two cells); the other waves pad y outside the image
    if (wave == 1) {
      if (lane < uint32_t(NC)) {
        opd[lane] = op[lane];
        op[lane] += ocnt[lane];
        ocnt[lane] = 0;
      }
      wave_lds_sync();
      wave_scan_into<1>(opre[par ^ 1], NC, [&](int c) { return min(oe[c] - op[c], uint32_t(OCAP)); });
    } else if (wave == 0) {
      wave_scan_into<ES>(spre, NSRC, [&](int sr) -> uint32_t {
        if (sp[sr] >= se[sr]) return 0u;
        const int last = (sr >= 2 * NH) ? (whi >> 1) : whi;
        const int yfs = yfirst[sr];
        return (last >= yfs) ? min(uint32_t(last - yfs + 1), se[sr] - sp[sr]) : 0u;
      });
    } else if (wlo < 0 || whi >= Dy) {   // y outside the image is zero padding
      const int span = whi - wlo + 1;
      for (int j = tid - 128; j < NH * span; j += NT - 128) {
        const int h = j / span, p = j % span;
        const int yy = wlo + p;
        if (yy < 0 || yy >= Dy) patch[h * PY + p] = pad;
      }
    }
    lds_barrier();

    // ---- C (one memory round): reconstruct the level-l patch over [wlo, whi]
    const uint32_t ns = spre[NSRC];
    const uint32_t nsf = spre[2 * NH];   // items of APR-l and tree-l rows come first
    // fine sources: one patch cell per element
    for (uint32_t base = tid; base < nsf; base += NT * kBatch) {
      int ss[kBatch], yv[kBatch], yn[kBatch];
      uint32_t ii[kBatch], jj[kBatch];
      PT val[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const uint32_t it = base + u * NT;
        const bool ok = it < nsf;
        ss[u] = ok ? find_row(spre, NSRC, it) : 0;
        jj[u] = ok ? it - spre[ss[u]] : 0u;
        ii[u] = sp[ss[u]] + jj[u];
        const bool istree = ss[u] >= NH;
        const uint16_t* ys = istree ? ty : py;
        yv[u] = ok ? int(ys[ii[u]]) : kBig;
        // next element of the row, if it is one of this chunk's items
        const bool has_next = ok && jj[u] + 1 < spre[ss[u] + 1] - spre[ss[u]];
        yn[u] = has_next ? int(ys[ii[u] + 1]) : kBig;
        if constexpr (INDEX)
          val[u] = PT((int64_t(istree ? 3 : 1) << 40) | int64_t(ii[u]));
        else
          val[u] = ok ? to_f32<TX>((istree ? tv : xv)[ii[u]]) : 0.f;
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        if (base + u * NT >= nsf) continue;
        const int s = ss[u];
        if (yv[u] >= wlo && yv[u] <= whi) patch[(s >= NH ? s - NH : s) * PY + (yv[u] - wlo)] = val[u];
        // consumed elements are a prefix of the row's items: the last one
        // records the count
        if (yv[u] < drop && !(yn[u] < drop)) scons[s] = jj[u] + 1;
      }
    }
    // coarse sources (APR level l-1): each element covers 2 x 2 x 2 level-l
    // cells, in up to four halo rows
    for (uint32_t base = nsf + tid; base < ns; base += NT * kBatch) {
      int ss[kBatch], yv[kBatch], yn[kBatch];
      uint32_t ii[kBatch], jj[kBatch];
      PT val[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const uint32_t it = base + u * NT;
        const bool ok = it < ns;
        ss[u] = ok ? find_row(spre, NSRC, it) : 2 * NH;
        jj[u] = ok ? it - spre[ss[u]] : 0u;
        ii[u] = sp[ss[u]] + jj[u];
        yv[u] = ok ? int(py[ii[u]]) : kBig;
        const bool has_next = ok && jj[u] + 1 < spre[ss[u] + 1] - spre[ss[u]];
        yn[u] = has_next ? int(py[ii[u] + 1]) : kBig;
        if constexpr (INDEX)
          val[u] = PT((int64_t(2) << 40) | int64_t(ii[u]));
        else
          val[u] = ok ? to_f32<TX>(xv[ii[u]]) : 0.f;
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        if (base + u * NT >= ns) continue;
        const int s = ss[u];
        const int lo = 2 * yv[u];
        const int js = s - 2 * NH;
        const int msk = cmask[js], hb = cbase[js];
        const bool w0 = lo >= wlo && lo <= whi;
        const bool w1 = lo + 1 >= wlo && lo + 1 <= whi && lo + 1 < Dy;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (!((msk >> q) & 1)) continue;
          PT* row = patch + (hb + (q >> 1) * HX + (q & 1)) * PY - wlo;
          if (w0) row[lo] = val[u];
          if (w1) row[lo + 1] = val[u];
        }
        if (lo + 1 < drop && !(2 * yn[u] + 1 < drop)) scons[s] = jj[u] + 1;
      }
    }
    lds_barrier();

    // ---- D: accumulate the taps of every listed particle
    for (int s = tid; s < NSRC; s += NT) {
      sp[s] += scons[s];
      scons[s] = 0;
    }
    if (tid == 0) s_y0 = ynx;
    if (tid < NC) {   // every wave has read them before the last barrier
      rymax[tid] = -1;
      rnext[tid] = int(kNoY);
    }
    for (uint32_t jt = tid; jt < nb; jt += NT) {
      const int pos = o_pos[jt];
      if (pos == kUnlisted) continue;
      const int c = pos >> 6, p0 = (pos & 63) + R;
      const uint32_t idx = opd[c] + (jt - ocap[c]);
      const int hz = c / TX_, hx = c % TX_;   // halo row of the tap (-R, -R) is (hz, hx)
      if constexpr (INDEX) {
        if (a.map32) {
          // tap-major layout [k^3][N_p]: consecutive particles are adjacent
          int q = 0;
          for (int dz = 0; dz < K; ++dz)
            for (int dx = 0; dx < K; ++dx)
              for (int dy = 0; dy < K; ++dy) {
                const int64_t code = int64_t(patch[((hz + dz) * HX + hx + dx) * PY + p0 - R + dy]);
                a.map32[size_t(q++) * size_t(a.n_sel) + idx] =
                    code < 0 ? -1 : int32_t(((code >> 40) << 30) | (code & ((int64_t(1) << 30) - 1)));
              }
          continue;
        }
        int64_t lo = 0, hi = a.n_sel;
        while (lo < hi) {
          const int64_t mid = (lo + hi) >> 1;
          if (a.sel[mid] < int64_t(idx)) lo = mid + 1; else hi = mid;
        }
        if (lo < a.n_sel && a.sel[lo] == int64_t(idx)) {
          int64_t* dst = a.map + lo * K3;
          int q = 0;
          for (int dz = 0; dz < K; ++dz)
            for (int dx = 0; dx < K; ++dx)
              for (int dy = 0; dy < K; ++dy)
                dst[q++] = int64_t(patch[((hz + dz) * HX + hx + dx) * PY + p0 - R + dy]);
        }
      } else if constexpr (NF == 3) {
        float g0 = 0.f, g1 = 0.f, g2 = 0.f;
#pragma unroll 1
        for (int dz = 0; dz < K; ++dz) {
          cfloat* wz = wl + dz * K * K;
#pragma unroll
          for (int dx = 0; dx < K; ++dx) {
            const float* row = &patch[((hz + dz) * HX + hx + dx) * PY + p0 - R];
#pragma unroll
            for (int dy = 0; dy < K; ++dy) {
              const float v = row[dy];
              g0 = fmaf(wz[dx * K + dy], v, g0);
              g1 = fmaf(wz[K3 + dx * K + dy], v, g1);
              g2 = fmaf(wz[2 * K3 + dx * K + dy], v, g2);
            }
          }
        }
        static_cast<TY*>(a.y)[idx] = from_f32<TY>(sqrtf(fmaf(g0, g0, fmaf(g1, g1, g2 * g2))));
      } else {
        float acc = 0.f;
#pragma unroll 1
        for (int dz = 0; dz < K; ++dz) {
          cfloat* wz = wl + dz * K * K;
#pragma unroll
          for (int dx = 0; dx < K; ++dx) {
            const float* row = &patch[((hz + dz) * HX + hx + dx) * PY + p0 - R];
#pragma unroll
            for (int dy = 0; dy < K; ++dy) acc = fmaf(wz[dx * K + dy], row[dy], acc);
          }
        }
        TY* yo = static_cast<TY*>(a.y);
        if (a.epi == APR_EPI_RATIO) {
          const float u = to_f32<TY>(static_cast<const TY*>(a.epi_arg)[idx]);
          acc = u / fmaxf(acc, a.eps_dev ? *a.eps_dev : a.eps);
        } else if (a.epi == APR_EPI_MUL) {
          acc *= to_f32<TY>(static_cast<const TY*>(a.epi_arg)[idx]);
        } else if (a.epi == APR_EPI_MULPOW) {
          acc = to_f32<TY>(static_cast<const TY*>(a.epi_arg)[idx]) * powf(fmaxf(acc, 0.f), a.power);
        }
        yo[idx] = from_f32<TY>(acc);
      }
    }
    lds_barrier();
    par ^= 1;
  }
}

template <int K, bool INDEX>
static apr_status launch_conv(const ConvArgs& args, int xdt, int ydt, hipStream_t s) {
  int64_t per = 0;
  for (int x = 0; x < 8; ++x) per = std::max(per, args.xcd_off[x + 1] - args.xcd_off[x]);
  const dim3 grid(unsigned(per * 8));
  if (!INDEX && args.epi == APR_EPI_GRADMAG) {
    if (K != 3) APR_FAIL(APR_EUNSUPPORTED, "apr_conv: APR_EPI_GRADMAG needs k = 3");
    if (xdt == APR_F32 && ydt == APR_F32)
      hipLaunchKernelGGL((conv1_kernel<3, float, float, false, 3>), grid, dim3(ConvShape<3>::kThreads), 0, s, args);
    else if (xdt == APR_BF16 && ydt == APR_F32)
      hipLaunchKernelGGL((conv1_kernel<3, __hip_bfloat16, float, false, 3>), grid, dim3(ConvShape<3>::kThreads), 0, s,
                         args);
    else
      APR_FAIL(APR_EUNSUPPORTED, "apr_conv: APR_EPI_GRADMAG takes F32 or BF16 x and F32 y");
    APR_HIP(hipGetLastError());
    return APR_OK;
  }
  if (xdt == APR_F32 && ydt == APR_F32)
    hipLaunchKernelGGL((conv1_kernel<K, float, float, INDEX>), grid, dim3(ConvShape<K>::kThreads), 0, s, args);
  else if (xdt == APR_BF16 && ydt == APR_BF16)
    hipLaunchKernelGGL((conv1_kernel<K, __hip_bfloat16, __hip_bfloat16, INDEX>), grid, dim3(ConvShape<K>::kThreads), 0,
                       s, args);
  else if (xdt == APR_BF16 && ydt == APR_F32)
    hipLaunchKernelGGL((conv1_kernel<K, __hip_bfloat16, float, INDEX>), grid, dim3(ConvShape<K>::kThreads), 0, s, args);
  else
    APR_FAIL(APR_EUNSUPPORTED, "apr_conv: unsupported dtype combination");
  APR_HIP(hipGetLastError());
  return APR_OK;
}

static ConvArgs base_args(const apr_handle* h) {
  ConvArgs a{};
  a.m = h->meta;
  a.py = h->py;
  a.pend = h->pend;
  a.ty = h->ty;
  a.tend = h->tend;
  a.tiles = h->tiles;
  a.n_tiles = h->n_tiles;
  for (int x = 0; x <= 8; ++x) a.xcd_off[x] = h->xcd_off[x];
  a.n_wlevels = 1;
  return a;
}

}  // namespace apr

using namespace apr;

namespace apr {
apr_status conv_impl(const apr_handle* h, const apr_conv_desc* d, const void* x, const void* tree,
                     const float* w, void* y, const float* eps_dev, void* stream);
apr_status mc_conv(const apr_handle* h, const apr_conv_desc* d, const void* x, const void* tree,
                   const float* w, void* y, hipStream_t s);
}

extern "C" apr_status apr_conv(const apr_handle* h, const apr_conv_desc* d, const void* x,
                               const void* tree, const float* w, void* y, void* stream) {
  return apr::conv_impl(h, d, x, tree, w, y, nullptr, stream);
}

apr_status apr::conv_impl(const apr_handle* h, const apr_conv_desc* d, const void* x,
                          const void* tree, const float* w, void* y, const float* eps_dev,
                          void* stream) {
  if (!h || !d) APR_FAIL(APR_EINVAL, "apr_conv: null handle or descriptor");
  if (d->k != 3 && d->k != 5) APR_FAIL(APR_EUNSUPPORTED, "apr_conv: k must be 3 or 5");
  if (d->c_in < 1 || d->c_out < 1) APR_FAIL(APR_EINVAL, "apr_conv: channel counts must be >= 1");
  const int nl = h->meta.l_max - h->meta.l_min + 1;
  if (d->n_wlevels != 1 && d->n_wlevels != nl)
    APR_FAIL(APR_EINVAL, "apr_conv: n_wlevels must be 1 or l_max - l_min + 1");
  if (d->epilogue < APR_EPI_NONE || d->epilogue > APR_EPI_GRADMAG)
    APR_FAIL(APR_EINVAL, "apr_conv: unknown epilogue");
  if (h->n_p == 0 || h->n_tiles == 0) return APR_OK;
  if (!x || !w || !y || (h->n_t && !tree)) APR_FAIL(APR_EINVAL, "apr_conv: null buffer");
  if (d->epilogue != APR_EPI_NONE && d->epilogue != APR_EPI_GRADMAG && !d->epi_arg)
    APR_FAIL(APR_EINVAL, "apr_conv: null epi_arg");
  if (y == x || y == tree) APR_FAIL(APR_EINVAL, "apr_conv: y must not alias x or tree");
  if (d->c_in != 1 || d->c_out != 1 || d->bias || d->relu || d->residual) {
    if (d->epilogue != APR_EPI_NONE) APR_FAIL(APR_EUNSUPPORTED, "apr_conv: epilogues need c_in = c_out = 1");
    return mc_conv(h, d, x, tree, w, y, static_cast<hipStream_t>(stream));
  }
  ConvArgs a = base_args(h);
  a.x = x;
  a.tree = tree;
  a.w = w;
  a.n_wlevels = d->n_wlevels;
  a.y = y;
  a.epi = d->epilogue;
  a.eps = d->eps;
  a.eps_dev = eps_dev;
  a.power = d->power;
  a.epi_arg = d->epi_arg;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return d->k == 3 ? launch_conv<3, false>(a, d->x_dtype, d->y_dtype, s)
                   : launch_conv<5, false>(a, d->x_dtype, d->y_dtype, s);
}

extern "C" apr_status apr_neighbor_map(const apr_handle* h, int32_t k, const int64_t* particles,
                                       int64_t n, int64_t* out, void* stream) {
  if (!h) APR_FAIL(APR_EINVAL, "apr_neighbor_map: null handle");
  if (k != 3 && k != 5) APR_FAIL(APR_EUNSUPPORTED, "apr_neighbor_map: k must be 3 or 5");
  if (n < 0 || (n > 0 && (!particles || !out))) APR_FAIL(APR_EINVAL, "apr_neighbor_map: bad list");
  if (n == 0 || h->n_tiles == 0) return APR_OK;
  ConvArgs a = base_args(h);
  a.sel = particles;
  a.n_sel = n;
  a.map = out;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return k == 3 ? launch_conv<3, true>(a, APR_F32, APR_F32, s)
                : launch_conv<5, true>(a, APR_F32, APR_F32, s);
}

namespace apr {
// gather map of every particle for stencil side k, written by the
// convolution's own patch builder (int32 code: type << 30 | index, -1 pad;
// type 1 = APR level l, 2 = APR level l-1, 3 = tree level l)
apr_status build_gather_map(const apr_handle* h, int k, int32_t* map32, hipStream_t s) {
  if (h->n_tiles == 0) return APR_OK;
  ConvArgs a = base_args(h);
  a.map32 = map32;
  a.n_sel = h->n_p;
  return k == 3 ? launch_conv<3, true>(a, APR_F32, APR_F32, s) : launch_conv<5, true>(a, APR_F32, APR_F32, s);
}
}  // namespace apr
