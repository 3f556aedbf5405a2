// Single-channel APR convolution (Section 4.1), GPU design after Section 5.2,
// re-shaped for wave64 / CDNA4.
//
// Work item: one tile of 4 x 4 particle rows (z, x) at one level l, taken from
// the non-empty tile list.  The workgroup (4 waves) sweeps the tile along y in
// chunks: each chunk starts at the smallest unprocessed y of the tile's output
// particles (empty stretches of the rows are skipped) and covers at most 64
// cells.  Per chunk:
//   B. the output particles of the 16 centre rows with y in [y0, y0+64) are
//      listed in LDS (ballot + rank per wave, one shared counter);
//   C. the level-l patch of the halo rows is reconstructed in LDS over
//      [y0 - r, ymax + r] from three sorted sources, streamed with running
//      pointers and coalesced lane-per-element loads: APR level l, tree level
//      l (cells containing finer particles), APR level l-1 (each element
//      covers 2 x 2 x 2 level-l cells).  With 26-neighbour 2:1 balance these
//      sources cover every cell within radius 2 of a level-l particle;
//   D. every listed particle accumulates its k^3 taps from the patch in FP32
//      and writes its output.
// The blockIdx -> tile map gives each XCD a contiguous run of tiles so that
// halo rows shared by neighbouring tiles are re-read from the same L2.
#include <type_traits>

#include "common.hpp"

namespace apr {

constexpr int kYC = 64;          // output cells per chunk along y
constexpr int kBig = 1 << 28;    // y of a lane past the end of its row

struct ConvArgs {
  Meta m;
  const uint16_t* py;
  const uint32_t* pend;
  const uint16_t* ty;
  const uint32_t* tend;
  const uint64_t* tiles;
  int64_t n_tiles;
  const void* x;
  const void* tree;
  const float* w;
  int32_t n_wlevels;
  void* y;
  int32_t epi;
  float eps;
  const void* epi_arg;
  const int64_t* sel;   // neighbour-map mode: sorted particle list
  int64_t n_sel;
  int64_t* map;         // neighbour-map mode output [n_sel][k^3]
};

template <int K, typename TX, typename TY, bool INDEX>
__global__ __launch_bounds__(256) void conv1_kernel(ConvArgs a) {
  constexpr int R = K / 2;
  constexpr int HZ = kTileZ + 2 * R, HX = kTileX + 2 * R;
  constexpr int NH = HZ * HX;                        // halo rows at level l
  constexpr int PZ = ((kTileZ - 1 + R) >> 1) + 2;    // parent rows (level l-1)
  constexpr int PX = ((kTileX - 1 + R) >> 1) + 2;
  constexpr int NSRC = 2 * NH + PZ * PX;             // [0,NH) APR l, [NH,2NH) tree l, rest APR l-1
  constexpr int NC = kTileZ * kTileX;                // centre (output) rows
  constexpr int PY = kYC + 2 * R;
  constexpr int K3 = K * K * K;
  using PT = typename std::conditional<INDEX, long long, float>::type;
  static_assert(PY <= 128, "patch position packs into 7 bits");

  __shared__ PT patch[NH][PY];
  __shared__ uint32_t sp[NSRC], se[NSRC];
  __shared__ uint32_t op[NC], oe[NC];
  __shared__ uint32_t o_idx[NC * kYC];
  __shared__ uint16_t o_pos[NC * kYC];
  __shared__ float wsh[K3];
  __shared__ int s_y0[2], s_n[2], s_ymax[2];

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const uint32_t lane = lane_id();

  // XCD-aware tile order: block b runs on XCD b % 8; give each XCD a
  // contiguous range of tiles.
  const int64_t per = (a.n_tiles + 7) / 8;
  const int64_t t = int64_t(blockIdx.x % 8) * per + int64_t(blockIdx.x / 8);
  if (t >= a.n_tiles) return;
  int l, tz, tx;
  tile_unpack(a.tiles[t], l, tz, tx);
  const Meta& m = a.m;
  const int z0 = tz * kTileZ, x0 = tx * kTileX;
  const int Dz = m.dz[l], Dx = m.dx[l], Dy = m.dy[l];
  const bool has_c = l > m.l_min;
  const bool has_t = l <= m.t_hi;
  const TX* __restrict__ xv = static_cast<const TX*>(a.x);
  const TX* __restrict__ tv = static_cast<const TX*>(a.tree);

  if constexpr (!INDEX) {
    const float* wl = a.w + (a.n_wlevels == 1 ? 0 : (l - m.l_min)) * K3;
    for (int i = tid; i < K3; i += 256) wsh[i] = wl[i];
  }
  const PT pad = INDEX ? PT(-1) : PT(0);
  for (int i = tid; i < NH * PY; i += 256) (&patch[0][0])[i] = pad;
  for (int s = tid; s < NSRC; s += 256) {
    uint32_t b = 0, e = 0;
    if (s < 2 * NH) {
      const int h = s < NH ? s : s - NH;
      const int z = z0 - R + h / HX, x = x0 - R + h % HX;
      const bool in = z >= 0 && x >= 0 && z < Dz && x < Dx;
      if (in && s < NH) row_range(a.pend, m.prow[l] + uint32_t(z) * Dx + x, b, e);
      if (in && s >= NH && has_t) row_range(a.tend, m.trow[l] + uint32_t(z) * Dx + x, b, e);
    } else if (has_c) {
      const int j = s - 2 * NH;
      const int pz = z0 / 2 - 1 + j / PX, px = x0 / 2 - 1 + j % PX;
      if (pz >= 0 && px >= 0 && pz < m.dz[l - 1] && px < m.dx[l - 1])
        row_range(a.pend, m.prow[l - 1] + uint32_t(pz) * m.dx[l - 1] + px, b, e);
    }
    sp[s] = b;
    se[s] = e;
  }
  for (int c = tid; c < NC; c += 256) {
    uint32_t b = 0, e = 0;
    const int z = z0 + c / kTileX, x = x0 + c % kTileX;
    if (z < Dz && x < Dx) row_range(a.pend, m.prow[l] + uint32_t(z) * Dx + x, b, e);
    op[c] = b;
    oe[c] = e;
  }
  if (tid == 0) {
    s_y0[0] = s_y0[1] = int(kNoY);
    s_n[0] = s_n[1] = 0;
    s_ymax[0] = s_ymax[1] = -1;
  }
  __syncthreads();
  for (int c = tid; c < NC; c += 256)
    if (op[c] < oe[c]) atomicMin(&s_y0[0], int(a.py[op[c]]));
  __syncthreads();

  int par = 0;
  while (true) {
    const int y0 = s_y0[par];
    if (y0 == int(kNoY)) break;

    // ---- B: list the outputs of this chunk
    for (int c = wave; c < NC; c += 4) {
      uint32_t base = op[c];
      const uint32_t end = oe[c];
      if (base >= end) continue;
      int ymx = -1, ynext = int(kNoY);
      while (true) {
        const uint32_t i = base + lane;
        const bool v = i < end;
        const int yv = v ? int(a.py[i]) : kBig;
        const bool in = v && yv < y0 + kYC;
        const uint64_t mk = ballot(in);
        const uint32_t cnt = __popcll(mk);
        if (cnt) {
          int slot0 = 0;
          if (lane == 0) slot0 = atomicAdd(&s_n[par], int(cnt));
          slot0 = __shfl(slot0, 0, 64);
          if (in) {
            const int q = slot0 + int(mask_rank(mk));
            o_idx[q] = i;
            o_pos[q] = uint16_t((c << 7) | (yv - y0 + R));
          }
          ymx = __shfl(yv, int(cnt) - 1, 64);
        }
        if (cnt == 64 && base + 64 < end) {
          base += 64;
          continue;
        }
        const int nxt = __shfl(yv, int(cnt & 63), 64);
        base += cnt;
        ynext = (base < end) ? nxt : int(kNoY);
        break;
      }
      if (lane == 0) {
        op[c] = base;
        if (ynext != int(kNoY)) atomicMin(&s_y0[par ^ 1], ynext);
        if (ymx >= 0) atomicMax(&s_ymax[par], ymx);
      }
    }
    __syncthreads();
    const int nout = s_n[par];
    const int ymax = s_ymax[par];
    const int ynx = s_y0[par ^ 1];
    const int wlo = y0 - R, whi = ymax + R;
    const int drop = (ynx == int(kNoY)) ? whi + 1 : ynx - R;   // cells below `drop` are never needed again

    // ---- C: reconstruct the level-l patch over [wlo, whi]
    for (int s = wave; s < NSRC; s += 4) {
      uint32_t base = sp[s];
      const uint32_t end = se[s];
      if (base >= end) continue;
      const bool coarse = s >= 2 * NH;
      const bool istree = s >= NH && !coarse;
      const uint16_t* __restrict__ ys = istree ? a.ty : a.py;
      uint32_t consumed = 0;
      while (true) {
        const uint32_t i = base + lane;
        const bool v = i < end;
        const int yv = v ? int(ys[i]) : kBig;
        const int lo = coarse ? 2 * yv : yv;
        const int hi = coarse ? 2 * yv + 1 : yv;
        if (v && hi >= wlo && lo <= whi) {
          PT val;
          if constexpr (INDEX)
            val = PT((int64_t(coarse ? 2 : (istree ? 3 : 1)) << 40) | int64_t(i));
          else
            val = to_f32<TX>(istree ? tv[i] : xv[i]);
          if (!coarse) {
            patch[s - (istree ? NH : 0)][yv - wlo] = val;
          } else {
            const int j = s - 2 * NH;
            const int hz0 = 2 * (j / PX) + R - 2, hx0 = 2 * (j % PX) + R - 2;
#pragma unroll
            for (int dz = 0; dz < 2; ++dz)
#pragma unroll
              for (int dx = 0; dx < 2; ++dx) {
                const int hz = hz0 + dz, hx = hx0 + dx;
                if (hz < 0 || hx < 0 || hz >= HZ || hx >= HX) continue;
                // a coarse cell on the far edge of an odd-sized grid covers
                // level-l cells outside the image: those stay zero padding
                if (z0 - R + hz >= Dz || x0 - R + hx >= Dx) continue;
                if (lo >= wlo) patch[hz * HX + hx][lo - wlo] = val;
                if (hi <= whi && hi < Dy) patch[hz * HX + hx][hi - wlo] = val;
              }
          }
        }
        consumed += __popcll(ballot(v && hi < drop));
        const bool v63 = base + 63 < end;
        const int lo63 = __shfl(lo, 63, 64), hi63 = __shfl(hi, 63, 64);
        if (v63 && (lo63 <= whi || hi63 < drop)) {
          base += 64;
          continue;
        }
        break;
      }
      if (lane == 0) sp[s] += consumed;
    }
    if (wlo < 0 || whi >= Dy) {
      const int span = whi - wlo + 1;
      for (int j = tid; j < NH * span; j += 256) {
        const int h = j / span, p = j % span;
        const int yy = wlo + p;
        if (yy < 0 || yy >= Dy) patch[h][p] = pad;
      }
    }
    __syncthreads();

    // ---- D: accumulate the taps of every listed particle
    if (tid == 0) {
      s_y0[par] = int(kNoY);
      s_n[par] = 0;
      s_ymax[par] = -1;
    }
    for (int j = tid; j < nout; j += 256) {
      const uint32_t idx = o_idx[j];
      const int pos = o_pos[j];
      const int c = pos >> 7, p0 = pos & 127;
      const int hz = c / kTileX, hx = c % kTileX;   // halo row of the tap (-R,-R) is (hz, hx)
      if constexpr (INDEX) {
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
                dst[q++] = int64_t(patch[(hz + dz) * HX + hx + dx][p0 - R + dy]);
        }
      } else {
        float acc = 0.f;
        int q = 0;
#pragma unroll
        for (int dz = 0; dz < K; ++dz)
#pragma unroll
          for (int dx = 0; dx < K; ++dx) {
            const float* row = &patch[(hz + dz) * HX + hx + dx][p0 - R];
#pragma unroll
            for (int dy = 0; dy < K; ++dy) acc = fmaf(wsh[q++], row[dy], acc);
          }
        TY* yo = static_cast<TY*>(a.y);
        if (a.epi == APR_EPI_RATIO) {
          const float u = to_f32<TY>(static_cast<const TY*>(a.epi_arg)[idx]);
          acc = u / fmaxf(acc, a.eps);
        } else if (a.epi == APR_EPI_MUL) {
          acc *= to_f32<TY>(static_cast<const TY*>(a.epi_arg)[idx]);
        }
        yo[idx] = from_f32<TY>(acc);
      }
    }
    __syncthreads();
    par ^= 1;
  }
}

template <int K, bool INDEX>
static apr_status launch_conv(const ConvArgs& args, int xdt, int ydt, hipStream_t s) {
  const int64_t per = (args.n_tiles + 7) / 8;
  const dim3 grid(unsigned(per * 8));
  if (xdt == APR_F32 && ydt == APR_F32)
    hipLaunchKernelGGL((conv1_kernel<K, float, float, INDEX>), grid, dim3(256), 0, s, args);
  else if (xdt == APR_BF16 && ydt == APR_BF16)
    hipLaunchKernelGGL((conv1_kernel<K, __hip_bfloat16, __hip_bfloat16, INDEX>), grid, dim3(256), 0,
                       s, args);
  else if (xdt == APR_BF16 && ydt == APR_F32)
    hipLaunchKernelGGL((conv1_kernel<K, __hip_bfloat16, float, INDEX>), grid, dim3(256), 0, s, args);
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
  a.n_wlevels = 1;
  return a;
}

}  // namespace apr

using namespace apr;

extern "C" apr_status apr_conv(const apr_handle* h, const apr_conv_desc* d, const void* x,
                               const void* tree, const float* w, void* y, void* stream) {
  if (!h || !d) APR_FAIL(APR_EINVAL, "apr_conv: null handle or descriptor");
  if (d->k != 3 && d->k != 5) APR_FAIL(APR_EUNSUPPORTED, "apr_conv: k must be 3 or 5");
  if (d->c_in != 1 || d->c_out != 1)
    APR_FAIL(APR_EUNSUPPORTED, "apr_conv: this build supports c_in = c_out = 1");
  const int nl = h->meta.l_max - h->meta.l_min + 1;
  if (d->n_wlevels != 1 && d->n_wlevels != nl)
    APR_FAIL(APR_EINVAL, "apr_conv: n_wlevels must be 1 or l_max - l_min + 1");
  if (d->epilogue < APR_EPI_NONE || d->epilogue > APR_EPI_MUL)
    APR_FAIL(APR_EINVAL, "apr_conv: unknown epilogue");
  if (h->n_p == 0 || h->n_tiles == 0) return APR_OK;
  if (!x || !w || !y || (h->n_t && !tree)) APR_FAIL(APR_EINVAL, "apr_conv: null buffer");
  if (d->epilogue != APR_EPI_NONE && !d->epi_arg) APR_FAIL(APR_EINVAL, "apr_conv: null epi_arg");
  if (y == x || y == tree) APR_FAIL(APR_EINVAL, "apr_conv: y must not alias x or tree");
  ConvArgs a = base_args(h);
  a.x = x;
  a.tree = tree;
  a.w = w;
  a.n_wlevels = d->n_wlevels;
  a.y = y;
  a.epi = d->epilogue;
  a.eps = d->eps;
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
