// Single-channel APR convolution (Section 4.1), GPU design after Section 5.2,
// re-shaped for wave64 / CDNA4.
//
// Work item: a run of the y windows of one tile of kTileZ x kTileX particle
// rows (z, x) at one level l, from the non-empty tile list (the pre-pass of
// Section 5.2).  The windows are made at access build: runs of the tile's
// output y spanning at most kWinY cells (empty stretches are skipped, the
// per-block y-range of Section 5.2); a long sweep is cut into several items.
// A workgroup sweeps its item's windows in y order.
//
// The level-l patch of a window covers the halo rows of the tile over
// [y0 - r, y1 + r] and is reconstructed in LDS from three sorted sources:
// APR level l, tree level l (cells that contain finer particles) and APR
// level l-1 (each element covers 2 x 2 x 2 level-l cells).  With 26-neighbour
// 2:1 balance these cover every cell within radius 2 of a level-l particle.
// Each source row is owned for the whole sweep by a group of lanes that keeps
// the row's cursor in registers and moves a batch of consecutive elements per
// memory round (coalesced, no searches); the first batch of the next window
// is loaded while the current window's taps run.  A row whose cursor falls
// far behind the window is advanced by a k-ary search, one probe per lane.
// Centre-row particles of the window are appended to an output list (one LDS
// atomic per wave), and every listed particle then accumulates its k^3 taps
// from the patch in FP32 with the weights in scalar registers.  Two barriers
// per window; barriers order LDS only (outputs are never read back, so stores
// stay in flight).
#include <algorithm>
#include <type_traits>

#include "common.hpp"

namespace apr {

constexpr int kBig = 1 << 28;    // key of a missing element
// Launch shape per stencil size: 3^3 in 1024-thread workgroups capped at 64
// registers (two per CU, eight waves per SIMD), 5^3 and 7^3 in 768-thread
// workgroups capped at 80 (two per CU, six waves per SIMD; 5^3 spills at 64,
// 9^3 at 80), 9^3 to 13^3 in 1024-thread workgroups at four waves per SIMD.
// Stencils above 5^3 sweep patches of at most 32 output cells (16: 15-34%
// slower).  Source rows are
// served by groups of kG lanes; each group moves kG * kNB elements of its row
// per memory round.  A
// patch holds output y spans of at most kW cells.  Within radius r of a
// level-l particle, 26-neighbour 2:1 balance admits particles of level l - j
// only at distances of at least 2^j - 1 cells, so stencils up to 5^3 read APR
// levels l and l-1 (and tree level l), stencils up to 13^3 also level l-2.
template <int K>
struct ConvShape {
  static_assert(K % 2 == 1 && K >= 3 && K <= 13, "odd stencil sides 3..13");
  static constexpr bool kLarge = K > 5;
  static constexpr int kThreads = (kLarge && K > 7) || K == 3 ? 1024 : 768;
  static constexpr int kG = 8;
  static constexpr int kNB = kLarge ? 1 : 2;
  static constexpr int kWavesPerSimd = kLarge && K > 7 ? 4 : K == 3 ? 8 : 6;
  static constexpr int kW = kLarge ? 32 : kWinY;
  static constexpr int kDepth = kLarge ? 2 : 1;   // coarsest APR source level: l - kDepth
  // patch row stride (floats): the y span plus the halo, padded up to 8 mod 32
  // words up to 5^3, which spreads the rows of a wave's reads and writes over
  // the LDS banks (measured: 3% and 4% faster 3^3 and 5^3 than unpadded)
  static constexpr int kPY = kLarge ? kW + 2 * (K / 2) : (kW + 2 * (K / 2) + 23) / 32 * 32 + 8;
};

struct ConvArgs {
  Meta m;
  const uint16_t* py;
  const uint32_t* pend;
  const uint16_t* ty;
  const uint32_t* tend;
  const uint64_t* tiles;
  const uint32_t* wins;      // sweep windows: y0 | (y1 << 16), outputs y0 <= y <= y1
  const uint32_t* items;     // work item i at items[4 i]: tile code (2 words), windows [first, end)
  int64_t n_tiles;
  int64_t xcd_off[9];     // work items of XCD x: [xcd_off[x], xcd_off[x + 1])
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

// the G bits of lane group `gbase / G` in a wave ballot
template <int G>
__device__ inline uint32_t group_bits(uint64_t bal, uint32_t gbase) {
  static_assert(G <= 16, "group masks are 32-bit");
  return uint32_t(bal >> gbase) & ((1u << G) - 1u);
}

// LDS of one workgroup of the K^3 launch
template <int K, bool INDEX>
struct ConvLds {
  static constexpr int R = K / 2, W = ConvShape<K>::kW;
  static constexpr int NH = (kTileZ + 2 * R) * (kTileX + 2 * R);
  static constexpr int PY = ConvShape<K>::kPY, NC = kTileZ * kTileX;
  using PT = typename std::conditional<INDEX, long long, float>::type;
  PT patch[NH * PY];
  uint32_t o_idx[NC * W];   // listed outputs of the patch: particle index
  uint16_t o_pos[NC * W];   // (centre row << 6) | (y - y0)
  uint32_t cnt[2];          // outputs listed, per window parity
};

// One work item: windows [w_beg, w_end) of tile (l, tz, tx), with the K^3
// stencil read as the central K^3 of each level's KW^3 weights.  The LDS
// buffers belong to a launch whose K is at least this K.
// NF = 3: three stencils per level on the same patch (the three directions of
// a gradient filter), output the magnitude sqrt(sum of squares).
template <int K, int KW, typename TX, typename TY, bool INDEX, int NF, int NT, typename PT>
__device__ __forceinline__ void conv_item(const ConvArgs& a, int l, int tz, int tx, uint32_t w_beg, uint32_t w_end,
                                          PT* __restrict__ patch, uint32_t* __restrict__ o_idx,
                                          uint16_t* __restrict__ o_pos, uint32_t* __restrict__ s_cnt) {
  constexpr int G = ConvShape<K>::kG, NB = ConvShape<K>::kNB, GB = G * NB;
  constexpr int NG = NT / G;                         // lane groups
  constexpr int R = K / 2;
  constexpr int TZ = kTileZ, TXr = kTileX;
  constexpr int HZ = TZ + 2 * R, HX = TXr + 2 * R;
  constexpr int NH = HZ * HX;                        // halo rows at level l
  constexpr int W = ConvShape<K>::kW, D = ConvShape<K>::kDepth;
  // rows of APR level l-j covering the halo: per axis from tile origin / 2^j
  // - CRj on (the tile origin is a multiple of 8)
  constexpr int CR1 = (R + 1) / 2, CR2 = (R + 3) / 4;
  constexpr int P1 = ((TXr - 1 + R) >> 1) + CR1 + 1;
  constexpr int P2 = D >= 2 ? ((TXr - 1 + R) >> 2) + CR2 + 1 : 0;
  constexpr int NCR1 = P1 * P1, NCR2 = P2 * P2;
  // source rows: [0,NH) APR l, [NH,2NH) tree l, then APR l-1, then APR l-2
  constexpr int NSRC = 2 * NH + NCR1 + NCR2;
  constexpr int RPG = (NSRC + NG - 1) / NG;          // source rows per group
  constexpr int NC = TZ * TXr;                       // centre (output) rows
  constexpr int PY = ConvShape<K>::kPY;
  constexpr int K3 = K * K * K;
  constexpr int KW3 = KW * KW * KW, WO = (KW - K) / 2;   // weight set size, offset of the central K^3
  constexpr uint32_t kNone = 0xffffffffu;
  constexpr int kUnknown = -1;                       // y at the cursor not yet read
  static_assert(std::is_same<PT, typename std::conditional<INDEX, long long, float>::type>::value, "patch type");
  static_assert(NC <= 64 && W <= 64 && TZ == TXr, "output positions pack into 12 bits");
  static_assert(64 % G == 0 && GB <= 32, "lane groups tile a wave; batch masks are 32-bit");
  static_assert(KW >= K && (KW - K) % 2 == 0 && (KW == K || (!INDEX && NF == 1)), "central sub-stencil");

  const int tid = threadIdx.x;
  const uint32_t lane = lane_id();
  const uint32_t gbase = lane & ~uint32_t(G - 1);   // first lane of this lane's group
  const int gj = int(lane) - int(gbase);            // lane within the group
  const int grp = tid / G;

  const Meta& m = a.m;
  const int z0 = tz * TZ, x0 = tx * TXr;
  const int Dz = m.dz[l], Dx = m.dx[l], Dy = m.dy[l];
  const bool has_t = l <= m.t_hi;
  const TX* __restrict__ xv = static_cast<const TX*>(a.x);
  const TX* __restrict__ tv = static_cast<const TX*>(a.tree);
  const uint16_t* __restrict__ py = a.py;
  const uint16_t* __restrict__ ty = a.ty;
  using cfloat = const __attribute__((address_space(4))) float;
  cfloat* wl = (cfloat*)(uintptr_t)(INDEX ? a.w
                                           : a.w + (a.n_wlevels == 1 ? 0 : (l - m.l_min)) * KW3 * NF +
                                                 (WO * KW + WO) * KW + WO);
  const PT pad = INDEX ? PT(-1) : PT(0);

  // ---- setup: each group owns source rows s = grp + r * NG for the whole
  // sweep.  Per row, in registers: the cursor (first element a later window
  // may need), the end, the y at the cursor when known, and the first batch
  // of the next window, loaded one window ahead.
  uint32_t cur[RPG], end[RPG];
  int ny[RPG];
  bool act[RPG];
  int pfy[RPG][NB];
  PT pfv[RPG][NB];
#pragma unroll
  for (int r = 0; r < RPG; ++r) {
    const int s = grp + r * NG;
    uint32_t b = 0, e = 0;
    if (s < 2 * NH) {
      const int h = s < NH ? s : s - NH;
      const int z = z0 - R + h / HX, x = x0 - R + h % HX;
      const bool in = z >= 0 && x >= 0 && z < Dz && x < Dx;
      if (in && s < NH) row_range(a.pend, m.prow[l] + uint32_t(z) * Dx + x, b, e);
      if (in && s >= NH && has_t) row_range(a.tend, m.trow[l] + uint32_t(z) * Dx + x, b, e);
    } else if (s < NSRC) {
      const int dep = s < 2 * NH + NCR1 ? 1 : 2;
      const int j = dep == 1 ? s - 2 * NH : s - 2 * NH - NCR1;
      const int P = dep == 1 ? P1 : P2, CR = dep == 1 ? CR1 : CR2;
      const int lc = l - dep;
      if (lc >= m.l_min) {
        const int pz = (z0 >> dep) - CR + j / P, px = (x0 >> dep) - CR + j % P;
        if (pz >= 0 && px >= 0 && pz < m.dz[lc] && px < m.dx[lc])
          row_range(a.pend, m.prow[lc] + uint32_t(pz) * m.dx[lc] + px, b, e);
      }
    }
    cur[r] = b;
    end[r] = e;
    ny[r] = kUnknown;
    act[r] = b < e;
  }
  // the first window's batches
#pragma unroll
  for (int r = 0; r < RPG; ++r) {
    const int s = grp + r * NG;
    const bool istree = s >= NH && s < 2 * NH;
    const uint16_t* __restrict__ ys = istree ? ty : py;
    const TX* __restrict__ vs = istree ? tv : xv;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const uint32_t i = cur[r] + uint32_t(u * G + gj);
      const bool ok = act[r] && i < end[r];
      pfy[r][u] = ok ? int(ys[i]) : kBig;
      if constexpr (INDEX)
        pfv[r][u] = PT((int64_t(s >= 2 * NH ? 2 : (istree ? 3 : 1)) << 40) | int64_t(i));
      else
        pfv[r][u] = ok ? to_f32<TX>(vs[i]) : 0.f;
    }
  }
  // halo rows outside the level-l grid are zero padding for the whole sweep
  // (no source ever writes them); other cells are written before use
  for (int i = tid; i < NH * PY; i += NT) {
    const int h = i / PY;
    const int z = z0 - R + h / HX, x = x0 - R + h % HX;
    if (z < 0 || x < 0 || z >= Dz || x >= Dx) patch[i] = pad;
  }
  if (tid < 2) s_cnt[tid] = 0;
  lds_barrier();

  // patches: each window of the tile in spans of at most W output cells
  int par = 0;
  uint32_t wi = w_beg;
  uint32_t wcur = a.wins[w_beg];
  int y0 = int(wcur & 0xffffu), y1 = min(int(wcur >> 16), y0 + W - 1);
  while (true) {
    const int wlo = y0 - R, whi = y1 + R;
    int ny0 = 0, ny1 = -1;
    bool has_next = true;
    if (y1 < int(wcur >> 16)) {
      ny0 = y1 + 1;
      ny1 = min(int(wcur >> 16), ny0 + W - 1);
    } else if (wi + 1 < w_end) {
      const uint32_t wn = a.wins[wi + 1];
      ny0 = int(wn & 0xffffu);
      ny1 = min(int(wn >> 16), ny0 + W - 1);
    } else {
      has_next = false;
    }
    const int nwlo = ny0 - R, nwhi = ny1 + R;

    // ---- sources: every element of the group's rows that covers a cell of
    // [wlo, whi] is written into the level-l patch; centre-row particles in
    // [y0, y1] are listed as outputs
#pragma unroll
    for (int r = 0; r < RPG; ++r) {
      const int s = grp + r * NG;
      const uint32_t e = end[r];
      // the kinds of row slot r can hold (constants after unrolling: the
      // code for the others is dropped)
      const bool r_apr = r * NG < NH, r_tree = r * NG < 2 * NH && (r + 1) * NG > NH;
      const bool r_coarse = (r + 1) * NG > 2 * NH;
      // element y covers cells [y << sh, ((y + 1) << sh) - 1]
      const int sh = !r_coarse || s < 2 * NH ? 0 : (D == 1 || s < 2 * NH + NCR1 ? 1 : 2);
      const bool coarse = sh > 0;
      if (s < NSRC && act[r]) {         // uniform per group
        const bool istree = r_tree && s >= NH && !coarse;
        const uint16_t* __restrict__ ys = istree ? ty : py;
        const TX* __restrict__ vs = istree ? tv : xv;
        const int h = s < NH ? s : s - NH;
        const bool centre =
            r_apr && s < NH && h / HX >= R && h / HX < R + TZ && h % HX >= R && h % HX < R + TXr;
        const int c = (h / HX - R) * TXr + (h % HX - R);
        // coarse row: its element covers 2^sh x 2^sh halo rows from hb (mask
        // of the ones inside the halo and the level-l grid)
        int hb = 0, msk = 0;
        if (D == 1 && coarse) {
          const int j = s - 2 * NH;
          const int hz0 = 2 * (j / P1 - CR1) + R, hx0 = 2 * (j % P1 - CR1) + R;
          hb = hz0 * HX + hx0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int hz = hz0 + (q >> 1), hx = hx0 + (q & 1);
            if (hz >= 0 && hx >= 0 && hz < HZ && hx < HX && z0 - R + hz < Dz && x0 - R + hx < Dx) msk |= 1 << q;
          }
        } else if (coarse) {
          const int j = sh == 1 ? s - 2 * NH : s - 2 * NH - NCR1;
          const int P = sh == 1 ? P1 : P2, CR = sh == 1 ? CR1 : CR2, n = 1 << sh;
          const int hz0 = n * (j / P - CR) + R, hx0 = n * (j % P - CR) + R;
          hb = hz0 * HX + hx0;
          for (int q = 0; q < n * n; ++q) {
            const int hz = hz0 + q / n, hx = hx0 + q % n;
            if (hz >= 0 && hx >= 0 && hz < HZ && hx < HX && z0 - R + hz < Dz && x0 - R + hx < Dx) msk |= 1 << q;
          }
        }
        uint32_t b = cur[r];
        uint32_t keep = kNone;
        int keep_y = kUnknown;
        int yv[NB];
        PT val[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
          yv[u] = pfy[r][u];
          val[u] = pfv[r][u];
        }
        bool more = true, loaded = true;
        while (more) {
          if (!loaded) {
#pragma unroll
            for (int u = 0; u < NB; ++u) {
              const uint32_t i = b + uint32_t(u * G + gj);
              const bool ok = i < e;
              yv[u] = ok ? int(ys[i]) : kBig;
              if constexpr (INDEX)
                val[u] = PT((int64_t(coarse ? 2 : (istree ? 3 : 1)) << 40) | int64_t(i));
              else
                val[u] = ok ? to_f32<TX>(vs[i]) : 0.f;
            }
          }
          loaded = false;
          uint32_t below = 0;
#pragma unroll
          for (int u = 0; u < NB; ++u)
            below |= group_bits<G>(ballot(((yv[u] + 1) << sh) - 1 < wlo), gbase) << (u * G);
          if (below == (1u << GB) - 1u && b + GB < e) {
            // the whole batch lies before the window: k-ary search of
            // [b + GB, e) for the first element covering a cell >= wlo
            uint32_t lo = b + GB, hi = e;
            while (hi - lo > uint32_t(GB)) {
              const uint32_t span = hi - lo;
              uint32_t bl = 0;
#pragma unroll
              for (int u = 0; u < NB; ++u) {
                const uint32_t k = uint32_t(u * G + gj);
                const uint32_t i = lo + span * (k + 1) / (GB + 1);
                bl |= group_bits<G>(ballot(((int(ys[i]) + 1) << sh) - 1 < wlo), gbase) << (u * G);
              }
              const uint32_t n = __builtin_popcount(bl);   // probes below form a prefix
              const uint32_t nlo = n ? lo + span * n / (GB + 1) + 1 : lo;
              if (n < uint32_t(GB)) hi = lo + span * (n + 1) / (GB + 1);
              lo = nlo;
            }
            b = lo;
            continue;
          }
          // write the covered cells of the window; list outputs
          bool isout[NB];
          uint32_t nout = 0;
          uint64_t ob[NB];
#pragma unroll
          for (int u = 0; u < NB; ++u) {
            const int y = yv[u];
            const bool ok = y != kBig;
            if (ok && (y << sh) <= whi && ((y + 1) << sh) - 1 >= wlo) {
              if (!coarse) {
                patch[h * PY + (y - wlo)] = val[u];
              } else if (D == 1 || sh == 1) {
                const int c0 = 2 * y;
                const bool w0 = c0 >= wlo, w1 = c0 + 1 <= whi && c0 + 1 < Dy;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  if (!((msk >> q) & 1)) continue;
                  PT* row = patch + (hb + (q >> 1) * HX + (q & 1)) * PY - wlo;
                  if (w0) row[c0] = val[u];
                  if (w1) row[c0 + 1] = val[u];
                }
              } else if constexpr (D >= 2) {
                const int c0 = 4 * y;
                for (int q = 0; q < 16; ++q) {
                  if (!((msk >> q) & 1)) continue;
                  PT* row = patch + (hb + (q >> 2) * HX + (q & 3)) * PY - wlo;
#pragma unroll
                  for (int tq = 0; tq < 4; ++tq) {
                    const int cc = c0 + tq;
                    if (cc >= wlo && cc <= whi && cc < Dy) row[cc] = val[u];
                  }
                }
              }
            }
            isout[u] = centre && y >= y0 && y <= y1;
            ob[u] = ballot(isout[u]);
            nout += __builtin_popcountll(ob[u]);
            // the next window's cursor: first element covering a cell >= its wlo
            if (has_next) {
              const uint32_t kb = group_bits<G>(ballot(ok && ((y + 1) << sh) - 1 >= nwlo), gbase);
              if (keep == kNone && kb) {
                keep = b + uint32_t(u * G) + uint32_t(__builtin_ctz(kb));
                keep_y = __shfl(y, int(gbase) + __builtin_ctz(kb), 64);
              }
            }
          }
          if (nout) {   // uniform across the wave's active lanes
            uint64_t all = 0;
#pragma unroll
            for (int u = 0; u < NB; ++u) all |= ob[u];
            const int leader = __builtin_ctzll(all);
            uint32_t base = 0;
            if (int(lane) == leader) base = atomicAdd(&s_cnt[par], nout);
            base = uint32_t(__shfl(int(base), leader, 64));
#pragma unroll
            for (int u = 0; u < NB; ++u) {
              if (isout[u]) {
                const uint32_t slot = base + mask_rank(ob[u]);
                o_idx[slot] = b + uint32_t(u * G + gj);
                o_pos[slot] = uint16_t((c << 6) | (yv[u] - y0));
              }
              base += __builtin_popcountll(ob[u]);
            }
          }
          // another batch if the row continues into the window
          const int ylast = __shfl(yv[NB - 1], int(gbase) + G - 1, 64);
          more = b + GB < e && ((ylast + 1) << sh) <= whi;
          b += GB;
        }
        if (keep != kNone) {
          cur[r] = keep;
          ny[r] = keep_y;
        } else {
          cur[r] = min(b, e);
          ny[r] = kUnknown;
        }
      }
      // is the row needed by the next window; if so, its first batch
      if (s < NSRC) {
        act[r] = has_next && cur[r] < e && (ny[r] == kUnknown || (ny[r] << sh) <= nwhi);
        const bool istree = r_tree && s >= NH && !coarse;
        const uint16_t* __restrict__ ys = istree ? ty : py;
        const TX* __restrict__ vs = istree ? tv : xv;
        if (act[r]) {
#pragma unroll
          for (int u = 0; u < NB; ++u) {
            const uint32_t i = cur[r] + uint32_t(u * G + gj);
            const bool ok = i < e;
            pfy[r][u] = ok ? int(ys[i]) : kBig;
            if constexpr (INDEX)
              pfv[r][u] = PT((int64_t(coarse ? 2 : (istree ? 3 : 1)) << 40) | int64_t(i));
            else
              pfv[r][u] = ok ? to_f32<TX>(vs[i]) : 0.f;
          }
        }
      }
    }
    // y outside the image is zero padding
    if (wlo < 0 || whi >= Dy) {
      for (int i = tid; i < NH * PY; i += NT) {
        const int yy = wlo + i % PY;
        if (yy < 0 || yy >= Dy) patch[i] = pad;
      }
    }
    lds_barrier();

    if (tid == 0) s_cnt[par ^ 1] = 0;   // read last in the previous window's tap phase
    const uint32_t nb = s_cnt[par];

    // ---- taps of every listed output
    for (uint32_t jt = tid; jt < nb; jt += NT) {
      const int pos = o_pos[jt];
      const uint32_t idx = o_idx[jt];
      const int c = pos >> 6, p0 = pos & 63;
      const int hz = c / TXr, hx = c % TXr;   // halo row of the tap (-R, -R) is (hz, hx)
      const PT* pb = patch + (hz * HX + hx) * PY + p0;
      if constexpr (INDEX) {
        if (a.map32) {
          // tap-major layout [k^3][N_p]: consecutive particles are adjacent
          int q = 0;
          for (int dz = 0; dz < K; ++dz)
            for (int dx = 0; dx < K; ++dx)
              for (int dy = 0; dy < K; ++dy) {
                const int64_t code = int64_t(pb[(dz * HX + dx) * PY + dy]);
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
              for (int dy = 0; dy < K; ++dy) dst[q++] = int64_t(pb[(dz * HX + dx) * PY + dy]);
        }
      } else if constexpr (NF == 3) {
        float g0 = 0.f, g1 = 0.f, g2 = 0.f;
#pragma unroll
        for (int dz = 0; dz < K; ++dz) {
          cfloat* wz = wl + dz * KW * KW;
#pragma unroll
          for (int dx = 0; dx < K; ++dx) {
            const float* row = pb + (dz * HX + dx) * PY;
#pragma unroll
            for (int dy = 0; dy < K; ++dy) {
              const float v = row[dy];
              g0 = fmaf(wz[dx * KW + dy], v, g0);
              g1 = fmaf(wz[KW3 + dx * KW + dy], v, g1);
              g2 = fmaf(wz[2 * KW3 + dx * KW + dy], v, g2);
            }
          }
        }
        static_cast<TY*>(a.y)[idx] = from_f32<TY>(sqrtf(fmaf(g0, g0, fmaf(g1, g1, g2 * g2))));
      } else {
        float acc = 0.f;
#pragma unroll(K == 3 ? K : 1)
        for (int dz = 0; dz < K; ++dz) {
          cfloat* wz = wl + dz * KW * KW;
#pragma unroll(K <= 5 ? K : 1)
          for (int dx = 0; dx < K; ++dx) {
            const float* row = pb + (dz * HX + dx) * PY;
#pragma unroll
            for (int dy = 0; dy < K; ++dy) acc = fmaf(wz[dx * KW + dy], row[dy], acc);
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
    if (!has_next) break;
    if (y1 >= int(wcur >> 16)) wcur = a.wins[++wi];
    y0 = ny0;
    y1 = ny1;
    par ^= 1;
  }
}

// true if the KW^3 weight set at w has only zeros outside its central 3^3
// (restricted stencils at the coarser levels, Eq. restrict_stenc); w uniform
template <int KW>
__device__ inline bool outer_shell_zero(const float* w) {
  using cfloat = const __attribute__((address_space(4))) float;
  cfloat* c = (cfloat*)(uintptr_t)w;
  uint32_t any = 0;
#pragma unroll
  for (int q = 0; q < KW * KW * KW; ++q) {
    const int z = q / (KW * KW), x = (q / KW) % KW, y = q % KW, o = KW / 2;
    if (abs(z - o) > 1 || abs(x - o) > 1 || abs(y - o) > 1) any |= __builtin_bit_cast(uint32_t, c[q]) << 1;
  }
  return any == 0;   // +0 and -0 both count as zero
}

// XCD-aware order: block b runs on XCD b % 8, which takes its own contiguous
// range of the work items (equal work per XCD, heaviest first).  A 5^3
// single-channel launch runs a tile with the 3^3 body when its level's weights
// vanish outside the central 3^3: every nonzero tap is then taken in the same
// order, so the outputs are the same (for finite values).
template <int K, typename TX, typename TY, bool INDEX, int NF = 1>
__global__ __launch_bounds__(ConvShape<K>::kThreads)
__attribute__((amdgpu_waves_per_eu(INDEX ? 3 : ConvShape<K>::kWavesPerSimd))) void conv1_kernel(ConvArgs a) {
  __shared__ ConvLds<K, INDEX> lds;
  const int xcd = int(blockIdx.x % 8);
  const int64_t it = a.xcd_off[xcd] + int64_t(blockIdx.x / 8);
  if (it >= a.xcd_off[xcd + 1]) return;
  const uint4 item = reinterpret_cast<const uint4*>(a.items)[it];
  int l, tz, tx, ty0;
  tile_unpack(uint64_t(__builtin_amdgcn_readfirstlane(item.x)) |
                  (uint64_t(__builtin_amdgcn_readfirstlane(item.y)) << 32),
              l, tz, tx, ty0);
  l = __builtin_amdgcn_readfirstlane(l);
  tz = __builtin_amdgcn_readfirstlane(tz);
  tx = __builtin_amdgcn_readfirstlane(tx);
  const uint32_t w_beg = __builtin_amdgcn_readfirstlane(item.z);
  const uint32_t w_end = __builtin_amdgcn_readfirstlane(item.w);
  if constexpr (K == 5 && !INDEX && NF == 1) {
    static_assert(sizeof(ConvLds<3, false>) <= sizeof(lds), "the 3^3 body runs in the 5^3 launch's LDS");
    const float* wl = a.w + (a.n_wlevels == 1 ? 0 : (l - a.m.l_min)) * 125;
    if (outer_shell_zero<5>(wl)) {
      conv_item<3, 5, TX, TY, false, 1, ConvShape<5>::kThreads>(a, l, tz, tx, w_beg, w_end, lds.patch, lds.o_idx,
                                                                lds.o_pos, lds.cnt);
      return;
    }
  }
  conv_item<K, K, TX, TY, INDEX, NF, ConvShape<K>::kThreads>(a, l, tz, tx, w_beg, w_end, lds.patch, lds.o_idx, lds.o_pos,
                                                             lds.cnt);
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
  else if (K > 5)
    APR_FAIL(APR_EUNSUPPORTED, "apr_conv: stencils above 5^3 take F32 values");
  else if (xdt == APR_BF16 && ydt == APR_BF16)
    hipLaunchKernelGGL((conv1_kernel<K <= 5 ? K : 3, __hip_bfloat16, __hip_bfloat16, INDEX>), grid,
                       dim3(ConvShape<K>::kThreads), 0, s, args);
  else if (xdt == APR_BF16 && ydt == APR_F32)
    hipLaunchKernelGGL((conv1_kernel<K <= 5 ? K : 3, __hip_bfloat16, float, INDEX>), grid,
                       dim3(ConvShape<K>::kThreads), 0, s, args);
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
  a.wins = h->wins;
  a.items = h->items;
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
  if (d->k < 3 || d->k > 13 || d->k % 2 == 0) APR_FAIL(APR_EUNSUPPORTED, "apr_conv: k must be 3, 5, 7, 9, 11 or 13");
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
    if (d->k > 5) APR_FAIL(APR_EUNSUPPORTED, "apr_conv: multichannel layers take k = 3 or 5");
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
  switch (d->k) {
    case 3: return launch_conv<3, false>(a, d->x_dtype, d->y_dtype, s);
    case 5: return launch_conv<5, false>(a, d->x_dtype, d->y_dtype, s);
    case 7: return launch_conv<7, false>(a, d->x_dtype, d->y_dtype, s);
    case 9: return launch_conv<9, false>(a, d->x_dtype, d->y_dtype, s);
    case 11: return launch_conv<11, false>(a, d->x_dtype, d->y_dtype, s);
    default: return launch_conv<13, false>(a, d->x_dtype, d->y_dtype, s);
  }
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

