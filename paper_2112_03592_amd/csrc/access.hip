// Access-structure build: host validation of the particle LinearAccess
// (Algorithm 1), device derivation of the APR tree (Section 3.4), optional
// device validation of partition and 2:1 balance, and the non-empty tile
// list of the convolution (the pre-pass of Section 5.2).
#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <vector>

#include "common.hpp"

namespace apr {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

// ---------------------------------------------------------------------------
// Exclusive scan of uint32 (block scan + recursive scan of block sums)
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 4;
constexpr int kScanBlock = kScanThreads * kScanPerThread;

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(v, o, 64);
    if (lane >= uint32_t(o)) v += t;
  }
  return v;
}

__global__ __launch_bounds__(kScanThreads) void scan_block_kernel(uint32_t* data, int64_t n,
                                                                  uint32_t* sums) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  const int64_t base = int64_t(blockIdx.x) * kScanBlock + int64_t(threadIdx.x) * kScanPerThread;
  uint32_t v[kScanPerThread];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanPerThread; ++j) {
    v[j] = (base + j < n) ? data[base + j] : 0u;
    s += v[j];
  }
  uint32_t incl = wave_incl_scan(s);
  const int w = threadIdx.x / 64;
  if (lane_id() == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t woff = 0;
  for (int i = 0; i < w; ++i) woff += wsum[i];
  uint32_t run = woff + incl - s;
#pragma unroll
  for (int j = 0; j < kScanPerThread; ++j) {
    if (base + j < n) data[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == kScanThreads - 1) {
    uint32_t tot = 0;
    for (int i = 0; i < kScanThreads / 64; ++i) tot += wsum[i];
    sums[blockIdx.x] = tot;
  }
}

__global__ void scan_add_kernel(uint32_t* data, int64_t n, const uint32_t* offs) {
  const int64_t base = int64_t(blockIdx.x) * kScanBlock;
  const uint32_t o = offs[blockIdx.x];
  for (int j = threadIdx.x; j < kScanBlock; j += blockDim.x)
    if (base + j < n) data[base + j] += o;
}

apr_status scan_u32(uint32_t* data, int64_t n, uint32_t* total_dev, hipStream_t stream) {
  if (n <= 0) {
    if (total_dev) APR_HIP(hipMemsetAsync(total_dev, 0, sizeof(uint32_t), stream));
    return APR_OK;
  }
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  uint32_t* sums = nullptr;
  APR_HIP(hipMalloc(&sums, sizeof(uint32_t) * (nb + 1)));
  hipLaunchKernelGGL(scan_block_kernel, dim3(unsigned(nb)), dim3(kScanThreads), 0, stream, data, n,
                     sums);
  APR_HIP(hipGetLastError());
  apr_status st = APR_OK;
  if (nb > 1) {
    st = scan_u32(sums, nb, total_dev, stream);
    if (st == APR_OK) {
      hipLaunchKernelGGL(scan_add_kernel, dim3(unsigned(nb)), dim3(kScanThreads), 0, stream, data,
                         n, sums);
      if (hipGetLastError() != hipSuccess) st = APR_EDEVICE;
    }
  } else if (total_dev) {
    if (hipMemcpyAsync(total_dev, sums, sizeof(uint32_t), hipMemcpyDeviceToDevice, stream) !=
        hipSuccess)
      st = APR_EDEVICE;
  }
  if (hipStreamSynchronize(stream) != hipSuccess) st = APR_EDEVICE;
  (void)hipFree(sums);
  if (st == APR_EDEVICE) set_error("scan_u32: device failure");
  return st;
}

// ---------------------------------------------------------------------------
// Tree derivation, one level L per launch, one wave per tree row.
// Tree row (L, z, x) holds the sorted distinct y/2 over the particles of the
// level-(L+1) rows (2z+a, 2x+b) and the tree nodes of those rows.
// Pass 1 (FILL=false) writes the row's node count into rows_io[row];
// pass 2 (FILL=true) reads the exclusive offset from rows_io[row], writes the
// nodes and replaces rows_io[row] by the inclusive end.
// ---------------------------------------------------------------------------
constexpr int kTreeWaves = 4;
constexpr int kMaxBitmapWords = (65536 / 2) / 32;   // parent y < 32768

template <bool FILL>
__global__ __launch_bounds__(64 * kTreeWaves) void tree_rows_kernel(
    Meta m, int L, const uint16_t* __restrict__ py, const uint32_t* __restrict__ pend,
    const uint16_t* __restrict__ cy, const uint32_t* __restrict__ cend, uint32_t* rows_io,
    uint16_t* __restrict__ out_y) {
  __shared__ uint32_t bitmap[kTreeWaves][kMaxBitmapWords];
  const int wave = threadIdx.x / 64;
  const uint32_t lane = lane_id();
  const int64_t nrows = int64_t(m.dz[L]) * m.dx[L];
  const int64_t row = int64_t(blockIdx.x) * kTreeWaves + wave;
  if (row >= nrows) return;
  const int z = int(row / m.dx[L]);
  const int x = int(row % m.dx[L]);
  const int C = L + 1;
  const bool has_p = (C >= m.l_min && C <= m.l_max);
  const bool has_t = (C <= m.t_hi);
  uint32_t lb[8], le[8];
  const uint16_t* ly[8];
  int nl = 0;
  uint32_t total = 0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int cz = 2 * z + a, cx = 2 * x + b;
      if (cz >= m.dz[C] || cx >= m.dx[C]) continue;
      if (has_p) {
        row_range(pend, m.prow[C] + uint32_t(cz) * m.dx[C] + cx, lb[nl], le[nl]);
        ly[nl] = py;
        total += le[nl] - lb[nl];
        ++nl;
      }
      if (has_t) {
        row_range(cend, uint32_t(cz) * m.dx[C] + cx, lb[nl], le[nl]);
        ly[nl] = cy;
        total += le[nl] - lb[nl];
        ++nl;
      }
    }
  if (total == 0) {
    // FILL: the inclusive end equals the exclusive offset already stored
    if (!FILL && lane == 0) rows_io[row] = 0;
    return;
  }
  uint32_t* bm = bitmap[wave];
  const int nwords = (m.dy[L] + 31) / 32;
  for (int w = lane; w < nwords; w += 64) bm[w] = 0u;
  wave_lds_sync();
  for (int j = 0; j < nl; ++j)
    for (uint32_t i = lb[j] + lane; i < le[j]; i += 64) {
      const uint32_t h = uint32_t(ly[j][i]) >> 1;
      atomicOr(&bm[h >> 5], 1u << (h & 31));
    }
  wave_lds_sync();
  if (!FILL) {
    uint32_t c = 0;
    for (int w = lane; w < nwords; w += 64) c += __popc(bm[w]);
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if (lane == 0) rows_io[row] = c;
    return;
  }
  uint32_t base = rows_io[row];
  for (int w0 = 0; w0 < nwords; w0 += 64) {
    const int w = w0 + int(lane);
    uint32_t word = (w < nwords) ? bm[w] : 0u;
    const uint32_t c = __popc(word);
    const uint32_t incl = wave_incl_scan(c);
    uint32_t pos = base + incl - c;
    while (word) {
      const int bit = __ffs(word) - 1;
      out_y[pos++] = uint16_t(w * 32 + bit);
      word &= word - 1u;
    }
    base += __shfl(incl, 63, 64);
  }
  if (lane == 0) rows_io[row] = base;
}

__global__ void add_offset_kernel(uint32_t* data, int64_t n, uint32_t off) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) data[i] += off;
}

// ---------------------------------------------------------------------------
// Validation: one wave per tree row, one lane per node.
// bit 0: partition (a node coincides with a particle, or an in-image child of
//        a node is neither particle nor node);
// bit 1: balance (a 26-neighbour of a node at level >= l_min lies inside a
//        coarser particle: neither particle nor node at the node's level).
// ---------------------------------------------------------------------------
__device__ inline bool row_has(const uint16_t* ys, const uint32_t* ends, uint32_t row, uint32_t y) {
  uint32_t b, e;
  row_range(ends, row, b, e);
  while (b < e) {
    const uint32_t mid = (b + e) >> 1;
    if (ys[mid] < y)
      b = mid + 1;
    else
      e = mid;
  }
  return b < ends[row] && ys[b] == y;
}

__device__ inline bool cell_exists(const Meta& m, const uint16_t* py, const uint32_t* pend,
                                   const uint16_t* ty, const uint32_t* tend, int l, int z, int x,
                                   int y) {
  if (l >= m.l_min && l <= m.l_max &&
      row_has(py, pend, m.prow[l] + uint32_t(z) * m.dx[l] + x, uint32_t(y)))
    return true;
  if (l >= m.t_lo && l <= m.t_hi &&
      row_has(ty, tend, m.trow[l] + uint32_t(z) * m.dx[l] + x, uint32_t(y)))
    return true;
  return false;
}

__global__ __launch_bounds__(256) void validate_kernel(Meta m, const uint16_t* __restrict__ py,
                                                       const uint32_t* __restrict__ pend,
                                                       const uint16_t* __restrict__ ty,
                                                       const uint32_t* __restrict__ tend,
                                                       int64_t n_trows, uint32_t* flags) {
  const int64_t row = int64_t(blockIdx.x) * 4 + threadIdx.x / 64;
  if (row >= n_trows) return;
  int L = m.t_lo;
  while (L < m.t_hi && uint32_t(row) >= m.trow[L + 1]) ++L;
  const uint32_t r = uint32_t(row) - m.trow[L];
  const int z = int(r / m.dx[L]), x = int(r % m.dx[L]);
  uint32_t b, e;
  row_range(tend, uint32_t(row), b, e);
  uint32_t bad = 0;
  for (uint32_t i = b + lane_id(); i < e; i += 64) {
    const int y = ty[i];
    if (L >= m.l_min && row_has(py, pend, m.prow[L] + uint32_t(z) * m.dx[L] + x, uint32_t(y)))
      bad |= 1u;
    const int C = L + 1;
    for (int a = 0; a < 2; ++a)
      for (int bb = 0; bb < 2; ++bb)
        for (int c = 0; c < 2; ++c) {
          const int cz = 2 * z + a, cx = 2 * x + bb, cyv = 2 * y + c;
          if (cz >= m.dz[C] || cx >= m.dx[C] || cyv >= m.dy[C]) continue;
          if (!cell_exists(m, py, pend, ty, tend, C, cz, cx, cyv)) bad |= 1u;
        }
    if (L >= m.l_min) {
      for (int dz = -1; dz <= 1; ++dz)
        for (int dx = -1; dx <= 1; ++dx)
          for (int dy = -1; dy <= 1; ++dy) {
            const int nz = z + dz, nx = x + dx, ny = y + dy;
            if (nz < 0 || nx < 0 || ny < 0 || nz >= m.dz[L] || nx >= m.dx[L] || ny >= m.dy[L])
              continue;
            if (!cell_exists(m, py, pend, ty, tend, L, nz, nx, ny)) bad |= 2u;
          }
    }
  }
  if (bad) atomicOr(flags, bad);
}

// ---------------------------------------------------------------------------
// Non-empty tile list (Section 5.2 pre-pass): a tile of kTileZ x kTileX
// particle rows at one level is kept if any of its rows holds a particle.
// Tiles are enumerated finest level first.
// ---------------------------------------------------------------------------
struct TileLevels {
  int32_t n_levels;
  int32_t level[kMaxL];
  int64_t first[kMaxL + 1];   // first tile index of each entry
  int32_t ntx[kMaxL];
};

__device__ inline void tile_locate(const TileLevels& tl, int64_t t, int& l, int& tz, int& tx) {
  int j = 0;
  while (j + 1 < tl.n_levels && t >= tl.first[j + 1]) ++j;
  l = tl.level[j];
  const int64_t r = t - tl.first[j];
  tz = int(r / tl.ntx[j]);
  tx = int(r % tl.ntx[j]);
}

// candidate tiles of every level, finest level first
static TileLevels tile_levels(const Meta& m) {
  TileLevels tl{};
  int64_t ntot = 0;
  for (int l = m.l_max; l >= m.l_min; --l) {
    const int j = tl.n_levels++;
    tl.level[j] = l;
    tl.first[j] = ntot;
    tl.ntx[j] = (m.dx[l] + kTileX - 1) / kTileX;
    ntot += int64_t((m.dz[l] + kTileZ - 1) / kTileZ) * tl.ntx[j];
  }
  tl.first[tl.n_levels] = ntot;
  return tl;
}

// flags[t] = tile t holds particles; ymin[t] = smallest y among them
__global__ void tile_flag_kernel(Meta m, TileLevels tl, const uint32_t* __restrict__ pend,
                                 const uint16_t* __restrict__ py, uint32_t* flags, uint32_t* ymin, int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  int l, tz, tx;
  tile_locate(tl, t, l, tz, tx);
  uint32_t any = 0, y0 = 0xffffu;
  for (int a = 0; a < kTileZ; ++a)
    for (int b = 0; b < kTileX; ++b) {
      const int z = tz * kTileZ + a, x = tx * kTileX + b;
      if (z >= m.dz[l] || x >= m.dx[l]) continue;
      uint32_t rb, re;
      row_range(pend, m.prow[l] + uint32_t(z) * m.dx[l] + x, rb, re);
      if (re > rb) {
        any = 1;
        y0 = min(y0, uint32_t(py[rb]));
      }
    }
  flags[t] = any;
  ymin[t] = y0;
}

__global__ void tile_compact_kernel(TileLevels tl, const uint32_t* __restrict__ flags_scanned,
                                    const uint32_t* __restrict__ flags_raw, const uint32_t* __restrict__ ymin,
                                    uint64_t* out, int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n || !flags_raw[t]) return;
  int l, tz, tx;
  tile_locate(tl, t, l, tz, tx);
  out[flags_scanned[t]] = tile_pack(l, tz, tx, int(ymin[t]));
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
apr_status build_gather_map(const apr_handle* h, int k, int32_t* map32, hipStream_t s);
apr_status build_child_map(const apr_handle* h, uint32_t* cmap, hipStream_t s);
apr_status build_inverse_map(apr_handle* h, int k, hipStream_t s,
                             apr_status (*alloc_u32)(apr_handle*, uint32_t**, int64_t),
                             apr_status (*scan)(uint32_t*, int64_t, uint32_t*, hipStream_t), uint32_t* total_dev);

static int finest_level(const int32_t* dims) {
  int32_t mx = std::max(dims[0], std::max(dims[1], dims[2]));
  int l = 0;
  while ((int64_t(1) << l) < mx) ++l;
  return l;
}

template <typename T>
static apr_status dev_alloc(apr_handle* h, T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) return APR_OK;
  void* q = nullptr;
  if (hipMalloc(&q, size_t(count) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    APR_FAIL(APR_ENOMEM, "hipMalloc failed (" + std::to_string(count * sizeof(T)) + " bytes)");
  }
  h->allocs.push_back(q);
  h->device_bytes += count * int64_t(sizeof(T));
  *p = static_cast<T*>(q);
  return APR_OK;
}

static void free_handle(apr_handle* h) {
  if (!h) return;
  for (void* p : h->allocs) (void)hipFree(p);
  delete h;
}

// Sweep windows and launch order of the convolution tiles (host copy of the
// access).  A tile's windows are the runs of its output y (union over the
// tile's rows): a window spans at most kWinY cells and ends before a stretch
// of more than kWinGap cells without outputs, so the patch is rebuilt only
// around the outputs.  A tile's cost is taken as the cells its windows span
// plus a fixed share per window (the memory rounds and barriers).  The list
// (finest level first, then z, x) is cut into eight contiguous ranges of equal
// cost, one per XCD (neighbouring tiles share halo rows in that XCD's L2), and
// each range runs its heaviest tiles first, so that no long tile starts last.
// Host threads for the O(N) checks and counts of the build: up to 16, one
// per 2^20 items.
static int host_threads(int64_t items) {
  const int hw = int(std::max(1u, std::thread::hardware_concurrency()));
  return int(std::max<int64_t>(1, std::min<int64_t>({int64_t(16), int64_t(hw), items >> 20})));
}

// Runs f(0) .. f(nth - 1) on nth threads (the caller's included).  An
// exception inside a worker (an allocation) is caught there and reported as
// false, as is a failure to start a worker (f then runs on the caller).
template <typename F>
static bool run_host_threads(int nth, F&& f) {
  std::atomic<bool> ok{true};
  auto guarded = [&](int t) {
    try {
      f(t);
    } catch (...) {
      ok = false;
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nth; ++t) {
    try {
      pool.emplace_back(guarded, t);
    } catch (...) {
      guarded(t);
    }
  }
  guarded(0);
  for (auto& th : pool) th.join();
  return ok;
}

// Work items of the conv launch.  Each tile's y sweep is cut into windows
// (runs of its output y spanning at most kWinY cells, gaps of at most kWinGap),
// counted on the host from the LinearAccess.  A work item is a run of one
// tile's windows: tiles whose sweep is long against the launch's ideal share
// per workgroup slot are cut into several items (each starts with its own row
// lookups), so that the longest item, not the longest tile, bounds the tail.
// The items are split into eight contiguous ranges of equal cost, one per XCD,
// each run heaviest first.
static apr_status order_tiles(apr_handle* h, const apr_access_desc* d, hipStream_t s) {
  const int64_t n = h->n_tiles;
  for (int x = 0; x <= 8; ++x) h->xcd_off[x] = 0;
  h->n_items = 0;
  if (n == 0) return APR_OK;
  std::vector<uint64_t> t(size_t(n), 0);
  APR_HIP(hipMemcpyAsync(t.data(), h->tiles, size_t(n) * 8, hipMemcpyDeviceToHost, s));
  APR_HIP(hipStreamSynchronize(s));
  const Meta& m = h->meta;
  // windows of every tile, tiles split over host threads (each fills its own
  // lists, concatenated in tile order)
  const int nth = host_threads(d->n_particles);
  std::vector<std::vector<uint32_t>> twins(static_cast<size_t>(nth)), tcost(static_cast<size_t>(nth));
  std::vector<int64_t> nwin(size_t(n), 0);
  auto tile_windows = [&](int th) {
    const int64_t i0 = n * th / nth, i1 = n * (th + 1) / nth;
    std::vector<uint64_t> bits;
    for (int64_t i = i0; i < i1; ++i) {
      int l, tz, tx, y0;
      tile_unpack(t[size_t(i)], l, tz, tx, y0);
      const int words = (m.dy[l] + 63) / 64;
      bits.assign(size_t(words), 0);
      for (int z = tz * kTileZ; z < std::min(m.dz[l], (tz + 1) * kTileZ); ++z)
        for (int x = tx * kTileX; x < std::min(m.dx[l], (tx + 1) * kTileX); ++x) {
          const uint64_t row = uint64_t(m.prow[l]) + uint64_t(z) * uint64_t(m.dx[l]) + uint64_t(x);
          const uint64_t b = row ? d->xz_end[row - 1] : 0, e = d->xz_end[row];
          for (uint64_t j = b; j < e; ++j) bits[d->y_idx[j] >> 6] |= uint64_t(1) << (d->y_idx[j] & 63);
        }
      // first occupied y at or after y (or -1)
      auto next = [&](int y) {
        if (y >= m.dy[l]) return -1;
        for (int w = y >> 6; w < words; ++w) {
          uint64_t v = bits[size_t(w)];
          if (w == (y >> 6)) v &= ~uint64_t(0) << (y & 63);
          if (v) return w * 64 + __builtin_ctzll(v);
        }
        return -1;
      };
      for (int y = next(0); y >= 0;) {
        const int w0 = y;
        int last = y, nx;
        while ((nx = next(last + 1)) >= 0 && nx - w0 < kWinY && nx - last - 1 <= kWinGap) last = nx;
        twins[size_t(th)].push_back(uint32_t(w0) | (uint32_t(last) << 16));
        tcost[size_t(th)].push_back(uint32_t(last - w0 + 1) + 16);
        ++nwin[size_t(i)];
        y = nx;
      }
    }
  };
  if (!run_host_threads(nth, tile_windows)) APR_FAIL(APR_ENOMEM, "apr_access_build: out of host memory (tile windows)");
  std::vector<uint32_t> wins;           // windows, tile by tile in list order
  std::vector<uint32_t> wcost;          // cost of each window: its span + 16 cells
  for (int th = 0; th < nth; ++th) {
    wins.insert(wins.end(), twins[size_t(th)].begin(), twins[size_t(th)].end());
    wcost.insert(wcost.end(), tcost[size_t(th)].begin(), tcost[size_t(th)].end());
  }
  std::vector<int64_t> woff(size_t(n) + 1, 0);
  for (int64_t i = 0; i < n; ++i) woff[size_t(i) + 1] = woff[size_t(i)] + nwin[size_t(i)];
  uint64_t total = 0;
  for (uint32_t c : wcost) total += c + kItemCost;
  if (wins.size() >= (size_t(1) << 32)) APR_FAIL(APR_EUNSUPPORTED, "apr_access_build: too many sweep windows");
  // items: runs of windows whose cost (item start included) stays within half
  // the ideal share of one of the launch's resident workgroups
  const uint64_t cap = std::max<uint64_t>(total / (2 * kConvSlots), 1);
  std::vector<uint32_t> items;          // [n_items][4]: tile code (low, high word), first window, end window
  std::vector<uint64_t> cost;
  for (int64_t i = 0; i < n; ++i) {
    uint64_t acc = kItemCost;
    int64_t start = woff[size_t(i)];
    for (int64_t w = woff[size_t(i)]; w < woff[size_t(i) + 1]; ++w) {
      if (w > start && acc + wcost[size_t(w)] > cap) {
        items.insert(items.end(), {uint32_t(t[size_t(i)]), uint32_t(t[size_t(i)] >> 32), uint32_t(start), uint32_t(w)});
        cost.push_back(acc);
        acc = kItemCost;
        start = w;
      }
      acc += wcost[size_t(w)];
    }
    items.insert(items.end(), {uint32_t(t[size_t(i)]), uint32_t(t[size_t(i)] >> 32), uint32_t(start),
                               uint32_t(woff[size_t(i) + 1])});
    cost.push_back(acc);
  }
  const int64_t ni = int64_t(cost.size());
  int64_t off[9];
  for (int x = 0; x <= 8; ++x) off[x] = ni * x / 8;
  std::vector<int64_t> idx(static_cast<size_t>(ni));
  for (int64_t i = 0; i < ni; ++i) idx[size_t(i)] = i;
  if (ni >= 16) {
    uint64_t all = 0;
    for (uint64_t c : cost) all += c;
    off[0] = 0;
    off[8] = ni;
    uint64_t acc = 0;
    int x = 1;
    for (int64_t i = 0; i < ni && x < 8; ++i) {
      acc += cost[size_t(i)];
      while (x < 8 && acc * 8 >= all * uint64_t(x)) off[x++] = i + 1;
    }
    while (x < 8) off[x++] = ni;
    for (int r = 0; r < 8; ++r)
      std::stable_sort(idx.begin() + off[r], idx.begin() + off[r + 1],
                       [&](int64_t a, int64_t b) { return cost[size_t(a)] > cost[size_t(b)]; });
  }
  std::vector<uint32_t> sorted(size_t(ni) * 4);
  for (int64_t i = 0; i < ni; ++i)
    std::copy_n(items.begin() + idx[size_t(i)] * 4, 4, sorted.begin() + i * 4);
  h->n_wins = int64_t(wins.size());
  h->n_items = ni;
  apr_status st = dev_alloc(h, &h->wins, h->n_wins);
  if (st == APR_OK) st = dev_alloc(h, &h->items, ni * 4);
  if (st != APR_OK) return st;
  APR_HIP(hipMemcpyAsync(h->wins, wins.data(), wins.size() * 4, hipMemcpyHostToDevice, s));
  APR_HIP(hipMemcpyAsync(h->items, sorted.data(), sorted.size() * 4, hipMemcpyHostToDevice, s));
  APR_HIP(hipStreamSynchronize(s));
  for (int r = 0; r <= 8; ++r) h->xcd_off[r] = off[r];
  return APR_OK;
}

#define APR_TRY(expr)                 \
  do {                                \
    apr_status _s = (expr);           \
    if (_s != APR_OK) {               \
      free_handle(h);                 \
      for (void* p : tmp) (void)hipFree(p); \
      return _s;                      \
    }                                 \
  } while (0)

#define APR_TRY_HIP(call)                                                       \
  do {                                                                          \
    hipError_t _e = (call);                                                     \
    if (_e != hipSuccess) {                                                     \
      set_error(std::string(#call) + ": " + hipGetErrorString(_e));             \
      free_handle(h);                                                           \
      for (void* p : tmp) (void)hipFree(p);                                           \
      return APR_EDEVICE;                                                       \
    }                                                                           \
  } while (0)

static apr_status build_impl(const apr_access_desc* d, hipStream_t s, apr_handle** out) {
  if (!d || !out) APR_FAIL(APR_EINVAL, "apr_access_build: null argument");
  *out = nullptr;
  for (int a = 0; a < 3; ++a)
    if (d->dims[a] <= 0) APR_FAIL(APR_EINVAL, "apr_access_build: image dims must be positive");
  if (d->dims[2] > 65535)
    APR_FAIL(APR_EUNSUPPORTED, "apr_access_build: y size above 65535 (16-bit y indices)");
  const int lmax = finest_level(d->dims);
  if (d->l_max != lmax)
    APR_FAIL(APR_EINVAL, "apr_access_build: l_max must be ceil(log2(max dim)) = " +
                             std::to_string(lmax));
  if (d->l_min < 0 || d->l_min > d->l_max)
    APR_FAIL(APR_EINVAL, "apr_access_build: need 0 <= l_min <= l_max");
  if (lmax >= kMaxL) APR_FAIL(APR_EUNSUPPORTED, "apr_access_build: too many levels");
  if (d->n_particles < 0 || d->n_particles >= int64_t(0xffffffffu))
    APR_FAIL(APR_EUNSUPPORTED, "apr_access_build: particle count must be below 2^32-1");
  if (d->n_particles > 0 && !d->y_idx) APR_FAIL(APR_EINVAL, "apr_access_build: y_idx is null");
  if (!d->xz_end) APR_FAIL(APR_EINVAL, "apr_access_build: xz_end is null");

  Meta m{};
  m.l_min = d->l_min;
  m.l_max = lmax;
  m.t_lo = std::max(d->l_min - 1, 0);
  m.t_hi = lmax - 1;
  for (int l = 0; l <= lmax; ++l) {
    const int64_t sh = int64_t(1) << (lmax - l);
    m.dz[l] = int32_t((d->dims[0] + sh - 1) / sh);
    m.dx[l] = int32_t((d->dims[1] + sh - 1) / sh);
    m.dy[l] = int32_t((d->dims[2] + sh - 1) / sh);
  }
  int64_t nrows = 0;
  for (int l = d->l_min; l <= lmax; ++l) {
    if (nrows > int64_t(0xffffffffu)) APR_FAIL(APR_EUNSUPPORTED, "too many rows");
    m.prow[l] = uint32_t(nrows);
    nrows += int64_t(m.dz[l]) * m.dx[l];
  }
  if (d->n_rows != nrows)
    APR_FAIL(APR_EINVAL, "apr_access_build: n_rows = " + std::to_string(d->n_rows) +
                             ", expected " + std::to_string(nrows));
  int64_t ntrows = 0;
  for (int l = m.t_lo; l <= m.t_hi; ++l) {
    m.trow[l] = uint32_t(ntrows);
    ntrows += int64_t(m.dz[l]) * m.dx[l];
  }

  // host validation of the LinearAccess arrays
  std::vector<uint32_t> ends(static_cast<size_t>(nrows));
  apr_handle* h = new apr_handle();
  std::vector<void*> tmp;
  h->meta = m;
  h->n_p = d->n_particles;
  h->n_rows = nrows;
  h->n_trows = ntrows;
  {
    // rows split over host threads; each chunk starts from the previous
    // row's end (a chunk whose start is invalid fails at its first row)
    const int nth = host_threads(nrows);
    std::vector<int64_t> bad(size_t(nth), -1);
    std::vector<int> why(size_t(nth), 0);
    auto check_rows = [&](int t) {
      const int64_t r0 = nrows * t / nth, r1 = nrows * (t + 1) / nth;
      int l = d->l_min;
      uint64_t prev = r0 ? d->xz_end[r0 - 1] : 0;
      for (int64_t row = r0; row < r1; ++row) {
        while (l < lmax && row >= int64_t(m.prow[l + 1])) ++l;
        const uint64_t e = d->xz_end[row];
        if (e < prev || e > uint64_t(d->n_particles)) {
          bad[size_t(t)] = row;
          why[size_t(t)] = 1;
          return;
        }
        for (uint64_t k = prev; k < e; ++k)
          if (d->y_idx[k] >= m.dy[l] || (k > prev && d->y_idx[k] <= d->y_idx[k - 1])) {
            bad[size_t(t)] = row;
            why[size_t(t)] = 2;
            return;
          }
        ends[size_t(row)] = uint32_t(e);
        prev = e;
      }
    };
    if (!run_host_threads(nth, check_rows)) {
      free_handle(h);
      APR_FAIL(APR_ENOMEM, "apr_access_build: host validation failed to run");
    }
    for (int t = 0; t < nth; ++t) {
      if (bad[size_t(t)] < 0) continue;
      free_handle(h);
      if (why[size_t(t)] == 1)
        APR_FAIL(APR_EINVAL, "apr_access_build: xz_end not monotone or beyond n_particles at row " +
                                 std::to_string(bad[size_t(t)]));
      APR_FAIL(APR_EINVAL, "apr_access_build: y_idx out of range or not strictly increasing in row " +
                               std::to_string(bad[size_t(t)]));
    }
    for (int l = d->l_min; l <= lmax; ++l) {
      const int64_t first = m.prow[l], last = first + int64_t(m.dz[l]) * m.dx[l] - 1;
      h->per_level_p[l] = int64_t(d->xz_end[last]) - (first ? int64_t(d->xz_end[first - 1]) : 0);
    }
    if (nrows && d->xz_end[nrows - 1] != uint64_t(d->n_particles)) {
      free_handle(h);
      APR_FAIL(APR_EINVAL, "apr_access_build: last xz_end must equal n_particles");
    }
    if (!nrows && d->n_particles) {
      free_handle(h);
      APR_FAIL(APR_EINVAL, "apr_access_build: last xz_end must equal n_particles");
    }
  }

  (void)hipGetDevice(&h->device);
  APR_TRY(dev_alloc(h, &h->py, h->n_p));
  APR_TRY(dev_alloc(h, &h->pend, nrows));
  if (h->n_p) APR_TRY_HIP(hipMemcpyAsync(h->py, d->y_idx, size_t(h->n_p) * 2, hipMemcpyHostToDevice, s));
  APR_TRY_HIP(hipMemcpyAsync(h->pend, ends.data(), size_t(nrows) * 4, hipMemcpyHostToDevice, s));
  APR_TRY_HIP(hipStreamSynchronize(s));

  // ---- tree, finest level first; per-level local arrays
  std::vector<uint16_t*> lev_y(kMaxL, nullptr);
  std::vector<uint32_t*> lev_end(kMaxL, nullptr);
  std::vector<uint32_t> lev_n(kMaxL, 0);
  uint32_t* d_total = nullptr;
  {
    void* q = nullptr;
    APR_TRY_HIP(hipMalloc(&q, sizeof(uint32_t)));
    tmp.push_back(q);
    d_total = static_cast<uint32_t*>(q);
  }
  for (int L = m.t_hi; L >= m.t_lo; --L) {
    const int64_t rows_l = int64_t(m.dz[L]) * m.dx[L];
    void* q = nullptr;
    APR_TRY_HIP(hipMalloc(&q, size_t(rows_l) * 4));
    tmp.push_back(q);
    lev_end[L] = static_cast<uint32_t*>(q);
    const unsigned grid = unsigned((rows_l + kTreeWaves - 1) / kTreeWaves);
    const uint16_t* cy = (L + 1 <= m.t_hi) ? lev_y[L + 1] : nullptr;
    const uint32_t* cend = (L + 1 <= m.t_hi) ? lev_end[L + 1] : nullptr;
    hipLaunchKernelGGL(tree_rows_kernel<false>, dim3(grid), dim3(64 * kTreeWaves), 0, s, m, L,
                       h->py, h->pend, cy, cend, lev_end[L], nullptr);
    APR_TRY_HIP(hipGetLastError());
    APR_TRY(scan_u32(lev_end[L], rows_l, d_total, s));
    uint32_t tot = 0;
    APR_TRY_HIP(hipMemcpyAsync(&tot, d_total, 4, hipMemcpyDeviceToHost, s));
    APR_TRY_HIP(hipStreamSynchronize(s));
    lev_n[L] = tot;
    if (tot) {
      APR_TRY_HIP(hipMalloc(&q, size_t(tot) * 2));
      tmp.push_back(q);
      lev_y[L] = static_cast<uint16_t*>(q);
    }
    hipLaunchKernelGGL(tree_rows_kernel<true>, dim3(grid), dim3(64 * kTreeWaves), 0, s, m, L,
                       h->py, h->pend, cy, cend, lev_end[L], lev_y[L]);
    APR_TRY_HIP(hipGetLastError());
  }
  int64_t nt = 0;
  for (int L = m.t_lo; L <= m.t_hi; ++L) {
    nt += lev_n[L];
    h->per_level_t[L] = lev_n[L];
  }
  if (nt >= int64_t(0xffffffffu)) APR_TRY(APR_EUNSUPPORTED);
  h->n_t = nt;
  APR_TRY(dev_alloc(h, &h->ty, nt));
  APR_TRY(dev_alloc(h, &h->tend, ntrows));
  {
    uint32_t base = 0;
    for (int L = m.t_lo; L <= m.t_hi; ++L) {
      const int64_t rows_l = int64_t(m.dz[L]) * m.dx[L];
      if (lev_n[L])
        APR_TRY_HIP(hipMemcpyAsync(h->ty + base, lev_y[L], size_t(lev_n[L]) * 2,
                                   hipMemcpyDeviceToDevice, s));
      APR_TRY_HIP(hipMemcpyAsync(h->tend + m.trow[L], lev_end[L], size_t(rows_l) * 4,
                                 hipMemcpyDeviceToDevice, s));
      if (base)
        hipLaunchKernelGGL(add_offset_kernel, dim3(unsigned((rows_l + 255) / 256)), dim3(256), 0,
                           s, h->tend + m.trow[L], rows_l, base);
      APR_TRY_HIP(hipGetLastError());
      base += lev_n[L];
    }
  }

  // ---- validation
  if (d->flags & (APR_VALIDATE_PARTITION | APR_VALIDATE_BALANCE)) {
    // level l_min must be fully covered by its particles and tree nodes
    const int64_t full = int64_t(m.dz[m.l_min]) * m.dx[m.l_min] * m.dy[m.l_min];
    const int64_t have = h->per_level_p[m.l_min] + (m.l_min <= m.t_hi ? h->per_level_t[m.l_min] : 0);
    uint32_t bad = (have != full) ? 1u : 0u;
    if (ntrows > 0) {
      APR_TRY_HIP(hipMemsetAsync(d_total, 0, 4, s));
      hipLaunchKernelGGL(validate_kernel, dim3(unsigned((ntrows + 3) / 4)), dim3(256), 0, s, m,
                         h->py, h->pend, h->ty, h->tend, ntrows, d_total);
      APR_TRY_HIP(hipGetLastError());
      uint32_t f = 0;
      APR_TRY_HIP(hipMemcpyAsync(&f, d_total, 4, hipMemcpyDeviceToHost, s));
      APR_TRY_HIP(hipStreamSynchronize(s));
      bad |= f;
    }
    if ((d->flags & APR_VALIDATE_PARTITION) && (bad & 1u)) {
      set_error("apr_access_build: particle cells do not partition the image");
      free_handle(h);
      for (void* p : tmp) (void)hipFree(p);
      return APR_EPARTITION;
    }
    if ((d->flags & APR_VALIDATE_BALANCE) && (bad & 2u)) {
      set_error("apr_access_build: neighbouring particle levels differ by more than one");
      free_handle(h);
      for (void* p : tmp) (void)hipFree(p);
      return APR_EUNBALANCED;
    }
  }

  // ---- tile list
  {
    const TileLevels tl = tile_levels(m);
    const int64_t ntot = tl.first[tl.n_levels];
    void* q = nullptr;
    APR_TRY_HIP(hipMalloc(&q, size_t(ntot + 1) * 4));
    tmp.push_back(q);
    uint32_t* raw = static_cast<uint32_t*>(q);
    void* q2 = nullptr;
    APR_TRY_HIP(hipMalloc(&q2, size_t(ntot + 1) * 4));
    tmp.push_back(q2);
    uint32_t* sc = static_cast<uint32_t*>(q2);
    void* q3 = nullptr;
    APR_TRY_HIP(hipMalloc(&q3, size_t(ntot + 1) * 4));
    tmp.push_back(q3);
    uint32_t* ymin = static_cast<uint32_t*>(q3);
    hipLaunchKernelGGL(tile_flag_kernel, dim3(unsigned((ntot + 255) / 256)), dim3(256), 0, s, m,
                       tl, h->pend, h->py, raw, ymin, ntot);
    APR_TRY_HIP(hipGetLastError());
    APR_TRY_HIP(hipMemcpyAsync(sc, raw, size_t(ntot) * 4, hipMemcpyDeviceToDevice, s));
    APR_TRY(scan_u32(sc, ntot, d_total, s));
    uint32_t nkeep = 0;
    APR_TRY_HIP(hipMemcpyAsync(&nkeep, d_total, 4, hipMemcpyDeviceToHost, s));
    APR_TRY_HIP(hipStreamSynchronize(s));
    h->n_tiles = nkeep;
    APR_TRY(dev_alloc(h, &h->tiles, std::max<int64_t>(nkeep, 1)));
    hipLaunchKernelGGL(tile_compact_kernel, dim3(unsigned((ntot + 255) / 256)), dim3(256), 0, s,
                       tl, sc, raw, ymin, h->tiles, ntot);
    APR_TRY_HIP(hipGetLastError());
    APR_TRY(order_tiles(h, d, s));
  }
  // ---- gather maps (multichannel convolution and the backward passes)
  for (int gi = 0; gi < 2; ++gi) {
    const int k = gi == 0 ? 3 : 5;
    if (!(d->flags & (gi == 0 ? APR_BUILD_GATHER3 : APR_BUILD_GATHER5))) continue;
    if (h->n_p >= (int64_t(1) << 30) - 1 || h->n_t >= (int64_t(1) << 30) - 1) {
      set_error("apr_access_build: gather maps need fewer than 2^30 particles and tree nodes");
      free_handle(h);
      for (void* p : tmp) (void)hipFree(p);
      return APR_EUNSUPPORTED;
    }
    APR_TRY(dev_alloc(h, &h->gmap[gi], h->n_p * int64_t(k * k * k)));
    APR_TRY(build_gather_map(h, k, h->gmap[gi], s));
    APR_TRY(build_inverse_map(h, k, s, &dev_alloc<uint32_t>, &scan_u32, d_total));
  }
  // ---- child map of the tree nodes (tree fills); codes hold 31-bit indices
  if (h->n_t > 0 && h->n_p < (int64_t(1) << 31) - 1) {
    APR_TRY(dev_alloc(h, &h->cmap, h->n_t * 8));
    APR_TRY(build_child_map(h, h->cmap, s));
  }
  APR_TRY_HIP(hipStreamSynchronize(s));
  for (void* p : tmp) (void)hipFree(p);
  *out = h;
  return APR_OK;
}

}  // namespace apr

using namespace apr;

extern "C" {

const char* apr_last_error(void) { return g_last_error.c_str(); }

apr_status apr_access_build(const apr_access_desc* desc, void* stream, apr_handle** out) {
  g_last_error.clear();
  try {
    return build_impl(desc, static_cast<hipStream_t>(stream), out);
  } catch (const std::exception& e) {
    set_error(std::string("apr_access_build: ") + e.what());
    return APR_ENOMEM;
  } catch (...) {
    set_error("apr_access_build: unknown failure");
    return APR_EDEVICE;
  }
}

apr_status apr_access_get_info(const apr_handle* h, apr_access_info* o) {
  if (!h || !o) APR_FAIL(APR_EINVAL, "apr_access_get_info: null argument");
  std::memset(o, 0, sizeof(*o));
  o->n_particles = h->n_p;
  o->n_tree = h->n_t;
  o->n_rows = h->n_rows;
  o->n_tree_rows = h->n_trows;
  o->l_min = h->meta.l_min;
  o->l_max = h->meta.l_max;
  o->tree_l_min = h->meta.t_lo;
  o->tree_l_max = h->meta.t_hi;
  for (int l = 0; l <= h->meta.l_max; ++l) {
    o->dims[l][0] = h->meta.dz[l];
    o->dims[l][1] = h->meta.dx[l];
    o->dims[l][2] = h->meta.dy[l];
    o->particles_per_level[l] = h->per_level_p[l];
    o->tree_per_level[l] = h->per_level_t[l];
  }
  o->n_tiles = h->n_tiles;
  o->device_bytes = h->device_bytes;
  o->n_work_items = h->n_items;
  return APR_OK;
}

apr_status apr_access_export_tree(const apr_handle* h, uint16_t* ty, uint64_t* tend) {
  if (!h) APR_FAIL(APR_EINVAL, "apr_access_export_tree: null handle");
  if (ty && h->n_t) APR_HIP(hipMemcpy(ty, h->ty, size_t(h->n_t) * 2, hipMemcpyDeviceToHost));
  if (tend && h->n_trows) {
    std::vector<uint32_t> e(static_cast<size_t>(h->n_trows));
    APR_HIP(hipMemcpy(e.data(), h->tend, size_t(h->n_trows) * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < h->n_trows; ++i) tend[i] = e[size_t(i)];
  }
  return APR_OK;
}

apr_status apr_access_export(const apr_handle* h, int32_t which, void* a, void* b) {
  if (!h) APR_FAIL(APR_EINVAL, "apr_access_export: null handle");
  switch (which) {
    case APR_EXPORT_APR: {
      if (a && h->n_p) APR_HIP(hipMemcpy(a, h->py, size_t(h->n_p) * 2, hipMemcpyDeviceToHost));
      if (b && h->n_rows) {
        std::vector<uint32_t> e(static_cast<size_t>(h->n_rows));
        APR_HIP(hipMemcpy(e.data(), h->pend, size_t(h->n_rows) * 4, hipMemcpyDeviceToHost));
        uint64_t* out = static_cast<uint64_t*>(b);
        for (int64_t i = 0; i < h->n_rows; ++i) out[i] = e[size_t(i)];
      }
      return APR_OK;
    }
    case APR_EXPORT_TREE:
      return apr_access_export_tree(h, static_cast<uint16_t*>(a), static_cast<uint64_t*>(b));
    case APR_EXPORT_TILES: {
      if (a && h->n_tiles) {
        std::vector<uint64_t> t(static_cast<size_t>(h->n_tiles));
        APR_HIP(hipMemcpy(t.data(), h->tiles, size_t(h->n_tiles) * 8, hipMemcpyDeviceToHost));
        int32_t* out = static_cast<int32_t*>(a);
        for (int64_t i = 0; i < h->n_tiles; ++i) {
          int l, tz, tx, y0;
          apr::tile_unpack(t[size_t(i)], l, tz, tx, y0);
          out[4 * i] = l;
          out[4 * i + 1] = tz;
          out[4 * i + 2] = tx;
          out[4 * i + 3] = y0;
        }
      }
      if (b) std::copy(h->xcd_off, h->xcd_off + 9, static_cast<int64_t*>(b));
      return APR_OK;
    }
    default:
      APR_FAIL(APR_EINVAL, "apr_access_export: which must be APR_EXPORT_APR, APR_EXPORT_TREE or APR_EXPORT_TILES");
  }
}

int64_t apr_tile_prepass_size(const apr_handle* h) {
  if (!h) return 0;
  const TileLevels tl = tile_levels(h->meta);
  return tl.first[tl.n_levels];
}

apr_status apr_tile_prepass(const apr_handle* h, uint32_t* flags, uint32_t* ymin, void* stream) {
  if (!h) APR_FAIL(APR_EINVAL, "apr_tile_prepass: null handle");
  const TileLevels tl = tile_levels(h->meta);
  const int64_t n = tl.first[tl.n_levels];
  if (n == 0) return APR_OK;
  if (!flags || !ymin) APR_FAIL(APR_EINVAL, "apr_tile_prepass: null buffer");
  hipLaunchKernelGGL(tile_flag_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), h->meta, tl, h->pend, h->py, flags, ymin, n);
  APR_HIP(hipGetLastError());
  return APR_OK;
}

apr_status apr_access_destroy(apr_handle* h) {
  free_handle(h);
  return APR_OK;
}

}  // extern "C"
