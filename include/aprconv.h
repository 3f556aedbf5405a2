/*
 * aprconv.h -- C ABI of the MI355X (gfx950) library for discrete convolution
 * computed directly on an Adaptive Particle Representation (APR) of an image.
 *
 * Paper: "Parallel Discrete Convolutions on Adaptive Particle Representations
 * of Images" (Jonsson, Cheeseman, Maddu, Gonciarz, Sbalzarini; arXiv
 * 2112.03592).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an apr_status.  On failure nothing has been
 *   launched and apr_last_error() returns a message for the calling thread.
 *   No C++ exception crosses this boundary.
 * - Axes are (z, x, y) with y contiguous (Section 3.1, footnote).  Levels are
 *   l in [l_min, l_max]; l_max = ceil(log2(max image edge)) (Section 2.1) and
 *   the grid at level l is ceil(N / 2^(l_max - l)) cells per axis.
 * - "device" pointers are HIP device memory owned by the caller unless stated
 *   otherwise; "host" pointers are ordinary host memory.  `stream` is a
 *   hipStream_t (NULL = the null stream).  Launches are asynchronous on that
 *   stream unless a function says it synchronizes.
 * - Particle values are stored as [N_p][C] (channel fastest); tree values as
 *   [N_t][C]; per-level weights as [n_wlevels][C_out][C_in][k][k][k] with the
 *   last three axes (dz, dx, dy) + r, r = (k-1)/2, in FP32.
 * - The library computes cross-correlation: out(c) = sum_o w[o] * V(c + o).
 *   Convolution in the sense of the paper equals correlation with the
 *   flipped stencil (apr_stencil_levels can flip).
 */
#ifndef APRCONV_H
#define APRCONV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t apr_status;
#define APR_OK 0
#define APR_EINVAL 1        /* bad pointer, size, order or argument value */
#define APR_EUNBALANCED 2   /* neighbouring particle levels differ by > 1 */
#define APR_EPARTITION 3    /* particle cells overlap or leave a gap */
#define APR_EUNSUPPORTED 4  /* valid request this build does not handle */
#define APR_ENOMEM 5        /* device allocation failed */
#define APR_EDEVICE 6       /* a HIP call failed; message holds its text */

/* storage types of particle / tree values */
#define APR_F32 0
#define APR_BF16 1
#define APR_FP8 2   /* FP8 E4M3, OCP "FN" encoding (bias 7, no infinities, NaN 0x7f,
                       largest finite 448): network activations on the gather path.
                       Stores round FP32 to nearest even and saturate to +-448. */

/* apr_access_desc.flags */
#define APR_VALIDATE_PARTITION 1u  /* check on the device that the cells partition the image */
#define APR_VALIDATE_BALANCE 2u    /* check 26-neighbour 2:1 level balance */
#define APR_BUILD_GATHER3 4u       /* also build the 3^3 gather map and its inverse (multichannel, backward) */
#define APR_BUILD_GATHER5 8u       /* also build the 5^3 gather map and its inverse */

#define APR_MAX_LEVELS 17          /* levels 0..16 (y_dim <= 65535) */

/* ----------------------------------------------------------------------
 * Access structure (Algorithm 1, "LinearAccess") and APR tree (Section 3.4)
 * ---------------------------------------------------------------------- */

typedef struct {
  int32_t dims[3];          /* image size in pixels (N_z, N_x, N_y); N_y <= 65535 */
  int32_t l_min;            /* coarsest particle level, 0 <= l_min <= l_max */
  int32_t l_max;            /* must equal ceil(log2(max(dims))) */
  const uint16_t* y_idx;    /* host [n_particles]: y of each particle, order l->z->x->y */
  int64_t n_particles;      /* < 2^32 - 1 */
  const uint64_t* xz_end;   /* host [n_rows]: inclusive prefix count of particles per
                               row; row = level_offset[l] + z * x_dim[l] + x for
                               l = l_min..l_max; the row begins at xz_end[row-1]
                               (0 for row 0) */
  int64_t n_rows;           /* sum over levels of z_dim[l] * x_dim[l] */
  uint32_t flags;           /* APR_VALIDATE_* */
} apr_access_desc;

typedef struct {
  int64_t n_particles, n_tree;           /* N_p, N_t */
  int64_t n_rows, n_tree_rows;
  int32_t l_min, l_max, tree_l_min, tree_l_max;  /* tree levels [max(l_min-1,0), l_max-1] */
  int32_t dims[APR_MAX_LEVELS][3];       /* grid size per level (z, x, y) */
  int64_t particles_per_level[APR_MAX_LEVELS];
  int64_t tree_per_level[APR_MAX_LEVELS];
  int64_t n_tiles;                       /* non-empty convolution tiles, all levels */
  int64_t device_bytes;                  /* device memory held by the handle */
  int64_t n_work_items;                  /* convolution work items (runs of a tile's y windows) */
} apr_access_info;

typedef struct apr_handle apr_handle;

/* Build the device-side access structure of one APR.
 * Reads the host arrays in `desc`, validates them (row ends monotone and equal
 * to n_particles at the end, y strictly increasing within each row and below
 * the level's y size), copies them to the current HIP device, derives the APR
 * tree (all interior nodes, Section 3.4: for every tree row the sorted union of
 * y/2 over the particles and tree nodes of its 2x2 child rows, finest level
 * first), the list of non-empty convolution tiles (the non-empty-row
 * pre-pass of Section 5.2, with each tile's first particle y), the
 * convolution's work items (each tile's y sweep cut on the host into windows,
 * runs of its particles' y spanning at most 64 cells; long sweeps cut into
 * several items; ordered for launch as eight contiguous ranges of equal work,
 * one per XCD, heaviest items first) and the child list of every tree node (which
 * apr_fill_tree gathers over).  Optional device validation per `desc->flags`
 * returns APR_EPARTITION / APR_EUNBALANCED.  Synchronizes `stream` before
 * returning.  The handle owns all its device memory; it is immutable after
 * the build and may be used from several streams.  Free with
 * apr_access_destroy. */
apr_status apr_access_build(const apr_access_desc* desc, void* stream, apr_handle** out);

/* Sizes and counts of a built handle (host struct filled in). */
apr_status apr_access_get_info(const apr_handle* h, apr_access_info* out);

/* Copy the APR tree's LinearAccess arrays to host memory: tree_y_idx [n_tree]
 * and tree_xz_end [n_tree_rows] (inclusive ends, rows ordered l->z->x over the
 * tree levels).  Either pointer may be NULL.  Synchronous. */
apr_status apr_access_export_tree(const apr_handle* h, uint16_t* tree_y_idx, uint64_t* tree_xz_end);

/* Copy one of the handle's canonical arrays to host memory (synchronous):
 *  APR_EXPORT_APR:   a = uint16 y_idx [n_particles], b = uint64 xz_end [n_rows]
 *                    (the LinearAccess of Algorithm 1 the handle was built from);
 *  APR_EXPORT_TREE:  a = uint16 tree_y_idx [n_tree], b = uint64 tree_xz_end
 *                    [n_tree_rows] (as apr_access_export_tree);
 *  APR_EXPORT_TILES: a = int32 [n_tiles][4] (level, tile z, tile x, first
 *                    particle y) of every tile of 8 x 8 (z, x) rows of one
 *                    level that holds a particle (Section 5.2's non-empty-row
 *                    pre-pass; tile (tz, tx) covers rows z in [8 tz, 8 tz + 8),
 *                    x in [8 tx, 8 tx + 8)), finest level first, then tile z,
 *                    tile x; b = int64 [9], the start of each XCD's range of
 *                    the launch list of work items, then its end (n_work_items).
 * Either pointer may be NULL.  Unknown `which`: APR_EINVAL. */
#define APR_EXPORT_APR 0
#define APR_EXPORT_TREE 1
#define APR_EXPORT_TILES 2
apr_status apr_access_export(const apr_handle* h, int32_t which, void* a, void* b);

/* Release the handle and its device memory. NULL is accepted. */
/* The non-empty-tile pre-pass of Section 5.2 on its own (apr_access_build
 * already ran it and keeps its result): for every candidate tile t of
 * 8 x 8 particle rows at one level (finest level first, then z, x),
 * flags[t] = 1 if one of its rows holds a particle, else 0, and ymin[t] =
 * the smallest y of those particles (0xffff if none).  For timing the paper's
 * pipeline (pre-pass + tree fill + convolution).  flags and ymin: device
 * uint32 [apr_tile_prepass_size(h)], caller-owned.  Asynchronous on stream.
 * Errors: APR_EINVAL (null handle or buffer). */
int64_t apr_tile_prepass_size(const apr_handle* h);
apr_status apr_tile_prepass(const apr_handle* h, uint32_t* flags, uint32_t* ymin, void* stream);

apr_status apr_access_destroy(apr_handle* h);

/* ----------------------------------------------------------------------
 * Tree values (Section 3.4, two-step fill)
 * ---------------------------------------------------------------------- */

/* tree[t][c] = mean over the in-image children c' of node t of V(c'), where
 * V is the particle value if c' is a particle and the tree value otherwise;
 * filled from level l_max-1 down to the coarsest tree level.
 * x: device [N_p][channels], tree: device [N_t][channels], both of `dtype`
 * (APR_F32, APR_BF16, or APR_FP8 with 16 channels; FP32 arithmetic, each
 * level's means rounded to the storage type).  Deterministic. Asynchronous. */
apr_status apr_fill_tree(const apr_handle* h, const void* x, void* tree, int32_t channels,
                         int32_t dtype, void* stream);

/* ----------------------------------------------------------------------
 * Stencils per level (Section 4.2, Eq. restrict_stenc; Section 4.3,
 * Eq. adapt_grad)
 * ---------------------------------------------------------------------- */

#define APR_STENCIL_SAME 0       /* w_l = w */
#define APR_STENCIL_RESTRICT 1   /* w_l = R_l K_w P_l: average of w applied at every
                                    position inside the level-l cell */
#define APR_STENCIL_ADAPTIVE 2   /* w_l = 2^-(l_max-l) w */

/* Host helper, FP64 arithmetic, FP32 output.  w: host [n_filters][k^3]
 * (n_filters = C_out*C_in); out: host [l_max-l_min+1][n_filters][k^3].
 * flip != 0 reverses w in every dimension first (the flipped PSF of
 * Section 6.2).  k odd, 3 to 13 (APR_EUNSUPPORTED otherwise). */
apr_status apr_stencil_levels(int32_t mode, int32_t k, int32_t n_filters, const double* w,
                              int32_t l_min, int32_t l_max, int32_t flip, float* out);

/* ----------------------------------------------------------------------
 * Convolution (Section 4.1; GPU design of Section 5.2)
 * ---------------------------------------------------------------------- */

#define APR_EPI_NONE 0
#define APR_EPI_RATIO 1   /* y = u / max(y, eps)   (Richardson-Lucy quotient, Section 6.2) */
#define APR_EPI_MUL 2     /* y = y * u             (Richardson-Lucy update) */
#define APR_EPI_MULPOW 3  /* y = u * max(y, 0)^power (update raised to a power; power 1 is MUL) */
#define APR_EPI_GRADMAG 4 /* three stencils per level, y = sqrt(sum_j (w_j * V)^2): the magnitude of a
                             gradient filter (Section 4.3, Eq. adapt_grad, with per-level stencils
                             2^-(l_max-l) w from APR_STENCIL_ADAPTIVE); k = 3, c_in = c_out = 1,
                             w is [n_wlevels][3][k^3], x F32 or BF16, y F32 */

typedef struct {
  int32_t k;             /* stencil side: 3 or 5; single channel also 7, 9, 11, 13 */
  int32_t c_in, c_out;   /* channels (this build: 1 and 1) */
  int32_t n_wlevels;     /* 1 (one stencil for every level) or l_max-l_min+1 */
  int32_t x_dtype;       /* APR_F32 / APR_BF16 / APR_FP8: storage of x and tree */
  int32_t y_dtype;       /* storage of y */
  int32_t epilogue;      /* APR_EPI_* */
  float eps;             /* clamp of APR_EPI_RATIO */
  const void* epi_arg;   /* device [N_p], same dtype as y: u for RATIO and MUL */
  const float* bias;     /* device FP32 [c_out] or NULL (gather path) */
  int32_t relu;          /* nonzero: y = max(y, 0) after bias and residual (gather path) */
  const void* residual;  /* device [N_p][c_out] of y's dtype added before relu, or NULL */
  float power;           /* exponent of APR_EPI_MULPOW */
} apr_conv_desc;

/* y[p] = sum_o w_{l_p}[o] * V_{l_p}(c_p + o) for every particle p, with V_l
 * the level-l reconstruction (Section 3.5): the value of the particle at a
 * level <= l containing the cell, else the tree value of the cell, 0 outside
 * the image.  Requires a balanced APR (neighbouring levels differ by <= 1),
 * so every tap of a stencil up to 5^3 is supplied by APR level l, APR level
 * l-1 or tree level l, and every tap up to 13^3 also by APR level l-2 (a
 * level-(l-j) particle lies at least 2^j - 1 level-l cells away).  Stencils
 * above 5^3 (Section 7's extension; single channel, FP32 x and y, any
 * epilogue but APR_EPI_GRADMAG) sum the k^2 lines of the stencil from
 * patches of at most 32 output cells along y.  Single-channel 5^3: a level
 * whose weights are zero outside the central 3^3 (the restricted stencil of
 * Eq. restrict_stenc at every level coarser than l_max) is evaluated with the
 * 3^3 neighbourhood, taking the same nonzero taps in the same order (equal
 * outputs for finite values).
 * x: device [N_p][c_in]; tree: device [N_t][c_in], filled from this exact x
 * by apr_fill_tree (not checked); w: device FP32 weights; y: device
 * [N_p][c_out], must not alias x or tree.  Asynchronous. */
apr_status apr_conv(const apr_handle* h, const apr_conv_desc* d, const void* x, const void* tree,
                    const float* w, void* y, void* stream);
/* Paths: c_in = c_out = 1 without bias / relu / residual runs the LDS-patch
 * kernels (so does APR_EPI_GRADMAG, three stencils on one patch); every other request (multichannel Y[p,co] = b[co] + sum_{ci,o}
 * W_l[co][ci][o] V_l[ci](c_p + o)) runs on the gather map and needs the handle
 * built with APR_BUILD_GATHER3 / APR_BUILD_GATHER5 for d->k.  Supported
 * (c_in, c_out): k = 3: (1,1) (1,16) (16,16) (16,1) (2,3); k = 5: (1,1) (2,3).
 * k = 3, 16 -> 16 runs on matrix cores: with BF16 x and tree (16-byte aligned)
 * the weights are rounded to BF16 (FP32 accumulation); with FP32 x and tree
 * (16-byte aligned) FP32 throughout.  FP8 storage (network activations):
 * k = 3 only; x FP8 with (16,16) (4-byte aligned x and tree; BF16 weights on
 * matrix cores, FP8 values widened exactly) or (16,1), y of any type; and
 * FP32 / BF16 x with (1,16) or (16,16) into FP8 y.  The single-channel
 * LDS-patch path and the gradients do not take FP8. */

/* Gradient of apr_conv with respect to x (the transpose of the linear map
 * x -> y, bias excluded): same-level taps, taps of level-(l+1) particles that
 * read a level-l particle as their coarser source, and tree taps routed down
 * through the child means (adjoint of Section 3.4's average).  The last two
 * come from the inverse of the gather map, built with it.  dy: device FP32
 * [N_p][c_out]; w: FP32 weights as in apr_conv; dx: device FP32 [N_p][c_in]
 * (overwritten); dtree: device FP32 [N_t][c_in] scratch.  Needs the gather map
 * for d->k.  Deterministic.  Asynchronous. */
apr_status apr_conv_bwd_data(const apr_handle* h, const apr_conv_desc* d, const float* dy, const float* w,
                             float* dx, float* dtree, void* stream);

/* Workspace bytes of apr_conv_bwd_weight (FP64 block partials). */
size_t apr_conv_bwd_weight_ws(const apr_handle* h, const apr_conv_desc* d);

/* dw[l][co][ci][o] = sum over particles p of level l of dy[p][co] V_l[ci](c_p + o)
 * (summed over levels when d->n_wlevels == 1).  x, tree: as in apr_conv
 * (tree filled from x); dy: FP32 [N_p][c_out]; dw: FP32 (overwritten); ws:
 * device workspace of apr_conv_bwd_weight_ws bytes.  FP32 block sums, FP64
 * partials reduced in a fixed order: deterministic.  Asynchronous.
 * The 16 -> 16, k = 3 kernels of both gradients address their gathers with
 * 32-bit buffer offsets while the gathered arrays (x and the tree here, dy in
 * apr_conv_bwd_data) stay below 0xF0000000 bytes, and with 64-bit addresses
 * above; the environment variable APR_WIDE_OFFSETS=1 selects the second form
 * at every size, and =2 the weight gradient's two-buffer form that it takes
 * when x and the tree lie too far apart for one buffer (all forms give the
 * same bits; the variable exists for testing). */
apr_status apr_conv_bwd_weight(const apr_handle* h, const apr_conv_desc* d, const void* x, const void* tree,
                               const float* dy, float* dw, void* ws, size_t ws_bytes, void* stream);

/* Test support: for each listed particle and each tap (dz, dx, dy ascending)
 * write which element supplies V_l(c_p + o), computed by the convolution's own
 * patch builder: -1 outside the image, else (source << 40) | index with
 * source 1 = APR level l, 2 = APR level l-1, 3 = tree level l; index is the
 * global particle or tree index.  particles: device int64 [n] (must be sorted
 * ascending and unique); out: device int64 [n][k^3].  Asynchronous. */
apr_status apr_neighbor_map(const apr_handle* h, int32_t k, const int64_t* particles, int64_t n,
                            int64_t* out, void* stream);

/* ----------------------------------------------------------------------
 * Richardson-Lucy deconvolution on the APR (Section 6.2)
 * ---------------------------------------------------------------------- */

/* Bytes of device workspace apr_richardson_lucy needs for this handle. */
size_t apr_richardson_lucy_workspace(const apr_handle* h);

/* n_iter iterations of  i <- i * corr(u / max(corr(i, w_flip_l), eps), w_l)^power
 * with i_0 = init (u when init is NULL) and eps = eps_rel * max|u|.  With
 * power = 1 this is the Richardson-Lucy update of Section 6.2 with both
 * convolutions replaced by APR convolutions and the PSF restricted to every
 * level (Eq. restrict_stenc); power > 1 over-relaxes the multiplicative
 * update (an accelerated variant, not in the paper).  w and w_flip: device
 * FP32 [n_wlevels][k^3], the per-level PSF and per-level flipped PSF
 * (apr_stencil_levels with flip = 0 and 1); u, init, out: device FP32 [N_p]
 * (out may alias neither); work: device workspace of
 * apr_richardson_lucy_workspace bytes.  Every tree is refilled from the array
 * it belongs to.  Asynchronous. */
apr_status apr_richardson_lucy(const apr_handle* h, int32_t k, int32_t n_wlevels, const float* w,
                               const float* w_flip, const float* u, const float* init, float* out,
                               int32_t n_iter, float eps_rel, float power, void* work, void* stream);

/* Allocation-free variant of apr_richardson_lucy, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments and results as
 * apr_richardson_lucy without `work`: the workspace is a static device array
 * of APR_RL_STATIC_FLOATS floats (64 MiB) per GPU, held until the process
 * ends, so the handle must satisfy N_t + 3 N_p + 1088 <= APR_RL_STATIC_FLOATS
 * (about 5.3M particles); larger handles return APR_EINVAL and launch
 * nothing.  Calls no allocating routine.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (several streams or threads)
 * race and give undefined results; serialize them.  Asynchronous. */
#define APR_RL_STATIC_FLOATS (1u << 24)
apr_status apr_richardson_lucy_static(const apr_handle* h, int32_t k, int32_t n_wlevels, const float* w,
                                      const float* w_flip, const float* u, const float* init, float* out,
                                      int32_t n_iter, float eps_rel, float power, void* stream);

/* ----------------------------------------------------------------------
 * Learned surrogate support.  Section 7 proposes CNNs made of APR
 * convolution layers whose filters are learned per resolution level by
 * back-propagating through the interpolation across levels.  These calls are
 * the non-convolution pieces of such a network's training and inference:
 * statistics, normalisation, activation and bias gradients, the loss, the
 * optimiser step and the per-level weight layout.  Reductions use a fixed
 * grid with FP64 partials summed in a fixed order (deterministic).
 * ---------------------------------------------------------------------- */

/* Bytes of device workspace of apr_moments / apr_relu_bias_grad (for up to
 * `channels` channels) / apr_rel_l2. */
size_t apr_nn_workspace(int32_t channels);

/* stats[0] = mean, stats[1] = population standard deviation (1 when zero) of
 * v_i = u_i (op 0) or v_i = log(max(u_i, 1)) (op 1) over n values, FP64.
 * u: device FP32 [n]; stats: device FP64 [2].  Asynchronous. */
apr_status apr_moments(int32_t op, const float* u, int64_t n, double* stats, void* ws, void* stream);

/* out_i = f_op(a_i, b_i) with (mu, sd) = stats, FP64 arithmetic, a+ = max(a, 1):
 *   0: (a - mu)/sd     1: (a - b)/sd               2: b + sd*a       3: sd*a
 *   4: (log a+ - mu)/sd  5: (log a+ - log b+)/sd   6: b*exp(sd*a)    7: sd*a*b
 * (ops 0-3: additive residual network, 4-7: multiplicative residual).
 * a, b, out: device FP32 [n] (b unused by ops 0, 3, 4; out may alias a or
 * b).  Asynchronous. */
apr_status apr_pointwise(int32_t op, const float* a, const float* b, int64_t n, const double* stats, float* out,
                         void* stream);

/* dy_pre = dy * [y > 0] (relu != 0) or dy (relu == 0) over rows*c values;
 * db[j] = sum_p dy_pre[p][j] (FP64 partials) when db != NULL.  y, dy, dy_pre:
 * device FP32 [rows][c] (dy_pre may alias dy); db: device FP32 [c], c <= 256.
 * Asynchronous. */
apr_status apr_relu_bias_grad(const float* y, const float* dy, int64_t rows, int32_t c, int32_t relu,
                              float* dy_pre, float* db, void* ws, void* stream);

/* out[0] = |a - b|^2 / |b|^2 and out[1] = |b|^2 (FP64; out[0] = |a - b|^2 when
 * b = 0); when grad != NULL, grad = grad_scale * 2 (a - b) / |b|^2, the
 * gradient of grad_scale * out[0] with respect to a.  a, b, grad: device FP32
 * [n]; out: device FP64 [2].  Asynchronous. */
apr_status apr_rel_l2(const float* a, const float* b, int64_t n, double* out, float* grad, float grad_scale,
                      void* ws, void* stream);

/* One Adam step (bias-corrected moments, step >= 1) on n parameters:
 * m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).  Device FP32.
 * Asynchronous. */
apr_status apr_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                    float eps, int32_t step, void* stream);

/* Per-level weights from weight sets: set s serves the levels at distance s
 * from the finest level (l = l_max - s), the last set every coarser level
 * too (Section 7's per-level filters, tied across images of different depth).
 * dir 0: out[l - l_min][:] = in[set(l)][:]  (in [n_sets][per_set] ->
 * out [l_max-l_min+1][per_set]);  dir 1: out[s][:] = sum of in[l - l_min][:]
 * over the levels of set s in ascending l (the gradient of dir 0).  Device
 * FP32, in and out must not alias.  Asynchronous. */
apr_status apr_level_weights(int32_t dir, const float* in, float* out, int64_t per_set, int32_t n_sets,
                             int32_t l_min, int32_t l_max, void* stream);

/* Message of the last failing call on this thread ("" if none). */
/* ---- APR construction on the device (Section 2.3) ------------------------
 * Builds the APR of a synthetic sphere-field image on the GPU: the particle
 * LinearAccess (Algorithm 1) and the particle values.
 *  - Level rule: a location at distance d from the nearest sphere surface
 *    asks for level l_max - floor(log2(1 + d/2)); a cell of side
 *    s = 2^(l_max - l) pixels is split when some point of the box spanned by
 *    its pixel centres lies at d < 2 (s - 1).  (The paper derives the level
 *    function from the image gradient and its local error scale; this rule
 *    stands in for it on the synthetic inputs.)
 *  - The Pulling Scheme's partition: from fine to coarse, the parent of every
 *    cell touching (26-neighbourhood) a split cell of its level is split, so
 *    neighbouring particle levels differ by at most one (Section 5.1); the
 *    particles are the unsplit cells under split parents (all of level
 *    l_min exist).
 *  - Values: average downsampling (Section 2.3) of the image
 *    clean = background + (foreground - background) (G * 1_union), G the
 *    normalised Gaussian of edge_sigma pixels truncated at 4 sigma (zeros
 *    outside the image; edge_sigma 0 = no blur), a pixel inside a sphere when
 *    its centre is within the radius.  With `noise`, the sum S over a cell of
 *    n pixels becomes S + sqrt(S) Z (the Gaussian limit of the Poisson law of
 *    S), Z = (sum of 12 uniforms) - 6 from Philox4x64-10 with counter
 *    (level << 48 | z << 32 | x << 16 | y, block 0..2, 0, 0) and key
 *    (seed, 0), each uniform (word >> 11) * 2^-53; value = sum / n.
 * Distance and inside tests are FP64 in a fixed order; blur and sums FP64
 * accumulation (the image itself is FP32).  Synchronizes `stream`.  Device
 * scratch: about 8 bytes per pixel during the call.
 * Errors: APR_EINVAL (dims, l_min, sphere list), APR_EUNSUPPORTED (y size
 * above 65535, 2^32 or more words of level bitmaps), APR_ENOMEM. */
typedef struct {
  int32_t dims[3];          /* image (N_z, N_x, N_y) */
  int32_t l_min;            /* coarsest particle level */
  int64_t n_spheres;
  const double* centres;    /* host [n_spheres][3], (z, x, y) in pixel units (pixel p spans [p, p+1)) */
  const double* radii;      /* host [n_spheres] */
  double background, foreground, edge_sigma;
  int32_t noise;            /* 1: cell noise as above */
  uint64_t seed;
} apr_sphere_field_desc;

typedef struct apr_field apr_field;   /* the built APR; owns its device arrays */

typedef struct {
  int32_t dims[3];
  int32_t l_min, l_max;
  int64_t n_particles, n_rows;
  const uint16_t* y_idx;    /* device [n_particles], Algorithm 1's y */
  const uint64_t* xz_end;   /* device [n_rows], inclusive row ends (rows l -> z -> x) */
  const float* values;      /* device [n_particles] */
} apr_field_info;

apr_status apr_sphere_field(const apr_sphere_field_desc* desc, void* stream, apr_field** out);
apr_status apr_field_get_info(const apr_field* f, apr_field_info* out);
apr_status apr_field_destroy(apr_field* f);   /* frees the field's device arrays */

const char* apr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* APRCONV_H */
