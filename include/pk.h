/*
 * pk.h -- C interface of libpk: line-of-sight-dependent power-spectrum multipoles
 * (P_0, P_2, P_4) of a galaxy catalogue with the FFT implementation of the Yamamoto
 * estimator (Bianchi, Gil-Marin, Ruggeri & Percival 2015), on one AMD MI355X (gfx950).
 *
 * What is computed (the paper's statement of the problem):
 *   Sec. 2, Eq. (1)   the FKP field F = w (n - alpha n_s) of galaxies and randoms, with
 *                     alpha = sum_g w / sum_r w and I = int w^2 nbar^2 dr;
 *   Sec. 3, Eq. (5)   A_n(k) = int (khat . rhat)^n F(r) e^{ik.r} dr, each particle using
 *                     its own line of sight rhat = (x - observer)/|x - observer|;
 *   Sec. 3, Eqs. (9)-(13)  A_2 and A_4 from the FFTs of 6 and 15 grids F rhat_i rhat_j
 *                     and F rhat_i^2 rhat_j rhat_l (1, 7 or 22 FFTs for ell_max 0, 2, 4);
 *                     ell_max = 6 adds A_6 from the 28 degree-6 grids (the higher-order
 *                     decomposition Sec. 3 mentions) and P_6 = 13/(16 I)
 *                     <A_0 (231 A_6 - 315 A_4 + 105 A_2 - 5 A_0)^*>;
 *   Sec. 3, Eqs. (6)-(8)   P_0 = <|A_0|^2>/I - noise, P_2 = 5/(2I) <A_0 (3A_2 - A_0)^*>,
 *                     P_4 = 9/(8I) <A_0 (35 A_4 - 30 A_2 + 3 A_0)^*>, shell-averaged;
 *   Sec. 2, Eq. (3)   shot noise subtracted from ell = 0 only;
 *   Sec. 4            cloud-in-cell (or triangular-shaped-cloud) assignment on a
 *                     periodic cube, corrected for the assignment window (Jing 2005).
 *
 * Discrete readings (where the paper leaves a choice):
 *   alpha = sum_g w / sum_r w;  I = alpha sum_r w^2 nbar (norm_from = 0) or
 *   sum_g w^2 nbar (norm_from = 1);  S = sum_g w^2 + alpha^2 sum_r w^2.
 *   Nodes at box_min + j H, H = L/N. CIC: i = floor(u), weights (1-f, f) on (i, i+1).
 *   TSC: i = floor(u + 1/2), d = u - i, weights (1/2 (1/2-d)^2, 3/4 - d^2, 1/2 (1/2+d)^2)
 *   on (i-1, i, i+1). Indices wrap modulo N.
 *   A mode n (integer vector, components in [-N/2, N/2)) belongs to bin b when
 *   b dn <= |n| < (b+1) dn (exact integer test on |n|^2); n = 0 is excluded.
 *   compensate = 0: no correction, noise S; 1: divide by W^2, noise S;
 *   2 (default): divide by W^2 and subtract the aliased noise S prod_i C_p(n_i) / W^2,
 *   W = prod_i sinc^p(pi n_i / N), p = 2 (CIC) or 3 (TSC),
 *   C_2 = 1 - 2/3 s^2, C_3 = 1 - s^2 + 2/15 s^4, s = sin(pi n_i / N).
 *
 * Memory: every device pointer below is borrowed and read only; the library
 * allocates no device memory. All scratch lives in the caller's workspace, sized by
 * pk_workspace_size(), and all work is queued on the caller's HIP stream.
 * Calls that share a workspace must not overlap.
 */
#ifndef PK_H
#define PK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pk_status;

#define PK_OK 0
#define PK_EINVAL (-1)      /* null pointer, bad enum, dn < 1, L <= 0, nbins*dn > N/2, n < 0, nbar missing */
#define PK_ERANGE (-2)      /* a particle outside [box_min, box_min + L) on some axis */
#define PK_EDOM (-3)        /* non-finite xyz / w / nbar, a particle at the observer, sum_r w = 0, I <= 0 */
#define PK_EWORKSPACE (-4)  /* workspace null or smaller than pk_workspace_size() */
#define PK_EDEVICE (-5)     /* a HIP runtime error */
#define PK_ENOTSUP (-6)     /* N not a supported FFT size, ell_max = 6 at N = 2048, or more than 2^31 - 1 particles */

#define PK_CIC 2
#define PK_TSC 3

/* One catalogue, in device memory.
 *   xyz   float32 (n, 3) row-major positions, same coordinates as box_min and observer
 *   w     float32 (n) weights
 *   nbar  float32 (n) expected number density at each point; may be NULL when the
 *         normalisation does not read it (galaxies with norm_from = 0, randoms with
 *         norm_from = 1)
 *   n     number of points (>= 0) */
typedef struct {
  const float* xyz;
  const float* w;
  const float* nbar;
  int64_t n;
} pk_catalog;

/* Estimator configuration (host memory). */
typedef struct {
  int32_t N;           /* grid side: 8, 16, 32, 64, 128, 256, 512, 1024 or 2048 */
  int32_t assign;      /* PK_CIC or PK_TSC */
  int32_t ell_max;     /* 0, 2, 4 or 6 -> 1, 7, 22 or 50 LOS-weighted grids (6: N <= 1024) */
  int32_t los;         /* 0: each particle's own line of sight; 1: fixed +z (plane-parallel) */
  int32_t compensate;  /* 0, 1 or 2 (see above) */
  int32_t dn;          /* bin width in units of the fundamental mode 2 pi / L, >= 1 */
  int32_t nbins;       /* number of bins, nbins * dn <= N / 2 */
  int32_t norm_from;   /* 0: I from the randoms, 1: I from the galaxies */
  double box_min[3];   /* lower corner of the periodic FFT cube */
  double L;            /* side of the cube */
  double observer[3];  /* origin of the lines of sight */
  int32_t x_planes;    /* z planes per slab of the x and y transforms: 0 = automatic (all
                        * N planes while the 1, 7, 22 or 50 x-transformed grids, 8 G N^2 Kx bytes
                        * with Kx = nbins dn rounded up to the kx tile, take at most 128 GiB,
                        * i.e. every N up to 1024; otherwise the largest power of two of
                        * planes whose two slabs fit in 8 GiB), or a power of two <= N. With
                        * x_planes < N the transforms run slab by slab and the x-transformed
                        * grids are held for two slabs only (out of core: at N = 2048 the 22
                        * grids would take 756 GB); the y transform of one slab runs on a
                        * second stream of the library while the x transform of the next runs
                        * on the caller's stream (not while the stream is being captured into
                        * a graph). The result is the same to FP32 rounding. */
} pk_config;

/* Results (host memory, caller-owned arrays).
 *   k_eff[nbins]   mode-averaged |k| of each bin (0 for an empty bin)
 *   P[(ell_max/2 + 1) * nbins]  P_0 then P_2, P_4 (and P_6), bin-fastest (0 for an empty bin)
 *   noise[nbins]   shell mean of the noise subtracted from P_0, divided by I
 *   nmodes[nbins]  number of modes of the full N^3 lattice in each bin
 *   wedges[2][nbins]  P_perp (mu in [0, 1/2]) then P_par (mu in [1/2, 1]) from the
 *                  multipoles, the wedges of Sec. 5: P_0 -+ 3/8 P_2 +- 15/128 P_4 (the
 *                  top-hat means of L_2 and L_4 over the two ranges); multipoles above
 *                  ell_max are taken as 0, and P_6 is not used (the paper's form)
 * Scalars alpha, I and S (sum_g w^2 + alpha^2 sum_r w^2) are filled in. Any array
 * pointer may be NULL to skip it. On error nothing is written. */
typedef struct {
  double* k_eff;
  double* P;
  double* noise;
  int64_t* nmodes;
  double alpha;
  double I;
  double S;
  double* wedges;
} pk_result;

/* Bytes of device workspace pk_multipoles needs for this configuration and these
 * catalogue sizes. Returns PK_EINVAL / PK_ENOTSUP for an invalid configuration. */
pk_status pk_workspace_size(const pk_config* cfg, int64_t n_gal, int64_t n_ran, size_t* bytes);

/* The whole estimator: catalogue scalars, LOS-weighted assignment, the batched FFTs,
 * the k-hat contraction, shell binning, shot noise and normalisation. Queues all work
 * on `hip_stream` (a hipStream_t; NULL = the default stream), then waits for it and
 * copies the FP64 results to `out`. `workspace` is device memory of at least
 * pk_workspace_size() bytes, 256-byte aligned; its prior contents do not matter. */
pk_status pk_multipoles(const pk_config* cfg, const pk_catalog* gal, const pk_catalog* ran,
                        void* workspace, size_t workspace_bytes, pk_result* out, void* hip_stream);

/* Bytes of the fixed scratch array that pk_multipoles_noalloc works in (64 MiB). */
#define PK_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code being captured into a HIP graph,
 * tight serving loops, harnesses that forbid allocation): pk_multipoles with its
 * workspace replaced by a fixed array of PK_NOALLOC_SCRATCH_BYTES in the library's device
 * image (each GPU the library runs on holds its own copy from the first launch of any
 * libpk kernel until the process ends). The call allocates nothing: no hipMalloc, no
 * stream or event creation, no second stream for slabs; the result is staged in a
 * per-thread host buffer. Same inputs, outputs, synchronous behaviour and errors as
 * pk_multipoles, plus PK_EWORKSPACE when the configuration and catalogue sizes need more
 * scratch than the array holds (pk_workspace_size() > PK_NOALLOC_SCRATCH_BYTES, e.g. a
 * 64^3 grid with about 1e6 particles fits, a 256^3 grid does not) or more than 1024
 * result values. All calls on one GPU share its array: calls that overlap in time on
 * one GPU (several host threads or streams) race and give wrong results; serialise them.
 * Every part of the array a call reads is written by that call first. */
pk_status pk_multipoles_noalloc(const pk_config* cfg, const pk_catalog* gal, const pk_catalog* ran,
                                pk_result* out, void* hip_stream);

/* Asynchronous form: queues the same work and leaves the results in device memory at
 * `d_result` (float64, pk_result_doubles(cfg) values: k_eff[nbins], P[(ell_max/2+1) nbins],
 * noise[nbins], nmodes[nbins] (as doubles), wedges[2 nbins], then alpha, I, S and the
 * error-flag word).
 * Returns after queueing; input errors found on the device appear only in the flag word
 * (bit 1 non-finite position, 2 out of box, 4 particle at the observer, 8 non-finite
 * weight or nbar, 16 sum_r w = 0 or I <= 0). Launch-time errors are returned. */
pk_status pk_multipoles_async(const pk_config* cfg, const pk_catalog* gal, const pk_catalog* ran,
                              void* workspace, size_t workspace_bytes, double* d_result,
                              void* hip_stream);

/* Batched estimator for ensembles of mocks (many catalogues of uneven size, each with
 * its own configuration). Mocks are processed in order over `lanes` (1 or 2) internal
 * HIP streams, each with its own slice of the workspace, so that one mock's short
 * kernels overlap another's transforms. Each mock's stages are captured into a hipGraph;
 * mocks of the same size class (N, assign, ell_max, nbins, dn, los, compensate,
 * norm_from and slab height) reuse
 * the instantiated graph of their lane. Work starts after everything already queued on
 * `hip_stream` and the call returns after all mocks are done.
 *   cfgs, gals, rans  arrays of n_mocks configurations and device catalogues
 *   workspace         device memory of pk_workspace_size_batch() bytes for the same
 *                     arguments and lanes, 256-byte aligned
 *   outs              n_mocks result structs (host arrays as for pk_multipoles)
 *   per_mock          n_mocks statuses (PK_OK or the mock's error; outs[i] is untouched
 *                     when per_mock[i] != PK_OK)
 * Returns PK_OK when every mock was run (per-mock input errors are reported in
 * per_mock), or the first argument / device error. */
pk_status pk_workspace_size_batch(const pk_config* cfgs, const pk_catalog* gals, const pk_catalog* rans,
                                  int32_t n_mocks, int32_t lanes, size_t* bytes);
pk_status pk_multipoles_batch(const pk_config* cfgs, const pk_catalog* gals, const pk_catalog* rans,
                              int32_t n_mocks, int32_t lanes, void* workspace, size_t workspace_bytes,
                              pk_result* outs, pk_status* per_mock, void* hip_stream);

/* Number of doubles pk_multipoles_async writes. */
int64_t pk_result_doubles(const pk_config* cfg);

/* Stage entry point for tests: runs the catalogue scalars, the row sort and the fused
 * LOS-weighted assignment with the FFT along x for the first slab of planes
 * [0, x_planes) (all planes when the plan holds them all), then stops, leaving the
 * x-transformed grids of that slab in the workspace (same kernels as pk_multipoles).
 * Queued on `hip_stream`. */
pk_status pk_stage_xgrids(const pk_config* cfg, const pk_catalog* gal, const pk_catalog* ran,
                          void* workspace, size_t workspace_bytes, void* hip_stream);

/* Where pk_stage_xgrids leaves grid `m` (a monomial with a power of rhat_z below 2: only
 * those are stored, 1, 6, 15 or 28 of the 1, 7, 22 or 50; any other monomial is an integer
 * combination of them through rhat_x^2 + rhat_y^2 + rhat_z^2 = 1, which the y transform
 * applies, and returns PK_EINVAL here): for z < x_planes (pk_x_planes), y < N,
 * kx < kx_count, the x-transformed (unnormalised, e^{-2 pi i kx x / N}) row of F rhat^m at
 * (y, z), complex64 values starting at byte `offset` of the workspace and stored
 * tile-major, X[z][kx / W][y][kx % W], with W the tile width pk_hgrid_layout reports
 * (16 up to N = 512, 8 at 1024, 4 at 2048), so that the y transform reads each tile of a
 * plane as one contiguous run. Monomial m has exponents (a, b, c) of rhat_x, rhat_y,
 * rhat_z as returned by pk_monomial. */
pk_status pk_xgrid_layout(const pk_config* cfg, int64_t n_gal, int64_t n_ran, int32_t m,
                          size_t* offset, int32_t* kx_count);

/* Stage entry point for tests: runs everything pk_multipoles runs up to and including
 * the transforms along y of every slab (same kernels), then stops, leaving in the
 * workspace the z-power groups H of the contraction of Sec. 3, Eqs. (10) and (12):
 * A_n = |t|^-n sum_{a+b+c=n} (n!/(a! b! c!)) tx^a ty^b tz^c G_abc with t = 2 n_vec / N
 * (k-hat = t / |t|) and G_abc the transform of F rhat_x^a rhat_y^b rhat_z^c, is regrouped by
 * the power c of tz before the transform along z:
 *   H_(n,c)(kx, ky, z) = sum_{a+b=n-c} (n!/(a! b! c!)) tx^a ty^b Y_abc(kx, ky, z),
 * Y_abc = the unnormalised transform along x and y (e^{-2 pi i (kx x + ky y)/N}) of plane z
 * of F rhat^(a,b,c), for kx in [0, Kx) and |ky| <= ky_max(kx tile) (the modes of the
 * binned sphere). Queued on `hip_stream`. Errors as pk_multipoles_async. */
pk_status pk_stage_fft(const pk_config* cfg, const pk_catalog* gal, const pk_catalog* ran,
                       void* workspace, size_t workspace_bytes, void* hip_stream);

/* Where pk_stage_fft leaves group `group` (0 .. 1/4/9/16 - 1, in the order of pk_zgroup)
 * for kx tile `kx_tile` (columns kx = kx_tile * tile_cols .. + tile_cols - 1, up to
 * Kx = nbins dn rounded up to tile_cols): complex64 values at byte `offset` of the
 * workspace, laid out [z][ky + ky_max][column] for z < N, |ky| <= ky_max. */
pk_status pk_hgrid_layout(const pk_config* cfg, int64_t n_gal, int64_t n_ran, int32_t group, int32_t kx_tile,
                          size_t* offset, int32_t* ky_max, int32_t* tile_cols);

/* Inspection entry point for tests (host only, no GPU): the weights with which the y
 * transform forms the z-power groups from the stored grids (pk_xgrid_layout), with sets of
 * up to `max_groups` groups per launch (6: the 8-value y schedule up to N = 512; 3: the
 * 16-value schedule, and the 8-value one from N = 1024 on). Term i adds
 * coef[i] tx^a[i] ty^b[i] Y_grid[i] to H_group[i] (Y: the grid transformed along x and y;
 * grid[i] a monomial index as for pk_monomial, group[i] as for pk_zgroup), in launch
 * set[i]; over all terms, sum_c tz^c H_(n,c) = sum_{a+b+c=n} (n!/(a! b! c!)) tx^a ty^b tz^c
 * Y_abc with every monomial of power of rhat_z of 2 or more written through
 * rhat_x^2 + rhat_y^2 + rhat_z^2 = 1 (Sec. 3, Eqs. 10 and 12). Writes the first `cap` terms
 * into the caller's arrays and returns the number of terms; -1 (PK_EINVAL detail) for an
 * unsupported ell_max or max_groups, or null arrays with cap > 0. */
int32_t pk_ygroup_terms(int32_t ell_max, int32_t max_groups, int32_t cap, int32_t* set, int32_t* group,
                        int32_t* grid, float* coef, int32_t* a, int32_t* b);

/* Degree n and power c of tz of z-power group `group`: the groups run over n = 0, 2, ..
 * ell_max and, for each n, c = 0 .. n. PK_EINVAL past the last group. */
pk_status pk_zgroup(int32_t ell_max, int32_t group, int32_t* degree, int32_t* z_power);

/* Stage entry point for tests: the transform along z, the k-hat contraction of Eqs. (10)
 * and (12), the compensation, the shell binning and the finalisation of Eqs. (6)-(8) and
 * (3), on the groups H and the catalogue scalars that pk_stage_fft left in `workspace`
 * for the same configuration and catalogue sizes (the same kernels as pk_multipoles).
 * Synchronous; fills `out` like pk_multipoles (input errors flagged by the earlier stage
 * are returned here). */
pk_status pk_stage_contract(const pk_config* cfg, int64_t n_gal, int64_t n_ran, void* workspace,
                            size_t workspace_bytes, pk_result* out, void* hip_stream);

/* The slab height the plan of this configuration uses (cfg->x_planes, or the automatic
 * choice when that is 0). PK_EINVAL / PK_ENOTSUP for an invalid configuration. */
pk_status pk_x_planes(const pk_config* cfg, int64_t n_gal, int64_t n_ran, int32_t* planes);

/* Schedules of the column transforms (the FFTs along y and along z): the values each
 * thread holds, 16 (radices 16, 8, 4 at N = 512: fewer threads per transform) or 8
 * (radices 8, 8, 8: half the registers). With 8 values the y pass sums up to 6 z-power
 * groups per launch, so each stored x-transformed grid is loaded once per parity of the
 * power of tz (ell_max <= 4); with 16 values its registers hold 3 groups, and grids that
 * several such sets need are loaded once per set. A process-wide table keyed by
 * (N, ell_max), default 8 for both passes, read when a call plans its work (not
 * thread-safe against concurrent changes). Both schedules compute the same transform;
 * results agree to FP32 rounding. At N = 2048 only the 8-value schedule is built (16
 * values per thread would need more than 256 registers): it is the only value reported
 * and accepted there. PK_EINVAL for an unsupported N or ell_max or values other than 8
 * and 16. */
pk_status pk_set_schedule(int32_t N, int32_t ell_max, int32_t y_values, int32_t z_values);
pk_status pk_get_schedule(int32_t N, int32_t ell_max, int32_t* y_values, int32_t* z_values);

/* Autotuner of those schedules: runs pk_multipoles once on the given inputs (same
 * arguments, workspace and errors), then times `reps` launches of every schedule of the
 * y pass (on the last slab when the plan runs several) and of the z pass on that data
 * with HIP events on hip_stream, stores the fastest pair in the table for (cfg->N,
 * cfg->ell_max) and returns it. Synchronous. */
pk_status pk_autotune(const pk_config* cfg, const pk_catalog* gal, const pk_catalog* ran, void* workspace,
                      size_t workspace_bytes, int32_t reps, int32_t* y_values, int32_t* z_values,
                      void* hip_stream);

/* Stage timing, for measurement. While enabled (process-wide, not thread-safe), each
 * pk_multipoles / pk_multipoles_async call records HIP events on its stream around its
 * stages: 0 workspace init, 1 catalogue scalars, 2 row sort, 3 LOS assignment + x FFT,
 * 4 y FFT + z-power grouping, 5 z FFT + contraction + binning, 6 finalize. When the
 * plan runs several slabs (x_planes < N), stage 3 covers the x and y transforms of all
 * slabs and stage 4 is empty.
 * pk_stage_times waits for the last call's events and writes up to n durations in
 * milliseconds; it returns the number of stages (7), or -1 if timing has no record. */
pk_status pk_set_stage_timing(int32_t enable);
int32_t pk_stage_times(double* ms, int32_t n);
const char* pk_stage_name(int32_t i);

/* ---------------------------------------------------------------------------------
 * Coarse-grid correction network. Callers: the correction that maps multipoles measured
 * on a coarse grid to the fine-grid estimate (aliasing and window), trained on pairs of
 * coarse- and fine-grid measurements made by pk_multipoles itself; the plain fine-grid
 * estimator stays the reference and the fallback.
 * Shape: din inputs (1..64), 3 hidden layers of width 128 with SiLU, dout outputs (1..16).
 * Canonical parameter vector (float32, device): for each of the 4 layers, W [in][out]
 * row-major then b [out]; pk_mlp_num_params() floats. The state buffer (device,
 * pk_mlp_state_bytes) holds FP32 master weights, Adam moments and BF16 copies; the
 * workspace (device, pk_mlp_workspace_bytes(rows)) holds activations for `rows` rows.
 * GEMMs run on BF16 MFMA with FP32 accumulation; reductions have a fixed order. All
 * calls queue work on hip_stream and return; results are valid after the stream syncs.
 * --------------------------------------------------------------------------------- */
typedef struct {
  int32_t din;
  int32_t dout;
  int32_t width;  /* must be 128 */
  int32_t depth;  /* must be 3 */
} pk_mlp_shape;

size_t pk_mlp_state_bytes(const pk_mlp_shape* shape);
size_t pk_mlp_workspace_bytes(const pk_mlp_shape* shape, int64_t rows);
int64_t pk_mlp_num_params(const pk_mlp_shape* shape);
/* Loads parameters (device float32, canonical order), zeroes the Adam moments. */
pk_status pk_mlp_set_params(const pk_mlp_shape* shape, void* state, const float* d_params, void* hip_stream);
pk_status pk_mlp_get_params(const pk_mlp_shape* shape, const void* state, float* d_params, void* hip_stream);
/* y[rows][dout] = network(x[rows][din]), float32 device arrays. */
pk_status pk_mlp_forward(const pk_mlp_shape* shape, const void* state, const float* d_x, int64_t rows, float* d_y,
                         void* workspace, size_t workspace_bytes, void* hip_stream);
/* Mean-squared-error loss against t[rows][dout] (to *d_loss, float32 device scalar) and
 * its gradient (canonical order, to d_grads unless NULL); parameters unchanged. */
pk_status pk_mlp_gradients(const pk_mlp_shape* shape, const void* state, const float* d_x, const float* d_t,
                           int64_t rows, float* d_grads, float* d_loss, void* workspace, size_t workspace_bytes,
                           void* hip_stream);
/* One Adam step (b1 0.9, b2 0.999, eps 1e-8; `step` counts from 1) on the batch. */
pk_status pk_mlp_train_step(const pk_mlp_shape* shape, void* state, const float* d_x, const float* d_t, int64_t rows,
                            float lr, int32_t step, float* d_loss, void* workspace, size_t workspace_bytes,
                            void* hip_stream);
/* The same Adam step (the kernel pk_mlp_train_step ends with) applied with a caller's
 * gradient vector d_grads (device float32, pk_mlp_num_params values, canonical order):
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * w -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps), in FP32 elementwise
 * (Kingma & Ba's Adam), then the BF16 copies of the weights are refreshed. */
pk_status pk_mlp_adam_apply(const pk_mlp_shape* shape, void* state, const float* d_grads, float lr, int32_t step,
                            void* hip_stream);

/* Number of LOS-weighted grids for ell_max (1, 7, 22, 50), and the exponents of grid m. */
int32_t pk_num_grids(int32_t ell_max);
pk_status pk_monomial(int32_t m, int32_t* a, int32_t* b, int32_t* c);

/* Static description of a status code. */
const char* pk_status_string(pk_status s);

/* Detail of the last error on the calling thread, copied into buf (NUL-terminated,
 * truncated to n bytes). Returns the full length of the message. */
size_t pk_last_error(char* buf, size_t n);

/* The same call under its longer name: copies the calling thread's last error detail into
 * buf exactly as pk_last_error does and returns the message's full length. */
size_t pk_last_error_detail(char* buf, size_t n);

#ifdef __cplusplus
}
#endif

#endif /* PK_H */
