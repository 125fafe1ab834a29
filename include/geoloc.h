/*
 * geoloc.h -- C ABI of the MI355X (gfx950) position-domain correlation library.
 *
 * Direct geolocation (Sec. III, Algorithm 1) searches a grid of candidate ground
 * points. For every point p, every snapshot (here: step k of L samples of one
 * contiguous capture) and every receiver pair (i, j), the expected TDOA and FDOA
 * follow from the receivers' known positions and velocities (Sec. II-B,
 * Eq. (3)-(10)); receiver j's samples are delay-shifted and the product with
 * receiver i is Doppler-rotated and summed (Eq. (11)); the per-step grids are
 * accumulated non-coherently and the peak is the emitter estimate.
 *
 *   J(p) = sum_pairs sum_k |C_k(p)|^2          (POWER, default)  or  sum |C_k(p)|  (MAG)
 *   C_k(p) = sum_{n=kL}^{kL+L-1} y_i[n] conj(yt_j[n]) exp(+j 2 pi nu_k(p) t_n)
 *   t_n = (n - kL - (L-1)/2) / f_s                       (time measured from the step centre)
 *   D_k(p) = (tau_j - tau_i) f_s, nu_k(p) = f_j - f_i    (Eq. (7)-(9), delay in samples)
 *   LINEAR: yt_j[n] = (1-a) y_j[n+d0] + a y_j[n+d0+1], d0 = floor(D), a = D - d0
 *   ROUND : yt_j[n] = y_j[n + round(D)]  (Eq. (9); halves round away from zero)
 *   SINC  : yt_j[n] = sum_{t=-3}^{4} w_t(a) y_j[n + d0 + t]  (eight-tap windowed sinc)
 *   y_j[m] = 0 for m outside [0, N).
 *
 * Conventions
 *   - Every call returns a status (GEOLOC_OK or a negative code); nothing throws or
 *     aborts across this boundary. Out-parameters are untouched on error, and
 *     geoloc_last_error() returns a thread-local detail string.
 *   - The caller owns every input and output buffer. A plan owns its device scratch
 *     until geoloc_destroy(). geoloc_map() and geoloc_geometry() are asynchronous on
 *     the caller's stream; geoloc_argmax() synchronises that stream.
 *   - A plan must not be used from two threads at once; different plans are
 *     independent.
 *   - Flat point index = row * n_cols + col, rows = latitude (RECT grids); the
 *     position in the lat/lon arrays for POINTS grids.
 *   - Units: SI; angles in radians: geocentric latitude / longitude on a sphere
 *     (GEOLOC_EARTH_SPHERE), or geodetic latitude / longitude on the WGS-84 ellipsoid
 *     (GEOLOC_EARTH_WGS84), heights along the ellipsoid normal. Receiver states are ECEF
 *     in both cases.
 *   - Requires a gfx950 device; anything else returns GEOLOC_EDEVICE.
 */
#ifndef GEOLOC_H
#define GEOLOC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GEOLOC_ABI_VERSION 4

/* status codes */
#define GEOLOC_OK            0
#define GEOLOC_EINVAL       -1   /* invalid argument or descriptor */
#define GEOLOC_ENOMEM       -2   /* device or host allocation failed */
#define GEOLOC_EDEVICE      -3   /* no usable gfx950 device */
#define GEOLOC_ESTATE       -4   /* call out of order (e.g. plan already destroyed) */
#define GEOLOC_ENAN         -5   /* NaN found in a map by geoloc_argmax */
#define GEOLOC_EUNSUPPORTED -6   /* valid request the library does not implement */
#define GEOLOC_ELAUNCH      -7   /* a HIP runtime call or kernel launch failed */

/* method */
#define GEOLOC_DIRECT_FP32   0   /* Eq. (11) in FP32 with FP64 geometry; the per-point sums
                                    are factored through lag moments shared by a tile of
                                    points (256, 512 or 1024 cells of a RECT grid in a slanted tile
                                    chosen per map, 256 consecutive points of a POINTS
                                    list), with a Taylor remainder of at
                                    most 2^-24 of each Taylor block's magnitude sum (blocks
                                    of 64 or 256 samples, chosen per map from the Doppler
                                    spread over the tiles, or fixed by
                                    geoloc_set_taylor_block);
                                    tiles whose lags or Doppler shifts spread too widely are
                                    summed point by point */
#define GEOLOC_DIRECT_FP32_POINTWISE 3  /* the same map, every point summed on its own      */
#define GEOLOC_CAF_BF16      1   /* CAF table on MFMA, BF16 inputs, FP32 accumulate        */
#define GEOLOC_CAF_FP16      2   /* CAF table on MFMA, FP16 inputs, FP32 accumulate        */

/* delay_mode */
#define GEOLOC_DELAY_LINEAR  0   /* two-tap linear fractional delay (default)              */
#define GEOLOC_DELAY_ROUND   1   /* integer delay round(D), the paper's Eq. (9)            */
#define GEOLOC_DELAY_SINC    2   /* eight-tap windowed-sinc fractional delay:
                                    yt[n] = sum_{t=-3}^{4} w_t y_j[n + floor(D) + t],
                                    w_t = g(t - a) / sum_s g(s - a), a = D - floor(D),
                                    g(x) = sinc(x) I0(6 sqrt(1 - (x/4)^2)) / I0(6), |x| < 4;
                                    flat to better than 1e-3 up to a quarter of f_s where the
                                    two-tap delay loses up to 3 dB                          */

/* accum_mode */
#define GEOLOC_ACC_POWER     0   /* J = sum |C|^2 */
#define GEOLOC_ACC_MAG       1   /* J = sum |C|   */

/* grid_kind */
#define GEOLOC_GRID_RECT     0   /* lat[n_rows] x lon[n_cols] */
#define GEOLOC_GRID_POINTS   1   /* lat[P], lon[P], P = n_rows * n_cols */

/* earth models (grid -> ECEF, the transformation that precedes Eq. (3)) */
#define GEOLOC_EARTH_SPHERE  0   /* radius earth_radius_m, geocentric latitude              */
#define GEOLOC_EARTH_WGS84   1   /* WGS-84 ellipsoid (a = 6378137 m, 1/f = 298.257223563),
                                    geodetic latitude, height along the ellipsoid normal */

/* geoloc_map flags */
#define GEOLOC_ACCUMULATE    1u  /* add into J_dev instead of overwriting it */

typedef struct geoloc_plan_s* geoloc_plan_t;

/* Plan descriptor. Pointers are host pointers read only during geoloc_plan(). */
typedef struct geoloc_desc {
    int32_t n_rx;              /* receivers in the captures (>= 2)                        */
    int32_t n_pairs;           /* pairs summed into J; 0 -> all i < j                     */
    const int32_t* pairs;      /* [n_pairs][2] = (reference i, shifted j); NULL if n_pairs == 0 */
    int64_t n_samples;         /* N, samples per receiver                                 */
    int64_t step_len;          /* L; N must be a multiple of L (K = N / L steps)          */
    double fs_hz;              /* sample rate f_s (> 0)                                   */
    double fc_hz;              /* carrier f_c (> 0); lambda = c / f_c, c = 299792458 m/s  */
    int32_t grid_kind;         /* GEOLOC_GRID_RECT or GEOLOC_GRID_POINTS                  */
    int32_t _pad0;
    int64_t n_rows, n_cols;    /* grid shape; P = n_rows * n_cols (> 0)                   */
    const double* lat;         /* RECT: [n_rows]; POINTS: [P]  (radians; geodetic for WGS-84) */
    const double* lon;         /* RECT: [n_cols]; POINTS: [P]  (radians)                  */
    double earth_radius_m;     /* sphere radius (e.g. 6371000); unused for WGS-84         */
    double alt_m;              /* height of every candidate point above the surface       */
    int32_t method;            /* GEOLOC_DIRECT_FP32 / GEOLOC_CAF_BF16 / GEOLOC_CAF_FP16  */
    int32_t delay_mode;        /* GEOLOC_DELAY_LINEAR / GEOLOC_DELAY_ROUND / GEOLOC_DELAY_SINC */
    int32_t accum_mode;        /* GEOLOC_ACC_POWER / GEOLOC_ACC_MAG                       */
    int32_t caf_lags;          /* CAF: integer lags per table; 0 -> fit to the footprint  */
    int32_t caf_bins;          /* CAF: Doppler bins per table; 0 -> 256                   */
    int32_t caf_lag_lo_set;    /* CAF: nonzero -> use caf_lag_lo instead of fitting it    */
    int32_t caf_lag_lo;        /* CAF: first lag of the table (samples)                   */
    int32_t _pad1;
    double caf_nu_lo_hz;       /* CAF: first bin centre; NaN -> fit to the footprint      */
    double caf_nu_hi_hz;       /* CAF: last bin centre;  NaN -> fit to the footprint      */
    int32_t earth_model;       /* GEOLOC_EARTH_SPHERE (earth_radius_m) or GEOLOC_EARTH_WGS84 */
    int32_t _pad2;
    const double* alt_grid;    /* NULL, or the height (m) of every candidate point above the
                                  sphere / ellipsoid, added to alt_m (a terrain model):
                                  RECT [n_rows][n_cols], POINTS [P]; read only during
                                  geoloc_plan(); such a plan takes no geoloc_set_grid() */
} geoloc_desc;

/* Per-map inputs. */
typedef struct geoloc_inputs {
    const void* captures;      /* DEVICE pointer: complex64 interleaved (re, im float32),
                                  [n_rx][n_samples], 8-byte aligned; read-only           */
    const double* rx_state;    /* HOST pointer: [K][n_rx][6] ECEF position (m), velocity
                                  (m/s) of each receiver at each step's centre instant   */
    void* stream;              /* hipStream_t to run on; NULL = the null stream          */
} geoloc_inputs;

/* Plan facts, and kernel times accumulated since the last geoloc_set_timing();
 * filled by geoloc_info(), which waits for the timed kernels to finish. */
typedef struct geoloc_plan_info {
    int64_t n_points, n_steps, n_pairs, n_samples, step_len;
    int32_t method, delay_mode;
    int32_t caf_lag_lo, caf_lags, caf_bins, _pad;
    double caf_nu_lo_hz, caf_nu_hi_hz;
    int64_t device_bytes;      /* device scratch owned by the plan                       */
    int64_t timed_maps;        /* maps run with timing enabled                           */
    int64_t correlate_launches;/* launches of the dominant correlation kernel            */
    double geometry_ms;        /* summed HIP-event times of the geometry kernels (CAF: the
                                  window fit; the direct method evaluates its geometry
                                  inside the correlation kernels and reports 0 here)       */
    double correlate_ms;       /* ... of the correlation kernels (direct, or CAF GEMM)   */
    double interp_ms;          /* ... of the CAF interpolation kernels; for the direct
                                  method, of the per-point pass over (tile, step) pairs the
                                  factored kernel left to it                              */
    double map_ms;             /* ... of whole geoloc_map calls, first to last kernel    */
    int32_t tile_rows, tile_cols;   /* tile of the last map: rows x cells per row (256, 512 or 1024 cells) */
    int32_t tile_shear;        /* column shift per tile row, in 1/256 columns (slanted tiles) */
    int32_t tile_transpose;    /* 1: rows and columns swap roles in the tile              */
    int32_t step_segments;     /* direct method: coherent segments each step is split into
                                  across workgroups (1 = not split); their complex partial
                                  sums are added before |C|^2 is taken                   */
    int32_t segment_len;       /* samples per segment (step_len when not split)          */
    int32_t taylor_block;      /* direct method: samples per Taylor block of the factored
                                  kernel in the last map (64, or 256 when the Doppler spread
                                  over the chosen tiles allows it)                        */
    int32_t _pad3;
} geoloc_plan_info;

/* ABI version of the loaded library (GEOLOC_ABI_VERSION when it matches). */
int geoloc_abi_version(void);

/* Validate the descriptor, check for a gfx950 device, convert the grid to ECEF on the
 * device (Algorithm 1, first step; sphere of radius R + h) and allocate scratch.
 * Errors: EINVAL (n_rx < 2, a pair out of range or i == j, N % L != 0, fs or fc <= 0,
 * empty grid, non-finite lat/lon, unknown enum), EDEVICE, ENOMEM. */
int geoloc_plan(const geoloc_desc* desc, geoloc_plan_t* out_plan);

/* Replace the grid coordinates of a plan (same grid kind and shape: RECT lat[n_rows],
 * lon[n_cols]; POINTS lat[P], lon[P]; host arrays, radians) and redo the ECEF conversion.
 * Synchronises the device; a previously fitted CAF window is refitted on the next map.
 * Errors: EINVAL (NULL or non-finite coordinates), ELAUNCH. */
int geoloc_set_grid(geoloc_plan_t plan, const double* lat, const double* lon);

/* Make a POINTS plan's points the cells of whole tiles of a rectilinear grid, tile by tile,
 * without a host round trip: lat_dev[rows] / lon_dev[cols] are DEVICE arrays (radians) of
 * the full grid, tile the tile side in cells (rows and cols multiples of it), tiles[n_tiles]
 * a HOST array of tile indices (tile row x cols / tile + tile column), and n_tiles x tile^2
 * must equal the plan's point count. Point p is cell w = p % tile^2 (row-major within the
 * tile) of tile tiles[p / tile^2]; a tile index outside the grid gives NaN points. Runs
 * asynchronously on `stream` (the grid -> ECEF conversion included); the next map on that
 * stream sees the new points. For the refinement of a tile proposal. Errors: EINVAL (not a
 * POINTS plan, a plan with per-point heights, bad sizes), ENOMEM, ELAUNCH. */
int geoloc_set_points_from_tiles(geoloc_plan_t plan, const double* lat_dev, const double* lon_dev, int64_t rows,
                                 int64_t cols, int32_t tile, const int32_t* tiles, int32_t n_tiles, void* stream);

/* Fix the tiling of the tile-factored kernel for the maps that follow (RECT grids, method
 * GEOLOC_DIRECT_FP32), instead of the per-map choice from the geometry: tiles of tile_h rows
 * of tile_w cells (tile_w x tile_h = 256, or 512 or 1024 for two or four cells per thread),
 * row i starting floor(shear * i / 256) columns further along, |shear| <= 1024, rows and
 * columns swapped if transpose. tile_w = 0 returns to the per-map choice. The map is the
 * same function of the inputs whatever the tiling (to FP32 rounding); only its speed and
 * which tile-steps go to the per-point kernel change (with a fixed tiling, tile-steps that
 * need more than four Taylor terms go there too). Errors: EINVAL (bad shape, shear or grid
 * kind / method). */
int geoloc_set_tiling(geoloc_plan_t plan, int32_t tile_w, int32_t tile_h, int32_t shear, int32_t transpose);

/* Fix the length of the factored kernel's Taylor blocks (Sec. III, Eq. (11): the Doppler
 * phase over a block is expanded in powers of the sample offset from the block centre) for
 * the maps that follow: 64 samples, or 256 (four 64-sample blocks whose moments are moved to
 * the long block's centre and summed, fewer per-point steps, more Taylor terms for the same
 * Doppler spread); 0 returns to the per-map choice from the geometry (for POINTS grids, which
 * have no per-map choice, 64). The map is the same function of the inputs to FP32 rounding.
 * Errors: EINVAL (other lengths). */
int geoloc_set_taylor_block(geoloc_plan_t plan, int32_t samples);

/* Enable (nonzero) or disable per-kernel HIP-event timing of subsequent maps; either
 * way the accumulated times in geoloc_info are reset. Events are recorded on the map's
 * stream around each kernel launch, so the times are those of the kernels alone. */
int geoloc_set_timing(geoloc_plan_t plan, int enable);

/* Compute the map J_dev[P] (float32, DEVICE pointer owned by the caller) from the
 * captures and receiver states (Algorithm 1: geometry, correlation, sum over steps
 * and pairs). With GEOLOC_ACCUMULATE the result is added to J_dev, which lets a
 * capture be processed in pieces. Asynchronous on in->stream for GEOLOC_DIRECT_FP32;
 * the CAF methods synchronise the stream once per map to size (or validate) the table
 * window from the footprint's delay and Doppler extent, then run asynchronously.
 * CAF window (Sec. I's cross-ambiguity function, one table per step and pair):
 *   lags  lag_lo .. lag_lo + caf_lags - 1: fitted to [floor(min D) - 1, floor(max D) + 2]
 *         unless caf_lags / caf_lag_lo are given (then they must cover it);
 *   bins  caf_bins centres nu_lo + m dnu, dnu = (nu_hi - nu_lo) / (caf_bins - 1), fitted to
 *         [min nu - dnu, min nu + (caf_bins - 2) dnu] unless caf_nu_lo_hz / caf_nu_hi_hz
 *         are given (then [min nu, max nu] must lie inside). Each point reads its table by
 *         bilinear interpolation in (delay, Doppler).
 * Errors: EINVAL (NULL pointers, non-finite state, CAF window not covering every
 * point and step), ELAUNCH, ENOMEM. */
int geoloc_map(geoloc_plan_t plan, const geoloc_inputs* in, float* J_dev, uint32_t flags);

/* Geometry alone (Eq. (3)-(9)) for pair index e (0..n_pairs-1) and steps
 * [step_lo, step_lo + n_steps): D_dev[k][P] = TDOA in samples, nu_dev[k][P] = FDOA in
 * Hz, both float64 DEVICE buffers owned by the caller. Asynchronous on in->stream
 * (in->captures is not read and may be NULL). */
int geoloc_geometry(geoloc_plan_t plan, const geoloc_inputs* in, int32_t pair_index, int64_t step_lo,
                    int64_t n_steps, double* D_dev, double* nu_dev);

/* CAF tables alone (CAF methods only; the window is fitted or validated as in
 * geoloc_map): T_dev[k][d][m] = sum over step step_lo + k of y_i[n] conj(y_j[n + lag_lo + d])
 * exp(+j 2 pi nu_m t_n), nu_m = nu_lo + m (nu_hi - nu_lo) / (bins - 1), t_n from the step
 * centre; complex64 interleaved DEVICE buffer of n_steps * caf_lags * caf_bins entries owned
 * by the caller (the window actually used is reported by geoloc_info). Pair index e as in
 * geoloc_geometry. Synchronises in->stream once to size the window. */
int geoloc_caf_table(geoloc_plan_t plan, const geoloc_inputs* in, int32_t pair_index, int64_t step_lo,
                     int64_t n_steps, void* T_dev, int64_t T_capacity);

/* Peaks of a map (the detection step at the end of Algorithm 1): the top_k largest
 * values of J_dev[P], ties to the lowest flat index; after each peak a
 * (2r+1) x (2r+1) window around it (RECT grids; r = nms_radius_cells) is excluded.
 * idx_host / val_host are HOST arrays of top_k entries; fewer peaks than top_k leave
 * idx = -1, val = -inf. Synchronises `stream`. Errors: EINVAL (top_k < 1, r < 0, r > 0
 * on a POINTS grid), ENAN (a NaN in J), ELAUNCH. */
int geoloc_argmax(geoloc_plan_t plan, const float* J_dev, int32_t top_k, int32_t nms_radius_cells,
                  int64_t* idx_host, float* val_host, void* stream);

/* geoloc_argmax without a plan and without any device allocation, for callers that cannot
 * allocate (code under stream capture, tight serving loops, hosts that forbid hipMalloc).
 * Same peaks, order, window and errors as geoloc_argmax on a plan with the same grid:
 * J_dev is the caller's float32 DEVICE map of n_rows * n_cols points (grid_kind RECT: rows =
 * latitude; POINTS: any n_rows x n_cols = P), idx_host / val_host HOST arrays of top_k.
 * Its scratch (block partials and the peaks found so far, 13 KB) is one static device
 * array per GPU, held until the process ends; it is looked up on the first call on each
 * device (which must be current) and needs no clearing. Calls that overlap on one GPU
 * (other threads or streams) race on that array: serialise them. Synchronises `stream`.
 * Errors: EINVAL (NULL pointer, unknown grid kind, empty grid, top_k outside [1, 64]: the
 * array holds 64 peaks, r < 0, r > 0 on a POINTS grid), ENAN, EDEVICE (no gfx950 device
 * current), ELAUNCH. */
int geoloc_argmax_noalloc(const float* J_dev, int32_t grid_kind, int64_t n_rows, int64_t n_cols, int32_t top_k,
                          int32_t nms_radius_cells, int64_t* idx_host, float* val_host, void* stream);

/* Threshold detection of several emitters (the threshold step of Algorithm 1, which the
 * paper leaves open), read as cell-averaging CFAR on a RECT map J_dev[rows][cols]: the noise
 * level of a cell is the mean of J over the cells within Chebyshev distance train_cells of
 * it, clipped to the grid, less those within guard_cells (0 <= guard < train); the cell is a
 * detection when J > scale x that mean. The detections are reported as peaks, largest
 * first (ties to the lowest flat index), each excluding a (2r+1) x (2r+1) window around it
 * (r = nms_radius_cells) as in geoloc_argmax, at most max_detections (1 .. 64) of them.
 * For independent Gamma(L) noise cells and N training cells, scale = N b / (1 - b) with b
 * the (1 - Pfa) quantile of Beta(L, N L) gives false-alarm probability Pfa (L = 1:
 * scale = N (Pfa^(-1/N) - 1)). idx_host / val_host / noise_host are HOST arrays of
 * max_detections entries (flat index, J, noise mean; unused entries -1, -inf, 0) and
 * *n_found the number of detections. The plan allocates 16 bytes per grid point of scratch
 * on the first call. Synchronises `stream`. Errors: EINVAL (POINTS grid, bad window, scale
 * or count), ENAN (a NaN in J), ENOMEM, ELAUNCH. */
int geoloc_detect(geoloc_plan_t plan, const float* J_dev, int32_t guard_cells, int32_t train_cells, double scale,
                  int32_t max_detections, int32_t nms_radius_cells, int64_t* idx_host, float* val_host,
                  float* noise_host, int32_t* n_found, void* stream);

/* Threshold scale of geoloc_detect for a false-alarm probability (the threshold step of
 * Algorithm 1, read as cell-averaging CFAR). For independent Gamma(L) noise cells, a cell x
 * and the sum z of N training cells give x / (x + z) ~ Beta(L, N L), so the scale a with
 * P(x > a z / N) = pfa is a = N b / (1 - b), b the (1 - pfa) quantile of Beta(L, N L).
 * The quantile is found by bisection on the upper tail 1 - I_b(L, N L), the regularised
 * incomplete beta function evaluated by its continued fraction (modified Lentz algorithm);
 * for L = 1 it equals the closed form N (pfa^(-1/N) - 1). Host computation only: needs no
 * device and no plan. *out (HOST) receives the scale. Errors: EINVAL (pfa outside (0, 1),
 * n_train < 1, looks < 1, NULL out). */
int geoloc_cfar_scale(double pfa, int32_t n_train, int32_t looks, double* out);

int geoloc_info(geoloc_plan_t plan, geoloc_plan_info* out);

/* Release the plan and its device scratch (synchronises the device first). */
int geoloc_destroy(geoloc_plan_t plan);

const char* geoloc_strerror(int status);
const char* geoloc_last_error(void);

/* Measurement helper, not a step of the method: the issue rate of unpacked FP32 FMA on the
 * current device, the ceiling of the library's FP32 VALU kernels (which are compiled
 * without the packed FP32 forms). Launches n_blocks workgroups of 256 threads, each thread
 * running *fma_per_lane FMAs in 16 independent chains, asynchronously on
 * `stream` (NULL = default); the caller times it (e.g. with events around the call) and
 * divides n_blocks x 256 x *fma_per_lane by the time. out_dev: DEVICE float[n_blocks x 256]
 * owned by the caller, receiving the chains' sums. *fma_per_lane (HOST) is set before the
 * call returns. Errors: EINVAL (NULL pointer, n_blocks outside 1..2^20, iters outside
 * 1..2^24), EDEVICE, ELAUNCH. */
int geoloc_fma_probe(int32_t n_blocks, int32_t iters, float* out_dev, int64_t* fma_per_lane, void* stream);

/* Sub-band split of complex captures (a DFT filter bank), the input of the learned tile
 * proposal's coarse map. Not a step of the paper's method: a coarse grid evaluated at
 * cell centres from full-band samples misses the one-sample-wide delay ridge of a
 * wideband emitter, while the same map over M decimated bands (delay resolution M
 * samples) summed over the bands does not, and a narrowband emitter stays in its band.
 *   out[b][c][m] = sum_{t=-h}^{h} g[t] exp(+j 2 pi (b - M/2) t / M) x_c[m M - t],
 * b = 0..M-1 (band centre (b - M/2) fs / M), m = 0..N/M-1, x_c = 0 outside [0, N);
 * g[t] = g0[t] w[t] / sum_s g0[s] w[s] with g0[t] = sin(pi t / M) / (pi t) (1/M at 0) and
 * the Blackman window w[t] = 0.42 + 0.5 cos(pi t / h) + 0.08 cos(2 pi t / h).
 * captures: DEVICE complex64 [n_ch][n_samples]; out: DEVICE complex64
 * [n_bands][n_ch][n_samples / n_bands], band-major, so that it reads as the captures of
 * n_bands * n_ch receivers (band b of channel c = receiver b * n_ch + c). Both owned by
 * the caller, 8-byte aligned, not overlapping. Asynchronous on `stream` (NULL = default).
 * Errors: EINVAL (null or misaligned buffer, n_ch < 1, n_samples < 1, n_bands outside
 * 1..32 or not dividing n_samples, half_taps outside 1..128, n_bands (2 half_taps + 1)
 * above 4096), EDEVICE, ELAUNCH. */
int geoloc_subbands(const void* captures, int32_t n_ch, int64_t n_samples, int32_t n_bands, int32_t half_taps,
                    void* out, void* stream);

/* ------------------------------------------------------------------------------------
 * Learned tile proposal. Not part of the paper: a small CNN reads a coarse map of the
 * same method (the map evaluated at coarse cell centres) and scores the tiles of the
 * fine grid, so that only the most likely tiles are mapped at full resolution; the
 * full-grid map stays the fallback and the reference. Network: `layers` 3x3
 * convolutions (zero padding 1) with bias, ReLU between layers, channels in_ch ->
 * hidden -> ... -> hidden -> 1, output = tile logits [height][width]; softmax over all
 * tiles; cross-entropy against a label distribution. Parameters: one flat float vector
 * [W0, b0, W1, b1, ...], W_l laid out [C_out][C_in][3][3]. The device keeps FP32 master
 * parameters (updated by Adam) and an FP16 working copy used by forward and backward;
 * activations and accumulations are FP32. Tensors are NCHW float32 DEVICE buffers owned
 * by the caller. A handle holds the activations of its last forward for backward.
 * ------------------------------------------------------------------------------------ */
typedef struct geoloc_cnn_s* geoloc_cnn_t;

typedef struct geoloc_cnn_desc {
    int32_t in_ch;       /* input channels (1..32); geoloc_cnn_prepare produces 3    */
    int32_t hidden;      /* hidden channels (1..32)                                   */
    int32_t layers;      /* convolution layers (>= 2)                                 */
    int32_t height, width;  /* tile grid, e.g. 64 x 64                                */
    int32_t max_batch;   /* largest batch passed to forward / backward                */
} geoloc_cnn_desc;

/* Allocate a network with all parameters zero (uniform tile probabilities). EINVAL for
 * out-of-range sizes, EDEVICE without a gfx950 device, ENOMEM. */
int geoloc_cnn_create(const geoloc_cnn_desc* desc, geoloc_cnn_t* out);
int geoloc_cnn_param_count(geoloc_cnn_t cnn, int64_t* n_params);
/* Load n FP32 parameters from a HOST array (master and FP16 copy); resets Adam. */
int geoloc_cnn_set_params(geoloc_cnn_t cnn, const float* theta_host, int64_t n);
/* Copy parameters to a HOST array: which = 0 FP32 master, 1 FP16 working copy (widened),
 * 2 last gradient. Synchronises the device. */
int geoloc_cnn_get_params(geoloc_cnn_t cnn, int32_t which, float* out_host, int64_t n);
/* Input features of a batch of coarse maps (in_ch must be 3): J_dev [batch][H*W] float,
 * D_dev / nu_dev [batch][H*W] float64 TDOA (samples) and FDOA (Hz) of one reference step
 * at the same points; x_dev [batch][3][H][W] = [log(J / mean J) clipped to +-8, D / 64,
 * (nu - mean nu) / 256]. */
int geoloc_cnn_prepare(geoloc_cnn_t cnn, const float* J_dev, const double* D_dev, const double* nu_dev,
                       int32_t batch, float* x_dev, void* stream);
/* logits_dev [batch][H][W] from x_dev [batch][in_ch][H][W]; keeps activations. */
int geoloc_cnn_forward(geoloc_cnn_t cnn, const float* x_dev, int32_t batch, float* logits_dev, void* stream);
/* Softmax cross-entropy per sample: loss_dev[batch], dlogits_dev = (softmax - label)/batch;
 * label_dev [batch][H*W] sums to 1 per sample. */
int geoloc_cnn_loss(geoloc_cnn_t cnn, const float* logits_dev, const float* label_dev, int32_t batch,
                    float* dlogits_dev, float* loss_dev, void* stream);
/* Parameter gradient of the loss (overwritten) from dlogits and the last forward's
 * activations (same batch). */
int geoloc_cnn_backward(geoloc_cnn_t cnn, const float* dlogits_dev, int32_t batch, void* stream);
/* One Adam step on the FP32 master parameters with the last gradient, then refresh the
 * FP16 copy: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, w -= lr m^ / (sqrt(v^) + eps). */
int geoloc_cnn_adam_step(geoloc_cnn_t cnn, float lr, float beta1, float beta2, float eps, void* stream);
/* The k (<= 64) highest-scoring tiles of each sample and their softmax probabilities
 * into HOST arrays [batch][k] (ties to the lower tile index). Synchronises `stream`. */
int geoloc_cnn_topk(geoloc_cnn_t cnn, const float* logits_dev, int32_t batch, int32_t k, int32_t* tiles_host,
                    float* probs_host, void* stream);
int geoloc_cnn_destroy(geoloc_cnn_t cnn);

#ifdef __cplusplus
}
#endif

#endif /* GEOLOC_H */
