// internal.h -- shared declarations of the gfx950 library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/geoloc.h"

namespace geoloc {

constexpr double kLightSpeed = 299792458.0;
constexpr double kWgs84A = 6378137.0;             // WGS-84 semi-major axis (m)
constexpr double kWgs84F = 1.0 / 298.257223563;   // WGS-84 flattening

// Points handled by one workgroup of the correlation kernels: a tile of 256 (or, for the
// factored kernel, 512 or 1024) cells of a RECT grid (neighbouring cells have neighbouring delays,
// so the lag spread a tile needs in LDS stays small), or 256 consecutive entries of a
// POINTS list.
//
// A RECT tile is tile_h rows of tile_w cells in which row i starts floor(shear * i / 256)
// columns further along, a parallelogram that can follow a line of equal delay at any
// slope (with `transpose`, rows and columns swap roles). Tiles stack in bands of tile_h
// rows; each band holds tiles_x tiles, enough to cover the sheared band, and cells outside
// the grid are invalid lanes. shear = 0, 16 x 16 is the plain square tiling.
constexpr int kTilePoints = 256;       // cells of the square tiling and of POINTS tiles
constexpr int kShearOne = 256;         // shear unit: one column per row

struct PointTiling {
    int64_t rows, cols;     // RECT: grid shape; POINTS: 1 x P
    int32_t tile_w, tile_h; // cells per tile row, rows per tile (POINTS: 256 x 1)
    int64_t tiles_x, tiles_y;   // tiles per band, bands
    int32_t shear;          // column shift per tile row in 1/256 columns (RECT)
    int32_t transpose;      // 1: the roles of rows and columns are swapped (RECT)
};

__host__ __device__ inline int tile_lanes(const PointTiling& t) { return t.tile_w * t.tile_h; }

// Column offset of row r: floor(shear * r / 256) (an arithmetic shift rounds down).
__host__ __device__ inline int64_t shear_offset(int32_t shear, int64_t r) { return ((int64_t)shear * r) >> 8; }

// Tile count of a tiling with the given shape over a rows x cols grid. Within a band the row
// offsets span at most floor(|shear| (tile_h - 1) / 256) + 1 columns.
__host__ __device__ inline void tiling_counts(PointTiling& t) {
    const int64_t R = t.transpose ? t.cols : t.rows, C = t.transpose ? t.rows : t.cols;
    const int64_t sh = t.shear < 0 ? -(int64_t)t.shear : (int64_t)t.shear;
    const int64_t span = sh ? ((sh * (t.tile_h - 1)) >> 8) + 1 : 0;
    t.tiles_y = (R + t.tile_h - 1) / t.tile_h;
    t.tiles_x = (C + span + t.tile_w - 1) / t.tile_w;
}

__host__ __device__ inline int64_t tile_point(const PointTiling& t, int64_t tile, int lane, bool* valid) {
    const int64_t ty = tile / t.tiles_x, tx = tile - ty * t.tiles_x;
    const int64_t R = t.transpose ? t.cols : t.rows, C = t.transpose ? t.rows : t.cols;
    const int64_t r0 = ty * t.tile_h;
    const int64_t r = r0 + lane / t.tile_w;
    // the band's largest row offset maps to column 0, so its rows cover [0, C)
    const int64_t b0 = -shear_offset(t.shear, t.shear > 0 ? r0 + t.tile_h - 1 : r0);
    const int64_t c = shear_offset(t.shear, r) + b0 + tx * t.tile_w + lane % t.tile_w;
    *valid = (r < R) && (c >= 0) && (c < C);
    const int64_t rr = t.transpose ? c : r, cc = t.transpose ? r : c;
    return *valid ? rr * t.cols + cc : 0;
}

struct DirectArgs {
    const float2* cap;       // [n_rx][N] complex64
    // geometry, evaluated inline per (point, step, pair) in FP64 (Eq. (3)-(9))
    const double* xyz;       // [P][3] ECEF of the grid points
    // rectilinear grid with a uniform height (else NULL): the ECEF of point p = r cols + c is
    // (ecef_row[r].x ecef_col[c].x, ecef_row[r].x ecef_col[c].y, ecef_row[r].y), the same
    // products xyz holds
    const double2* ecef_row;
    const double2* ecef_col;
    const double* states;    // [K][n_rx][6] receiver position and velocity per step
    int32_t n_rx;
    double fs, inv_lambda;
    const int2* pairs;       // [n_pairs]
    float* J;                // [P]
    PointTiling tiling;
    int64_t n_tiles;         // tiles_x * tiles_y
    int64_t N, P;
    int32_t L, k0, kc, n_pairs;
    double inv_fs;
    int32_t accum_mode;
    int32_t load_J;          // add onto the existing J values
    int32_t n_groups;        // groups of (pair, step) items per chunk (1: each workgroup owns its points' J)
    float* partial;          // [n_groups][P] partial sums when n_groups > 1
    // [n_pairs][kc][n_tiles] deferral bytes, bit h for the tile's 256-cell part h (cells
    // 256 h .. 256 h + 255 of the tile): set = this pass handles that part; NULL = all
    const uint8_t* mask;
    // deferral flag of this launch: the factored kernel stores defer_seq into *defer_flag
    // when it leaves any (tile, step) to a later pass, which returns at once unless the
    // flag holds defer_seq (a per-map sequence number, so the flag never needs clearing)
    uint32_t* defer_flag;
    uint32_t defer_seq;
    // factored kernel with a mask (a second pass, over the (tile, step) pairs the first
    // pass deferred, with shorter Taylor blocks and tiles cut into parts): returns at once
    // unless *gate_flag (the first pass's flag) holds defer_seq; adds only the flagged
    // parts, clears the bits of those it completes and raises its own defer_flag for
    // those it defers again
    const uint32_t* gate_flag;
    // factored kernel with a mask: workgroups per tile, each taking tile_lanes / parts
    // consecutive cells (256); without a mask always one
    int32_t parts;
    // factored kernel only: each step split into n_segs coherent segments of seg_len samples
    // (a multiple of 64) whose complex sums go to cpart [n_segs][n_pairs * kc][P]; 1 = off
    int32_t n_segs, seg_len;
    float2* cpart;
};

// Masked passes: the first item at or after `it` and below it_hi whose deferral byte for
// `tile` has any of `bits` set, or it_hi if none. A wave reads the bytes of 64 items at once
// (lane l that of item base + l, base a multiple of 64) and takes the first set bit of their
// ballot, instead of one dependent byte read per item. Every lane of the wave must be active
// and pass the same arguments; the result is the same in every wave of the workgroup.
__device__ inline int64_t next_flagged(const uint8_t* mask, int64_t n_tiles, int64_t tile, uint32_t bits, int64_t it,
                                       int64_t it_hi) {
    const int lane = (int)(threadIdx.x & 63);
    while (it < it_hi) {
        const int64_t j = (it & ~(int64_t)63) + lane;
        const unsigned long long w = __ballot(j >= it && j < it_hi && (mask[j * n_tiles + tile] & bits) != 0);
        if (w) return (it & ~(int64_t)63) + __builtin_ctzll(w);
        it = (it & ~(int64_t)63) + 64;
    }
    return it_hi;
}

// exp(j 2 pi cyc) with the argument reduced in FP64 and evaluated in FP32.
__device__ inline float2 cis_cycles(double cyc) {
    const double f = cyc - rint(cyc);
    float s, c;
    sincospif((float)(2.0 * f), &s, &c);
    return make_float2(c, s);
}

// Windowed-sinc fractional delay (GEOLOC_DELAY_SINC): eight taps t = -3 .. 4 around
// floor(D), w_t = g(t - alpha) / sum_s g(s - alpha), g(x) = sinc(x) I0(6 sqrt(1 - (x/4)^2)) / I0(6)
// for |x| < 4. I0 by its power series (20 terms reach FP32 precision for arguments <= 6).
constexpr int kSincTaps = 8;
constexpr int kSincLo = 3;     // taps before floor(D)

__device__ inline float bessel_i0f(float x) {
    const float q = 0.25f * x * x;
    float term = 1.f, sum = 1.f;
#pragma unroll
    for (int k = 1; k <= 20; ++k) {
        term *= q / (float)(k * k);
        sum += term;
    }
    return sum;
}

__device__ inline void sinc_taps(float alpha, float (&w)[kSincTaps]) {
    const float inv_i0 = 1.f / bessel_i0f(6.f);
    float sum = 0.f;
#pragma unroll
    for (int t = 0; t < kSincTaps; ++t) {
        const float x = (float)(t - kSincLo) - alpha;
        float g = 0.f;
        if (fabsf(x) < 4.f) {
            const float sn = x == 0.f ? 1.f : sinpif(x) / (3.14159265358979f * x);
            const float u = 0.25f * x;
            g = sn * bessel_i0f(6.f * sqrtf(fmaxf(1.f - u * u, 0.f))) * inv_i0;
        }
        w[t] = g;
        sum += g;
    }
    const float inv = 1.f / sum;
#pragma unroll
    for (int t = 0; t < kSincTaps; ++t) w[t] *= inv;
}

// sub_blocks: 64-sample sub-blocks per Taylor block, 1 or 4; a tile of 256, 512 or 1024
// cells. With a mask: a.parts workgroups of 256 cells per tile and sub_blocks 1.
hipError_t launch_direct_fact(const DirectArgs& a, uint8_t* deferred, int32_t delay_mode, bool wide_doppler,
                              int32_t sub_blocks, hipStream_t s);
hipError_t launch_direct_sinc(const DirectArgs& a, hipStream_t s);
// J[p] = (J[p] if loading) + sum over items of |sum over segments of cpart|^2 (or |.|)
// CFAR detection (k_cfar.hip): summed-area table of J in sat [rows][cols], then masked[p] =
// J[p] where J exceeds scale x the training-window mean (noise[p]), -inf elsewhere.
hipError_t launch_cfar(const float* J, int64_t rows, int64_t cols, int32_t guard, int32_t train, double scale,
                       double* sat, float* masked, float* noise, hipStream_t s);
hipError_t launch_gather_noise(const float* noise, const int64_t* idx, int32_t k, float* out, hipStream_t s);
hipError_t launch_direct_seg_reduce(const DirectArgs& a, hipStream_t s);

constexpr int32_t kMaxItemGroups = 64;
// Items of at least this many samples (a step, or a segment of one) take the four-wave
// budget in the factored kernel's LINEAR mode with 256-sample blocks; shorter ones pay its
// spills too often (on the 1e6-point map, steps of 10,000 samples, it ran 2 % slower, while
// 250,000-sample steps ran 23 % faster).
constexpr int64_t kLongItem = 32768;
int32_t direct_groups(int64_t n_tiles, int64_t n_items);   // n_items = pairs x steps per chunk

struct GeomArgs {
    const double* xyz;       // [P][3]
    const double* states;    // [K][n_rx][6]
    const int2* pairs;
    double* D;               // [n_pairs][kc][P]
    double* nu;
    int64_t P;
    int32_t n_rx, n_pairs, k0, kc;
    double fs, inv_lambda;
};

// Delay and Doppler of one receiver state s = [p; v] against ECEF point q (Sec. II-B,
// Eq. (3)-(6)): rho = |p - q|, tau = rho / c, f = -(1/lambda) (p - q)/rho . v, with 1/rho
// taken once (one FP64 division instead of four) and no FMA contraction; the result
// differs from the expressions written out term by term in the last bits only.
__device__ inline void delay_doppler(double q0, double q1, double q2, const double* __restrict__ s, double inv_lambda,
                                     double* tau, double* f) {
#pragma clang fp contract(off)
    const double r0 = s[0] - q0, r1 = s[1] - q1, r2 = s[2] - q2;
    const double rr = r0 * r0 + r1 * r1 + r2 * r2;
    // 1/rho from the hardware reciprocal square root (relative error up to about 2^-23) and two
    // Newton steps y <- y + (y/2)(1 - rr y^2), each of which squares the error: the result is
    // within a few units in the last place, like sqrt and a division, at about half their cost;
    // rho = rr (1/rho)
    double inv = __builtin_amdgcn_rsq(rr);
    inv = fma(0.5 * inv, fma(-rr * inv, inv, 1.0), inv);
    inv = fma(0.5 * inv, fma(-rr * inv, inv, 1.0), inv);
    const double rho = rr * inv;
    *tau = rho * (1.0 / kLightSpeed);
    *f = -inv_lambda * ((r0 * s[3] + r1 * s[4] + r2 * s[5]) * inv);
}

// TDOA in samples and FDOA in Hz of the receiver pair pr at ECEF point q and step k
// (Eq. (7)-(9)) from the states [K][n_rx][6]. Every kernel that needs the geometry of a
// (point, step, pair) evaluates it through this function, so they all see the same values.
__device__ inline void pair_geometry(double q0, double q1, double q2, const double* __restrict__ states, int32_t n_rx,
                                     int32_t k, int2 pr, double fs, double inv_lambda, double* D, double* nu) {
#pragma clang fp contract(off)
    double ti, fi, tj, fj;
    delay_doppler(q0, q1, q2, states + ((int64_t)k * n_rx + pr.x) * 6, inv_lambda, &ti, &fi);
    delay_doppler(q0, q1, q2, states + ((int64_t)k * n_rx + pr.y) * 6, inv_lambda, &tj, &fj);
    *D = (tj - ti) * fs;
    *nu = fj - fi;
}

// Everything the CAF kernels need to evaluate the geometry of (point, step, pair) inline.
struct CafGeomArgs {
    const double* xyz;       // [P][3]
    const double* states;    // [K][n_rx][6]
    const int2* pairs;       // [n_pairs]
    int64_t P;
    int32_t K, n_rx, n_pairs, _pad;
    double fs, inv_lambda;
};

// TDOA in samples and FDOA in Hz of pair e at point p and step k (Eq. (7)-(9)).
__device__ inline void pair_delay_doppler(const CafGeomArgs& g, int64_t p, int32_t k, int32_t e, double* D,
                                          double* nu) {
#pragma clang fp contract(off)
    pair_geometry(g.xyz[3 * p], g.xyz[3 * p + 1], g.xyz[3 * p + 2], g.states, g.n_rx, k, g.pairs[e], g.fs,
                  g.inv_lambda, D, nu);
}

// CAF GEMM workgroup tile: table rows (lags) x columns (Doppler bins); the table is padded
// to whole tiles
constexpr int kCafTileLags = 128;
constexpr int kCafTileBins = 128;

struct CafGemmArgs {
    const float2* cap;             // [n_rx][N]
    const int2* pairs;
    const unsigned short* Fr;      // phasor table planes, [L_pad / 8][M_pad][8] 16-bit floats
    const unsigned short* Fi;
    float2* out;                   // [n_split][n_pairs * kc][n_lags_pad][M_pad]
    int64_t N;
    int32_t L, k0, kc, n_pairs;
    int32_t n_split, chunk;        // split of each step's samples (chunk is a multiple of 256)
    int32_t lag_lo, n_lags_pad, M_pad;
    float scale, unscale;          // input scale 2^-s applied to y_i; output multiplied by unscale
};

struct CafInterpArgs {
    CafGeomArgs g;
    PointTiling tiling;
    const float2* T;               // [n_pairs * kc][n_lags_pad][M_pad]
    float* J;
    int64_t lag_lo;
    int32_t n_lags, n_lags_pad, M, M_pad;
    int32_t k0, kc;
    double nu_lo, dnu;
    int32_t accum_mode, load_J;
};

// launchers (return hipError_t of the launch)
hipError_t launch_grid_ecef(const double* lat, const double* lon, int32_t grid_kind, int64_t rows, int64_t cols,
                            int32_t model, double radius, double alt, const double* alt_p, double2* row_tab,
                            double2* col_tab, double* xyz, hipStream_t s);
hipError_t launch_geometry(const GeomArgs& a, hipStream_t s);
hipError_t launch_tile_points(const double* glat, const double* glon, int64_t rows, int64_t cols, int32_t tile,
                              const int32_t* tiles, int64_t P, double* lat, double* lon, hipStream_t s);
hipError_t launch_direct(const DirectArgs& a, int32_t delay_mode, hipStream_t s);
// with item groups, adds the [n_groups][P] partial sums into J (onto J when load_J)
hipError_t launch_direct_reduce(const DirectArgs& a, hipStream_t s);

struct ArgmaxScratch {
    float* part_val = nullptr;
    int64_t* part_idx = nullptr;
    int64_t* found_idx = nullptr;  // [kMaxTopK]
    float* found_val = nullptr;
    int32_t n_blocks = 0;
};
constexpr int kMaxTopK = 64;
constexpr int kArgmaxMaxBlocks = 1024;   // most block partials of one argmax pass
hipError_t launch_argmax(const float* J, int64_t P, int64_t cols, int32_t rect, int32_t radius, int32_t top_k,
                         ArgmaxScratch& s, hipStream_t st);
// measurement helper (k_calib.hip): n_blocks x 256 threads of independent FP32 FMA chains,
// fma_ceiling_chains() x iters FMAs per thread; out holds n_blocks x 256 floats
hipError_t launch_fma_ceiling(int32_t n_blocks, int32_t iters, float* out, hipStream_t s);
int32_t fma_ceiling_chains();
// Record a detail string for geoloc_last_error() and return code.
int set_last_error(int code, const char* msg);
int32_t argmax_blocks(int64_t P);

int32_t caf_extent_blocks(int64_t points);
hipError_t launch_caf_extent(const CafGeomArgs& a, double* part, int32_t blocks, hipStream_t s);
hipError_t launch_caf_power(const float2* cap, int64_t N, int32_t n_rx, double* part, int32_t blocks, hipStream_t s);
hipError_t launch_caf_phasor(bool f16, int32_t L_pad, int32_t L, int32_t M, int32_t M_pad, double nu_lo, double dnu,
                             double inv_fs, unsigned short* Fr, unsigned short* Fi, hipStream_t s);
hipError_t launch_caf_gemm(bool f16, const CafGemmArgs& a, hipStream_t s);
hipError_t launch_caf_reduce(const float2* part, int64_t n, int32_t n_split, float unscale, float2* T, hipStream_t s);
hipError_t launch_caf_interp(const CafInterpArgs& a, int32_t delay_mode, hipStream_t s);

hipError_t launch_cnn_conv_fwd(bool relu_in, const float* in, const _Float16* w, const _Float16* b, float* out, int B,
                               int C, int O, int H, int W, hipStream_t s);
hipError_t launch_cnn_conv_dgrad(bool mask, const float* g, const _Float16* w, const float* zprev, float* gin, int B,
                                 int C, int O, int H, int W, hipStream_t s);
hipError_t launch_cnn_conv_wgrad(bool relu_in, const float* g, const float* in, float* dw, float* db, int B, int C,
                                 int O, int H, int W, hipStream_t s);
hipError_t launch_cnn_softmax_ce(const float* z, const float* q, int T, int B, float* dz, float* loss, hipStream_t s);
hipError_t launch_cnn_adam(float* master, float* m, float* v, const float* g, _Float16* w16, int64_t n, float lr,
                           float b1, float b2, float eps, float bc1, float bc2, hipStream_t s);
hipError_t launch_cnn_to_half(const float* src, _Float16* dst, int64_t n, hipStream_t s);
hipError_t launch_cnn_topk(const float* z, int T, int B, int k, int32_t* tiles, float* probs, hipStream_t s);
hipError_t launch_cnn_prep(const float* J, const double* D, const double* nu, int T, int B, float* x, hipStream_t s);

// sub-band split (the proposal's coarse-map input)
constexpr int kSubbandMaxBands = 32;
constexpr int kSubbandMaxHalf = 128;
constexpr int kSubbandMaxTable = 4096;   // bands x taps
struct SubbandArgs {
    const float2* in;        // [n_ch][N]
    float2* out;             // [n_bands][n_ch][N / n_bands]
    int64_t N;
    int32_t n_ch, n_bands, half_taps;
    float taps[2 * kSubbandMaxHalf + 1];   // low-pass g[-h..h]
};
hipError_t launch_subband(const SubbandArgs& a, hipStream_t s);

}  // namespace geoloc
