// api.hip -- the C-ABI host layer: validation, device checks, buffer ownership, dispatch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <array>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using namespace geoloc;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

}  // namespace

int geoloc::set_last_error(int code, const char* msg) {
    g_last_error = msg;
    return code;
}

namespace {

#define HIP_TRY(call)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return fail(GEOLOC_ELAUNCH, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

constexpr uint32_t kMagic = 0x67656f6cu;  // "geol"
constexpr int64_t kMaskChunkBytes = 64ll << 20;  // deferral mask of one correlation launch
constexpr int64_t kBalanceBytes = 256ll << 20;   // partial rows of a balanced factored launch
constexpr int32_t kMaxBalanceGroups = 16;
constexpr int32_t kMaxShear = 4 * kShearOne;   // steepest tile shear: 4 columns per row

struct TimedSpan {
    int kind;  // 0 geometry, 1 correlate, 2 interp, 3 whole map
    hipEvent_t a, b;
};

}  // namespace

struct geoloc_plan_s {
    uint32_t magic = kMagic;
    int device = 0;
    // descriptor facts
    int32_t n_rx = 0, n_pairs = 0, method = 0, delay_mode = 0, accum_mode = 0, grid_kind = 0;
    int64_t N = 0, L = 0, K = 0, P = 0, rows = 0, cols = 0;
    double fs = 0, fc = 0, radius = 0, alt = 0;
    std::vector<int2> pairs;
    PointTiling tiling{};            // tiling of the current map
    PointTiling base_tiling{};       // 16 x 16 squares (RECT; CAF and per-point paths) or runs of 256 points (POINTS)
    std::vector<PointTiling> tile_shapes;   // RECT: candidate tilings of the factored kernel
    int64_t max_tiles = 0;           // most tiles of any candidate (scratch is sized for it)
    bool tiling_fixed = false;       // geoloc_set_tiling: use fixed_tiling instead of the per-map choice
    int32_t* d_tiles = nullptr;      // geoloc_set_points_from_tiles: the tile list
    int32_t d_tiles_cap = 0;
    PointTiling fixed_tiling{};
    std::vector<double> h_lat, h_lon;       // grid coordinates (host copy, for the tile choice)
    std::vector<double> h_alt;              // per-point terrain height (host copy), empty if none
    int32_t earth_model = GEOLOC_EARTH_SPHERE;
    double* d_alt = nullptr;         // [P] per-point terrain height, or null
    int32_t kc = 1;  // steps per correlation launch
    // device scratch
    double* d_xyz = nullptr;
    double2* d_ecef_row = nullptr;   // RECT grid with a uniform height: ECEF row and column factors
    double2* d_ecef_col = nullptr;
    double* d_lat = nullptr;         // grid coordinates as given (kept for geoloc_set_grid)
    double* d_lon = nullptr;
    double* d_states = nullptr;
    int2* d_pairs = nullptr;
    uint32_t* d_defer_flags = nullptr;   // [2][step chunks] deferral flags of the two factored passes
    int64_t n_chunks = 0;                // step chunks (correlation launches per map)
    uint32_t defer_seq = 0;              // sequence number of the current map (never 0)
    float* d_partial = nullptr;      // [item groups][P]: small grids, or the balanced split of a large one
    int32_t n_groups = 1;            // item groups of a grid too small to fill the GPU
    int32_t max_balance_groups = 1;  // large grids: most item groups a factored launch may be split into
    uint8_t* d_deferred = nullptr;   // [n_pairs][kc][n_tiles] steps left to the per-point kernel
    bool use_fact = false;           // factored direct kernel (method GEOLOC_DIRECT_FP32)
    bool fact_wide = false;          // its variant with up to 6 Taylor terms (wide Doppler spreads)
    int32_t fact_sub = 1;            // 64-sample sub-blocks per Taylor block of the factored kernel (1 or 4)
    int32_t taylor_fixed = 0;        // geoloc_set_taylor_block: that many sub-blocks (0: chosen per map)
    int32_t n_segs = 1, seg_len = 0; // factored kernel: coherent segments per step (few tiles, long steps)
    float2* d_cpart = nullptr;       // [n_segs][n_pairs * kc][P] complex partial sums
    // detection (allocated by the first geoloc_detect)
    double* d_sat = nullptr;         // [rows][cols] summed-area table of J
    float* d_masked = nullptr;       // [P] J where a detection, -inf elsewhere
    float* d_noise = nullptr;        // [P] training-window mean
    float* d_found_noise = nullptr;  // [kMaxTopK]
    ArgmaxScratch am;
    int64_t device_bytes = 0;
    // host staging for receiver states (pinned) and its reuse guard
    double* h_states = nullptr;
    hipEvent_t states_copied = nullptr;
    bool states_pending = false;
    // CAF table path
    int32_t caf_lags_req = 0, caf_bins = 256, caf_lag_lo_req = 0;
    bool caf_lag_lo_set = false;
    double caf_nu_lo_req = NAN, caf_nu_hi_req = NAN;
    int64_t caf_lag_lo = 0;
    int32_t caf_n_lags = 0, caf_n_lags_pad = 0, caf_M_pad = 0, caf_L_pad = 0;
    double caf_nu_lo = NAN, caf_nu_hi = NAN, caf_dnu = 0;
    int32_t caf_scale_exp = 0;
    unsigned short* d_Fr = nullptr;
    unsigned short* d_Fi = nullptr;
    size_t F_elems = 0;
    bool F_valid = false;
    double F_nu_lo = 0, F_dnu = 0;
    int32_t F_M = 0, F_L = 0;
    float2* d_T = nullptr;
    size_t T_elems = 0;
    float2* d_Tpart = nullptr;
    size_t Tpart_elems = 0;
    double* d_part = nullptr;
    double* h_part = nullptr;
    int32_t part_elems = 0;
    // timing
    bool timing = false;
    std::vector<TimedSpan> spans;
    std::vector<hipEvent_t> event_pool;
    int64_t timed_maps = 0, correlate_launches = 0;
    double t_geom = 0, t_corr = 0, t_interp = 0, t_map = 0;
};

namespace {

bool plan_ok(geoloc_plan_t p) { return p != nullptr && p->magic == kMagic; }

int check_device(int* dev) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) return fail(GEOLOC_EDEVICE, "no HIP device (%s)", hipGetErrorString(e));
    if (hipGetDevice(dev) != hipSuccess) return fail(GEOLOC_EDEVICE, "hipGetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, *dev) != hipSuccess) return fail(GEOLOC_EDEVICE, "hipGetDeviceProperties failed");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(GEOLOC_EDEVICE, "device %d is %s, this library is built for gfx950", *dev, prop.gcnArchName);
    return GEOLOC_OK;
}

template <typename T>
int dev_alloc(geoloc_plan_t p, T** out, size_t count) {
    if (count == 0) count = 1;
    void* ptr = nullptr;
    if (hipMalloc(&ptr, count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GEOLOC_ENOMEM, "hipMalloc of %zu bytes failed", count * sizeof(T));
    }
    *out = (T*)ptr;
    p->device_bytes += (int64_t)(count * sizeof(T));
    return GEOLOC_OK;
}

void release(geoloc_plan_t p) {
    (void)hipDeviceSynchronize();
    (void)hipFree(p->d_xyz);
    (void)hipFree(p->d_ecef_row);
    (void)hipFree(p->d_ecef_col);
    (void)hipFree(p->d_alt);
    (void)hipFree(p->d_tiles);
    (void)hipFree(p->d_lat);
    (void)hipFree(p->d_lon);
    (void)hipFree(p->d_states);
    (void)hipFree(p->d_pairs);
    (void)hipFree(p->d_defer_flags);
    (void)hipFree(p->d_partial);
    (void)hipFree(p->d_cpart);
    (void)hipFree(p->d_sat);
    (void)hipFree(p->d_masked);
    (void)hipFree(p->d_noise);
    (void)hipFree(p->d_found_noise);
    (void)hipFree(p->d_deferred);
    (void)hipFree(p->am.part_val);
    (void)hipFree(p->am.part_idx);
    (void)hipFree(p->am.found_idx);
    (void)hipFree(p->am.found_val);
    (void)hipFree(p->d_Fr);
    (void)hipFree(p->d_Fi);
    (void)hipFree(p->d_T);
    (void)hipFree(p->d_Tpart);
    (void)hipFree(p->d_part);
    if (p->h_part) (void)hipHostFree(p->h_part);
    if (p->h_states) (void)hipHostFree(p->h_states);
    if (p->states_copied) (void)hipEventDestroy(p->states_copied);
    for (auto& s : p->spans) {
        (void)hipEventDestroy(s.a);
        (void)hipEventDestroy(s.b);
    }
    for (auto e : p->event_pool) (void)hipEventDestroy(e);
    p->magic = 0;
    delete p;
}

int get_event(geoloc_plan_t p, hipEvent_t* e) {
    if (!p->event_pool.empty()) {
        *e = p->event_pool.back();
        p->event_pool.pop_back();
        return GEOLOC_OK;
    }
    HIP_TRY(hipEventCreate(e));
    return GEOLOC_OK;
}

// Record the start of a timed span on stream s (no-op when timing is off).
int span_begin(geoloc_plan_t p, hipStream_t s, TimedSpan* sp, int kind) {
    if (!p->timing) return GEOLOC_OK;
    sp->kind = kind;
    int rc = get_event(p, &sp->a);
    if (rc) return rc;
    rc = get_event(p, &sp->b);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(sp->a, s));
    return GEOLOC_OK;
}

int span_end(geoloc_plan_t p, hipStream_t s, TimedSpan* sp) {
    if (!p->timing) return GEOLOC_OK;
    HIP_TRY(hipEventRecord(sp->b, s));
    p->spans.push_back(*sp);
    return GEOLOC_OK;
}

int drain_spans(geoloc_plan_t p) {
    for (auto& s : p->spans) {
        HIP_TRY(hipEventSynchronize(s.b));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, s.a, s.b));
        switch (s.kind) {
            case 0: p->t_geom += ms; break;
            case 1: p->t_corr += ms; break;
            case 2: p->t_interp += ms; break;
            default: p->t_map += ms; break;
        }
        p->event_pool.push_back(s.a);
        p->event_pool.push_back(s.b);
    }
    p->spans.clear();
    return GEOLOC_OK;
}

// Copy the [K][n_rx][6] receiver states to the device through the pinned staging buffer.
int upload_states(geoloc_plan_t p, const double* host, hipStream_t s) {
    const size_t n = (size_t)p->K * p->n_rx * 6;
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(host[i])) return fail(GEOLOC_EINVAL, "rx_state[%zu] is not finite", i);
    if (p->states_pending) HIP_TRY(hipEventSynchronize(p->states_copied));
    memcpy(p->h_states, host, n * sizeof(double));
    HIP_TRY(hipMemcpyAsync(p->d_states, p->h_states, n * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(p->states_copied, s));
    p->states_pending = true;
    return GEOLOC_OK;
}

// Delay (samples) and Doppler (radians per sample) of RECT grid cell (r, c) for one pair at
// one step, in FP64 on the host (Eq. (3)-(8), on the plan's earth model): only the tile
// choice uses it.
void host_delay_doppler(const geoloc_plan_s* p, int64_t r, int64_t c, const double* si, const double* sj, double* D,
                        double* th) {
    const double lat = p->h_lat[r], lon = p->h_lon[c];
    const double h = p->alt + (p->h_alt.empty() ? 0.0 : p->h_alt[r * p->cols + c]);
    const double lambda = kLightSpeed / p->fc;
    const double cl = std::cos(lat), sl = std::sin(lat);
    double x[3];
    if (p->earth_model == GEOLOC_EARTH_WGS84) {
        const double e2 = kWgs84F * (2.0 - kWgs84F), N = kWgs84A / std::sqrt(1.0 - e2 * sl * sl);
        x[0] = (N + h) * cl * std::cos(lon);
        x[1] = (N + h) * cl * std::sin(lon);
        x[2] = (N * (1.0 - e2) + h) * sl;
    } else {
        const double R = p->radius + h;
        x[0] = R * cl * std::cos(lon);
        x[1] = R * cl * std::sin(lon);
        x[2] = R * sl;
    }
    double tau[2], f[2];
    const double* st[2] = {si, sj};
    for (int k = 0; k < 2; ++k) {
        const double dx[3] = {st[k][0] - x[0], st[k][1] - x[1], st[k][2] - x[2]};
        const double rho = std::sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
        tau[k] = rho / kLightSpeed;
        f[k] = -(dx[0] * st[k][3] + dx[1] * st[k][4] + dx[2] * st[k][5]) / (rho * lambda);
    }
    *D = (tau[1] - tau[0]) * p->fs;
    *th = 2.0 * 3.14159265358979323846 * (f[1] - f[0]) / p->fs;
}

// Tile shape for the factored kernel: from the delay and Doppler gradients at the grid
// centre (middle step) of every pair, the candidate (shape of 256, 512 or 1024 cells, shear of
// whole columns per row or along a pair's lines of equal delay) with the least predicted
// VALU work per correlation summed over the pairs, counting the lanes its tiles leave
// outside the grid. The lag moments cost about (4 + 4Q) instructions per lag pair and
// sample, shared by the tile's cells (waves without a (block, lag pair) item skip them),
// and the per-point combination about (4Q + 6) / B per Taylor block of B samples (LINEAR;
// fewer for ROUND, more for SINC), or the time of its LDS reads where that is longer; a tile that the factored kernel would defer costs about
// 13. Blocks of 256 samples (four 64-sample sub-blocks whose moments are moved to the long
// block's centre and summed) cut the per-point share fourfold but need more Taylor terms
// for the same Doppler spread; both block lengths are priced. A tiling whose launch has
// fewer than 768 workgroups (three per CU) is charged for the idle share of the chip, and
// SINC keeps to tiles at most 8 cells wide, or 16 x 64. Taylor orders 5 and 6 need the kernel's
// wide-Doppler variant, whose larger LDS footprint costs a third of its occupancy: they
// are counted 1.5 times, and the variant is launched when the chosen tiling needs them.
// Tiles of 1024 cells (four per thread, at most four Taylor terms) share
// each moment among twice as many cells; LINEAR runs them at three waves per SIMD like its
// 256- and 512-cell kernels, and where those run four (items of at least kLongItem samples,
// with 256-sample blocks) the 1024-cell work is counted 1.15 times. ROUND runs every
// kernel with 256-sample blocks at four waves. SINC runs its 16 x 64 tiles at three
// against four for 512 cells, uncharged: they measured faster (above). On the 1e6-point
// map the LINEAR map took
// 10.3 ms on 16 x 64 tiles against 13.7 ms on 8 x 64 (the model's ratio 0.81). A
// fixed tiling (geoloc_set_tiling) keeps its shape and never takes the wide variant; only its
// block length is chosen.
void choose_tiling(geoloc_plan_t p, const double* states) {
    p->tiling = p->tiling_fixed ? p->fixed_tiling : p->base_tiling;
    p->fact_wide = false;
    p->fact_sub = 1;
    if (p->grid_kind != GEOLOC_GRID_RECT || p->method != GEOLOC_DIRECT_FP32 ||
        (p->tile_shapes.empty() && !p->tiling_fixed)) {
        if (p->taylor_fixed) p->fact_sub = p->taylor_fixed;   // POINTS plans: the caller's block length
        return;
    }
    const int64_t r0 = p->rows / 2, c0 = p->cols / 2, k = p->K / 2;
    const bool has_r = p->rows >= 3, has_c = p->cols >= 3;
    // per pair, a quadratic model of the delay D (samples) and the Doppler th (radians per
    // sample) about the grid centre, in cells: [D_r, D_c, th_r, th_c, D_rr, D_cc, D_rc,
    // th_rr, th_cc, th_rc] from the 3 x 3 stencil of neighbouring cells
    std::vector<std::array<double, 10>> grads;
    std::vector<double> weight;
    for (const int2 pr : p->pairs) {
        const double* si = states + ((size_t)k * p->n_rx + pr.x) * 6;
        const double* sj = states + ((size_t)k * p->n_rx + pr.y) * 6;
        double D[3][3], T[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const int64_t r = has_r ? r0 + i - 1 : r0, c = has_c ? c0 + j - 1 : c0;
                host_delay_doppler(p, r, c, si, sj, &D[i][j], &T[i][j]);
            }
        std::array<double, 10> g{};
        if (has_r) {
            g[0] = 0.5 * (D[2][1] - D[0][1]);
            g[2] = 0.5 * (T[2][1] - T[0][1]);
            g[4] = D[2][1] + D[0][1] - 2.0 * D[1][1];
            g[7] = T[2][1] + T[0][1] - 2.0 * T[1][1];
        }
        if (has_c) {
            g[1] = 0.5 * (D[1][2] - D[1][0]);
            g[3] = 0.5 * (T[1][2] - T[1][0]);
            g[5] = D[1][2] + D[1][0] - 2.0 * D[1][1];
            g[8] = T[1][2] + T[1][0] - 2.0 * T[1][1];
        }
        if (has_r && has_c) {
            g[6] = 0.25 * (D[2][2] - D[2][0] - D[0][2] + D[0][0]);
            g[9] = 0.25 * (T[2][2] - T[2][0] - T[0][2] + T[0][0]);
        }
        double sum = 0.0;
        for (double v : g) sum += v;
        if (!std::isfinite(sum)) return;
        // pairs of the same geometry (stacked sub-bands of one capture) count once, weighted
        bool seen = false;
        for (size_t i = 0; i < grads.size() && !seen; ++i)
            if (grads[i] == g) {
                weight[i] += 1.0;
                seen = true;
            }
        if (!seen) {
            grads.push_back(g);
            weight.push_back(1.0);
        }
    }
    // workgroups of a launch with this tiling: too few to fill the chip cost their idle share
    const double groups = (double)p->n_groups * (p->n_segs > 1 ? p->n_segs : 1);
    auto fill = [&](const PointTiling& t) {
        return std::max(1.0, 768.0 / ((double)(t.tiles_x * t.tiles_y) * groups));
    };
    // per-point instructions per block: Taylor terms times lags read, plus one Horner step;
    // or the LDS reads of those moments when they take longer (8 bytes per moment at 128
    // bytes per CU-cycle against one 64-lane instruction per CU-cycle: 4 instructions' worth)
    auto combine = [&](int Q) {
        const double reads = p->delay_mode == GEOLOC_DELAY_SINC ? 8.0 : (p->delay_mode == GEOLOC_DELAY_ROUND ? 1.0 : 2.0);
        const double valu = p->delay_mode == GEOLOC_DELAY_SINC ? 18.0 * Q + 6.0
                                                                : (p->delay_mode == GEOLOC_DELAY_ROUND ? 2.0 : 4.0) * Q + 6.0;
        return std::max(valu, 4.0 * reads * Q);
    };
    const double taps = p->delay_mode == GEOLOC_DELAY_SINC ? 8.0 : 2.0;   // lags each cell reads
    auto cost = [&](const PointTiling& t, int sub, int* q_need) {
        double total = 0.0;
        *q_need = 0;
        const double sh = (double)t.shear / kShearOne;
        const double jag = (t.shear % kShearOne) ? 1.0 : 0.0;   // rounding of fractional row offsets
        const int lanes = tile_lanes(t);
        const int q_allowed = (p->tiling_fixed || lanes == 1024) ? 4 : 6;
        const double Rn = (double)(t.transpose ? p->cols : p->rows), Cn = (double)(t.transpose ? p->rows : p->cols);
        const double hl = t.tile_h - 1.0, wl = t.tile_w - 1.0 + jag;
        // spread over a tile of a quantity with gradient (fr, fc) and second derivatives
        // (frr, fcc, frc): the linear part, the bend along the tile, and the drift of the
        // slope between the grid centre and an average tile
        auto spread = [&](double fr, double fc, double frr, double fcc, double frc) {
            const double fuu = frr + 2.0 * sh * frc + sh * sh * fcc;
            return std::fabs(fr + sh * fc) * hl + std::fabs(fc) * wl + 0.25 * std::fabs(fuu) * hl * hl +
                   0.25 * std::fabs(fcc) * wl * wl +
                   0.25 * (std::fabs(frr + sh * frc) * Rn + std::fabs(frc + sh * fcc) * Cn) * hl;
        };
        for (size_t gi = 0; gi < grads.size(); ++gi) {
            const auto& g = grads[gi];
            const bool tr = t.transpose != 0;
            const double H = spread(tr ? g[1] : g[0], tr ? g[0] : g[1], tr ? g[5] : g[4], tr ? g[4] : g[5], g[6]) + taps + 1.0;
            const double xr = 0.5 * spread(tr ? g[3] : g[2], tr ? g[2] : g[3], tr ? g[8] : g[7], tr ? g[7] : g[8], g[9]) *
                              (0.5 * 64.0 * sub);
            int Q = 0;
            double term = 1.0;
            for (int q = 1; q <= q_allowed && xr < 1.0; ++q) {
                term *= xr / q;
                if (term <= 5.9604645e-8) {
                    Q = q;
                    break;
                }
            }
            double c = 13.0;
            if (Q > 0 && H <= 128.0) {
                const int Hg = (int)std::ceil(H / 2.0);
                const int NB = std::min(32 / sub, 256 / (sub * Hg));     // Taylor blocks per round
                const double waves = std::ceil(NB * sub * Hg / 64.0);   // waves busy with moments
                // per lane and sub-block: the moments' basis change, and for long blocks the shift
                // to the long block's centre and the quad sums
                const double extra = 2.0 * (Q - 1) * (Q + 2) + (sub > 1 ? 2.0 * Q * (Q - 1) + 8.0 * Q : 0.0);
                c = ((4.0 + 4.0 * Q + extra / 64.0) * waves * 64.0 / (NB * sub * lanes) + combine(Q) / (64.0 * sub)) *
                    (Q > 4 ? 1.5 : 1.0);
                *q_need = std::max(*q_need, Q);
            }
            total += weight[gi] * c;
        }
        double occupancy = 1.0;
        if (lanes == 1024) {
            const int64_t item = p->n_segs > 1 ? p->seg_len : p->L;
            const bool four = sub == 4 && p->delay_mode != GEOLOC_DELAY_ROUND && item >= kLongItem;
            occupancy = four ? 1.15 : 1.0;
        }
        return total * (double)(t.tiles_x * t.tiles_y * lanes) / (double)p->P * fill(t) * occupancy;
    };
    int q_best = 0, q = 0;
    std::vector<int> subs = {1, 4};
    if (p->taylor_fixed) subs = {p->taylor_fixed};
    p->fact_sub = subs[0];
    double best = cost(p->tiling, subs[0], &q_best);
    for (size_t i = 1; i < subs.size(); ++i) {
        const int sub = subs[i];
        const double c = cost(p->tiling, sub, &q);
        if (c < 0.97 * best) {
            best = c;
            q_best = q;
            p->fact_sub = sub;
        }
    }
    if (p->tiling_fixed) return;
    for (const auto& shape : p->tile_shapes) {
        // the SINC combination is bound by per-point work, registers and LDS reads: tiles of
        // 256 or 512 cells at most 8 cells wide (on the 1e6-point map 16-wide tiles of two
        // cells per thread ran 1.4x slower, each wave's cells reading twice as many distinct
        // lags per block; 8 x 64 took 23.4 ms against 30.8 ms on 4 x 64), and of the 1024-cell
        // shapes 16 x 64 (21.3 ms; 32 x 32 23.9 ms, 8 x 128 24.4 ms)
        if (p->delay_mode == GEOLOC_DELAY_SINC &&
            (tile_lanes(shape) == 1024 ? shape.tile_w != 16 : shape.tile_w > 8))
            continue;
        // shears: whole columns per row, and the slope of each pair's lines of equal delay
        std::vector<int32_t> shears = {-2 * kShearOne, -kShearOne, 0, kShearOne, 2 * kShearOne};
        for (const auto& g : grads) {
            const double gr = shape.transpose ? g[1] : g[0], gc = shape.transpose ? g[0] : g[1];
            if (std::fabs(gc) > 1e-12) {
                const double sg = std::max(-4.0, std::min(4.0, -gr / gc));
                shears.push_back((int32_t)std::lround(sg * kShearOne));
            }
        }
        std::sort(shears.begin(), shears.end());
        shears.erase(std::unique(shears.begin(), shears.end()), shears.end());
        for (const int32_t sh : shears) {
            PointTiling t = shape;
            t.shear = std::max(-kMaxShear, std::min(kMaxShear, sh));
            tiling_counts(t);
            for (const int sub : subs) {
                const double c = cost(t, sub, &q);
                if (c < 0.97 * best) {
                    best = c;
                    q_best = q;
                    p->tiling = t;
                    p->fact_sub = sub;
                }
            }
        }
    }
    p->fact_wide = q_best > 4;
}

// Item groups for a factored launch of `items` (pair, step) items over a large grid. The
// workgroups of a launch run in rounds of as many as fit on the chip at once; a last round
// that is only partly filled leaves the rest of the chip idle (2160 tiles on 768 slots:
// three rounds for 2.8 rounds of work), and tiles of unequal work (lag spreads, Taylor
// orders, cells past the grid edge) leave the same kind of tail. Splitting every tile's
// items into G groups (G workgroups per tile, each adding its items into a partial row)
// makes the workgroups G times shorter, and the tail with them. G is the largest the
// partial rows allow (on the 1e6-point map: 16.2 ms with one group, 14.4 with six, 13.9
// with sixteen).
int32_t balance_groups(int64_t items, int32_t max_groups) {
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(max_groups, items));
}

int run_geometry(geoloc_plan_t p, int32_t pair_lo, int32_t n_pairs, int64_t k0, int32_t kc, double* D, double* nu,
                 hipStream_t s) {
    GeomArgs g{};
    g.xyz = p->d_xyz;
    g.states = p->d_states;
    g.pairs = p->d_pairs + pair_lo;
    g.D = D;
    g.nu = nu;
    g.P = p->P;
    g.n_rx = p->n_rx;
    g.n_pairs = n_pairs;
    g.k0 = (int32_t)k0;
    g.kc = kc;
    g.fs = p->fs;
    g.inv_lambda = p->fc / kLightSpeed;
    HIP_TRY(launch_geometry(g, s));
    return GEOLOC_OK;
}

constexpr int64_t kCafTableBytes = 1ll << 30;   // budget for one step-chunk of CAF tables
constexpr int32_t kCafPowerBlocks = 64;

// Grow-only device buffer.
template <typename T>
int ensure(geoloc_plan_t p, T** buf, size_t* cap, size_t need) {
    if (*cap >= need && *buf) return GEOLOC_OK;
    if (*buf) {
        (void)hipFree(*buf);
        p->device_bytes -= (int64_t)(*cap * sizeof(T));
        *buf = nullptr;
        *cap = 0;
    }
    int rc = dev_alloc(p, buf, need);
    if (rc) return rc;
    *cap = need;
    return GEOLOC_OK;
}

CafGeomArgs caf_geom(geoloc_plan_t p, int32_t pair_lo, int32_t n_pairs) {
    CafGeomArgs g{};
    g.xyz = p->d_xyz;
    g.states = p->d_states;
    g.pairs = p->d_pairs + pair_lo;
    g.P = p->P;
    g.K = (int32_t)p->K;
    g.n_rx = p->n_rx;
    g.n_pairs = n_pairs;
    g.fs = p->fs;
    g.inv_lambda = p->fc / kLightSpeed;
    return g;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Size (or validate) the CAF window from the footprint's delay / Doppler extent, choose the
// input scale, and (re)build the phasor table. Synchronises stream s once.
int caf_prepare(geoloc_plan_t p, const float2* cap, hipStream_t s) {
    const bool f16 = p->method == GEOLOC_CAF_FP16;
    CafGeomArgs g = caf_geom(p, 0, p->n_pairs);
    const int32_t eb = caf_extent_blocks(p->P);
    const int32_t need = eb * 4 + kCafPowerBlocks * p->n_rx;
    if (p->part_elems < need) {
        (void)hipFree(p->d_part);
        if (p->h_part) (void)hipHostFree(p->h_part);
        p->d_part = nullptr;
        p->h_part = nullptr;
        int rc = dev_alloc(p, &p->d_part, (size_t)need);
        if (rc) return rc;
        if (hipHostMalloc((void**)&p->h_part, need * sizeof(double)) != hipSuccess) {
            p->h_part = nullptr;
            return fail(GEOLOC_ENOMEM, "pinned host allocation failed");
        }
        p->part_elems = need;
    }
    HIP_TRY(launch_caf_extent(g, p->d_part, eb, s));
    HIP_TRY(launch_caf_power(cap, p->N, p->n_rx, p->d_part + eb * 4, kCafPowerBlocks, s));
    HIP_TRY(hipMemcpyAsync(p->h_part, p->d_part, need * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double dmin = INFINITY, dmax = -INFINITY, nmin = INFINITY, nmax = -INFINITY, pw = 0.0;
    for (int b = 0; b < eb; ++b) {
        dmin = std::min(dmin, p->h_part[4 * b]);
        dmax = std::max(dmax, -p->h_part[4 * b + 1]);
        nmin = std::min(nmin, p->h_part[4 * b + 2]);
        nmax = std::max(nmax, -p->h_part[4 * b + 3]);
    }
    for (int b = 0; b < kCafPowerBlocks * p->n_rx; ++b) pw += p->h_part[eb * 4 + b];
    if (!std::isfinite(dmin) || !std::isfinite(dmax) || !std::isfinite(nmin) || !std::isfinite(nmax) ||
        std::fabs(dmin) > 1e9 || std::fabs(dmax) > 1e9)
        return fail(GEOLOC_EINVAL, "geometry out of range for a CAF table (D in [%g, %g], nu in [%g, %g])", dmin,
                    dmax, nmin, nmax);
    // lag window
    // lags the interpolation reads: floor(D) and floor(D) + 1 (LINEAR, ROUND), floor(D) - 3 ..
    // floor(D) + 4 (SINC), with one lag of margin either side
    const int64_t tap_lo = p->delay_mode == GEOLOC_DELAY_SINC ? kSincLo : 0;
    const int64_t tap_hi = p->delay_mode == GEOLOC_DELAY_SINC ? kSincTaps - 1 - kSincLo : 1;
    const int64_t need_lo = (int64_t)std::floor(dmin) - tap_lo - 1, need_hi = (int64_t)std::floor(dmax) + tap_hi + 1;
    const int64_t n_lags = p->caf_lags_req > 0 ? p->caf_lags_req : need_hi - need_lo + 1;
    int64_t lag_lo = need_lo;
    if (p->caf_lag_lo_set)
        lag_lo = p->caf_lag_lo_req;
    else if (p->caf_lags_req > 0)
        lag_lo = (int64_t)std::floor(0.5 * (dmin + dmax)) - n_lags / 2;
    if (lag_lo > need_lo || lag_lo + n_lags - 1 < need_hi)
        return fail(GEOLOC_EINVAL, "CAF lag window [%lld, %lld] does not cover the footprint's [%lld, %lld]",
                    (long long)lag_lo, (long long)(lag_lo + n_lags - 1), (long long)need_lo, (long long)need_hi);
    if (n_lags > (1 << 20) || lag_lo < INT32_MIN / 2 || lag_lo > INT32_MAX / 2)
        return fail(GEOLOC_EINVAL, "CAF lag window too large");
    // Doppler bins
    const int32_t M = p->caf_bins;
    double lo, hi, dnu;
    if (std::isfinite(p->caf_nu_lo_req) && std::isfinite(p->caf_nu_hi_req)) {
        lo = p->caf_nu_lo_req;
        hi = p->caf_nu_hi_req;
        dnu = (hi - lo) / (M - 1);
        if (!(hi > lo) || nmin < lo || nmax > hi)
            return fail(GEOLOC_EINVAL, "CAF Doppler window [%g, %g] Hz does not cover the footprint's [%g, %g] Hz", lo,
                        hi, nmin, nmax);
    } else {
        dnu = std::max(nmax - nmin, 1.0) / (M - 3);
        lo = nmin - dnu;
        hi = lo + (M - 1) * dnu;
    }
    p->caf_lag_lo = lag_lo;
    p->caf_n_lags = (int32_t)n_lags;
    p->caf_n_lags_pad = (int32_t)round_up(n_lags, kCafTileLags);
    p->caf_M_pad = (int32_t)round_up(M, kCafTileBins);
    p->caf_L_pad = (int32_t)round_up(p->L, 16);
    p->caf_nu_lo = lo;
    p->caf_nu_hi = hi;
    p->caf_dnu = dnu;
    // power-of-two input scale: lag products near unit magnitude (keeps FP16 in range)
    const double mean_pw = pw / ((double)p->N * p->n_rx);
    int32_t se = mean_pw > 0 ? (int32_t)std::lround(std::log2(mean_pw)) : 0;
    p->caf_scale_exp = std::min(60, std::max(-60, se));
    // phasor table
    const size_t felems = (size_t)p->caf_L_pad * p->caf_M_pad;
    if (!p->F_valid || p->F_nu_lo != lo || p->F_dnu != dnu || p->F_M != M || p->F_L != p->L) {
        size_t cap_r = p->F_elems, cap_i = p->F_elems;
        int rc = ensure(p, &p->d_Fr, &cap_r, felems);
        if (rc) return rc;
        rc = ensure(p, &p->d_Fi, &cap_i, felems);
        if (rc) return rc;
        p->F_elems = std::min(cap_r, cap_i);
        HIP_TRY(launch_caf_phasor(f16, p->caf_L_pad, (int32_t)p->L, M, p->caf_M_pad, lo, dnu, 1.0 / p->fs, p->d_Fr,
                                  p->d_Fi, s));
        p->F_valid = true;
        p->F_nu_lo = lo;
        p->F_dnu = dnu;
        p->F_M = M;
        p->F_L = (int32_t)p->L;
    }
    return GEOLOC_OK;
}

// Work split of the CAF GEMM for n_pairs pairs: steps per chunk and split-K of each step.
void caf_split(geoloc_plan_t p, int32_t n_pairs, int64_t n_steps, int32_t* kc_out, int32_t* n_split_out,
               int32_t* chunk_out) {
    const int64_t per_step = (int64_t)n_pairs * p->caf_n_lags_pad * p->caf_M_pad * 8;
    int64_t kc = std::max<int64_t>(1, std::min<int64_t>(n_steps, kCafTableBytes / per_step));
    const int64_t wgs = (int64_t)(p->caf_n_lags_pad / kCafTileLags) * (p->caf_M_pad / kCafTileBins) * n_pairs * kc;
    int64_t n_split = 1, chunk = p->L;
    if (wgs < 1024) {
        n_split = std::min<int64_t>((1024 + wgs - 1) / wgs, (p->L + 255) / 256);
        chunk = round_up((p->L + n_split - 1) / n_split, 256);
        n_split = (p->L + chunk - 1) / chunk;
        while (n_split > 1 && per_step * kc * n_split > kCafTableBytes) {
            chunk *= 2;
            n_split = (p->L + chunk - 1) / chunk;
        }
    }
    *kc_out = (int32_t)kc;
    *n_split_out = (int32_t)n_split;
    *chunk_out = (int32_t)chunk;
}

// CAF tables of pairs [pair_lo, pair_lo + n_pairs) for steps [k0, k0 + kc) into p->d_T.
int caf_tables(geoloc_plan_t p, const float2* cap, int32_t pair_lo, int32_t n_pairs, int64_t k0, int32_t kc,
               int32_t n_split, int32_t chunk, hipStream_t s) {
    const bool f16 = p->method == GEOLOC_CAF_FP16;
    const size_t tel = (size_t)n_pairs * kc * p->caf_n_lags_pad * p->caf_M_pad;
    int rc = ensure(p, &p->d_T, &p->T_elems, tel);
    if (rc) return rc;
    if (n_split > 1 && (rc = ensure(p, &p->d_Tpart, &p->Tpart_elems, tel * n_split))) return rc;
    CafGemmArgs a{};
    a.cap = cap;
    a.pairs = p->d_pairs + pair_lo;
    a.Fr = p->d_Fr;
    a.Fi = p->d_Fi;
    a.out = n_split > 1 ? p->d_Tpart : p->d_T;
    a.N = p->N;
    a.L = (int32_t)p->L;
    a.k0 = (int32_t)k0;
    a.kc = kc;
    a.n_pairs = n_pairs;
    a.n_split = n_split;
    a.chunk = chunk;
    a.lag_lo = (int32_t)p->caf_lag_lo;
    a.n_lags_pad = p->caf_n_lags_pad;
    a.M_pad = p->caf_M_pad;
    a.scale = std::ldexp(1.0f, -p->caf_scale_exp);
    const float unscale = std::ldexp(1.0f, p->caf_scale_exp);
    a.unscale = n_split > 1 ? 1.0f : unscale;
    HIP_TRY(launch_caf_gemm(f16, a, s));
    if (n_split > 1) HIP_TRY(launch_caf_reduce(p->d_Tpart, (int64_t)tel, n_split, unscale, p->d_T, s));
    return GEOLOC_OK;
}

int caf_map(geoloc_plan_t p, const geoloc_inputs* in, float* J, uint32_t flags, hipStream_t s) {
    const float2* cap = (const float2*)in->captures;
    TimedSpan sp{};
    int rc = span_begin(p, s, &sp, 0);
    if (rc) return rc;
    if ((rc = caf_prepare(p, cap, s))) return rc;
    if ((rc = span_end(p, s, &sp))) return rc;
    int32_t kc, n_split, chunk;
    caf_split(p, p->n_pairs, p->K, &kc, &n_split, &chunk);
    for (int64_t k0 = 0; k0 < p->K; k0 += kc) {
        const int32_t kn = (int32_t)std::min<int64_t>(kc, p->K - k0);
        TimedSpan sg{}, si{};
        if ((rc = span_begin(p, s, &sg, 1))) return rc;
        if ((rc = caf_tables(p, cap, 0, p->n_pairs, k0, kn, n_split, chunk, s))) return rc;
        if ((rc = span_end(p, s, &sg))) return rc;
        if (p->timing) p->correlate_launches++;
        CafInterpArgs a{};
        a.g = caf_geom(p, 0, p->n_pairs);
        a.tiling = p->tiling;
        a.T = p->d_T;
        a.J = J;
        a.lag_lo = p->caf_lag_lo;
        a.n_lags = p->caf_n_lags;
        a.n_lags_pad = p->caf_n_lags_pad;
        a.M = p->caf_bins;
        a.M_pad = p->caf_M_pad;
        a.k0 = (int32_t)k0;
        a.kc = kn;
        a.nu_lo = p->caf_nu_lo;
        a.dnu = p->caf_dnu;
        a.accum_mode = p->accum_mode;
        a.load_J = (k0 > 0) || (flags & GEOLOC_ACCUMULATE);
        if ((rc = span_begin(p, s, &si, 2))) return rc;
        HIP_TRY(launch_caf_interp(a, p->delay_mode, s));
        if ((rc = span_end(p, s, &si))) return rc;
    }
    return GEOLOC_OK;
}

}  // namespace

extern "C" {

int geoloc_abi_version(void) { return GEOLOC_ABI_VERSION; }

const char* geoloc_strerror(int status) {
    switch (status) {
        case GEOLOC_OK: return "ok";
        case GEOLOC_EINVAL: return "invalid argument";
        case GEOLOC_ENOMEM: return "out of memory";
        case GEOLOC_EDEVICE: return "no usable gfx950 device";
        case GEOLOC_ESTATE: return "invalid state";
        case GEOLOC_ENAN: return "NaN in map";
        case GEOLOC_EUNSUPPORTED: return "unsupported";
        case GEOLOC_ELAUNCH: return "HIP launch or runtime error";
        default: return "unknown status";
    }
}

const char* geoloc_last_error(void) { return g_last_error.c_str(); }

int geoloc_plan(const geoloc_desc* d, geoloc_plan_t* out) {
    if (!d || !out) return fail(GEOLOC_EINVAL, "NULL descriptor or output");
    if (d->n_rx < 2) return fail(GEOLOC_EINVAL, "n_rx must be >= 2 (got %d)", d->n_rx);
    if (d->n_samples <= 0 || d->step_len <= 0 || d->n_samples % d->step_len != 0)
        return fail(GEOLOC_EINVAL, "n_samples (%lld) must be a positive multiple of step_len (%lld)",
                    (long long)d->n_samples, (long long)d->step_len);
    if (d->step_len > (1ll << 30) || d->n_samples > (1ll << 40)) return fail(GEOLOC_EINVAL, "capture too long");
    if (!(d->fs_hz > 0) || !(d->fc_hz > 0) || !std::isfinite(d->fs_hz) || !std::isfinite(d->fc_hz))
        return fail(GEOLOC_EINVAL, "fs_hz and fc_hz must be finite and > 0");
    if (d->earth_model != GEOLOC_EARTH_SPHERE && d->earth_model != GEOLOC_EARTH_WGS84)
        return fail(GEOLOC_EINVAL, "unknown earth_model %d", d->earth_model);
    if ((d->earth_model == GEOLOC_EARTH_SPHERE && (!(d->earth_radius_m > 0) || !std::isfinite(d->earth_radius_m))) ||
        !std::isfinite(d->alt_m))
        return fail(GEOLOC_EINVAL, "earth_radius_m must be > 0 (sphere) and alt_m finite");
    if (d->grid_kind != GEOLOC_GRID_RECT && d->grid_kind != GEOLOC_GRID_POINTS)
        return fail(GEOLOC_EINVAL, "unknown grid_kind %d", d->grid_kind);
    if (d->n_rows <= 0 || d->n_cols <= 0) return fail(GEOLOC_EINVAL, "empty grid");
    if (d->n_rows > (1ll << 31) || d->n_cols > (1ll << 31) || d->n_rows * d->n_cols > (1ll << 34))
        return fail(GEOLOC_EINVAL, "grid too large");
    if (!d->lat || !d->lon) return fail(GEOLOC_EINVAL, "NULL lat or lon");
    if (d->method != GEOLOC_DIRECT_FP32 && d->method != GEOLOC_CAF_BF16 && d->method != GEOLOC_CAF_FP16 &&
        d->method != GEOLOC_DIRECT_FP32_POINTWISE)
        return fail(GEOLOC_EINVAL, "unknown method %d", d->method);
    if (d->delay_mode != GEOLOC_DELAY_LINEAR && d->delay_mode != GEOLOC_DELAY_ROUND &&
        d->delay_mode != GEOLOC_DELAY_SINC)
        return fail(GEOLOC_EINVAL, "unknown delay_mode %d", d->delay_mode);
    if (d->accum_mode != GEOLOC_ACC_POWER && d->accum_mode != GEOLOC_ACC_MAG)
        return fail(GEOLOC_EINVAL, "unknown accum_mode %d", d->accum_mode);

    std::vector<int2> pairs;
    if (d->n_pairs < 0) return fail(GEOLOC_EINVAL, "n_pairs < 0");
    if (d->n_pairs == 0) {
        for (int i = 0; i < d->n_rx; ++i)
            for (int j = i + 1; j < d->n_rx; ++j) pairs.push_back(make_int2(i, j));
    } else {
        if (!d->pairs) return fail(GEOLOC_EINVAL, "n_pairs > 0 but pairs is NULL");
        for (int e = 0; e < d->n_pairs; ++e) {
            int i = d->pairs[2 * e], j = d->pairs[2 * e + 1];
            if (i < 0 || j < 0 || i >= d->n_rx || j >= d->n_rx || i == j)
                return fail(GEOLOC_EINVAL, "pair %d = (%d, %d) invalid for n_rx = %d", e, i, j, d->n_rx);
            pairs.push_back(make_int2(i, j));
        }
    }
    const int64_t P = d->n_rows * d->n_cols;
    const int64_t n_lat = d->grid_kind == GEOLOC_GRID_RECT ? d->n_rows : P;
    const int64_t n_lon = d->grid_kind == GEOLOC_GRID_RECT ? d->n_cols : P;
    for (int64_t i = 0; i < n_lat; ++i)
        if (!std::isfinite(d->lat[i])) return fail(GEOLOC_EINVAL, "lat[%lld] not finite", (long long)i);
    for (int64_t i = 0; i < n_lon; ++i)
        if (!std::isfinite(d->lon[i])) return fail(GEOLOC_EINVAL, "lon[%lld] not finite", (long long)i);
    if (d->alt_grid)
        for (int64_t i = 0; i < P; ++i)
            if (!std::isfinite(d->alt_grid[i]) || std::fabs(d->alt_grid[i]) > 1.0e6)
                return fail(GEOLOC_EINVAL, "alt_grid[%lld] not finite or beyond 1000 km", (long long)i);
    const bool caf = d->method == GEOLOC_CAF_BF16 || d->method == GEOLOC_CAF_FP16;
    if (caf) {
        if (d->caf_bins != 0 && (d->caf_bins < 4 || d->caf_bins > 65536))
            return fail(GEOLOC_EINVAL, "caf_bins must be 0 or in [4, 65536]");
        if (d->caf_lags < 0 || (d->caf_lags > 0 && d->caf_lags < 3) || d->caf_lags > (1 << 20))
            return fail(GEOLOC_EINVAL, "caf_lags must be 0 or in [3, 2^20]");
        if (std::isfinite(d->caf_nu_lo_hz) != std::isfinite(d->caf_nu_hi_hz))
            return fail(GEOLOC_EINVAL, "give both caf_nu_lo_hz and caf_nu_hi_hz, or neither");
        if (std::isfinite(d->caf_nu_lo_hz) && !(d->caf_nu_hi_hz > d->caf_nu_lo_hz))
            return fail(GEOLOC_EINVAL, "caf_nu_hi_hz must exceed caf_nu_lo_hz");
        if (d->step_len > (1ll << 28)) return fail(GEOLOC_EINVAL, "step_len too long for a CAF table");
    }

    int dev = 0;
    int rc = check_device(&dev);
    if (rc) return rc;

    geoloc_plan_t p = new (std::nothrow) geoloc_plan_s();
    if (!p) return fail(GEOLOC_ENOMEM, "host allocation failed");
    p->device = dev;
    p->n_rx = d->n_rx;
    p->n_pairs = (int32_t)pairs.size();
    p->pairs = pairs;
    p->method = d->method;
    p->delay_mode = d->delay_mode;
    p->accum_mode = d->accum_mode;
    p->grid_kind = d->grid_kind;
    p->N = d->n_samples;
    p->L = d->step_len;
    p->K = d->n_samples / d->step_len;
    p->P = P;
    p->rows = d->n_rows;
    p->cols = d->n_cols;
    p->fs = d->fs_hz;
    p->fc = d->fc_hz;
    p->caf_lags_req = d->caf_lags;
    p->caf_bins = d->caf_bins > 0 ? d->caf_bins : 256;
    p->caf_lag_lo_set = d->caf_lag_lo_set != 0;
    p->caf_lag_lo_req = d->caf_lag_lo;
    p->caf_nu_lo_req = d->caf_nu_lo_hz;
    p->caf_nu_hi_req = d->caf_nu_hi_hz;
    p->radius = d->earth_radius_m;
    p->alt = d->alt_m;
    p->earth_model = d->earth_model;
    if (d->alt_grid) p->h_alt.assign(d->alt_grid, d->alt_grid + P);
    {
        PointTiling t{};
        if (d->grid_kind == GEOLOC_GRID_RECT) {
            t.rows = d->n_rows;
            t.cols = d->n_cols;
            t.tile_w = 16;
            t.tile_h = 16;
        } else {
            t.rows = 1;
            t.cols = P;
            t.tile_w = kTilePoints;
            t.tile_h = 1;
        }
        tiling_counts(t);
        p->base_tiling = p->tiling = t;
        p->max_tiles = t.tiles_x * t.tiles_y;
        if (d->grid_kind == GEOLOC_GRID_RECT) {
            // tile shapes of 256, 512 and 1024 cells, either way round; the map picks one and
            // its shear from the geometry, with |shear| <= kMaxShear (scratch is sized for that)
            const int shapes[10][2] = {{16, 16}, {8, 32}, {4, 64}, {16, 32}, {8, 64},
                                       {4, 128}, {32, 32}, {16, 64}, {8, 128}, {4, 256}};
            for (int tr = 0; tr < 2; ++tr)
                for (const auto& wh : shapes) {
                    PointTiling c = t;
                    c.tile_w = wh[0];
                    c.tile_h = wh[1];
                    c.transpose = tr;
                    p->tile_shapes.push_back(c);
                    for (int sg = -1; sg <= 1; sg += 2) {
                        c.shear = sg * kMaxShear;
                        tiling_counts(c);
                        p->max_tiles = std::max(p->max_tiles, c.tiles_x * c.tiles_y);
                    }
                }
        }
        p->h_lat.assign(d->lat, d->lat + (d->grid_kind == GEOLOC_GRID_RECT ? d->n_rows : P));
        p->h_lon.assign(d->lon, d->lon + (d->grid_kind == GEOLOC_GRID_RECT ? d->n_cols : P));
    }

    // steps per correlation launch: all of them, unless the deferral mask of one launch
    // ([pairs][steps][tiles] bytes) would exceed its budget
    const int64_t per_step = (int64_t)p->n_pairs * std::max<int64_t>(p->max_tiles, 1);
    int64_t kc = kMaskChunkBytes / per_step;
    if (kc < 1) kc = 1;
    if (kc > p->K) kc = p->K;
    const int64_t n_chunks = (p->K + kc - 1) / kc;
    p->kc = (int32_t)((p->K + n_chunks - 1) / n_chunks);
    p->n_chunks = n_chunks;

    do {
        if ((rc = dev_alloc(p, &p->d_xyz, (size_t)P * 3))) break;
        if (d->grid_kind == GEOLOC_GRID_RECT && !d->alt_grid &&
            ((rc = dev_alloc(p, &p->d_ecef_row, (size_t)d->n_rows)) ||
             (rc = dev_alloc(p, &p->d_ecef_col, (size_t)d->n_cols))))
            break;
        if ((rc = dev_alloc(p, &p->d_states, (size_t)p->K * p->n_rx * 6))) break;
        if ((rc = dev_alloc(p, &p->d_pairs, pairs.size()))) break;
        if ((rc = dev_alloc(p, &p->d_defer_flags, (size_t)(2 * n_chunks)))) break;
        if (hipMemset(p->d_defer_flags, 0, (size_t)(2 * n_chunks) * sizeof(uint32_t)) != hipSuccess) {
            rc = fail(GEOLOC_ELAUNCH, "hipMemset failed");
            break;
        }
        p->use_fact = p->method == GEOLOC_DIRECT_FP32;
        const int64_t base_tiles = p->base_tiling.tiles_x * p->base_tiling.tiles_y;
        const int64_t items = (int64_t)p->kc * p->n_pairs;
        p->n_groups = direct_groups(base_tiles, items);
        const int64_t wgs = base_tiles * p->n_groups;
        if (p->use_fact && wgs < 1024 && p->L >= 8192) {
            // too few (tile, item group) workgroups to fill the GPU, and long steps: also
            // split every step into coherent segments of a multiple of 2,048 samples
            int64_t ns = std::min<int64_t>({(1024 + wgs - 1) / wgs, 16, p->L / 2048});
            if (ns >= 2) {
                const int64_t len = round_up((p->L + ns - 1) / ns, 2048);
                p->seg_len = (int32_t)len;
                p->n_segs = (int32_t)((p->L + len - 1) / len);
                if ((rc = dev_alloc(p, &p->d_cpart, (size_t)p->n_segs * items * P))) break;
            }
        }
        if (p->n_groups > 1 && p->n_segs <= 1 && (rc = dev_alloc(p, &p->d_partial, (size_t)p->n_groups * P)))
            break;
        if (p->use_fact && p->n_groups == 1 && p->n_segs <= 1 && items > 1) {
            // a large grid: its factored launches may be split into item groups so that the
            // workgroup count fills whole rounds of the chip (partial rows within a budget)
            p->max_balance_groups = (int32_t)std::max<int64_t>(
                1, std::min<int64_t>({kMaxBalanceGroups, items, kBalanceBytes / ((int64_t)sizeof(float) * P)}));
            if (p->max_balance_groups > 1 &&
                (rc = dev_alloc(p, &p->d_partial, (size_t)p->max_balance_groups * P)))
                break;
        }
        // (whole 32-bit words: the second pass clears bits with word atomics)
        if (p->use_fact &&
            (rc = dev_alloc(p, &p->d_deferred, ((size_t)p->n_pairs * p->kc * p->max_tiles + 3) & ~(size_t)3)))
            break;
        p->am.n_blocks = argmax_blocks(P);
        if ((rc = dev_alloc(p, &p->am.part_val, p->am.n_blocks))) break;
        if ((rc = dev_alloc(p, &p->am.part_idx, p->am.n_blocks))) break;
        if ((rc = dev_alloc(p, &p->am.found_idx, kMaxTopK))) break;
        if ((rc = dev_alloc(p, &p->am.found_val, kMaxTopK))) break;
        if (hipHostMalloc((void**)&p->h_states, (size_t)p->K * p->n_rx * 6 * sizeof(double)) != hipSuccess) {
            p->h_states = nullptr;
            rc = fail(GEOLOC_ENOMEM, "pinned host allocation failed");
            break;
        }
        if (hipEventCreateWithFlags(&p->states_copied, hipEventDisableTiming) != hipSuccess) {
            rc = fail(GEOLOC_ELAUNCH, "hipEventCreate failed");
            break;
        }
        // grid -> ECEF on the device, once per plan (and again on geoloc_set_grid)
        if ((rc = dev_alloc(p, &p->d_lat, (size_t)n_lat))) break;
        if ((rc = dev_alloc(p, &p->d_lon, (size_t)n_lon))) break;
        if (d->alt_grid && (rc = dev_alloc(p, &p->d_alt, (size_t)P))) break;
        hipError_t e = hipMemcpy(p->d_lat, d->lat, n_lat * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess && d->alt_grid)
            e = hipMemcpy(p->d_alt, d->alt_grid, P * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(p->d_lon, d->lon, n_lon * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(p->d_pairs, pairs.data(), pairs.size() * sizeof(int2), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_grid_ecef(p->d_lat, p->d_lon, d->grid_kind, d->n_rows, d->n_cols, p->earth_model, p->radius,
                                 p->alt, p->d_alt, p->d_ecef_row, p->d_ecef_col, p->d_xyz, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            rc = fail(GEOLOC_ELAUNCH, "plan set-up: %s", hipGetErrorString(e));
            break;
        }
    } while (0);
    if (rc) {
        release(p);
        return rc;
    }
    *out = p;
    return GEOLOC_OK;
}

int geoloc_set_grid(geoloc_plan_t p, const double* lat, const double* lon) {
    if (!plan_ok(p)) return fail(GEOLOC_ESTATE, "invalid plan");
    if (!lat || !lon) return fail(GEOLOC_EINVAL, "NULL lat or lon");
    if (p->d_alt) return fail(GEOLOC_EINVAL, "the plan has a height per point: make a new plan for a new grid");
    const int64_t n_lat = p->grid_kind == GEOLOC_GRID_RECT ? p->rows : p->P;
    const int64_t n_lon = p->grid_kind == GEOLOC_GRID_RECT ? p->cols : p->P;
    for (int64_t i = 0; i < n_lat; ++i)
        if (!std::isfinite(lat[i])) return fail(GEOLOC_EINVAL, "lat[%lld] not finite", (long long)i);
    for (int64_t i = 0; i < n_lon; ++i)
        if (!std::isfinite(lon[i])) return fail(GEOLOC_EINVAL, "lon[%lld] not finite", (long long)i);
    HIP_TRY(hipDeviceSynchronize());
    p->h_lat.assign(lat, lat + n_lat);
    p->h_lon.assign(lon, lon + n_lon);
    HIP_TRY(hipMemcpy(p->d_lat, lat, n_lat * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->d_lon, lon, n_lon * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(launch_grid_ecef(p->d_lat, p->d_lon, p->grid_kind, p->rows, p->cols, p->earth_model, p->radius, p->alt,
                             nullptr, p->d_ecef_row, p->d_ecef_col, p->d_xyz, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    return GEOLOC_OK;
}

int geoloc_set_points_from_tiles(geoloc_plan_t p, const double* lat_dev, const double* lon_dev, int64_t rows,
                                 int64_t cols, int32_t tile, const int32_t* tiles, int32_t n_tiles, void* stream) {
    if (!plan_ok(p)) return fail(GEOLOC_ESTATE, "invalid plan");
    if (!lat_dev || !lon_dev || !tiles) return fail(GEOLOC_EINVAL, "NULL pointer");
    if (p->grid_kind != GEOLOC_GRID_POINTS) return fail(GEOLOC_EINVAL, "needs a POINTS plan");
    if (p->d_alt) return fail(GEOLOC_EINVAL, "the plan has a height per point: make a new plan for a new grid");
    if (tile < 1 || rows < tile || cols < tile || rows % tile || cols % tile)
        return fail(GEOLOC_EINVAL, "rows and cols must be positive multiples of tile");
    if (n_tiles < 1 || (int64_t)n_tiles * tile * tile != p->P)
        return fail(GEOLOC_EINVAL, "n_tiles x tile^2 must equal the plan's %lld points", (long long)p->P);
    hipStream_t s = (hipStream_t)stream;
    if (p->d_tiles_cap < n_tiles) {
        (void)hipFree(p->d_tiles);
        p->d_tiles = nullptr;
        p->d_tiles_cap = 0;
        int rc = dev_alloc(p, &p->d_tiles, (size_t)n_tiles);
        if (rc) return rc;
        p->d_tiles_cap = n_tiles;
    }
    HIP_TRY(hipMemcpyAsync(p->d_tiles, tiles, (size_t)n_tiles * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_tile_points(lat_dev, lon_dev, rows, cols, tile, p->d_tiles, p->P, p->d_lat, p->d_lon, s));
    HIP_TRY(launch_grid_ecef(p->d_lat, p->d_lon, p->grid_kind, p->rows, p->cols, p->earth_model, p->radius, p->alt,
                             nullptr, nullptr, nullptr, p->d_xyz, s));
    // the host copy of the grid serves the tile choice of RECT plans only
    p->h_lat.clear();
    p->h_lon.clear();
    return GEOLOC_OK;
}

int geoloc_set_tiling(geoloc_plan_t p, int32_t tile_w, int32_t tile_h, int32_t shear, int32_t transpose) {
    if (!plan_ok(p)) return fail(GEOLOC_ESTATE, "invalid plan");
    if (tile_w == 0) {
        p->tiling_fixed = false;
        return GEOLOC_OK;
    }
    if (p->grid_kind != GEOLOC_GRID_RECT || p->method != GEOLOC_DIRECT_FP32)
        return fail(GEOLOC_EINVAL, "a fixed tiling needs a RECT grid and GEOLOC_DIRECT_FP32");
    const int64_t cells = (int64_t)tile_w * tile_h;
    if (tile_w < 1 || tile_h < 1 || (cells != 256 && cells != 512 && cells != 1024))
        return fail(GEOLOC_EINVAL, "tile must hold 256, 512 or 1024 cells (got %d x %d)", tile_w, tile_h);
    if (shear < -kMaxShear || shear > kMaxShear) return fail(GEOLOC_EINVAL, "|shear| must be <= %d", kMaxShear);
    if (transpose != 0 && transpose != 1) return fail(GEOLOC_EINVAL, "transpose must be 0 or 1");
    PointTiling t = p->base_tiling;
    t.tile_w = tile_w;
    t.tile_h = tile_h;
    t.shear = shear;
    t.transpose = transpose;
    tiling_counts(t);
    if (t.tiles_x * t.tiles_y > p->max_tiles)
        return fail(GEOLOC_EINVAL, "tiling exceeds the plan's scratch");
    p->fixed_tiling = t;
    p->tiling_fixed = true;
    return GEOLOC_OK;
}

int geoloc_set_taylor_block(geoloc_plan_t p, int32_t samples) {
    if (!plan_ok(p)) return fail(GEOLOC_ESTATE, "invalid plan");
    if (samples != 0 && samples != 64 && samples != 256)
        return fail(GEOLOC_EINVAL, "Taylor block must be 0 (per map), 64 or 256 samples (got %d)", samples);
    p->taylor_fixed = samples / 64;
    return GEOLOC_OK;
}

int geoloc_set_timing(geoloc_plan_t p, int enable) {
    if (!plan_ok(p)) return fail(GEOLOC_ESTATE, "invalid plan");
    int rc = drain_spans(p);
    if (rc) return rc;
    p->timing = enable != 0;
    p->timed_maps = p->correlate_launches = 0;
    p->t_geom = p->t_corr = p->t_interp = p->t_map = 0;
    return GEOLOC_OK;
}

int geoloc_map(geoloc_plan_t p, const geoloc_inputs* in, float* J, uint32_t flags) {
    if (!plan_ok(p)) return fail(GEOLOC_ESTATE, "invalid plan");
    if (!in || !in->captures || !in->rx_state || !J) return fail(GEOLOC_EINVAL, "NULL input or output");
    if (((uintptr_t)in->captures & 7) != 0) return fail(GEOLOC_EINVAL, "captures must be 8-byte aligned");
    if (flags & ~GEOLOC_ACCUMULATE) return fail(GEOLOC_EINVAL, "unknown flags 0x%x", flags);
    hipStream_t s = (hipStream_t)in->stream;
    int rc = upload_states(p, in->rx_state, s);
    if (rc) return rc;
    choose_tiling(p, in->rx_state);
    TimedSpan whole{};
    if ((rc = span_begin(p, s, &whole, 3))) return rc;
    if (p->method == GEOLOC_CAF_BF16 || p->method == GEOLOC_CAF_FP16) {
        if ((rc = caf_map(p, in, J, flags, s))) return rc;
        if ((rc = span_end(p, s, &whole))) return rc;
        if (p->timing) p->timed_maps++;
        return GEOLOC_OK;
    }
    // a new sequence number per map: a deferral flag holds it only if this map's factored
    // launch deferred something (0 is the flags' initial value, never a sequence number)
    if (++p->defer_seq == 0) p->defer_seq = 1;
    for (int64_t k0 = 0; k0 < p->K; k0 += p->kc) {
        const int32_t kc = (int32_t)std::min<int64_t>(p->kc, p->K - k0);
        TimedSpan sc{};
        DirectArgs a{};
        a.cap = (const float2*)in->captures;
        a.xyz = p->d_xyz;
        a.ecef_row = p->d_ecef_row;
        a.ecef_col = p->d_ecef_col;
        a.states = p->d_states;
        a.n_rx = p->n_rx;
        a.fs = p->fs;
        a.inv_lambda = p->fc / kLightSpeed;
        a.pairs = p->d_pairs;
        a.J = J;
        a.tiling = p->tiling;
        a.n_tiles = p->tiling.tiles_x * p->tiling.tiles_y;   // <= max_tiles
        a.N = p->N;
        a.P = p->P;
        a.L = (int32_t)p->L;
        a.k0 = (int32_t)k0;
        a.kc = kc;
        a.n_pairs = p->n_pairs;
        a.inv_fs = 1.0 / p->fs;
        a.accum_mode = p->accum_mode;
        a.load_J = (k0 > 0) || (flags & GEOLOC_ACCUMULATE);
        a.n_groups = (int32_t)std::min<int64_t>(p->n_groups, (int64_t)kc * p->n_pairs);
        a.partial = p->d_partial;
        a.mask = nullptr;
        a.n_segs = p->use_fact ? p->n_segs : 1;
        a.seg_len = p->seg_len;
        a.cpart = p->d_cpart;
        a.defer_flag = p->d_defer_flags + k0 / p->kc;
        a.defer_seq = p->defer_seq;
        if (p->use_fact && a.n_groups == 1 && a.n_segs <= 1 && p->max_balance_groups > 1)
            a.n_groups = balance_groups((int64_t)kc * p->n_pairs, p->max_balance_groups);
        if ((rc = span_begin(p, s, &sc, 1))) return rc;
        if (p->use_fact) {
            HIP_TRY(launch_direct_fact(a, p->d_deferred, p->delay_mode, p->fact_wide, p->fact_sub, s));
            if (a.n_segs > 1) {
                // the segment reduction writes J itself: later passes add to it in place
                HIP_TRY(launch_direct_seg_reduce(a, s));
                a.n_groups = 1;
            }
        } else if (p->delay_mode == GEOLOC_DELAY_SINC)
            HIP_TRY(launch_direct_sinc(a, s));
        else
            HIP_TRY(launch_direct(a, p->delay_mode, s));
        if ((rc = span_end(p, s, &sc))) return rc;
        if (p->timing) p->correlate_launches++;
        if (p->use_fact) {
            TimedSpan sd{};
            DirectArgs m = a;
            m.mask = p->d_deferred;
            m.load_J = 1;
            if ((rc = span_begin(p, s, &sd, 2))) return rc;
            const int parts = tile_lanes(a.tiling) / 256;
            if (p->fact_sub == 4 || parts > 1) {
                // the deferred (tile, step) pairs go through the factored kernel again in
                // 256-cell parts of the tile (a part spans fewer lags) with 64-sample Taylor
                // blocks (a quarter of the Doppler phase spread over a block) and up to six
                // terms; the parts it defers again fall to the per-point kernel, gated on this
                // pass's flag. Whole steps: after a segment reduction J holds the rest.
                DirectArgs b = m;
                b.parts = parts;
                b.n_segs = 1;
                b.gate_flag = a.defer_flag;
                b.defer_flag = a.defer_flag + p->n_chunks;
                HIP_TRY(launch_direct_fact(b, p->d_deferred, p->delay_mode, true, 1, s));
                m.defer_flag = b.defer_flag;
            }
            // the per-point kernel adds the (tile, step) pairs the factored kernel deferred
            if (p->delay_mode == GEOLOC_DELAY_SINC)
                HIP_TRY(launch_direct_sinc(m, s));
            else
                HIP_TRY(launch_direct(m, p->delay_mode, s));
            if ((rc = span_end(p, s, &sd))) return rc;
        }
        HIP_TRY(launch_direct_reduce(a, s));
    }
    if ((rc = span_end(p, s, &whole))) return rc;
    if (p->timing) p->timed_maps++;
    return GEOLOC_OK;
}

int geoloc_geometry(geoloc_plan_t p, const geoloc_inputs* in, int32_t pair_index, int64_t step_lo, int64_t n_steps,
                    double* D, double* nu) {
    if (!plan_ok(p)) return fail(GEOLOC_ESTATE, "invalid plan");
    if (!in || !in->rx_state || !D || !nu) return fail(GEOLOC_EINVAL, "NULL input or output");
    if (pair_index < 0 || pair_index >= p->n_pairs) return fail(GEOLOC_EINVAL, "pair_index out of range");
    if (step_lo < 0 || n_steps < 1 || step_lo + n_steps > p->K || n_steps > INT32_MAX)
        return fail(GEOLOC_EINVAL, "step range [%lld, +%lld) outside [0, %lld)", (long long)step_lo,
                    (long long)n_steps, (long long)p->K);
    hipStream_t s = (hipStream_t)in->stream;
    int rc = upload_states(p, in->rx_state, s);
    if (rc) return rc;
    return run_geometry(p, pair_index, 1, step_lo, (int32_t)n_steps, D, nu, s);
}

int geoloc_caf_table(geoloc_plan_t p, const geoloc_inputs* in, int32_t pair_index, int64_t step_lo, int64_t n_steps,
                     void* T_dev, int64_t T_capacity) {
    if (!plan_ok(p)) return fail(GEOLOC_ESTATE, "invalid plan");
    if (p->method != GEOLOC_CAF_BF16 && p->method != GEOLOC_CAF_FP16)
        return fail(GEOLOC_EINVAL, "geoloc_caf_table needs a CAF method");
    if (!in || !in->captures || !in->rx_state || !T_dev) return fail(GEOLOC_EINVAL, "NULL input or output");
    if (((uintptr_t)in->captures & 7) != 0 || ((uintptr_t)T_dev & 7) != 0)
        return fail(GEOLOC_EINVAL, "captures and T_dev must be 8-byte aligned");
    if (pair_index < 0 || pair_index >= p->n_pairs) return fail(GEOLOC_EINVAL, "pair_index out of range");
    if (step_lo < 0 || n_steps < 1 || step_lo + n_steps > p->K)
        return fail(GEOLOC_EINVAL, "step range outside [0, %lld)", (long long)p->K);
    hipStream_t s = (hipStream_t)in->stream;
    int rc = upload_states(p, in->rx_state, s);
    if (rc) return rc;
    const float2* cap = (const float2*)in->captures;
    if ((rc = caf_prepare(p, cap, s))) return rc;
    const int64_t per = (int64_t)p->caf_n_lags * p->caf_bins;
    if (T_capacity < per * n_steps)
        return fail(GEOLOC_EINVAL, "T_capacity %lld < %lld entries needed", (long long)T_capacity,
                    (long long)(per * n_steps));
    int32_t kc, n_split, chunk;
    caf_split(p, 1, n_steps, &kc, &n_split, &chunk);
    for (int64_t k = 0; k < n_steps; k += kc) {
        const int32_t kn = (int32_t)std::min<int64_t>(kc, n_steps - k);
        if ((rc = caf_tables(p, cap, pair_index, 1, step_lo + k, kn, n_split, chunk, s))) return rc;
        for (int32_t q = 0; q < kn; ++q)
            HIP_TRY(hipMemcpy2DAsync((float2*)T_dev + (k + q) * per, (size_t)p->caf_bins * sizeof(float2),
                                     p->d_T + (size_t)q * p->caf_n_lags_pad * p->caf_M_pad,
                                     (size_t)p->caf_M_pad * sizeof(float2), (size_t)p->caf_bins * sizeof(float2),
                                     (size_t)p->caf_n_lags, hipMemcpyDeviceToDevice, s));
    }
    return GEOLOC_OK;
}

int geoloc_argmax(geoloc_plan_t p, const float* J, int32_t top_k, int32_t radius, int64_t* idx_host, float* val_host,
                  void* stream) {
    if (!plan_ok(p)) return fail(GEOLOC_ESTATE, "invalid plan");
    if (!J || !idx_host || !val_host) return fail(GEOLOC_EINVAL, "NULL pointer");
    if (top_k < 1 || top_k > kMaxTopK) return fail(GEOLOC_EINVAL, "top_k must be in [1, %d]", kMaxTopK);
    if (radius < 0) return fail(GEOLOC_EINVAL, "nms radius < 0");
    if (radius > 0 && p->grid_kind != GEOLOC_GRID_RECT) return fail(GEOLOC_EINVAL, "nms radius needs a RECT grid");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_argmax(J, p->P, p->cols, p->grid_kind == GEOLOC_GRID_RECT, radius, top_k, p->am, s));
    std::vector<int64_t> idx(top_k);
    std::vector<float> val(top_k);
    HIP_TRY(hipMemcpyAsync(idx.data(), p->am.found_idx, top_k * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(val.data(), p->am.found_val, top_k * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (std::isnan(val[0])) return fail(GEOLOC_ENAN, "NaN in map");
    for (int t = 0; t < top_k; ++t) {
        idx_host[t] = idx[t];
        val_host[t] = idx[t] < 0 ? -INFINITY : val[t];
    }
    return GEOLOC_OK;
}

int geoloc_detect(geoloc_plan_t p, const float* J, int32_t guard, int32_t train, double scale, int32_t max_det,
                  int32_t radius, int64_t* idx_host, float* val_host, float* noise_host, int32_t* n_found,
                  void* stream) {
    if (!plan_ok(p)) return fail(GEOLOC_ESTATE, "invalid plan");
    if (!J || !idx_host || !val_host || !noise_host || !n_found) return fail(GEOLOC_EINVAL, "NULL pointer");
    if (p->grid_kind != GEOLOC_GRID_RECT) return fail(GEOLOC_EINVAL, "detection needs a RECT grid");
    if (guard < 0 || train <= guard) return fail(GEOLOC_EINVAL, "need 0 <= guard < train");
    if (max_det < 1 || max_det > kMaxTopK) return fail(GEOLOC_EINVAL, "max_detections must be in [1, %d]", kMaxTopK);
    if (radius < 0) return fail(GEOLOC_EINVAL, "exclusion radius < 0");
    if (!(scale > 0.0) || !std::isfinite(scale)) return fail(GEOLOC_EINVAL, "scale must be finite and > 0");
    int rc = GEOLOC_OK;
    if (!p->d_sat) {
        if ((rc = dev_alloc(p, &p->d_sat, (size_t)p->P))) return rc;
        if ((rc = dev_alloc(p, &p->d_masked, (size_t)p->P))) return rc;
        if ((rc = dev_alloc(p, &p->d_noise, (size_t)p->P))) return rc;
        if ((rc = dev_alloc(p, &p->d_found_noise, (size_t)kMaxTopK))) return rc;
    }
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_cfar(J, p->rows, p->cols, guard, train, scale, p->d_sat, p->d_masked, p->d_noise, s));
    HIP_TRY(launch_argmax(p->d_masked, p->P, p->cols, 1, radius, max_det, p->am, s));
    HIP_TRY(launch_gather_noise(p->d_noise, p->am.found_idx, max_det, p->d_found_noise, s));
    std::vector<int64_t> idx(max_det);
    std::vector<float> val(max_det), nz(max_det);
    HIP_TRY(hipMemcpyAsync(idx.data(), p->am.found_idx, max_det * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(val.data(), p->am.found_val, max_det * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(nz.data(), p->d_found_noise, max_det * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (std::isnan(val[0])) return fail(GEOLOC_ENAN, "NaN in map");
    int32_t n = 0;
    for (int t = 0; t < max_det; ++t) {
        const bool ok = idx[t] >= 0 && val[t] > -INFINITY;   // masked cells are not detections
        idx_host[t] = ok ? idx[t] : -1;
        val_host[t] = ok ? val[t] : -INFINITY;
        noise_host[t] = ok ? nz[t] : 0.f;
        if (ok) ++n;
    }
    *n_found = n;
    return GEOLOC_OK;
}

// Regularised incomplete beta function I_x(a, b) from its continued fraction
//   I_x(a, b) = x^a (1 - x)^b / (a B(a, b)) * 1 / (1 + e_1 / (1 + e_2 / (1 + ...))),
//   e_{2m+1} = -(a + m)(a + b + m) x / ((a + 2m)(a + 2m + 1)),
//   e_{2m}   = m (b - m) x / ((a + 2m - 1)(a + 2m)),
// (Abramowitz & Stegun 26.5.8), evaluated by the modified Lentz algorithm (Lentz 1976;
// Thompson & Barnett 1986). The fraction converges fast for x < (a + 1) / (a + b + 2); above
// that I_x(a, b) = 1 - I_{1-x}(b, a) is used, and `upper` asks for 1 - I_x(a, b) directly so
// that small tail probabilities keep their relative precision.
static double beta_cf(double a, double b, double x) {
    constexpr double kTiny = 1e-300;
    double c = 1.0, d = 1.0 - (a + b) * x / (a + 1.0);
    if (std::fabs(d) < kTiny) d = kTiny;
    d = 1.0 / d;
    double f = d;
    for (int m = 1; m <= 100000; ++m) {
        const double e_even = m * (b - m) * x / ((a + 2.0 * m - 1.0) * (a + 2.0 * m));
        d = 1.0 + e_even * d;
        c = 1.0 + e_even / c;
        if (std::fabs(d) < kTiny) d = kTiny;
        if (std::fabs(c) < kTiny) c = kTiny;
        d = 1.0 / d;
        f *= c * d;
        const double e_odd = -(a + m) * (a + b + m) * x / ((a + 2.0 * m) * (a + 2.0 * m + 1.0));
        d = 1.0 + e_odd * d;
        c = 1.0 + e_odd / c;
        if (std::fabs(d) < kTiny) d = kTiny;
        if (std::fabs(c) < kTiny) c = kTiny;
        d = 1.0 / d;
        const double delta = c * d;
        f *= delta;
        if (std::fabs(delta - 1.0) < 1e-16) break;
    }
    return f;
}

static double beta_inc(double a, double b, double x, bool upper) {
    if (x <= 0.0) return upper ? 1.0 : 0.0;
    if (x >= 1.0) return upper ? 0.0 : 1.0;
    const double lfront = std::lgamma(a + b) - std::lgamma(a) - std::lgamma(b) + a * std::log(x) + b * std::log1p(-x);
    if (x < (a + 1.0) / (a + b + 2.0)) {
        const double v = std::exp(lfront) * beta_cf(a, b, x) / a;
        return upper ? 1.0 - v : v;
    }
    const double v = std::exp(lfront) * beta_cf(b, a, 1.0 - x) / b;   // 1 - I_x(a, b)
    return upper ? v : 1.0 - v;
}

int geoloc_cfar_scale(double pfa, int32_t n_train, int32_t looks, double* out) {
    if (!out) return fail(GEOLOC_EINVAL, "NULL output");
    if (!(pfa > 0.0 && pfa < 1.0)) return fail(GEOLOC_EINVAL, "false-alarm probability must be in (0, 1)");
    if (n_train < 1 || looks < 1) return fail(GEOLOC_EINVAL, "need n_train >= 1 and looks >= 1");
    // x / (x + z) ~ Beta(L, N L): find the b with P(Beta > b) = pfa by bisection on [0, 1]
    // (the tail falls monotonically in b), then scale = N b / (1 - b).
    const double a = (double)looks, bb = (double)n_train * (double)looks;
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (beta_inc(a, bb, mid, true) > pfa)
            lo = mid;
        else
            hi = mid;
    }
    const double b = 0.5 * (lo + hi);
    const double scale = (double)n_train * b / (1.0 - b);
    if (!std::isfinite(scale) || !(scale > 0.0)) return fail(GEOLOC_EINVAL, "no finite scale for this request");
    *out = scale;
    return GEOLOC_OK;
}

int geoloc_info(geoloc_plan_t p, geoloc_plan_info* out) {
    if (!plan_ok(p)) return fail(GEOLOC_ESTATE, "invalid plan");
    if (!out) return fail(GEOLOC_EINVAL, "NULL output");
    int rc = drain_spans(p);
    if (rc) return rc;
    geoloc_plan_info r{};
    r.n_points = p->P;
    r.n_steps = p->K;
    r.n_pairs = p->n_pairs;
    r.n_samples = p->N;
    r.step_len = p->L;
    r.method = p->method;
    r.delay_mode = p->delay_mode;
    r.caf_lag_lo = (int32_t)p->caf_lag_lo;
    r.caf_lags = p->caf_n_lags;
    r.caf_bins = (p->method == GEOLOC_CAF_BF16 || p->method == GEOLOC_CAF_FP16) ? p->caf_bins : 0;
    r.caf_nu_lo_hz = p->caf_nu_lo;
    r.caf_nu_hi_hz = p->caf_nu_hi;
    r.device_bytes = p->device_bytes;
    r.timed_maps = p->timed_maps;
    r.correlate_launches = p->correlate_launches;
    r.geometry_ms = p->t_geom;
    r.correlate_ms = p->t_corr;
    r.interp_ms = p->t_interp;
    r.map_ms = p->t_map;
    r.tile_rows = p->tiling.tile_h;
    r.tile_cols = p->tiling.tile_w;
    r.tile_shear = p->tiling.shear;
    r.tile_transpose = p->tiling.transpose;
    r.step_segments = p->n_segs > 1 ? p->n_segs : 1;
    r.segment_len = p->n_segs > 1 ? p->seg_len : (int32_t)p->L;
    r.taylor_block = 64 * p->fact_sub;
    *out = r;
    return GEOLOC_OK;
}

int geoloc_fma_probe(int32_t n_blocks, int32_t iters, float* out_dev, int64_t* fma_per_lane, void* stream) {
    if (!out_dev || !fma_per_lane) return fail(GEOLOC_EINVAL, "geoloc_fma_probe: NULL pointer");
    if (n_blocks < 1 || n_blocks > (1 << 20) || iters < 1 || iters > (1 << 24))
        return fail(GEOLOC_EINVAL, "geoloc_fma_probe: n_blocks %d or iters %d out of range", n_blocks, iters);
    int dev = 0;
    int rc = check_device(&dev);
    if (rc) return rc;
    HIP_TRY(launch_fma_ceiling(n_blocks, iters, out_dev, (hipStream_t)stream));
    *fma_per_lane = (int64_t)iters * fma_ceiling_chains();
    return GEOLOC_OK;
}

int geoloc_subbands(const void* captures, int32_t n_ch, int64_t n_samples, int32_t n_bands, int32_t half_taps,
                    void* out, void* stream) {
    if (captures == nullptr || out == nullptr) return fail(GEOLOC_EINVAL, "geoloc_subbands: null buffer");
    if ((reinterpret_cast<uintptr_t>(captures) & 7u) || (reinterpret_cast<uintptr_t>(out) & 7u))
        return fail(GEOLOC_EINVAL, "geoloc_subbands: buffers must be 8-byte aligned");
    if (n_ch < 1 || n_samples < 1) return fail(GEOLOC_EINVAL, "geoloc_subbands: empty input");
    if (n_bands < 1 || n_bands > kSubbandMaxBands)
        return fail(GEOLOC_EINVAL, "geoloc_subbands: n_bands %d outside 1..%d", n_bands, kSubbandMaxBands);
    if (n_samples % n_bands)
        return fail(GEOLOC_EINVAL, "geoloc_subbands: n_samples %lld not divisible by n_bands %d",
                    (long long)n_samples, n_bands);
    if (half_taps < 1 || half_taps > kSubbandMaxHalf)
        return fail(GEOLOC_EINVAL, "geoloc_subbands: half_taps %d outside 1..%d", half_taps, kSubbandMaxHalf);
    if ((int64_t)n_bands * (2 * half_taps + 1) > kSubbandMaxTable)
        return fail(GEOLOC_EINVAL, "geoloc_subbands: n_bands x (2 half_taps + 1) exceeds %d", kSubbandMaxTable);
    const int64_t n_seg = (n_samples / n_bands + 63) / 64;
    if (n_seg * n_ch > (int64_t)INT32_MAX) return fail(GEOLOC_EINVAL, "geoloc_subbands: input too long");
    int dev = 0;
    int rc = check_device(&dev);
    if (rc) return rc;
    SubbandArgs a{};
    a.in = static_cast<const float2*>(captures);
    a.out = static_cast<float2*>(out);
    a.N = n_samples;
    a.n_ch = n_ch;
    a.n_bands = n_bands;
    a.half_taps = half_taps;
    // Blackman-windowed sinc, cut-off 1/(2M) cycles per sample, unit DC gain (FP64)
    const double pi = 3.14159265358979323846;
    double g[2 * kSubbandMaxHalf + 1];
    double sum = 0.0;
    for (int t = -half_taps; t <= half_taps; ++t) {
        const double g0 = t == 0 ? 1.0 / n_bands : std::sin(pi * t / n_bands) / (pi * t);
        const double w = 0.42 + 0.5 * std::cos(pi * t / half_taps) + 0.08 * std::cos(2.0 * pi * t / half_taps);
        g[t + half_taps] = g0 * w;
        sum += g0 * w;
    }
    for (int i = 0; i < 2 * half_taps + 1; ++i) a.taps[i] = (float)(g[i] / sum);
    HIP_TRY(launch_subband(a, static_cast<hipStream_t>(stream)));
    return GEOLOC_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------------ CNN

struct geoloc_cnn_s {
    uint32_t magic = 0x636e6e31u;  // "cnn1"
    int32_t in_ch = 0, hidden = 0, layers = 0, H = 0, W = 0, max_batch = 0;
    int64_t n_params = 0, step = 0;
    std::vector<int32_t> cin, cout;
    std::vector<int64_t> w_off, b_off;
    float* d_master = nullptr;
    float* d_grad = nullptr;
    float* d_m = nullptr;
    float* d_v = nullptr;
    _Float16* d_w16 = nullptr;
    float* d_x = nullptr;            // copy of the last forward input
    std::vector<float*> d_z;         // pre-activations of layers 0 .. layers-2
    float* d_g0 = nullptr;
    float* d_g1 = nullptr;
    int32_t* d_tiles = nullptr;
    float* d_probs = nullptr;
    int32_t last_batch = -1;
};

namespace {

bool cnn_ok(geoloc_cnn_t c) { return c != nullptr && c->magic == 0x636e6e31u; }

void cnn_release(geoloc_cnn_t c) {
    (void)hipDeviceSynchronize();
    for (void* ptr : {(void*)c->d_master, (void*)c->d_grad, (void*)c->d_m, (void*)c->d_v, (void*)c->d_w16,
                      (void*)c->d_x, (void*)c->d_g0, (void*)c->d_g1, (void*)c->d_tiles, (void*)c->d_probs})
        (void)hipFree(ptr);
    for (float* z : c->d_z) (void)hipFree(z);
    c->magic = 0;
    delete c;
}

template <typename T>
int cnn_alloc(T** out, size_t count) {
    void* ptr = nullptr;
    if (hipMalloc(&ptr, (count ? count : 1) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GEOLOC_ENOMEM, "hipMalloc of %zu bytes failed", count * sizeof(T));
    }
    *out = (T*)ptr;
    return GEOLOC_OK;
}

int cnn_batch_ok(geoloc_cnn_t c, int32_t batch) {
    if (batch < 1 || batch > c->max_batch)
        return fail(GEOLOC_EINVAL, "batch %d outside [1, %d]", batch, c->max_batch);
    return GEOLOC_OK;
}

}  // namespace

extern "C" {

int geoloc_cnn_create(const geoloc_cnn_desc* d, geoloc_cnn_t* out) {
    if (!d || !out) return fail(GEOLOC_EINVAL, "NULL descriptor or output");
    if (d->in_ch < 1 || d->in_ch > 32 || d->hidden < 1 || d->hidden > 32 || d->layers < 2 || d->layers > 16 ||
        d->height < 1 || d->width < 1 || (int64_t)d->height * d->width > (1 << 20) || d->max_batch < 1 ||
        d->max_batch > 4096)
        return fail(GEOLOC_EINVAL, "CNN sizes out of range");
    int dev = 0;
    int rc = check_device(&dev);
    if (rc) return rc;
    geoloc_cnn_t c = new (std::nothrow) geoloc_cnn_s();
    if (!c) return fail(GEOLOC_ENOMEM, "host allocation failed");
    c->in_ch = d->in_ch;
    c->hidden = d->hidden;
    c->layers = d->layers;
    c->H = d->height;
    c->W = d->width;
    c->max_batch = d->max_batch;
    int64_t o = 0;
    for (int l = 0; l < c->layers; ++l) {
        const int ci = l == 0 ? c->in_ch : c->hidden, co = l == c->layers - 1 ? 1 : c->hidden;
        c->cin.push_back(ci);
        c->cout.push_back(co);
        c->w_off.push_back(o);
        o += (int64_t)co * ci * 9;
        c->b_off.push_back(o);
        o += co;
    }
    c->n_params = o;
    const size_t plane = (size_t)c->H * c->W;
    do {
        if ((rc = cnn_alloc(&c->d_master, o)) || (rc = cnn_alloc(&c->d_grad, o)) || (rc = cnn_alloc(&c->d_m, o)) ||
            (rc = cnn_alloc(&c->d_v, o)) || (rc = cnn_alloc(&c->d_w16, o)) ||
            (rc = cnn_alloc(&c->d_x, (size_t)c->max_batch * c->in_ch * plane)) ||
            (rc = cnn_alloc(&c->d_g0, (size_t)c->max_batch * c->hidden * plane)) ||
            (rc = cnn_alloc(&c->d_g1, (size_t)c->max_batch * c->hidden * plane)) ||
            (rc = cnn_alloc(&c->d_tiles, (size_t)c->max_batch * 64)) ||
            (rc = cnn_alloc(&c->d_probs, (size_t)c->max_batch * 64)))
            break;
        for (int l = 0; l + 1 < c->layers && !rc; ++l) {
            float* z = nullptr;
            rc = cnn_alloc(&z, (size_t)c->max_batch * c->hidden * plane);
            if (!rc) c->d_z.push_back(z);
        }
        if (rc) break;
        hipError_t e = hipMemset(c->d_master, 0, o * sizeof(float));
        if (e == hipSuccess) e = hipMemset(c->d_grad, 0, o * sizeof(float));
        if (e == hipSuccess) e = hipMemset(c->d_m, 0, o * sizeof(float));
        if (e == hipSuccess) e = hipMemset(c->d_v, 0, o * sizeof(float));
        if (e == hipSuccess) e = hipMemset(c->d_w16, 0, o * sizeof(_Float16));
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) rc = fail(GEOLOC_ELAUNCH, "CNN set-up: %s", hipGetErrorString(e));
    } while (0);
    if (rc) {
        cnn_release(c);
        return rc;
    }
    *out = c;
    return GEOLOC_OK;
}

int geoloc_cnn_param_count(geoloc_cnn_t c, int64_t* n) {
    if (!cnn_ok(c)) return fail(GEOLOC_ESTATE, "invalid CNN handle");
    if (!n) return fail(GEOLOC_EINVAL, "NULL output");
    *n = c->n_params;
    return GEOLOC_OK;
}

int geoloc_cnn_set_params(geoloc_cnn_t c, const float* theta, int64_t n) {
    if (!cnn_ok(c)) return fail(GEOLOC_ESTATE, "invalid CNN handle");
    if (!theta || n != c->n_params) return fail(GEOLOC_EINVAL, "expected %lld parameters", (long long)c->n_params);
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(theta[i])) return fail(GEOLOC_EINVAL, "parameter %lld not finite", (long long)i);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(c->d_master, theta, n * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(c->d_m, 0, n * sizeof(float)));
    HIP_TRY(hipMemset(c->d_v, 0, n * sizeof(float)));
    HIP_TRY(launch_cnn_to_half(c->d_master, c->d_w16, n, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    c->step = 0;
    return GEOLOC_OK;
}

int geoloc_cnn_get_params(geoloc_cnn_t c, int32_t which, float* out, int64_t n) {
    if (!cnn_ok(c)) return fail(GEOLOC_ESTATE, "invalid CNN handle");
    if (!out || n != c->n_params || which < 0 || which > 2) return fail(GEOLOC_EINVAL, "bad arguments");
    HIP_TRY(hipDeviceSynchronize());
    if (which == 1) {
        std::vector<_Float16> h(n);
        HIP_TRY(hipMemcpy(h.data(), c->d_w16, n * sizeof(_Float16), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i) out[i] = (float)h[i];
        return GEOLOC_OK;
    }
    HIP_TRY(hipMemcpy(out, which == 0 ? c->d_master : c->d_grad, n * sizeof(float), hipMemcpyDeviceToHost));
    return GEOLOC_OK;
}

int geoloc_cnn_prepare(geoloc_cnn_t c, const float* J, const double* D, const double* nu, int32_t batch, float* x,
                       void* stream) {
    if (!cnn_ok(c)) return fail(GEOLOC_ESTATE, "invalid CNN handle");
    if (c->in_ch != 3) return fail(GEOLOC_EINVAL, "geoloc_cnn_prepare makes 3 input channels");
    if (!J || !D || !nu || !x) return fail(GEOLOC_EINVAL, "NULL pointer");
    if (batch < 1) return fail(GEOLOC_EINVAL, "batch < 1");
    HIP_TRY(launch_cnn_prep(J, D, nu, c->H * c->W, batch, x, (hipStream_t)stream));
    return GEOLOC_OK;
}

int geoloc_cnn_forward(geoloc_cnn_t c, const float* x, int32_t batch, float* logits, void* stream) {
    if (!cnn_ok(c)) return fail(GEOLOC_ESTATE, "invalid CNN handle");
    if (!x || !logits) return fail(GEOLOC_EINVAL, "NULL pointer");
    int rc = cnn_batch_ok(c, batch);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const size_t plane = (size_t)c->H * c->W;
    HIP_TRY(hipMemcpyAsync(c->d_x, x, (size_t)batch * c->in_ch * plane * sizeof(float), hipMemcpyDeviceToDevice, s));
    for (int l = 0; l < c->layers; ++l) {
        const float* in = l == 0 ? c->d_x : c->d_z[l - 1];
        float* out = l == c->layers - 1 ? logits : c->d_z[l];
        HIP_TRY(launch_cnn_conv_fwd(l > 0, in, c->d_w16 + c->w_off[l], c->d_w16 + c->b_off[l], out, batch, c->cin[l],
                                    c->cout[l], c->H, c->W, s));
    }
    c->last_batch = batch;
    return GEOLOC_OK;
}

int geoloc_cnn_loss(geoloc_cnn_t c, const float* logits, const float* label, int32_t batch, float* dlogits,
                    float* loss, void* stream) {
    if (!cnn_ok(c)) return fail(GEOLOC_ESTATE, "invalid CNN handle");
    if (!logits || !label || !dlogits || !loss) return fail(GEOLOC_EINVAL, "NULL pointer");
    if (batch < 1) return fail(GEOLOC_EINVAL, "batch < 1");
    HIP_TRY(launch_cnn_softmax_ce(logits, label, c->H * c->W, batch, dlogits, loss, (hipStream_t)stream));
    return GEOLOC_OK;
}

int geoloc_cnn_backward(geoloc_cnn_t c, const float* dlogits, int32_t batch, void* stream) {
    if (!cnn_ok(c)) return fail(GEOLOC_ESTATE, "invalid CNN handle");
    if (!dlogits) return fail(GEOLOC_EINVAL, "NULL pointer");
    if (batch != c->last_batch) return fail(GEOLOC_ESTATE, "backward needs the batch of the last forward");
    hipStream_t s = (hipStream_t)stream;
    const float* g = dlogits;
    float* bufs[2] = {c->d_g0, c->d_g1};
    for (int l = c->layers - 1; l >= 0; --l) {
        const float* in = l == 0 ? c->d_x : c->d_z[l - 1];
        HIP_TRY(launch_cnn_conv_wgrad(l > 0, g, in, c->d_grad + c->w_off[l], c->d_grad + c->b_off[l], batch,
                                      c->cin[l], c->cout[l], c->H, c->W, s));
        if (l > 0) {
            float* gn = bufs[l & 1];
            HIP_TRY(launch_cnn_conv_dgrad(true, g, c->d_w16 + c->w_off[l], c->d_z[l - 1], gn, batch, c->cin[l],
                                          c->cout[l], c->H, c->W, s));
            g = gn;
        }
    }
    return GEOLOC_OK;
}

int geoloc_cnn_adam_step(geoloc_cnn_t c, float lr, float b1, float b2, float eps, void* stream) {
    if (!cnn_ok(c)) return fail(GEOLOC_ESTATE, "invalid CNN handle");
    if (!(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
        return fail(GEOLOC_EINVAL, "bad Adam hyper-parameters");
    c->step++;
    const float bc1 = (float)(1.0 - std::pow((double)b1, (double)c->step));
    const float bc2 = (float)(1.0 - std::pow((double)b2, (double)c->step));
    HIP_TRY(launch_cnn_adam(c->d_master, c->d_m, c->d_v, c->d_grad, c->d_w16, c->n_params, lr, b1, b2, eps, bc1, bc2,
                            (hipStream_t)stream));
    return GEOLOC_OK;
}

int geoloc_cnn_topk(geoloc_cnn_t c, const float* logits, int32_t batch, int32_t k, int32_t* tiles, float* probs,
                    void* stream) {
    if (!cnn_ok(c)) return fail(GEOLOC_ESTATE, "invalid CNN handle");
    if (!logits || !tiles || !probs) return fail(GEOLOC_EINVAL, "NULL pointer");
    int rc = cnn_batch_ok(c, batch);
    if (rc) return rc;
    if (k < 1 || k > 64 || k > c->H * c->W) return fail(GEOLOC_EINVAL, "k must be in [1, min(64, tiles)]");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_cnn_topk(logits, c->H * c->W, batch, k, c->d_tiles, c->d_probs, s));
    HIP_TRY(hipMemcpyAsync(tiles, c->d_tiles, (size_t)batch * k * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(probs, c->d_probs, (size_t)batch * k * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return GEOLOC_OK;
}

int geoloc_cnn_destroy(geoloc_cnn_t c) {
    if (!cnn_ok(c)) return fail(GEOLOC_ESTATE, "invalid CNN handle");
    cnn_release(c);
    return GEOLOC_OK;
}

int geoloc_destroy(geoloc_plan_t p) {
    if (!plan_ok(p)) return fail(GEOLOC_ESTATE, "invalid plan");
    release(p);
    return GEOLOC_OK;
}

}  // extern "C"
