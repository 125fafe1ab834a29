// api.hip -- the C-ABI host layer: validation, device checks, buffer ownership, dispatch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
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

#define HIP_TRY(call)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return fail(GEOLOC_ELAUNCH, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

constexpr uint32_t kMagic = 0x67656f6cu;  // "geol"
constexpr int64_t kGeomChunkBytes = 512ll << 20;

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
    PointTiling tiling{};
    int32_t kc = 1;  // steps per geometry chunk
    // device scratch
    double* d_xyz = nullptr;
    double* d_states = nullptr;
    int2* d_pairs = nullptr;
    double* d_D = nullptr;
    double* d_nu = nullptr;
    ArgmaxScratch am;
    int64_t device_bytes = 0;
    // host staging for receiver states (pinned) and its reuse guard
    double* h_states = nullptr;
    hipEvent_t states_copied = nullptr;
    bool states_pending = false;
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
    (void)hipFree(p->d_states);
    (void)hipFree(p->d_pairs);
    (void)hipFree(p->d_D);
    (void)hipFree(p->d_nu);
    (void)hipFree(p->am.part_val);
    (void)hipFree(p->am.part_idx);
    (void)hipFree(p->am.found_idx);
    (void)hipFree(p->am.found_val);
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

int run_geometry(geoloc_plan_t p, int32_t pair_lo, int32_t n_pairs, int64_t k0, int32_t kc, double* D, double* nu,
                 bool tile_major, hipStream_t s) {
    GeomArgs g{};
    g.tiling = p->tiling;
    g.tile_major = tile_major ? 1 : 0;
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
    if (!(d->earth_radius_m > 0) || !std::isfinite(d->earth_radius_m) || !std::isfinite(d->alt_m))
        return fail(GEOLOC_EINVAL, "earth_radius_m must be > 0 and alt_m finite");
    if (d->grid_kind != GEOLOC_GRID_RECT && d->grid_kind != GEOLOC_GRID_POINTS)
        return fail(GEOLOC_EINVAL, "unknown grid_kind %d", d->grid_kind);
    if (d->n_rows <= 0 || d->n_cols <= 0) return fail(GEOLOC_EINVAL, "empty grid");
    if (d->n_rows > (1ll << 31) || d->n_cols > (1ll << 31) || d->n_rows * d->n_cols > (1ll << 34))
        return fail(GEOLOC_EINVAL, "grid too large");
    if (!d->lat || !d->lon) return fail(GEOLOC_EINVAL, "NULL lat or lon");
    if (d->method != GEOLOC_DIRECT_FP32 && d->method != GEOLOC_CAF_BF16 && d->method != GEOLOC_CAF_FP16)
        return fail(GEOLOC_EINVAL, "unknown method %d", d->method);
    if (d->delay_mode != GEOLOC_DELAY_LINEAR && d->delay_mode != GEOLOC_DELAY_ROUND)
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
    if (d->method != GEOLOC_DIRECT_FP32) return fail(GEOLOC_EUNSUPPORTED, "CAF methods are not built yet");

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
    p->radius = d->earth_radius_m;
    p->alt = d->alt_m;
    if (d->grid_kind == GEOLOC_GRID_RECT) {
        p->tiling.rows = d->n_rows;
        p->tiling.cols = d->n_cols;
        p->tiling.tile_w = 16;
        p->tiling.tile_h = 16;
    } else {
        p->tiling.rows = 1;
        p->tiling.cols = P;
        p->tiling.tile_w = kTilePoints;
        p->tiling.tile_h = 1;
    }
    p->tiling.tiles_x = (p->tiling.cols + p->tiling.tile_w - 1) / p->tiling.tile_w;
    p->tiling.tiles_y = (p->tiling.rows + p->tiling.tile_h - 1) / p->tiling.tile_h;

    const int64_t table_points = p->tiling.tiles_x * p->tiling.tiles_y * kTilePoints;  // tile-major >= P
    const int64_t per_step = (int64_t)p->n_pairs * table_points * 16;
    int64_t kc = kGeomChunkBytes / per_step;
    if (kc < 1) kc = 1;
    if (kc > p->K) kc = p->K;
    const int64_t n_chunks = (p->K + kc - 1) / kc;
    p->kc = (int32_t)((p->K + n_chunks - 1) / n_chunks);

    double* d_lat = nullptr;
    double* d_lon = nullptr;
    do {
        if ((rc = dev_alloc(p, &p->d_xyz, (size_t)P * 3))) break;
        if ((rc = dev_alloc(p, &p->d_states, (size_t)p->K * p->n_rx * 6))) break;
        if ((rc = dev_alloc(p, &p->d_pairs, pairs.size()))) break;
        if ((rc = dev_alloc(p, &p->d_D, (size_t)p->n_pairs * p->kc * table_points))) break;
        if ((rc = dev_alloc(p, &p->d_nu, (size_t)p->n_pairs * p->kc * table_points))) break;
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
        // grid -> ECEF on the device, once per plan
        if ((rc = dev_alloc(p, &d_lat, (size_t)n_lat))) break;
        if ((rc = dev_alloc(p, &d_lon, (size_t)n_lon))) break;
        hipError_t e = hipMemcpy(d_lat, d->lat, n_lat * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_lon, d->lon, n_lon * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(p->d_pairs, pairs.data(), pairs.size() * sizeof(int2), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_grid_ecef(d_lat, d_lon, d->grid_kind, d->n_rows, d->n_cols, d->earth_radius_m + d->alt_m,
                                 p->d_xyz, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            rc = fail(GEOLOC_ELAUNCH, "plan set-up: %s", hipGetErrorString(e));
            break;
        }
    } while (0);
    if (d_lat) {
        (void)hipFree(d_lat);
        p->device_bytes -= n_lat * sizeof(double);
    }
    if (d_lon) {
        (void)hipFree(d_lon);
        p->device_bytes -= n_lon * sizeof(double);
    }
    if (rc) {
        release(p);
        return rc;
    }
    *out = p;
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
    TimedSpan whole{};
    if ((rc = span_begin(p, s, &whole, 3))) return rc;
    for (int64_t k0 = 0; k0 < p->K; k0 += p->kc) {
        const int32_t kc = (int32_t)std::min<int64_t>(p->kc, p->K - k0);
        TimedSpan sg{}, sc{};
        if ((rc = span_begin(p, s, &sg, 0))) return rc;
        if ((rc = run_geometry(p, 0, p->n_pairs, k0, kc, p->d_D, p->d_nu, true, s))) return rc;
        if ((rc = span_end(p, s, &sg))) return rc;

        DirectArgs a{};
        a.cap = (const float2*)in->captures;
        a.D = p->d_D;
        a.nu = p->d_nu;
        a.pairs = p->d_pairs;
        a.J = J;
        a.tiling = p->tiling;
        a.n_tiles = p->tiling.tiles_x * p->tiling.tiles_y;
        a.N = p->N;
        a.P = p->P;
        a.L = (int32_t)p->L;
        a.k0 = (int32_t)k0;
        a.kc = kc;
        a.n_pairs = p->n_pairs;
        a.inv_fs = 1.0 / p->fs;
        a.accum_mode = p->accum_mode;
        a.load_J = (k0 > 0) || (flags & GEOLOC_ACCUMULATE);
        if ((rc = span_begin(p, s, &sc, 1))) return rc;
        HIP_TRY(launch_direct(a, p->delay_mode, s));
        if ((rc = span_end(p, s, &sc))) return rc;
        if (p->timing) p->correlate_launches++;
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
    return run_geometry(p, pair_index, 1, step_lo, (int32_t)n_steps, D, nu, false, s);
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
    r.caf_nu_lo_hz = NAN;
    r.caf_nu_hi_hz = NAN;
    r.device_bytes = p->device_bytes;
    r.timed_maps = p->timed_maps;
    r.correlate_launches = p->correlate_launches;
    r.geometry_ms = p->t_geom;
    r.correlate_ms = p->t_corr;
    r.interp_ms = p->t_interp;
    r.map_ms = p->t_map;
    *out = r;
    return GEOLOC_OK;
}

int geoloc_destroy(geoloc_plan_t p) {
    if (!plan_ok(p)) return fail(GEOLOC_ESTATE, "invalid plan");
    release(p);
    return GEOLOC_OK;
}

}  // extern "C"
