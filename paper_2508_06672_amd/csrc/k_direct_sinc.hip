// k_direct_sinc.hip -- Eq. (11) point by point with the eight-tap windowed-sinc delay
// (GEOLOC_DELAY_SINC): the kernel of GEOLOC_DIRECT_FP32_POINTWISE in that mode, and the
// pass over the (tile, step) pairs the factored kernel defers.
//
// One lane per point, one workgroup per 256 points of a tile and group of (pair, step)
// items, as in the other correlation kernels (same tiling, masks and partial rows). Per
// sample a lane reads y_i[n] (the same address for every lane: one broadcast load) and the
// eight taps y_j[n + floor(D) - 3 .. n + floor(D) + 4] from global memory; the taps slide in
// registers, so each sample loads one new y_j value. The Doppler phasor advances by a
// per-lane step and is re-anchored from an exact FP64 phase every 64 samples.
#include "internal.h"

namespace geoloc {

constexpr int kSincAnchor = 64;   // samples between FP64 phase re-anchors

__global__ __launch_bounds__(256) void k_direct_sinc(DirectArgs a) {
    const int tid = threadIdx.x;
    // (a tile of 512 cells is two workgroups, one per half)
    // a masked pass after a factored launch that deferred nothing has nothing to add
    if (a.mask && *a.defer_flag != a.defer_seq) return;
    const int halves = tile_lanes(a.tiling) / 256;
    const int64_t sub = blockIdx.x % (a.n_tiles * halves);
    const int64_t tile = sub / halves;
    const int half = (int)(sub - tile * halves);
    const int lane = half * 256 + tid;
    const int group = (int)(blockIdx.x / (a.n_tiles * halves));
    const int64_t n_items = (int64_t)a.n_pairs * a.kc;
    const int64_t it_lo = n_items * group / a.n_groups;
    const int64_t it_hi = n_items * (group + 1) / a.n_groups;
    bool valid;
    const int64_t p = tile_point(a.tiling, tile, lane, &valid);
    // a wave without a grid cell has nothing to do (this kernel has no barriers)
    if (__ballot(valid) == 0) return;
    double jacc = 0.0;
    if (valid && a.n_groups == 1 && a.load_J) jacc = (double)a.J[p];
    if (valid && a.n_groups > 1 && a.mask) jacc = (double)a.partial[(int64_t)group * a.P + p];
    const double centre = 0.5 * (double)(a.L - 1);

    for (int64_t it = it_lo; it < it_hi; ++it) {
        // with a mask, only this 256-cell part of the (tile, step) pairs the factored kernel
        // left over (the search needs every lane of the wave: the lanes without a cell run
        // the body on point 0 and never store their sum)
        if (a.mask) {
            it = next_flagged(a.mask, a.n_tiles, tile, 1u << half, it, it_hi);
            if (it >= it_hi) break;
        }
        const int e = (int)(it / a.kc);
        const int kk = (int)(it - (int64_t)e * a.kc);
        const int2 pr = a.pairs[e];
        const float2* __restrict__ yi = a.cap + (int64_t)pr.x * a.N;
        const float2* __restrict__ yj = a.cap + (int64_t)pr.y * a.N;
        const int64_t n_step = (int64_t)(a.k0 + kk) * a.L;
        // delay (samples) and Doppler shift (Hz) of this point, Eq. (3)-(9) in FP64
        double D, nu;
        pair_geometry(a.xyz[3 * p], a.xyz[3 * p + 1], a.xyz[3 * p + 2], a.states, a.n_rx, a.k0 + kk, pr, a.fs,
                      a.inv_lambda, &D, &nu);
        if (!(fabs(D) < 1.0e9)) D = 1.0e9;
        const double f = floor(D);
        const int64_t d0 = (int64_t)f;
        float w[kSincTaps];
        sinc_taps((float)(D - f), w);
        const double cyc = nu * a.inv_fs;
        const float2 E = cis_cycles(cyc);
        // sliding window of the eight taps for sample n: y_j[n + d0 - 3 + t]
        auto yj_at = [&](int64_t m) { return (m >= 0 && m < a.N) ? yj[m] : make_float2(0.f, 0.f); };
        float2 win[kSincTaps];
#pragma unroll
        for (int t = 0; t < kSincTaps - 1; ++t) win[t + 1] = yj_at(n_step + d0 - kSincLo + t);
        float cr = 0.f, ci = 0.f;
        for (int s0 = 0; s0 < a.L; s0 += kSincAnchor) {
            float2 W = cis_cycles(cyc * ((double)s0 - centre));
            const int s1 = min(a.L, s0 + kSincAnchor);
            for (int n = s0; n < s1; ++n) {
#pragma unroll
                for (int t = 0; t < kSincTaps - 1; ++t) win[t] = win[t + 1];
                win[kSincTaps - 1] = yj_at(n_step + n + d0 - kSincLo + kSincTaps - 1);
                float yr = 0.f, yim = 0.f;
#pragma unroll
                for (int t = 0; t < kSincTaps; ++t) {
                    yr = fmaf(w[t], win[t].x, yr);
                    yim = fmaf(w[t], win[t].y, yim);
                }
                const float2 x = yi[n_step + n];
                // x * conj(yt) * W
                const float pr_ = fmaf(x.x, yr, x.y * yim);
                const float pi_ = fmaf(x.y, yr, -(x.x * yim));
                cr = fmaf(pr_, W.x, fmaf(-pi_, W.y, cr));
                ci = fmaf(pr_, W.y, fmaf(pi_, W.x, ci));
                const float wr = fmaf(W.x, E.x, -(W.y * E.y));
                W.y = fmaf(W.x, E.y, W.y * E.x);
                W.x = wr;
            }
        }
        const double pw = (double)cr * cr + (double)ci * ci;
        jacc += (a.accum_mode == GEOLOC_ACC_MAG) ? sqrt(pw) : pw;
    }
    if (!valid) return;
    if (a.n_groups == 1)
        a.J[p] = (float)jacc;
    else
        a.partial[(int64_t)group * a.P + p] = (float)jacc;
}

hipError_t launch_direct_sinc(const DirectArgs& a, hipStream_t s) {
    dim3 grid((unsigned)(a.n_tiles * (tile_lanes(a.tiling) / 256) * a.n_groups)), block(256);
    hipLaunchKernelGGL(k_direct_sinc, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace geoloc
