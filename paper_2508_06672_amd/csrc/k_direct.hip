// k_direct.hip -- direct position-domain correlation in FP32 (Sec. III, Eq. (11)), with
// the non-coherent sum over steps and pairs of Algorithm 1 fused in.
//
// Per candidate point p, step k and pair (i, j), with D = d0 + a and FDOA nu from the
// FP64 geometry (Eq. (3)-(9), evaluated inline per point and step):
//   C = sum_{n in step k} y_i[n] conj(yt_j[n]) exp(+j 2 pi nu t_n),  t_n from the step centre
//   yt_j[n] = y_j[n+d0] + a (y_j[n+d0+1] - y_j[n+d0])   (LINEAR; ROUND uses y_j[n+round(D)])
//   J(p) += |C|^2  (or |C|).
//
// Mapping on gfx950 (64-wide wavefronts, 160 KiB LDS per CU):
//  * one workgroup = 256 candidate points (a tile of a rectilinear grid, or one half of a 512-cell tile),
//    one point per lane; a point owns its J value for the whole launch, so the sums
//    over steps and pairs need no atomics and are deterministic;
//  * per step the tile's lag range [dlo, dhi] is found by a wave-shuffle + LDS
//    reduction; a sample tile of y_j[n0+dlo .. n0+T+dhi] (zero outside the capture) is
//    staged through LDS with coalesced loads and every lane reads its own delayed taps
//    from it (the second tap of the linear delay is the next sample's first tap, kept in
//    registers); y_i, the same for every lane, comes in through scalar loads and is used
//    as an SGPR operand, which leaves the LDS bandwidth to the taps;
//  * the Doppler rotation uses a per-lane table E_r = exp(j 2 pi nu r / f_s),
//    r < R, computed once per step from the FP64 FDOA, so a block of R samples needs
//    no per-sample phasor update: C += W_b * sum_r y_i conj(yt) E_r, and the block
//    phasor W_b advances by exp(j 2 pi nu R / f_s); W is re-anchored from an FP64 phase
//    at the start of every LDS tile, which bounds the FP32 drift to T / R products;
//  * a tile whose lag spread exceeds the LDS halo reads its taps from global memory
//    (same arithmetic) instead.
#include "internal.h"

#include <climits>

namespace geoloc {

#ifndef GEOLOC_DIRECT_R
#define GEOLOC_DIRECT_R 16
#endif
#ifndef GEOLOC_DIRECT_T
#define GEOLOC_DIRECT_T 1024
#endif
#ifndef GEOLOC_DIRECT_WAVES_PER_EU
#define GEOLOC_DIRECT_WAVES_PER_EU 4
#endif

constexpr int kR = GEOLOC_DIRECT_R;   // samples per phasor block
constexpr int kT = GEOLOC_DIRECT_T;   // samples per LDS tile (multiple of kR)
constexpr int kHalo = 2048;           // largest lag spread of a tile staged in LDS
static_assert(kT % kR == 0, "LDS tile must hold whole phasor blocks");


__device__ inline void wg_minmax(int& lo, int& hi, int (*s_mm)[4]) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o));
        hi = max(hi, __shfl_xor(hi, o));
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        s_mm[0][w] = lo;
        s_mm[1][w] = hi;
    }
    __syncthreads();
    lo = min(min(s_mm[0][0], s_mm[0][1]), min(s_mm[0][2], s_mm[0][3]));
    hi = max(max(s_mm[1][0], s_mm[1][1]), max(s_mm[1][2], s_mm[1][3]));
}

// Blocks [b0, b1) of one sample tile, kR samples each. xs points at y_i for the tile's
// first sample: every lane reads the same address, so these are scalar (SGPR) loads and
// y_i enters the FMAs as a scalar operand. tap(m) returns y_j at tile offset m relative to
// this lane's integer delay. kTail masks samples at or beyond `tl` (last, partial block).
template <bool kRound, bool kTail, typename Tap>
__device__ inline void correlate_blocks(const float2* __restrict__ xs, int b0, int b1, int tl, float alpha,
                                        const float2 (&E)[kR], float2 ER, float2& W, float& cr, float& ci,
                                        Tap tap) {
    for (int b = b0; b < b1; ++b) {
        const int m = b * kR;
        float ar = 0.f, ai = 0.f;
        float2 tp[kR + 1];
#pragma unroll
        for (int r = 0; r <= kR; ++r) tp[r] = (kRound && r == kR) ? make_float2(0.f, 0.f) : tap(m + r);
        float2 t0 = tp[0];
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            float2 xv;
            if constexpr (kTail) {
                xv = xs[min(m + r, tl - 1)];  // address kept inside the capture, value masked
                if (m + r >= tl) xv = make_float2(0.f, 0.f);
            } else {
                xv = xs[m + r];
            }
            float tr, ti;
            if constexpr (kRound) {
                tr = t0.x;
                ti = t0.y;
                t0 = tp[r + 1];
            } else {
                const float2 t1 = tp[r + 1];
                tr = fmaf(alpha, t1.x - t0.x, t0.x);
                ti = fmaf(alpha, t1.y - t0.y, t0.y);
                t0 = t1;
            }
            // v = y_i * E_r ; acc += v * conj(yt)
            const float vr = fmaf(xv.x, E[r].x, -(xv.y * E[r].y));
            const float vi = fmaf(xv.x, E[r].y, xv.y * E[r].x);
            ar = fmaf(vi, ti, fmaf(vr, tr, ar));
            ai = fmaf(-vr, ti, fmaf(vi, tr, ai));
        }
        cr = fmaf(-ai, W.y, fmaf(ar, W.x, cr));
        ci = fmaf(ai, W.x, fmaf(ar, W.y, ci));
        const float wr = fmaf(W.x, ER.x, -(W.y * ER.y));
        W.y = fmaf(W.x, ER.y, W.y * ER.x);
        W.x = wr;
    }
}

template <bool kRound, typename Tap>
__device__ inline void correlate_tile(const float2* __restrict__ xs, int tl, float alpha, const float2 (&E)[kR],
                                      float2 ER, float2 W, float& cr, float& ci, Tap tap) {
    const int nfull = tl / kR;
    correlate_blocks<kRound, false>(xs, 0, nfull, tl, alpha, E, ER, W, cr, ci, tap);
    if (nfull * kR < tl)
        correlate_blocks<kRound, true>(xs, nfull, nfull + 1, tl, alpha, E, ER, W, cr, ci, tap);
}

template <bool kRound>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GEOLOC_DIRECT_WAVES_PER_EU)))
void k_direct(DirectArgs a) {
    __shared__ float2 s_y[kT + kHalo + 2];
    __shared__ int s_mm[2][4];

    const int tid = threadIdx.x;
    // workgroup -> (point tile, group): with n_groups > 1 each group sums its share of the
    // chunk's (pair, step) items, pair-major, into its own partial row, reduced afterwards
    // in a fixed order
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
    // item groups: a masked pass adds onto the partial sums the factored kernel wrote
    double jacc = 0.0;
    if (valid && a.n_groups == 1 && a.load_J) jacc = (double)a.J[p];
    if (valid && a.n_groups > 1 && a.mask) jacc = (double)a.partial[(int64_t)group * a.P + p];
    const double centre = 0.5 * (double)(a.L - 1);

    for (int64_t it = it_lo; it < it_hi; ++it) {
        // with a mask, only this 256-cell part of the (tile, step) pairs the factored kernel
        // left over
        if (a.mask) {
            it = next_flagged(a.mask, a.n_tiles, tile, 1u << half, it, it_hi);
            if (it >= it_hi) break;
        }
        const int e = (int)(it / a.kc);
        const int kk = (int)(it - (int64_t)e * a.kc);
        const int2 pr = a.pairs[e];
        const float2* __restrict__ yi = a.cap + (int64_t)pr.x * a.N;
        const float2* __restrict__ yj = a.cap + (int64_t)pr.y * a.N;
        {
            const int64_t n_step = (int64_t)(a.k0 + kk) * a.L;
            // delay (samples) and Doppler shift (Hz) of this point, Eq. (3)-(9) in FP64
            double D = 0.0, nu = 0.0;
            if (valid)
                pair_geometry(a.xyz[3 * p], a.xyz[3 * p + 1], a.xyz[3 * p + 2], a.states, a.n_rx, a.k0 + kk, pr, a.fs,
                              a.inv_lambda, &D, &nu);
            // keep the integer lag representable whatever the geometry (NaN included);
            // such a lag lies outside any capture and reads zeros
            if (!(fabs(D) < 1.0e9)) D = 1.0e9;
            int d0;
            float alpha;
            if constexpr (kRound) {
                d0 = (int)round(D);
                alpha = 0.f;
            } else {
                const double f = floor(D);
                d0 = (int)f;
                alpha = (float)(D - f);
            }
            int dlo = valid ? d0 : INT_MAX, dhi = valid ? d0 : INT_MIN;
            wg_minmax(dlo, dhi, s_mm);
            const int64_t spread64 = (int64_t)dhi - (int64_t)dlo;
            const bool in_lds = spread64 <= kHalo;
            const int spread = in_lds ? (int)spread64 : 0;
            const int off = valid ? d0 - dlo : 0;

            const double cyc = nu * a.inv_fs;
            float2 E[kR];
#pragma unroll
            for (int r = 0; r < kR; ++r) E[r] = cis_cycles(cyc * (double)r);
            const float2 ER = cis_cycles(cyc * (double)kR);

            float cr = 0.f, ci = 0.f;
            for (int s0 = 0; s0 < a.L; s0 += kT) {
                const int tl = min(kT, a.L - s0);
                const int nblk = (tl + kR - 1) / kR;
                __syncthreads();
                if (in_lds) {
                    const int64_t m0 = n_step + s0 + dlo;
                    const int len = nblk * kR + spread + 1;
                    for (int t = tid; t < len; t += 256) {
                        const int64_t m = m0 + t;
                        s_y[t] = (m >= 0 && m < a.N) ? yj[m] : make_float2(0.f, 0.f);
                    }
                }
                __syncthreads();
                const float2 W = cis_cycles(cyc * ((double)s0 - centre));
                const float2* xs = yi + n_step + s0;
                if (in_lds) {
                    // 64-bit LDS reads (ds_read2_b64 pairs) of the complex taps
                    const double* ys = reinterpret_cast<const double*>(s_y + off);
                    correlate_tile<kRound>(xs, tl, alpha, E, ER, W, cr, ci,
                                           [&](int m) { return __builtin_bit_cast(float2, ys[m]); });
                } else {
                    const int64_t base = n_step + s0 + d0;
                    const int64_t N = a.N;
                    correlate_tile<kRound>(xs, tl, alpha, E, ER, W, cr, ci, [&](int m) {
                        const int64_t q = base + m;
                        return (q >= 0 && q < N) ? yj[q] : make_float2(0.f, 0.f);
                    });
                }
            }
            const double pw = (double)cr * cr + (double)ci * ci;
            jacc += (a.accum_mode == GEOLOC_ACC_MAG) ? sqrt(pw) : pw;
        }
    }
    if (!valid) return;
    if (a.n_groups == 1)
        a.J[p] = (float)jacc;
    else
        a.partial[(int64_t)group * a.P + p] = (float)jacc;
}

// J[p] = (J[p] if loading) + sum over item groups of the partial sums, in group order.
__global__ __launch_bounds__(256) void k_direct_reduce(const float* __restrict__ partial, int32_t n_groups, int64_t P,
                                                       int32_t load_J, float* __restrict__ J) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    double acc = load_J ? (double)J[p] : 0.0;
    for (int g = 0; g < n_groups; ++g) acc += (double)partial[(int64_t)g * P + p];
    J[p] = (float)acc;
}

int32_t direct_groups(int64_t n_tiles, int64_t n_items) {
    // enough workgroups to cover 256 CUs several times over
    int64_t g = (1024 + n_tiles - 1) / n_tiles;
    if (g > n_items) g = n_items;
    if (g > kMaxItemGroups) g = kMaxItemGroups;
    return (int32_t)(g < 1 ? 1 : g);
}

hipError_t launch_direct(const DirectArgs& a, int32_t delay_mode, hipStream_t s) {
    dim3 grid((unsigned)(a.n_tiles * (tile_lanes(a.tiling) / 256) * a.n_groups)), block(256);
    if (delay_mode == GEOLOC_DELAY_ROUND)
        hipLaunchKernelGGL(k_direct<true>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(k_direct<false>, grid, block, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_direct_reduce(const DirectArgs& a, hipStream_t s) {
    if (a.n_groups == 1) return hipSuccess;
    hipLaunchKernelGGL(k_direct_reduce, dim3((unsigned)((a.P + 255) / 256)), dim3(256), 0, s,
                       (const float*)a.partial, a.n_groups, a.P, a.load_J, a.J);
    return hipGetLastError();
}

}  // namespace geoloc
