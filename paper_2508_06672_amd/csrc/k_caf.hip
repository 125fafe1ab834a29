// k_caf.hip -- the CAF-table form of the position-domain correlation on MFMA.
//
// Eq. (11) for every integer lag d of a window and every Doppler bin nu_m of a uniform
// grid is a cross-ambiguity (CAF) table per step (the CAF of the two-step method,
// Sec. I, evaluated once per step instead of once per candidate):
//
//   T_k[d, m] = sum_{n in step k} y_i[n] conj(y_j[n + d]) exp(+j 2 pi nu_m t_n)
//             = (L_k F)[d, m],  L_k[d, n] = y_i[n] conj(y_j[n + d]),  F[n, m] = exp(j 2 pi nu_m t_n)
//
// with t_n measured from the step centre. Each candidate point then reads its table by
// bilinear interpolation of the complex values at (D, nu) and adds |C|^2 to J
// (Algorithm 1's sum over steps and pairs). With the two-tap linear delay the lag
// interpolation is exact; the Doppler interpolation is the approximation of this form.
//
// Kernels
//   k_caf_extent  FP64 geometry of every (point, step, pair), a thread per point; block min / max
//                 of D and nu
//                 (sizes and validates the table window on the host)
//   k_caf_power   sum of |y|^2 per receiver (power-of-two input scale for FP16 range)
//   k_caf_phasor  F in BF16 or FP16, bin-interleaved: [n / 8][m][8] per plane (re, im), so
//                 one 16-byte load per lane is one MFMA B fragment
//   k_caf_gemm    MFMA complex GEMM, lag products formed in the prologue from LDS-staged
//                 samples (never written to HBM), FP32 accumulation, optional split-K
//   k_caf_reduce  sums split-K partials and undoes the input scale
//   k_caf_interp  FP64 geometry inline, complex interpolation (linear in Doppler; linear,
//                 nearest or eight windowed-sinc taps in lag), J += |C|^2
//
// MFMA: v_mfma_f32_32x32x16_{bf16,f16}. Lane l holds A[l % 32][8 (l / 32) + j] and
// B[8 (l / 32) + j][l % 32], j < 8; accumulator i of lane l is C[8 (i / 4) + 4 (l / 32) +
// (i % 4)][l % 32]. Complex product as four real MFMAs:
//   Tr += Ar Fr + (-Ai) Fi,   Ti += Ar Fi + Ai Fr.
// A wave owns 64 lags x 64 bins (2 x 2 blocks of 32 x 32, 128 FP32 accumulators), so that
// every F fragment it loads feeds two row blocks and every lag-product fragment two column
// blocks; a workgroup of 4 waves owns 128 lags x 128 bins. Two waves per SIMD (the
// accumulators then live in VGPRs) let one wave form lag products while another's MFMAs run.
#include "internal.h"

#include <cfloat>

namespace geoloc {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(unsigned int)))) unsigned int u32x4;

#ifndef GEOLOC_CAF_KC
#define GEOLOC_CAF_KC 256
#endif
constexpr int kCafKc = GEOLOC_CAF_KC;  // samples staged in LDS per chunk (multiple of 16)
#ifndef GEOLOC_CAF_WAVES_PER_EU
#define GEOLOC_CAF_WAVES_PER_EU 2
#endif

// --------------------------------------------------------------------------- extent

__global__ __launch_bounds__(256) void k_caf_extent(CafGeomArgs a, double* __restrict__ part) {
    __shared__ double s[4][256];
    double dmin = DBL_MAX, dmax = -DBL_MAX, nmin = DBL_MAX, nmax = -DBL_MAX;
    // a thread per point (grid-stride over the points), every pair and step of it in turn:
    // the point's ECEF is loaded once and the states are the same for the whole block
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < a.P; p += (int64_t)gridDim.x * 256) {
        const double q0 = a.xyz[3 * p], q1 = a.xyz[3 * p + 1], q2 = a.xyz[3 * p + 2];
        for (int32_t e = 0; e < a.n_pairs; ++e) {
            const int2 pr = a.pairs[e];
            for (int32_t k = 0; k < a.K; ++k) {
                double D, nu;
                pair_geometry(q0, q1, q2, a.states, a.n_rx, k, pr, a.fs, a.inv_lambda, &D, &nu);
                dmin = fmin(dmin, D);
                dmax = fmax(dmax, D);
                nmin = fmin(nmin, nu);
                nmax = fmax(nmax, nu);
            }
        }
    }
    const int t = threadIdx.x;
    s[0][t] = dmin;
    s[1][t] = -dmax;
    s[2][t] = nmin;
    s[3][t] = -nmax;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
            for (int q = 0; q < 4; ++q) s[q][t] = fmin(s[q][t], s[q][t + h]);
        __syncthreads();
    }
    if (t < 4) part[blockIdx.x * 4 + t] = s[t][0];
}

// --------------------------------------------------------------------------- capture power

__global__ __launch_bounds__(256) void k_caf_power(const float2* __restrict__ cap, int64_t N, int32_t n_rx,
                                                   double* __restrict__ part) {
    __shared__ double s[256];
    const int rx = blockIdx.y;
    const float2* y = cap + (int64_t)rx * N;
    double acc = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < N; n += (int64_t)gridDim.x * 256) {
        const float2 v = y[n];
        acc += (double)v.x * v.x + (double)v.y * v.y;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[rx * gridDim.x + blockIdx.x] = s[0];
}

// --------------------------------------------------------------------------- phasor table

template <bool kF16>
__global__ __launch_bounds__(256) void k_caf_phasor(int32_t L_pad, int32_t L, int32_t M, int32_t M_pad,
                                                    double nu_lo, double dnu, double inv_fs,
                                                    unsigned short* __restrict__ Fr, unsigned short* __restrict__ Fi) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;  // over [L_pad][M_pad]
    if (idx >= (int64_t)L_pad * M_pad) return;
    const int32_t n = (int32_t)(idx / M_pad);
    const int32_t m = (int32_t)(idx % M_pad);
    float re = 0.f, im = 0.f;
    if (n < L && m < M) {
        const double t = ((double)n - 0.5 * (double)(L - 1)) * inv_fs;
        const double cyc = (nu_lo + dnu * (double)m) * t;
        const double f = cyc - rint(cyc);
        double s, c;
        sincospi(2.0 * f, &s, &c);
        re = (float)c;
        im = (float)s;
    }
    const int64_t o = ((int64_t)(n >> 3) * M_pad + m) * 8 + (n & 7);
    if constexpr (kF16) {
        Fr[o] = __builtin_bit_cast(unsigned short, (_Float16)re);
        Fi[o] = __builtin_bit_cast(unsigned short, (_Float16)im);
    } else {
        Fr[o] = __builtin_bit_cast(unsigned short, (__bf16)re);
        Fi[o] = __builtin_bit_cast(unsigned short, (__bf16)im);
    }
}

// --------------------------------------------------------------------------- GEMM

template <bool kF16>
struct MfmaTypes;
template <>
struct MfmaTypes<false> {
    typedef bf16x8 vec;
    static __device__ inline f32x16 mfma(vec a, vec b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
    static __device__ inline unsigned short cvt(float x) { return __builtin_bit_cast(unsigned short, (__bf16)x); }
    // two values rounded to nearest even and packed, low half first (one conversion instruction)
    static __device__ inline unsigned int cvt2(float lo, float hi) {
        typedef float f2 __attribute__((ext_vector_type(2)));
        typedef __bf16 b2 __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(unsigned int, __builtin_convertvector((f2){lo, hi}, b2));
    }
};
template <>
struct MfmaTypes<true> {
    typedef f16x8 vec;
    static __device__ inline f32x16 mfma(vec a, vec b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
    static __device__ inline unsigned short cvt(float x) { return __builtin_bit_cast(unsigned short, (_Float16)x); }
    static __device__ inline unsigned int cvt2(float lo, float hi) {
        typedef float f2 __attribute__((ext_vector_type(2)));
        typedef _Float16 h2 __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(unsigned int, __builtin_convertvector((f2){lo, hi}, h2));
    }
};

template <bool kF16>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GEOLOC_CAF_WAVES_PER_EU))) void k_caf_gemm(CafGemmArgs a) {
    using MT = MfmaTypes<kF16>;
    using vec = typename MT::vec;
    __shared__ float2 s_yi[kCafKc];
    __shared__ float2 s_yj[kCafKc + kCafTileLags + 16];

    // workgroup: 128 lags x 128 bins; wave (wrow, wcol): 64 lags x 64 bins, four 32 x 32
    // blocks, so that each B fragment of F feeds two row blocks and each A fragment two
    // column blocks
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wrow = wave >> 1, wcol = wave & 1;
    const int lag_base = blockIdx.x * kCafTileLags;    // table row of this workgroup
    const int bin_base = blockIdx.y * kCafTileBins + wcol * 64;
    const int z = blockIdx.z;                          // (split, pair, step)
    const int split = z % a.n_split;
    const int ek = z / a.n_split;                      // pair * kc + step-in-chunk
    const int e = ek / a.kc, kk = ek % a.kc;
    const int2 pr = a.pairs[e];
    const float2* __restrict__ yi = a.cap + (int64_t)pr.x * a.N;
    const float2* __restrict__ yj = a.cap + (int64_t)pr.y * a.N;
    const int64_t n_step = (int64_t)(a.k0 + kk) * a.L;
    const int c0 = split * a.chunk;                    // sample range of this split within the step
    const int c1 = min(a.L, c0 + a.chunk);
    const int64_t lag0 = (int64_t)a.lag_lo + lag_base; // lag of table row lag_base

    f32x16 tr[2][2], ti[2][2];                         // [row block][column block]
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int i = 0; i < 16; ++i) tr[rb][cb][i] = ti[rb][cb][i] = 0.f;

    const int kg = lane >> 5;                          // which 8 samples of the 16-sample K step

    for (int s0 = c0; s0 < c1; s0 += kCafKc) {
        const int len = min(kCafKc, c1 - s0);
        __syncthreads();
        for (int t = tid; t < kCafKc; t += 256) {
            float2 v = make_float2(0.f, 0.f);
            if (t < len) {
                v = yi[n_step + s0 + t];
                v.x *= a.scale;
                v.y *= a.scale;
            }
            s_yi[t] = v;
        }
        for (int t = tid; t < kCafKc + kCafTileLags + 16; t += 256) {
            const int64_t m = n_step + s0 + lag0 + t;
            s_yj[t] = (m >= 0 && m < a.N) ? yj[m] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        const int nks = (len + 15) >> 4;
        for (int ks = 0; ks < nks; ++ks) {
            // B fragments: F at this lane's 8 samples for bins bin_base + 32 cb + lane % 32
            const int64_t g = (int64_t)((s0 + ks * 16) >> 3) + kg;
            vec fr[2], fi[2];
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const int64_t o = (g * a.M_pad + bin_base + cb * 32 + (lane & 31)) * 8;
                fr[cb] = __builtin_bit_cast(vec, *reinterpret_cast<const u32x4*>(a.Fr + o));
                fi[cb] = __builtin_bit_cast(vec, *reinterpret_cast<const u32x4*>(a.Fi + o));
            }
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                // A fragments: lag products of this lane's row at 8 consecutive samples
                const int row = wrow * 64 + rb * 32 + (lane & 31);
                u32x4 par, pai;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float lr[2], li[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int t = ks * 16 + kg * 8 + 2 * q + h;
                        const float2 x = s_yi[t];
                        const float2 y = s_yj[t + row];
                        lr[h] = fmaf(x.x, y.x, x.y * y.y);  // x * conj(y)
                        li[h] = fmaf(x.y, y.x, -(x.x * y.y));
                    }
                    par[q] = MT::cvt2(lr[0], lr[1]);
                    pai[q] = MT::cvt2(li[0], li[1]);
                }
                const u32x4 pnai = pai ^ 0x80008000u;   // -Ai: flip both sign bits of each word
                const vec va = __builtin_bit_cast(vec, par);
                const vec vai = __builtin_bit_cast(vec, pai);
                const vec vnai = __builtin_bit_cast(vec, pnai);
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    tr[rb][cb] = MT::mfma(va, fr[cb], tr[rb][cb]);
                    tr[rb][cb] = MT::mfma(vnai, fi[cb], tr[rb][cb]);
                    ti[rb][cb] = MT::mfma(va, fi[cb], ti[rb][cb]);
                    ti[rb][cb] = MT::mfma(vai, fr[cb], ti[rb][cb]);
                }
            }
        }
    }

    // epilogue: rows 8 (i/4) + 4 (lane/32) + i%4 of each 32-row block, column lane % 32
    float2* out = a.out + ((int64_t)split * a.n_pairs * a.kc + ek) * (int64_t)a.n_lags_pad * a.M_pad;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int r = lag_base + wrow * 64 + rb * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
                const int c = bin_base + cb * 32 + (lane & 31);
                out[(int64_t)r * a.M_pad + c] = make_float2(tr[rb][cb][i] * a.unscale, ti[rb][cb][i] * a.unscale);
            }
}

__global__ __launch_bounds__(256) void k_caf_reduce(const float2* __restrict__ part, int64_t n, int32_t n_split,
                                                    float unscale, float2* __restrict__ T) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= n) return;
    float sr = 0.f, si = 0.f;
    for (int s = 0; s < n_split; ++s) {
        const float2 v = part[(int64_t)s * n + idx];
        sr += v.x;
        si += v.y;
    }
    T[idx] = make_float2(sr * unscale, si * unscale);
}

// --------------------------------------------------------------------------- interpolation

template <int kMode>   // GEOLOC_DELAY_LINEAR, _ROUND or _SINC
__global__ __launch_bounds__(256) void k_caf_interp(CafInterpArgs a) {
    const int tid = threadIdx.x;
    bool valid;
    const int64_t p = tile_point(a.tiling, blockIdx.x, tid, &valid);
    if (!valid) return;
    double jacc = a.load_J ? (double)a.J[p] : 0.0;
    for (int e = 0; e < a.g.n_pairs; ++e) {
        for (int kk = 0; kk < a.kc; ++kk) {
            double D, nu;
            pair_delay_doppler(a.g, p, a.k0 + kk, e, &D, &nu);
            if (!(fabs(D) < 1.0e9)) D = 1.0e9;
            int64_t d0;
            double al;
            if constexpr (kMode == GEOLOC_DELAY_ROUND) {
                d0 = (int64_t)round(D);
                al = 0.0;
            } else {
                const double f = floor(D);
                d0 = (int64_t)f;
                al = D - f;
            }
            const double u = (nu - a.nu_lo) / a.dnu;
            const double mf = floor(u);
            int64_t m0 = (int64_t)mf;
            double be = u - mf;
            if (m0 == a.M - 1 && be == 0.0) {
                m0 = a.M - 2;
                be = 1.0;
            }
            m0 = min(max(m0, (int64_t)0), (int64_t)a.M - 2);
            const float2* T = a.T + ((int64_t)e * a.kc + kk) * (int64_t)a.n_lags_pad * a.M_pad;
            const float fb = (float)be;
            float cr, ci;
            if constexpr (kMode == GEOLOC_DELAY_SINC) {
                // eight lag taps floor(D) - 3 .. floor(D) + 4, each linear in Doppler
                float w[kSincTaps];
                sinc_taps((float)al, w);
                int64_t r0 = d0 - kSincLo - a.lag_lo;
                // the host checked coverage; clamping only keeps every read inside the table
                r0 = min(max(r0, (int64_t)0), (int64_t)a.n_lags - kSincTaps);
                cr = 0.f;
                ci = 0.f;
#pragma unroll
                for (int t = 0; t < kSincTaps; ++t) {
                    const float2 v0 = T[(r0 + t) * a.M_pad + m0], v1 = T[(r0 + t) * a.M_pad + m0 + 1];
                    cr = fmaf(w[t], fmaf(fb, v1.x - v0.x, v0.x), cr);
                    ci = fmaf(w[t], fmaf(fb, v1.y - v0.y, v0.y), ci);
                }
            } else {
                int64_t r0 = d0 - a.lag_lo;
                if (r0 == a.n_lags - 1 && al == 0.0) {
                    r0 = a.n_lags - 2;
                    al = 1.0;
                }
                // the host checked coverage; clamping only keeps every read inside the table
                r0 = min(max(r0, (int64_t)0), (int64_t)a.n_lags - 2);
                const float2 t00 = T[r0 * a.M_pad + m0], t01 = T[r0 * a.M_pad + m0 + 1];
                const float2 t10 = T[(r0 + 1) * a.M_pad + m0], t11 = T[(r0 + 1) * a.M_pad + m0 + 1];
                const float fa = (float)al;
                const float w00 = (1.f - fa) * (1.f - fb), w10 = fa * (1.f - fb), w01 = (1.f - fa) * fb,
                            w11 = fa * fb;
                cr = w00 * t00.x + w10 * t10.x + w01 * t01.x + w11 * t11.x;
                ci = w00 * t00.y + w10 * t10.y + w01 * t01.y + w11 * t11.y;
            }
            const double pw = (double)cr * cr + (double)ci * ci;
            jacc += (a.accum_mode == GEOLOC_ACC_MAG) ? sqrt(pw) : pw;
        }
    }
    a.J[p] = (float)jacc;
}

// --------------------------------------------------------------------------- launchers

int32_t caf_extent_blocks(int64_t points) {
    int64_t b = (points + 255) / 256;
    return (int32_t)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

hipError_t launch_caf_extent(const CafGeomArgs& a, double* part, int32_t blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_caf_extent, dim3(blocks), dim3(256), 0, s, a, part);
    return hipGetLastError();
}

hipError_t launch_caf_power(const float2* cap, int64_t N, int32_t n_rx, double* part, int32_t blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_caf_power, dim3(blocks, n_rx), dim3(256), 0, s, cap, N, n_rx, part);
    return hipGetLastError();
}

hipError_t launch_caf_phasor(bool f16, int32_t L_pad, int32_t L, int32_t M, int32_t M_pad, double nu_lo, double dnu,
                             double inv_fs, unsigned short* Fr, unsigned short* Fi, hipStream_t s) {
    const int64_t total = (int64_t)L_pad * M_pad;
    dim3 grid((unsigned)((total + 255) / 256));
    if (f16)
        hipLaunchKernelGGL(k_caf_phasor<true>, grid, dim3(256), 0, s, L_pad, L, M, M_pad, nu_lo, dnu, inv_fs, Fr, Fi);
    else
        hipLaunchKernelGGL(k_caf_phasor<false>, grid, dim3(256), 0, s, L_pad, L, M, M_pad, nu_lo, dnu, inv_fs, Fr, Fi);
    return hipGetLastError();
}

hipError_t launch_caf_gemm(bool f16, const CafGemmArgs& a, hipStream_t s) {
    dim3 grid((unsigned)(a.n_lags_pad / kCafTileLags), (unsigned)(a.M_pad / kCafTileBins),
              (unsigned)(a.n_split * a.n_pairs * a.kc));
    if (f16)
        hipLaunchKernelGGL(k_caf_gemm<true>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_caf_gemm<false>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_caf_reduce(const float2* part, int64_t n, int32_t n_split, float unscale, float2* T, hipStream_t s) {
    hipLaunchKernelGGL(k_caf_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, n, n_split, unscale, T);
    return hipGetLastError();
}

hipError_t launch_caf_interp(const CafInterpArgs& a, int32_t delay_mode, hipStream_t s) {
    dim3 grid((unsigned)(a.tiling.tiles_x * a.tiling.tiles_y));
    if (delay_mode == GEOLOC_DELAY_ROUND)
        hipLaunchKernelGGL(k_caf_interp<GEOLOC_DELAY_ROUND>, grid, dim3(256), 0, s, a);
    else if (delay_mode == GEOLOC_DELAY_SINC)
        hipLaunchKernelGGL(k_caf_interp<GEOLOC_DELAY_SINC>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_caf_interp<GEOLOC_DELAY_LINEAR>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace geoloc
