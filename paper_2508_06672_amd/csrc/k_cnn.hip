// k_cnn.hip -- forward / backward / optimiser kernels of the tile-proposal CNN.
//
// The network (not part of the paper; an addition of this library) reads a coarse
// position-domain map and predicts which tiles of the fine grid hold the emitter:
// L layers of 3x3 convolution (zero padding 1), bias, ReLU between layers, a 1-channel
// tile-logit map at the end, softmax over all tiles, cross-entropy against a label
// distribution. Weights and biases are used in FP16 (working copy of FP32 master
// weights kept for Adam); activations and every accumulation are FP32. All tensors are
// NCHW. Every reduction is done by exactly one workgroup in a fixed order, so results
// are run-to-run deterministic.
#include "internal.h"

#include <cfloat>

namespace geoloc {

constexpr int kCnnMaxCh = 32;

__device__ inline float act(float v, bool relu) { return (relu && v < 0.f) ? 0.f : v; }

// z[b][o][p] = bias[o] + sum_{c,dy,dx} W[o][c][dy][dx] act(in[b][c][p + (dy-1, dx-1)]).
// One thread per output pixel and group of kCnnOG output channels (blockIdx.z), so a
// single image still spreads over several workgroups; the group's weights sit in LDS as
// FP32 ordered [c][dy][dx][o], so that one 16-byte read fetches four output channels.
constexpr int kCnnOG = 8;

template <bool kReluIn>
__global__ __launch_bounds__(256) void k_cnn_conv_fwd(const float* __restrict__ in, const _Float16* __restrict__ w,
                                                      const _Float16* __restrict__ bias, float* __restrict__ out,
                                                      int C, int O, int H, int W) {
    __shared__ __align__(16) float s_w[kCnnMaxCh * 9 * kCnnOG];
    const int o0 = blockIdx.z * kCnnOG;
    const int og = min(kCnnOG, O - o0);            // output channels of this group
    for (int i = threadIdx.x; i < C * 9 * kCnnOG; i += 256) {
        const int oo = i % kCnnOG, ck = i / kCnnOG; // ck = c * 9 + dy * 3 + dx
        s_w[i] = oo < og ? (float)w[(int64_t)(o0 + oo) * C * 9 + ck] : 0.f;
    }
    __syncthreads();
    const int b = blockIdx.y;
    const int pix = blockIdx.x * 256 + threadIdx.x;
    if (pix >= H * W) return;
    const int h = pix / W, x = pix - h * W;
    float acc[kCnnOG];
#pragma unroll
    for (int oo = 0; oo < kCnnOG; ++oo) acc[oo] = oo < og ? (float)bias[o0 + oo] : 0.f;
    const float* src = in + (int64_t)b * C * H * W;
    for (int c = 0; c < C; ++c) {
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const int hh = h + dy - 1;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int ww = x + dx - 1;
                float v = 0.f;
                if (hh >= 0 && hh < H && ww >= 0 && ww < W) v = act(src[((int64_t)c * H + hh) * W + ww], kReluIn);
                const float4* wp = reinterpret_cast<const float4*>(s_w + (c * 9 + dy * 3 + dx) * kCnnOG);
#pragma unroll
                for (int q = 0; q < kCnnOG / 4; ++q) {
                    const float4 w4 = wp[q];
                    acc[4 * q + 0] = fmaf(w4.x, v, acc[4 * q + 0]);
                    acc[4 * q + 1] = fmaf(w4.y, v, acc[4 * q + 1]);
                    acc[4 * q + 2] = fmaf(w4.z, v, acc[4 * q + 2]);
                    acc[4 * q + 3] = fmaf(w4.w, v, acc[4 * q + 3]);
                }
            }
        }
    }
    float* dst = out + (int64_t)b * O * H * W;
#pragma unroll
    for (int oo = 0; oo < kCnnOG; ++oo)
        if (oo < og) dst[(int64_t)(o0 + oo) * H * W + pix] = acc[oo];
}

// gin[b][c][p] = mask(zprev[b][c][p] > 0) * sum_{o,dy,dx} W[o][c][2-dy][2-dx] g[b][o][p + (dy-1, dx-1)]
// (the input gradient of a 3x3 same-padded correlation, with the previous layer's ReLU).
template <bool kMask>
__global__ __launch_bounds__(256) void k_cnn_conv_dgrad(const float* __restrict__ g, const _Float16* __restrict__ w,
                                                        const float* __restrict__ zprev, float* __restrict__ gin,
                                                        int C, int O, int H, int W) {
    __shared__ float s_w[kCnnMaxCh * kCnnMaxCh * 9];
    for (int i = threadIdx.x; i < O * C * 9; i += 256) s_w[i] = (float)w[i];
    __syncthreads();
    const int b = blockIdx.y;
    const int pix = blockIdx.x * 256 + threadIdx.x;
    if (pix >= H * W) return;
    const int h = pix / W, x = pix - h * W;
    float acc[kCnnMaxCh];
#pragma unroll
    for (int c = 0; c < kCnnMaxCh; ++c) acc[c] = 0.f;
    const float* src = g + (int64_t)b * O * H * W;
    for (int o = 0; o < O; ++o) {
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const int hh = h + dy - 1;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int ww = x + dx - 1;
                if (hh < 0 || hh >= H || ww < 0 || ww >= W) continue;
                const float gv = src[((int64_t)o * H + hh) * W + ww];
                const float* wp = s_w + o * C * 9 + (2 - dy) * 3 + (2 - dx);
#pragma unroll
                for (int c = 0; c < kCnnMaxCh; ++c)
                    if (c < C) acc[c] = fmaf(wp[c * 9], gv, acc[c]);
            }
        }
    }
    float* dst = gin + (int64_t)b * C * H * W;
    const float* zp = zprev + (int64_t)b * C * H * W;
#pragma unroll
    for (int c = 0; c < kCnnMaxCh; ++c)
        if (c < C) {
            float v = acc[c];
            if (kMask && !(zp[(int64_t)c * H * W + pix] > 0.f)) v = 0.f;
            dst[(int64_t)c * H * W + pix] = v;
        }
}

// dW[o][c][t] = sum_{b,p} g[b][o][p] act(in[b][c][p + tap t]),  db[o] = sum_{b,p} g[b][o][p].
// One workgroup per (o, c); threads stride over pixels and samples, then an LDS tree.
template <bool kReluIn>
__global__ __launch_bounds__(256) void k_cnn_conv_wgrad(const float* __restrict__ g, const float* __restrict__ in,
                                                        float* __restrict__ dw, float* __restrict__ db, int B, int C,
                                                        int O, int H, int W) {
    __shared__ float s[10][256];
    const int o = blockIdx.x / C, c = blockIdx.x % C;
    float acc[10];
#pragma unroll
    for (int t = 0; t < 10; ++t) acc[t] = 0.f;
    for (int b = 0; b < B; ++b) {
        const float* gp = g + ((int64_t)b * O + o) * H * W;
        const float* ip = in + ((int64_t)b * C + c) * H * W;
        for (int pix = threadIdx.x; pix < H * W; pix += 256) {
            const int h = pix / W, x = pix - h * W;
            const float gv = gp[pix];
            acc[9] += gv;
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const int hh = h + dy - 1, ww = x + dx - 1;
                    const float v = (hh >= 0 && hh < H && ww >= 0 && ww < W) ? act(ip[hh * W + ww], kReluIn) : 0.f;
                    acc[dy * 3 + dx] = fmaf(gv, v, acc[dy * 3 + dx]);
                }
        }
    }
#pragma unroll
    for (int t = 0; t < 10; ++t) s[t][threadIdx.x] = acc[t];
    __syncthreads();
    for (int hs = 128; hs > 0; hs >>= 1) {
        if (threadIdx.x < hs)
#pragma unroll
            for (int t = 0; t < 10; ++t) s[t][threadIdx.x] += s[t][threadIdx.x + hs];
        __syncthreads();
    }
    if (threadIdx.x < 9) dw[((int64_t)o * C + c) * 9 + threadIdx.x] = s[threadIdx.x][0];
    if (threadIdx.x == 9 && c == 0) db[o] = s[9][0];
}

// Per sample: p = softmax(z), loss = -sum q log p, dz = (p - q) / B.
__global__ __launch_bounds__(256) void k_cnn_softmax_ce(const float* __restrict__ z, const float* __restrict__ q, int T,
                                                        int B, float* __restrict__ dz, float* __restrict__ loss) {
    __shared__ float s[256];
    __shared__ double sd[256];
    const int b = blockIdx.x;
    const float* zb = z + (int64_t)b * T;
    const float* qb = q + (int64_t)b * T;
    float m = -FLT_MAX;
    for (int t = threadIdx.x; t < T; t += 256) m = fmaxf(m, zb[t]);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] = fmaxf(s[threadIdx.x], s[threadIdx.x + h]);
        __syncthreads();
    }
    m = s[0];
    __syncthreads();
    double se = 0.0;
    for (int t = threadIdx.x; t < T; t += 256) se += exp((double)(zb[t] - m));
    sd[threadIdx.x] = se;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) sd[threadIdx.x] += sd[threadIdx.x + h];
        __syncthreads();
    }
    const double lse = (double)m + log(sd[0]);
    __syncthreads();
    double l = 0.0;
    for (int t = threadIdx.x; t < T; t += 256) {
        const double lp = (double)zb[t] - lse;
        l -= (double)qb[t] * lp;
        dz[(int64_t)b * T + t] = (float)((exp(lp) - (double)qb[t]) / B);
    }
    sd[threadIdx.x] = l;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) sd[threadIdx.x] += sd[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[b] = (float)sd[0];
}

__global__ __launch_bounds__(256) void k_cnn_adam(float* __restrict__ master, float* __restrict__ m,
                                                  float* __restrict__ v, const float* __restrict__ g,
                                                  _Float16* __restrict__ w16, int64_t n, float lr, float b1, float b2,
                                                  float eps, float bc1, float bc2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = master[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    master[i] = wi;
    w16[i] = (_Float16)wi;
}

__global__ __launch_bounds__(256) void k_cnn_to_half(const float* __restrict__ src, _Float16* __restrict__ dst,
                                                     int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = (_Float16)src[i];
}

// Per sample: the k largest logits (ties to the lower tile index) and their softmax
// probabilities.
__global__ __launch_bounds__(256) void k_cnn_topk(const float* __restrict__ z, int T, int k, int32_t* __restrict__ tiles,
                                                  float* __restrict__ probs) {
    __shared__ float sv[256];
    __shared__ int si[256];
    __shared__ double sd[256];
    __shared__ int chosen[64];
    const int b = blockIdx.x;
    const float* zb = z + (int64_t)b * T;
    float m = -FLT_MAX;
    for (int t = threadIdx.x; t < T; t += 256) m = fmaxf(m, zb[t]);
    sv[threadIdx.x] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) sv[threadIdx.x] = fmaxf(sv[threadIdx.x], sv[threadIdx.x + h]);
        __syncthreads();
    }
    m = sv[0];
    __syncthreads();
    double se = 0.0;
    for (int t = threadIdx.x; t < T; t += 256) se += exp((double)(zb[t] - m));
    sd[threadIdx.x] = se;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) sd[threadIdx.x] += sd[threadIdx.x + h];
        __syncthreads();
    }
    const double tot = sd[0];
    for (int r = 0; r < k; ++r) {
        float bv = -FLT_MAX;
        int bi = T;
        for (int t = threadIdx.x; t < T; t += 256) {
            bool taken = false;
            for (int q = 0; q < r; ++q) taken |= (chosen[q] == t);
            const float v = zb[t];
            if (!taken && (v > bv || (v == bv && t < bi))) {
                bv = v;
                bi = t;
            }
        }
        __syncthreads();
        sv[threadIdx.x] = bv;
        si[threadIdx.x] = bi;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) {
                const float ov = sv[threadIdx.x + h];
                const int oi = si[threadIdx.x + h];
                if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                    sv[threadIdx.x] = ov;
                    si[threadIdx.x] = oi;
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const int t = si[0] < T ? si[0] : -1;
            chosen[r] = t;
            tiles[(int64_t)b * k + r] = t;
            probs[(int64_t)b * k + r] = t >= 0 ? (float)(exp((double)(zb[t] - m)) / tot) : 0.f;
        }
        __syncthreads();
    }
}

// Input features of one coarse map: [log(J / mean J) clipped to +-8, D / 64, (nu - mean nu) / 256 Hz].
__global__ __launch_bounds__(256) void k_cnn_prep(const float* __restrict__ J, const double* __restrict__ D,
                                                  const double* __restrict__ nu, int T, float* __restrict__ x) {
    __shared__ double s[2][256];
    const int b = blockIdx.x;
    const float* Jb = J + (int64_t)b * T;
    const double* Db = D + (int64_t)b * T;
    const double* nb = nu + (int64_t)b * T;
    double sj = 0.0, sn = 0.0;
    for (int t = threadIdx.x; t < T; t += 256) {
        sj += (double)Jb[t];
        sn += nb[t];
    }
    s[0][threadIdx.x] = sj;
    s[1][threadIdx.x] = sn;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            s[0][threadIdx.x] += s[0][threadIdx.x + h];
            s[1][threadIdx.x] += s[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    const double mj = s[0][0] / T, mn = s[1][0] / T;
    float* xb = x + (int64_t)b * 3 * T;
    for (int t = threadIdx.x; t < T; t += 256) {
        double lj = (mj > 0.0 && Jb[t] > 0.f) ? log((double)Jb[t] / mj) : -8.0;
        lj = lj < -8.0 ? -8.0 : (lj > 8.0 ? 8.0 : lj);
        xb[t] = (float)lj;
        xb[T + t] = (float)(Db[t] / 64.0);
        xb[2 * T + t] = (float)((nb[t] - mn) / 256.0);
    }
}

// --------------------------------------------------------------------------- launchers

hipError_t launch_cnn_conv_fwd(bool relu_in, const float* in, const _Float16* w, const _Float16* b, float* out, int B,
                               int C, int O, int H, int W, hipStream_t s) {
    dim3 grid((unsigned)((H * W + 255) / 256), (unsigned)B, (unsigned)((O + kCnnOG - 1) / kCnnOG));
    if (relu_in)
        hipLaunchKernelGGL(k_cnn_conv_fwd<true>, grid, dim3(256), 0, s, in, w, b, out, C, O, H, W);
    else
        hipLaunchKernelGGL(k_cnn_conv_fwd<false>, grid, dim3(256), 0, s, in, w, b, out, C, O, H, W);
    return hipGetLastError();
}

hipError_t launch_cnn_conv_dgrad(bool mask, const float* g, const _Float16* w, const float* zprev, float* gin, int B,
                                 int C, int O, int H, int W, hipStream_t s) {
    dim3 grid((unsigned)((H * W + 255) / 256), (unsigned)B);
    if (mask)
        hipLaunchKernelGGL(k_cnn_conv_dgrad<true>, grid, dim3(256), 0, s, g, w, zprev, gin, C, O, H, W);
    else
        hipLaunchKernelGGL(k_cnn_conv_dgrad<false>, grid, dim3(256), 0, s, g, w, zprev, gin, C, O, H, W);
    return hipGetLastError();
}

hipError_t launch_cnn_conv_wgrad(bool relu_in, const float* g, const float* in, float* dw, float* db, int B, int C,
                                 int O, int H, int W, hipStream_t s) {
    dim3 grid((unsigned)(O * C));
    if (relu_in)
        hipLaunchKernelGGL(k_cnn_conv_wgrad<true>, grid, dim3(256), 0, s, g, in, dw, db, B, C, O, H, W);
    else
        hipLaunchKernelGGL(k_cnn_conv_wgrad<false>, grid, dim3(256), 0, s, g, in, dw, db, B, C, O, H, W);
    return hipGetLastError();
}

hipError_t launch_cnn_softmax_ce(const float* z, const float* q, int T, int B, float* dz, float* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_cnn_softmax_ce, dim3(B), dim3(256), 0, s, z, q, T, B, dz, loss);
    return hipGetLastError();
}

hipError_t launch_cnn_adam(float* master, float* m, float* v, const float* g, _Float16* w16, int64_t n, float lr,
                           float b1, float b2, float eps, float bc1, float bc2, hipStream_t s) {
    hipLaunchKernelGGL(k_cnn_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, master, m, v, g, w16, n, lr, b1,
                       b2, eps, bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_cnn_to_half(const float* src, _Float16* dst, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_cnn_to_half, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_cnn_topk(const float* z, int T, int B, int k, int32_t* tiles, float* probs, hipStream_t s) {
    hipLaunchKernelGGL(k_cnn_topk, dim3(B), dim3(256), 0, s, z, T, k, tiles, probs);
    return hipGetLastError();
}

hipError_t launch_cnn_prep(const float* J, const double* D, const double* nu, int T, int B, float* x, hipStream_t s) {
    hipLaunchKernelGGL(k_cnn_prep, dim3(B), dim3(256), 0, s, J, D, nu, T, x);
    return hipGetLastError();
}

}  // namespace geoloc
