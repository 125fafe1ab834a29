// k_subband.hip -- split complex captures into M frequency bands, each decimated by M
// (a DFT filter bank): the input of the coarse map of the learned tile proposal.
//
//   z_b[m] = sum_{t=-h}^{h} g[t] exp(+j 2 pi (b - M/2) t / M) x[m M - t],   x = 0 outside
//
// g is the Blackman-windowed low-pass with cut-off 1/(2M) cycles per sample and unit DC
// gain (its FP64 taps come from the host). A workgroup produces 64 consecutive outputs of
// one channel for every band: it stages the input span in LDS in polyphase order
// (sample s = q M + rho at [rho][q]), so that the 64 lanes of a wave, one output each,
// read consecutive words for every tap, and each wave writes 64 consecutive outputs of
// one band (512 contiguous bytes). The band phasors exp(j 2 pi k / M) use an exactly
// reduced argument k = (b - M/2) t mod M.
#include "internal.h"

namespace geoloc {

constexpr int kSbOut = 64;                      // outputs per workgroup
// polyphase rows: M rows of at most kSbOut + 2h / M + 1 samples
constexpr int kSbX = kSubbandMaxBands * (kSbOut + 1) + 2 * kSubbandMaxHalf;

__global__ __launch_bounds__(256) void k_subband(SubbandArgs a) {
    __shared__ float2 s_x[kSbX];
    __shared__ float2 s_t[kSubbandMaxTable];

    const int M = a.n_bands, h = a.half_taps, K = 2 * h + 1;
    const int64_t n_out = a.N / M;
    const int64_t seg = blockIdx.x;                       // (channel, output segment)
    const int64_t n_seg = (n_out + kSbOut - 1) / kSbOut;
    const int c = (int)(seg / n_seg);
    const int64_t m0 = (seg - (int64_t)c * n_seg) * kSbOut;
    const float2* __restrict__ x = a.in + (int64_t)c * a.N;
    const int tid = threadIdx.x;

    // band taps T[b][u] = g[h - u] exp(j 2 pi (b - M/2)(h - u) / M), u = 0 .. 2h
    for (int i = tid; i < M * K; i += 256) {
        const int b = i / K, u = i - b * K;
        const int t = h - u;
        int k = ((b - M / 2) * t) % M;
        if (k < 0) k += M;
        float s, co;
        sincospif(2.0f * (float)k / (float)M, &s, &co);
        const float g = a.taps[t + h];
        s_t[i] = make_float2(g * co, g * s);
    }
    // input span: samples m0 M - h .. (m0 + 64) M + h - M, polyphase order
    const int R = kSbOut + (2 * h) / M + 1;               // row length
    const int span = (kSbOut - 1) * M + 2 * h + 1;
    const int64_t n0 = m0 * M - h;
    for (int s = tid; s < span; s += 256) {
        const int64_t n = n0 + s;
        const int rho = s % M, q = s / M;
        s_x[rho * R + q] = (n >= 0 && n < a.N) ? x[n] : make_float2(0.f, 0.f);
    }
    __syncthreads();

    const int ml = tid & (kSbOut - 1);                    // this lane's output
    const int64_t m = m0 + ml;
    for (int b = tid >> 6; b < M; b += 4) {               // one band per wave at a time
        const float2* T = s_t + b * K;
        float ar = 0.f, ai = 0.f;
        // tap u = qq M + rho reads sample (ml + qq) M + rho of the span
        for (int qq = 0, u0 = 0; u0 < K; ++qq, u0 += M) {
            const float2* xq = s_x + ml + qq;
            const int nr = min(M, K - u0);
            for (int rho = 0; rho < nr; ++rho) {
                const float2 v = xq[rho * R];
                const float2 w = T[u0 + rho];
                ar = fmaf(w.x, v.x, fmaf(-w.y, v.y, ar));
                ai = fmaf(w.x, v.y, fmaf(w.y, v.x, ai));
            }
        }
        if (m < n_out) a.out[((int64_t)b * a.n_ch + c) * n_out + m] = make_float2(ar, ai);
    }
}

hipError_t launch_subband(const SubbandArgs& a, hipStream_t s) {
    const int64_t n_out = a.N / a.n_bands;
    const int64_t n_seg = (n_out + kSbOut - 1) / kSbOut;
    dim3 grid((unsigned)(n_seg * a.n_ch)), block(256);
    hipLaunchKernelGGL(k_subband, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace geoloc
