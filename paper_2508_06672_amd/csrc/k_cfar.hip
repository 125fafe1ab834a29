// k_cfar.hip -- threshold detection of several emitters on a RECT map (the detection step
// that ends Algorithm 1), read as cell-averaging CFAR.
//
// The noise level at a cell is the mean of J over its training window: the cells within
// Chebyshev distance t, clipped to the grid, less those within the guard distance g. Box
// sums come from a summed-area table S[r][c] = sum of J over rows <= r, cols <= c, built in
// FP64 (a block scan along every row, then a running sum down every column), so that each
// cell costs eight table reads whatever the window. A cell is a detection when J exceeds
// scale x noise; the mask kernel writes J there and -inf elsewhere (NaN stays NaN), and the
// peaks of the masked map are then taken by the top-k kernels with their exclusion window.
#include "internal.h"

#include <cmath>

namespace geoloc {

constexpr int kScanThreads = 256;

// S[r][c] = sum_{c' <= c} J[r][c'] for one row per workgroup: a block scan per chunk of
// 256 cells, carried across chunks.
__global__ __launch_bounds__(kScanThreads) void k_sat_rows(const float* __restrict__ J, int64_t cols,
                                                           double* __restrict__ S) {
    __shared__ double s_x[kScanThreads];
    __shared__ double s_carry;
    const int tid = threadIdx.x;
    const int64_t row = blockIdx.x;
    const float* Jr = J + row * cols;
    double* Sr = S + row * cols;
    if (tid == 0) s_carry = 0.0;
    for (int64_t c0 = 0; c0 < cols; c0 += kScanThreads) {
        const int64_t c = c0 + tid;
        double v = c < cols ? (double)Jr[c] : 0.0;
        __syncthreads();                            // previous chunk done with s_x, s_carry
        s_x[tid] = v;
        __syncthreads();
        // Hillis-Steele inclusive scan in LDS
        for (int o = 1; o < kScanThreads; o <<= 1) {
            const double add = tid >= o ? s_x[tid - o] : 0.0;
            __syncthreads();
            s_x[tid] += add;
            __syncthreads();
        }
        const double carry = s_carry;
        if (c < cols) Sr[c] = carry + s_x[tid];
        __syncthreads();
        if (tid == kScanThreads - 1) s_carry = carry + s_x[tid];
    }
}

// S[r][c] += S[r - 1][c] down every column: one thread per column, rows in order, eight
// rows' loads in flight at a time.
__global__ __launch_bounds__(kScanThreads) void k_sat_cols(int64_t rows, int64_t cols, double* __restrict__ S) {
    const int64_t c = (int64_t)blockIdx.x * kScanThreads + threadIdx.x;
    if (c >= cols) return;
    double acc = 0.0;
    int64_t r = 0;
    for (; r + 8 <= rows; r += 8) {
        double v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = S[(r + i) * cols + c];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            acc += v[i];
            S[(r + i) * cols + c] = acc;
        }
    }
    for (; r < rows; ++r) {
        acc += S[r * cols + c];
        S[r * cols + c] = acc;
    }
}

// Sum of J over rows [r0, r1] x cols [c0, c1] (inclusive, already clipped to the grid).
__device__ inline double box_sum(const double* __restrict__ S, int64_t cols, int64_t r0, int64_t r1, int64_t c0,
                                 int64_t c1) {
    const double a = S[r1 * cols + c1];
    const double b = r0 > 0 ? S[(r0 - 1) * cols + c1] : 0.0;
    const double d = c0 > 0 ? S[r1 * cols + c0 - 1] : 0.0;
    const double e = (r0 > 0 && c0 > 0) ? S[(r0 - 1) * cols + c0 - 1] : 0.0;
    return (a - b) - (d - e);
}

__global__ __launch_bounds__(256) void k_cfar_mask(const float* __restrict__ J, const double* __restrict__ S,
                                                   int64_t rows, int64_t cols, int32_t guard, int32_t train,
                                                   double scale, float* __restrict__ masked,
                                                   float* __restrict__ noise) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= rows * cols) return;
    const int64_t r = p / cols, c = p - r * cols;
    const int64_t r0 = r - train > 0 ? r - train : 0, r1 = r + train < rows - 1 ? r + train : rows - 1;
    const int64_t c0 = c - train > 0 ? c - train : 0, c1 = c + train < cols - 1 ? c + train : cols - 1;
    const int64_t g0 = r - guard > 0 ? r - guard : 0, g1 = r + guard < rows - 1 ? r + guard : rows - 1;
    const int64_t h0 = c - guard > 0 ? c - guard : 0, h1 = c + guard < cols - 1 ? c + guard : cols - 1;
    const int64_t n = (r1 - r0 + 1) * (c1 - c0 + 1) - (g1 - g0 + 1) * (h1 - h0 + 1);
    const double sum = box_sum(S, cols, r0, r1, c0, c1) - box_sum(S, cols, g0, g1, h0, h1);
    const double mean = n > 0 ? sum / (double)n : 0.0;
    const float v = J[p];
    const bool hit = n > 0 && (double)v > scale * mean;
    masked[p] = isnan(v) ? v : (hit ? v : -INFINITY);
    noise[p] = (float)mean;
}

__global__ void k_gather_noise(const float* __restrict__ noise, const int64_t* __restrict__ idx, int32_t k,
                               float* __restrict__ out) {
    const int t = threadIdx.x;
    if (t < k) out[t] = idx[t] >= 0 ? noise[idx[t]] : 0.f;
}

hipError_t launch_cfar(const float* J, int64_t rows, int64_t cols, int32_t guard, int32_t train, double scale,
                       double* sat, float* masked, float* noise, hipStream_t s) {
    hipLaunchKernelGGL(k_sat_rows, dim3((unsigned)rows), dim3(kScanThreads), 0, s, J, cols, sat);
    hipLaunchKernelGGL(k_sat_cols, dim3((unsigned)((cols + kScanThreads - 1) / kScanThreads)), dim3(kScanThreads), 0,
                       s, rows, cols, sat);
    const int64_t P = rows * cols;
    hipLaunchKernelGGL(k_cfar_mask, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, J, (const double*)sat, rows,
                       cols, guard, train, scale, masked, noise);
    return hipGetLastError();
}

hipError_t launch_gather_noise(const float* noise, const int64_t* idx, int32_t k, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_noise, dim3(1), dim3(kMaxTopK), 0, s, noise, idx, k, out);
    return hipGetLastError();
}

}  // namespace geoloc
