// k_argmax.hip -- peak extraction from a map (the detection step that ends Algorithm 1).
//
// Deterministic two-pass block argmax: pass 1 scans J with a grid-stride loop and
// reduces (value, flat index) per block in LDS; pass 2 reduces the block partials in
// one block. Ties go to the lowest flat index, a NaN anywhere poisons the result.
// Top-k repeats both passes, skipping every index inside a (2r+1) x (2r+1) window
// (Chebyshev distance <= r on a RECT grid; the index itself on a POINTS list) around
// the peaks already found; the found list stays on the device until the end.
#include "internal.h"

#include <cmath>

namespace geoloc {

constexpr int kArgThreads = 256;

int32_t argmax_blocks(int64_t P) {
    int64_t b = (P + 4 * kArgThreads - 1) / (4 * kArgThreads);
    if (b < 1) b = 1;
    if (b > kArgmaxMaxBlocks) b = kArgmaxMaxBlocks;
    return (int32_t)b;
}

__device__ inline bool better(float v, int64_t i, float bv, int64_t bi) { return (v > bv) || (v == bv && i < bi); }

__device__ inline bool suppressed(int64_t idx, int64_t cols, int32_t rect, int32_t radius,
                                  const int64_t* __restrict__ found, int32_t n_found) {
    for (int32_t t = 0; t < n_found; ++t) {
        const int64_t f = found[t];
        if (f < 0) continue;
        if (!rect) {
            if (f == idx) return true;
            continue;
        }
        const int64_t r = idx / cols, c = idx - r * cols;
        const int64_t fr = f / cols, fc = f - fr * cols;
        const int64_t dr = r > fr ? r - fr : fr - r, dc = c > fc ? c - fc : fc - c;
        if (dr <= radius && dc <= radius) return true;
    }
    return false;
}

// Reduce (v, i, nan) over the block through LDS; thread 0 ends with the result.
__device__ inline void block_reduce(float& v, int64_t& i, int& nan, float* sv, int64_t* si, int* sn) {
    const int tid = threadIdx.x;
    sv[tid] = v;
    si[tid] = i;
    sn[tid] = nan;
    __syncthreads();
    for (int s = kArgThreads / 2; s > 0; s >>= 1) {
        if (tid < s) {
            if (better(sv[tid + s], si[tid + s], sv[tid], si[tid])) {
                sv[tid] = sv[tid + s];
                si[tid] = si[tid + s];
            }
            sn[tid] |= sn[tid + s];
        }
        __syncthreads();
    }
    v = sv[0];
    i = si[0];
    nan = sn[0];
}

__global__ __launch_bounds__(kArgThreads) void k_argmax_blocks(const float* __restrict__ J, int64_t P, int64_t cols,
                                                               int32_t rect, int32_t radius,
                                                               const int64_t* __restrict__ found, int32_t n_found,
                                                               float* __restrict__ part_val,
                                                               int64_t* __restrict__ part_idx) {
    __shared__ float sv[kArgThreads];
    __shared__ int64_t si[kArgThreads];
    __shared__ int sn[kArgThreads];
    float bv = -INFINITY;
    int64_t bi = INT64_MAX;
    int nan = 0;
    const int64_t stride = (int64_t)gridDim.x * kArgThreads;
    for (int64_t idx = (int64_t)blockIdx.x * kArgThreads + threadIdx.x; idx < P; idx += stride) {
        const float v = J[idx];
        if (v != v) {
            nan = 1;
            continue;
        }
        if (n_found > 0 && suppressed(idx, cols, rect, radius, found, n_found)) continue;
        if (better(v, idx, bv, bi)) {
            bv = v;
            bi = idx;
        }
    }
    block_reduce(bv, bi, nan, sv, si, sn);
    if (threadIdx.x == 0) {
        part_val[blockIdx.x] = nan ? NAN : bv;
        part_idx[blockIdx.x] = bi;
    }
}

__global__ __launch_bounds__(kArgThreads) void k_argmax_final(const float* __restrict__ part_val,
                                                              const int64_t* __restrict__ part_idx, int32_t n,
                                                              int64_t* __restrict__ found_idx,
                                                              float* __restrict__ found_val, int32_t slot) {
    __shared__ float sv[kArgThreads];
    __shared__ int64_t si[kArgThreads];
    __shared__ int sn[kArgThreads];
    float bv = -INFINITY;
    int64_t bi = INT64_MAX;
    int nan = 0;
    for (int t = threadIdx.x; t < n; t += kArgThreads) {
        const float v = part_val[t];
        if (v != v) {
            nan = 1;
            continue;
        }
        if (better(v, part_idx[t], bv, bi)) {
            bv = v;
            bi = part_idx[t];
        }
    }
    block_reduce(bv, bi, nan, sv, si, sn);
    if (threadIdx.x == 0) {
        const bool none = !(bv > -INFINITY);
        found_idx[slot] = none ? -1 : bi;
        found_val[slot] = nan ? NAN : bv;
    }
}

hipError_t launch_argmax(const float* J, int64_t P, int64_t cols, int32_t rect, int32_t radius, int32_t top_k,
                         ArgmaxScratch& s, hipStream_t st) {
    for (int32_t t = 0; t < top_k; ++t) {
        hipLaunchKernelGGL(k_argmax_blocks, dim3(s.n_blocks), dim3(kArgThreads), 0, st, J, P, cols, rect, radius,
                           (const int64_t*)s.found_idx, t, s.part_val, s.part_idx);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(kArgThreads), 0, st, (const float*)s.part_val,
                           (const int64_t*)s.part_idx, s.n_blocks, s.found_idx, s.found_val, t);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace geoloc
