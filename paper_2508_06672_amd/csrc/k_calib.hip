// k_calib.hip -- measurement helper: the rate at which the chip issues unpacked FP32 FMAs,
// the ceiling of the FP32 VALU kernels of this library (they are compiled without the
// packed FP32 forms). Every thread runs `iters` rounds of 16 independent FMA chains, so
// that each wave has independent work for every issue slot; the results are stored so
// that none of the work is removed.
#include "internal.h"

namespace geoloc {

constexpr int kCalibChains = 16;

__global__ __launch_bounds__(256) void k_fma_ceiling(float* __restrict__ out, int32_t iters, float a, float b) {
    float x[kCalibChains];
#pragma unroll
    for (int i = 0; i < kCalibChains; ++i) x[i] = (float)threadIdx.x * 1e-3f + (float)i;
    for (int32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kCalibChains; ++i) x[i] = fmaf(x[i], a, b);
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < kCalibChains; ++i) s += x[i];
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

hipError_t launch_fma_ceiling(int32_t n_blocks, int32_t iters, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_fma_ceiling, dim3((unsigned)n_blocks), dim3(256), 0, s, out, iters, 0.999f, 1e-4f);
    return hipGetLastError();
}

int32_t fma_ceiling_chains() { return kCalibChains; }

}  // namespace geoloc
