// noalloc.hip -- geoloc_argmax_noalloc: the peaks of a map without a plan and without any
// device allocation, for callers that cannot allocate (code under stream capture, tight
// serving loops, hosts that forbid hipMalloc).
//
// The two-pass argmax kernels need block partials and the list of peaks found so far.
// Here they live in one file-scope device array, `scratch`, that every call on a GPU
// shares. Host code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): the device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept in g_scratch[device].
// Nothing in the array needs clearing between calls: every partial is written by pass 1
// before pass 2 reads it, and peak slot t is written before the pass for peak t + 1
// reads it. Calls that overlap on one GPU (two streams, two threads) race on the array.
#include "internal.h"

#include <cmath>
#include <mutex>

namespace geoloc {
namespace {

constexpr int kMaxDevices = 64;
// byte layout of the array: part_val float[kArgmaxMaxBlocks], part_idx int64[...],
// found_idx int64[kMaxTopK], found_val float[kMaxTopK], each at a 256-byte boundary
constexpr size_t kOffVal = 0;
constexpr size_t kOffIdx = kOffVal + ((kArgmaxMaxBlocks * sizeof(float) + 255) & ~size_t(255));
constexpr size_t kOffFoundIdx = kOffIdx + ((kArgmaxMaxBlocks * sizeof(int64_t) + 255) & ~size_t(255));
constexpr size_t kOffFoundVal = kOffFoundIdx + ((kMaxTopK * sizeof(int64_t) + 255) & ~size_t(255));
constexpr size_t kScratchBytes = kOffFoundVal + ((kMaxTopK * sizeof(float) + 255) & ~size_t(255));

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first call there.
int scratch_address(unsigned char** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return set_last_error(GEOLOC_EDEVICE, "no current HIP device");
    if (dev >= kMaxDevices) return set_last_error(GEOLOC_EDEVICE, "device index beyond the static table");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess || std::string(prop.gcnArchName).rfind("gfx950", 0) != 0)
            return set_last_error(GEOLOC_EDEVICE, "the current device is not a gfx950");
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return set_last_error(GEOLOC_EDEVICE, "hipGetSymbolAddress of the argmax scratch failed");
        g_scratch[dev] = ptr;
    }
    *out = static_cast<unsigned char*>(g_scratch[dev]);
    return GEOLOC_OK;
}

}  // namespace
}  // namespace geoloc

extern "C" int geoloc_argmax_noalloc(const float* J_dev, int32_t grid_kind, int64_t n_rows, int64_t n_cols,
                                     int32_t top_k, int32_t nms_radius_cells, int64_t* idx_host, float* val_host,
                                     void* stream) {
    using namespace geoloc;
    if (!J_dev || !idx_host || !val_host) return set_last_error(GEOLOC_EINVAL, "NULL pointer");
    if (grid_kind != GEOLOC_GRID_RECT && grid_kind != GEOLOC_GRID_POINTS)
        return set_last_error(GEOLOC_EINVAL, "unknown grid kind");
    if (n_rows < 1 || n_cols < 1 || n_rows > INT64_MAX / n_cols) return set_last_error(GEOLOC_EINVAL, "empty or oversized grid");
    if (top_k < 1 || top_k > kMaxTopK)
        return set_last_error(GEOLOC_EINVAL, "top_k must be in [1, 64]: the static scratch holds 64 peaks");
    if (nms_radius_cells < 0) return set_last_error(GEOLOC_EINVAL, "nms radius < 0");
    if (nms_radius_cells > 0 && grid_kind != GEOLOC_GRID_RECT)
        return set_last_error(GEOLOC_EINVAL, "nms radius needs a RECT grid");
    unsigned char* base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    const int64_t P = n_rows * n_cols;
    ArgmaxScratch sc;
    sc.part_val = reinterpret_cast<float*>(base + kOffVal);
    sc.part_idx = reinterpret_cast<int64_t*>(base + kOffIdx);
    sc.found_idx = reinterpret_cast<int64_t*>(base + kOffFoundIdx);
    sc.found_val = reinterpret_cast<float*>(base + kOffFoundVal);
    sc.n_blocks = argmax_blocks(P);   // at most kArgmaxMaxBlocks
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_argmax(J_dev, P, n_cols, grid_kind == GEOLOC_GRID_RECT, nms_radius_cells, top_k, sc, s);
    int64_t idx[kMaxTopK];
    float val[kMaxTopK];
    if (e == hipSuccess) e = hipMemcpyAsync(idx, sc.found_idx, top_k * sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(val, sc.found_val, top_k * sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_last_error(GEOLOC_ELAUNCH, hipGetErrorString(e));
    if (std::isnan(val[0])) return set_last_error(GEOLOC_ENAN, "NaN in map");
    for (int t = 0; t < top_k; ++t) {
        idx_host[t] = idx[t];
        val_host[t] = idx[t] < 0 ? -INFINITY : val[t];
    }
    return GEOLOC_OK;
}
