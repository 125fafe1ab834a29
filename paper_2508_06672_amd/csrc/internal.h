// internal.h -- shared declarations of the gfx950 library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/geoloc.h"

namespace geoloc {

constexpr double kLightSpeed = 299792458.0;

// Points handled by one workgroup of the correlation kernels: a 16 x 16 tile of a
// RECT grid (neighbouring cells have neighbouring delays, so the lag spread a tile
// needs in LDS stays small), or 256 consecutive entries of a POINTS list.
constexpr int kTilePoints = 256;

struct PointTiling {
    int64_t rows, cols;     // RECT: grid shape; POINTS: 1 x P
    int32_t tile_w, tile_h; // 16 x 16 (RECT) or 256 x 1 (POINTS)
    int64_t tiles_x, tiles_y;
};

__host__ __device__ inline int64_t tile_point(const PointTiling& t, int64_t tile, int lane, bool* valid) {
    int64_t ty = tile / t.tiles_x, tx = tile - ty * t.tiles_x;
    int64_t r = ty * t.tile_h + lane / t.tile_w;
    int64_t c = tx * t.tile_w + lane % t.tile_w;
    *valid = (r < t.rows) && (c < t.cols);
    return r * t.cols + c;
}

struct DirectArgs {
    const float2* cap;       // [n_rx][N] complex64
    const double* D;         // delay in samples, tile-major (see n_tiles)
    const double* nu;        // FDOA in Hz, tile-major
    const int2* pairs;       // [n_pairs]
    float* J;                // [P]
    PointTiling tiling;
    int64_t n_tiles;         // tiles_x * tiles_y; D / nu are [n_pairs][kc][n_tiles][256]
    int64_t N, P;
    int32_t L, k0, kc, n_pairs;
    double inv_fs;
    int32_t accum_mode;
    int32_t load_J;          // add onto the existing J values
};

struct GeomArgs {
    const double* xyz;       // [P][3]
    const double* states;    // [K][n_rx][6]
    const int2* pairs;
    double* D;               // [n_pairs][kc][P], or tile-major [n_pairs][kc][n_tiles][256]
    double* nu;
    PointTiling tiling;
    int32_t tile_major;      // write the tile-major layout read by the correlation kernels
    int64_t P;
    int32_t n_rx, n_pairs, k0, kc;
    double fs, inv_lambda;
};

// launchers (return hipError_t of the launch)
hipError_t launch_grid_ecef(const double* lat, const double* lon, int32_t grid_kind, int64_t rows, int64_t cols,
                            double radius, double* xyz, hipStream_t s);
hipError_t launch_geometry(const GeomArgs& a, hipStream_t s);
hipError_t launch_direct(const DirectArgs& a, int32_t delay_mode, hipStream_t s);

struct ArgmaxScratch {
    float* part_val = nullptr;
    int64_t* part_idx = nullptr;
    int64_t* found_idx = nullptr;  // [kMaxTopK]
    float* found_val = nullptr;
    int32_t n_blocks = 0;
};
constexpr int kMaxTopK = 64;
hipError_t launch_argmax(const float* J, int64_t P, int64_t cols, int32_t rect, int32_t radius, int32_t top_k,
                         ArgmaxScratch& s, hipStream_t st);
int32_t argmax_blocks(int64_t P);

}  // namespace geoloc
