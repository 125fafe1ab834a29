// k_geometry.hip -- candidate grid to ECEF, and per-(pair, step, point) TDOA / FDOA in FP64.
//
// Grid conversion: Sec. III (candidate points given in latitude / longitude, put on the
// surface and converted to ECEF), first step of Algorithm 1; a sphere of radius R + h.
// Geometry: Sec. II-B, Eq. (3)-(8), delay expressed in samples as in Eq. (9):
//   r = p_rx - q,  rho = |r|,  tau = rho / c,  f = -(1/lambda) (r / rho) . v_rx,
//   D = (tau_j - tau_i) f_s,   nu = f_j - f_i.
// Both kernels evaluate every product and sum as written (no contraction into FMA), which
// keeps them within a few units in the last place of a plain FP64 implementation of the
// same expressions (the geometry forms 1/rho by a reciprocal square root refined by Newton
// steps and rho as rr / rho; the device's sincos rounds differently).
#include "internal.h"

namespace geoloc {

#pragma clang fp contract(off)

// Candidate point -> ECEF (m). Sphere: radius (+ altitude) times the unit vector of the
// geocentric latitude / longitude. WGS-84: geodetic latitude / longitude and a height above
// the ellipsoid along its normal, with the prime-vertical radius N = a / sqrt(1 - e^2
// sin^2 lat): x = (N + h) cos lat cos lon, y = (N + h) cos lat sin lon, z = (N (1 - e^2) +
// h) sin lat. The height is alt (uniform) plus alt_p[p] when a per-point terrain is given.
// The latitude part (A, Z) = ((N + h) cos lat, (N (1 - e^2) + h) sin lat) and the longitude
// part (cos lon, sin lon) are formed separately and give x = A cos lon, y = A sin lon, z = Z.
__device__ inline double2 ecef_lat_part(double la, double h, int32_t model, double radius) {
    const double cl = cos(la), sl = sin(la);
    if (model == GEOLOC_EARTH_WGS84) {
        const double a = kWgs84A, e2 = kWgs84F * (2.0 - kWgs84F);
        const double N = a / sqrt(1.0 - e2 * sl * sl);
        return make_double2((N + h) * cl, (N * (1.0 - e2) + h) * sl);
    }
    const double R = radius + h;
    return make_double2(R * cl, R * sl);
}

__device__ inline double2 ecef_lon_part(double lo) { return make_double2(cos(lo), sin(lo)); }

// Row and column factors of a rectilinear grid with a uniform height: row_tab[r] = the
// latitude part of row r, col_tab[c] = the longitude part of column c.
__global__ __launch_bounds__(256) void k_grid_ecef_factors(const double* __restrict__ lat, const double* __restrict__ lon,
                                                           int64_t rows, int64_t cols, int32_t model, double radius,
                                                           double alt, double2* __restrict__ row_tab,
                                                           double2* __restrict__ col_tab) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < rows)
        row_tab[i] = ecef_lat_part(lat[i], alt, model, radius);
    else if (i < rows + cols)
        col_tab[i - rows] = ecef_lon_part(lon[i - rows]);
}

// ECEF of every point; a rectilinear grid with a uniform height takes the products of its
// row and column factors (the same products the factored correlation kernel forms).
__global__ __launch_bounds__(256) void k_grid_ecef(const double* __restrict__ lat, const double* __restrict__ lon,
                                                   int32_t grid_kind, int64_t rows, int64_t cols, int32_t model,
                                                   double radius, double alt, const double* __restrict__ alt_p,
                                                   const double2* __restrict__ row_tab,
                                                   const double2* __restrict__ col_tab, double* __restrict__ xyz) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= rows * cols) return;
    double2 A, C;
    if (row_tab) {
        const int64_t r = p / cols;
        A = row_tab[r];
        C = col_tab[p - r * cols];
    } else {
        double la, lo;
        if (grid_kind == GEOLOC_GRID_RECT) {
            const int64_t r = p / cols;
            la = lat[r];
            lo = lon[p - r * cols];
        } else {
            la = lat[p];
            lo = lon[p];
        }
        A = ecef_lat_part(la, alt + (alt_p ? alt_p[p] : 0.0), model, radius);
        C = ecef_lon_part(lo);
    }
    xyz[3 * p + 0] = A.x * C.x;
    xyz[3 * p + 1] = A.x * C.y;
    xyz[3 * p + 2] = A.y;
}

// Points of whole tiles of a rectilinear grid, tile by tile (a POINTS plan's grid): point p
// is cell (tile_row * tile + w / tile, tile_col * tile + w % tile) of tile tiles[p / tile^2],
// w = p % tile^2, with tile index tile_row * (cols / tile) + tile_col. An index outside the
// grid gives NaN coordinates (and a NaN map there) instead of a read out of bounds.
__global__ __launch_bounds__(256) void k_tile_points(const double* __restrict__ glat, const double* __restrict__ glon,
                                                     int64_t rows, int64_t cols, int32_t tile,
                                                     const int32_t* __restrict__ tiles, int64_t P,
                                                     double* __restrict__ lat, double* __restrict__ lon) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const int64_t cells = (int64_t)tile * tile;
    const int64_t t = tiles[p / cells], w = p % cells;
    const int64_t tcols = cols / tile, n_tiles = (rows / tile) * tcols;
    if (t < 0 || t >= n_tiles) {
        lat[p] = lon[p] = __builtin_nan("");
        return;
    }
    const int64_t r = (t / tcols) * tile + w / tile, c = (t % tcols) * tile + w % tile;
    lat[p] = glat[r];
    lon[p] = glon[c];
}

hipError_t launch_tile_points(const double* glat, const double* glon, int64_t rows, int64_t cols, int32_t tile,
                              const int32_t* tiles, int64_t P, double* lat, double* lon, hipStream_t s) {
    hipLaunchKernelGGL(k_tile_points, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, glat, glon, rows, cols, tile,
                       tiles, P, lat, lon);
    return hipGetLastError();
}

// One thread per (pair, step, point), idx = (e * kc + kk) * P + p: the geometry alone, for
// geoloc_geometry (the correlation kernels evaluate the same function inline).
__global__ __launch_bounds__(256) void k_geometry(GeomArgs a) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = a.P * a.kc * a.n_pairs;
    if (idx >= total) return;
    const int64_t p = idx % a.P;
    const int64_t rest = idx / a.P;
    const int32_t kk = (int32_t)(rest % a.kc);
    const int32_t e = (int32_t)(rest / a.kc);
    double D, nu;
    pair_geometry(a.xyz[3 * p], a.xyz[3 * p + 1], a.xyz[3 * p + 2], a.states, a.n_rx, a.k0 + kk, a.pairs[e], a.fs,
                  a.inv_lambda, &D, &nu);
    a.D[idx] = D;
    a.nu[idx] = nu;
}

hipError_t launch_grid_ecef(const double* lat, const double* lon, int32_t grid_kind, int64_t rows, int64_t cols,
                            int32_t model, double radius, double alt, const double* alt_p, double2* row_tab,
                            double2* col_tab, double* xyz, hipStream_t s) {
    const bool factors = grid_kind == GEOLOC_GRID_RECT && !alt_p && row_tab && col_tab;
    if (factors) {
        hipLaunchKernelGGL(k_grid_ecef_factors, dim3((unsigned)((rows + cols + 255) / 256)), dim3(256), 0, s, lat, lon,
                           rows, cols, model, radius, alt, row_tab, col_tab);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    int64_t P = rows * cols;
    dim3 grid((unsigned)((P + 255) / 256));
    hipLaunchKernelGGL(k_grid_ecef, grid, dim3(256), 0, s, lat, lon, grid_kind, rows, cols, model, radius, alt, alt_p,
                       factors ? row_tab : nullptr, factors ? col_tab : nullptr, xyz);
    return hipGetLastError();
}

hipError_t launch_geometry(const GeomArgs& a, hipStream_t s) {
    const int64_t total = a.P * a.kc * a.n_pairs;
    dim3 grid((unsigned)((total + 255) / 256));
    hipLaunchKernelGGL(k_geometry, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace geoloc
