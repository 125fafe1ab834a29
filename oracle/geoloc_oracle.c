/*
 * geoloc_oracle.c -- plain FP64 CPU oracle of the position-domain correlation map.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load this library. It shares no code, header, table or constant
 * with the GPU library; it is deliberately slow and written to be checked by eye
 * against the paper:
 *
 *   grid -> ECEF ............ Sec. III (candidate points in LLA, "standard transformations"),
 *                             Algorithm 1 (first step); spherical Earth, altitude h.
 *   geometry ................ Sec. II-B, Eq. (3)-(8): range vector, range / delay, unit range
 *                             vector, Doppler f = -(1/lambda) r_hat . v, TDOA, FDOA.
 *   delay in samples ........ Eq. (9) with the dimensional reading D = dTau * f_s; the
 *                             paper's integer rounding (ROUND mode), a two-tap linear
 *                             fractional delay (LINEAR mode, default) and an eight-tap
 *                             Kaiser-windowed sinc fractional delay (SINC mode).
 *   correlation ............. Eq. (10)-(11) per snapshot (step) k, with the sample time t_n
 *                             measured from the step centre and y_j = 0 outside the capture.
 *   map ..................... Algorithm 1 "sum the grids": J(p) = sum over pairs and steps of
 *                             |C_k(p)|^2 (POWER, default) or |C_k(p)| (MAG).
 *
 * Every multiply-add is evaluated as written (compile with -ffp-contract=off); the Doppler
 * phasor is computed from scratch with cos/sin for every sample.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_C_LIGHT 299792458.0
#define ORC_PI 3.14159265358979323846

enum { ORC_LINEAR = 0, ORC_ROUND = 1, ORC_SINC = 2 };
#define ORC_SINC_HALF 4        /* taps t = -3 .. 4 around floor(D) */
#define ORC_SINC_BETA 6.0      /* Kaiser window shape */
enum { ORC_POWER = 0, ORC_MAG = 1 };

int oracle_abi_version(void) { return 1; }

void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Candidate point (geocentric lat, lon in radians; sphere of radius R; altitude h) to ECEF. */
void oracle_grid_ecef(int64_t n, const double* lat, const double* lon, double radius, double alt,
                      double* xyz /* [n][3] */) {
    for (int64_t p = 0; p < n; ++p) {
        double r = radius + alt;
        xyz[3 * p + 0] = r * cos(lat[p]) * cos(lon[p]);
        xyz[3 * p + 1] = r * cos(lat[p]) * sin(lon[p]);
        xyz[3 * p + 2] = r * sin(lat[p]);
    }
}

/* Candidate point on the WGS-84 ellipsoid (geodetic lat, lon in radians; height h[p] above
 * the ellipsoid along its normal, e.g. a terrain model) to ECEF: with the prime-vertical
 * radius of curvature N = a / sqrt(1 - e^2 sin^2 lat),
 *   x = (N + h) cos lat cos lon, y = (N + h) cos lat sin lon, z = (N (1 - e^2) + h) sin lat,
 * a = 6378137 m, f = 1 / 298.257223563, e^2 = f (2 - f). */
void oracle_ecef_wgs84(int64_t n, const double* lat, const double* lon, const double* h, double* xyz) {
    const double a = 6378137.0, f = 1.0 / 298.257223563;
    const double e2 = f * (2.0 - f);
    for (int64_t p = 0; p < n; ++p) {
        double sl = sin(lat[p]), cl = cos(lat[p]);
        double N = a / sqrt(1.0 - e2 * sl * sl);
        xyz[3 * p + 0] = (N + h[p]) * cl * cos(lon[p]);
        xyz[3 * p + 1] = (N + h[p]) * cl * sin(lon[p]);
        xyz[3 * p + 2] = (N * (1.0 - e2) + h[p]) * sl;
    }
}

/* Delay and Doppler of one receiver state s = [p; v] against point q: Eq. (3)-(6). */
static void receiver_delay_doppler(const double q[3], const double* s, double lambda,
                                   double* tau, double* f) {
    double r[3] = {s[0] - q[0], s[1] - q[1], s[2] - q[2]};           /* Eq. (3) */
    double rho = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);      /* Eq. (4) */
    double rhat[3] = {r[0] / rho, r[1] / rho, r[2] / rho};           /* Eq. (5) */
    *tau = rho / ORC_C_LIGHT;
    *f = -(1.0 / lambda) * (rhat[0] * s[3] + rhat[1] * s[4] + rhat[2] * s[5]); /* Eq. (6) */
}

/* TDOA in samples and FDOA (Hz) of the pair (i reference, j shifted): Eq. (7)-(9). */
static void pair_geometry(const double q[3], const double* si, const double* sj, double fs, double fc,
                          double* D, double* nu) {
    double lambda = ORC_C_LIGHT / fc;
    double tau_i, f_i, tau_j, f_j;
    receiver_delay_doppler(q, si, lambda, &tau_i, &f_i);
    receiver_delay_doppler(q, sj, lambda, &tau_j, &f_j);
    *D = (tau_j - tau_i) * fs;   /* Eq. (7), in samples */
    *nu = f_j - f_i;             /* Eq. (8) */
}

/* Geometry table for one pair: D[k][p] (samples) and nu[k][p] (Hz). states: [K][n_rx][6]. */
void oracle_geometry(int64_t n_points, const double* xyz, int32_t n_steps, int32_t n_rx,
                     const double* states, int32_t i, int32_t j, double fs, double fc,
                     double* D, double* nu) {
    for (int32_t k = 0; k < n_steps; ++k)
        for (int64_t p = 0; p < n_points; ++p)
            pair_geometry(&xyz[3 * p], &states[(k * n_rx + i) * 6], &states[(k * n_rx + j) * 6], fs, fc,
                          &D[(int64_t)k * n_points + p], &nu[(int64_t)k * n_points + p]);
}

/* Sample m of a capture (interleaved complex64), zero outside [0, N). */
static void sample_at(const float* y, int64_t n_samples, int64_t m, double* re, double* im) {
    if (m < 0 || m >= n_samples) { *re = 0.0; *im = 0.0; return; }
    *re = (double)y[2 * m];
    *im = (double)y[2 * m + 1];
}

/* Integer lag and fractional weight for a delay of D samples. */
static void split_delay(double D, int mode, int64_t* d0, double* alpha) {
    if (mode == ORC_ROUND) {
        *d0 = (int64_t)round(D);        /* round half away from zero */
        *alpha = 0.0;
    } else {
        double f = floor(D);
        *d0 = (int64_t)f;
        *alpha = D - f;
    }
}

/* Modified Bessel function of the first kind, order 0: sum_k ((x/2)^k / k!)^2. */
static double bessel_i0(double x) {
    double q = 0.25 * x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

/* Kaiser-windowed sinc g(x) = sinc(x) I0(beta sqrt(1 - (x/4)^2)) / I0(beta) for |x| < 4,
 * 0 outside; sinc(x) = sin(pi x) / (pi x). */
static double windowed_sinc(double x) {
    const double h = (double)ORC_SINC_HALF;
    if (fabs(x) >= h) return 0.0;
    const double s = x == 0.0 ? 1.0 : sin(ORC_PI * x) / (ORC_PI * x);
    const double u = x / h;
    return s * bessel_i0(ORC_SINC_BETA * sqrt(1.0 - u * u)) / bessel_i0(ORC_SINC_BETA);
}

/* The eight weights of a delay with fractional part alpha: w[t + 3] = g(t - alpha) /
 * sum_s g(s - alpha), t = -3 .. 4 (unit gain at zero frequency). */
void oracle_sinc_taps(double alpha, double* w) {
    double sum = 0.0;
    for (int t = -ORC_SINC_HALF + 1; t <= ORC_SINC_HALF; ++t) {
        w[t + ORC_SINC_HALF - 1] = windowed_sinc((double)t - alpha);
        sum += w[t + ORC_SINC_HALF - 1];
    }
    for (int i = 0; i < 2 * ORC_SINC_HALF; ++i) w[i] /= sum;
}

/* One correlation C_k for delay D (samples) and FDOA nu (Hz), Eq. (11) over step k:
 *   C = sum_{n=kL}^{kL+L-1} y_i[n] * conj(ytilde_j[n]) * exp(+j 2 pi nu t_n),
 *   t_n = (n - kL - (L-1)/2) / f_s,
 *   ytilde_j[n] = (1-alpha) y_j[n+d0] + alpha y_j[n+d0+1]. */
void oracle_corr(const float* yi, const float* yj, int64_t n_samples, int64_t k, int64_t step_len,
                 double D, double nu, double fs, int32_t delay_mode, double* c_re, double* c_im) {
    int64_t d0;
    double alpha;
    split_delay(D, delay_mode, &d0, &alpha);
    double w[2 * ORC_SINC_HALF];
    if (delay_mode == ORC_SINC) oracle_sinc_taps(alpha, w);
    double sr = 0.0, si = 0.0;
    for (int64_t n = k * step_len; n < (k + 1) * step_len; ++n) {
        double ar, ai, br, bi, xr, xi;
        sample_at(yj, n_samples, n + d0, &ar, &ai);
        sample_at(yj, n_samples, n + d0 + 1, &br, &bi);
        double ytr = (1.0 - alpha) * ar + alpha * br;
        double yti = (1.0 - alpha) * ai + alpha * bi;
        if (delay_mode == ORC_SINC) {
            /* ytilde_j[n] = sum_{t=-3}^{4} w[t] y_j[n + d0 + t] */
            ytr = 0.0;
            yti = 0.0;
            for (int t = -ORC_SINC_HALF + 1; t <= ORC_SINC_HALF; ++t) {
                double cr, ci;
                sample_at(yj, n_samples, n + d0 + t, &cr, &ci);
                ytr += w[t + ORC_SINC_HALF - 1] * cr;
                yti += w[t + ORC_SINC_HALF - 1] * ci;
            }
        }
        sample_at(yi, n_samples, n, &xr, &xi);
        /* x * conj(ytilde) */
        double pr = xr * ytr + xi * yti;
        double pi = xi * ytr - xr * yti;
        double t = ((double)(n - k * step_len) - 0.5 * (double)(step_len - 1)) / fs;
        double ph = 2.0 * ORC_PI * nu * t;
        double wr = cos(ph), wi = sin(ph);
        sr += pr * wr - pi * wi;
        si += pr * wi + pi * wr;
    }
    *c_re = sr;
    *c_im = si;
}

/* Full map over an explicit point list.
 *   captures: [n_rx][N] interleaved complex64; states: [K][n_rx][6];
 *   pairs: [n_pairs][2] (reference i, shifted j); lat/lon: [n_points] (radians).
 *   J: [n_points] float64 (overwritten). */
static double point_J(const double q[3], int32_t n_rx, int64_t n_samples, int64_t step_len, const float* captures,
                      const double* states, int32_t n_pairs, const int32_t* pairs, double fs, double fc,
                      int32_t delay_mode, int32_t accum_mode);

void oracle_map(int64_t n_points, const double* lat, const double* lon, double radius, double alt,
                int32_t n_rx, int64_t n_samples, int64_t step_len, const float* captures,
                const double* states, int32_t n_pairs, const int32_t* pairs, double fs, double fc,
                int32_t delay_mode, int32_t accum_mode, double* J) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < n_points; ++p) {
        double q[3];
        oracle_grid_ecef(1, &lat[p], &lon[p], radius, alt, q);
        J[p] = point_J(q, n_rx, n_samples, step_len, captures, states, n_pairs, pairs, fs, fc, delay_mode, accum_mode);
    }
}

/* The same map at candidate points given in ECEF (xyz: [n_points][3], m). */
void oracle_map_xyz(int64_t n_points, const double* xyz, int32_t n_rx, int64_t n_samples, int64_t step_len,
                    const float* captures, const double* states, int32_t n_pairs, const int32_t* pairs, double fs,
                    double fc, int32_t delay_mode, int32_t accum_mode, double* J) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < n_points; ++p)
        J[p] = point_J(&xyz[3 * p], n_rx, n_samples, step_len, captures, states, n_pairs, pairs, fs, fc, delay_mode,
                       accum_mode);
}

static double point_J(const double q[3], int32_t n_rx, int64_t n_samples, int64_t step_len, const float* captures,
                      const double* states, int32_t n_pairs, const int32_t* pairs, double fs, double fc,
                      int32_t delay_mode, int32_t accum_mode) {
    int64_t n_steps = n_samples / step_len;
    {
        double acc = 0.0;
        for (int32_t e = 0; e < n_pairs; ++e) {
            int32_t i = pairs[2 * e], j = pairs[2 * e + 1];
            const float* yi = captures + 2 * (int64_t)i * n_samples;
            const float* yj = captures + 2 * (int64_t)j * n_samples;
            for (int64_t k = 0; k < n_steps; ++k) {
                double D, nu, cr, ci;
                pair_geometry(q, &states[(k * n_rx + i) * 6], &states[(k * n_rx + j) * 6], fs, fc, &D, &nu);
                oracle_corr(yi, yj, n_samples, k, step_len, D, nu, fs, delay_mode, &cr, &ci);
                double pw = cr * cr + ci * ci;
                acc += (accum_mode == ORC_MAG) ? sqrt(pw) : pw;
            }
        }
        return acc;
    }
}
