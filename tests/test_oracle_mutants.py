"""Plant plausible mistakes in the oracle's C source (on the CPU) and check that the pins
catch every one: a wrong sign, a swapped weight, a missing conjugate, an index off by one,
broken zero padding, a swapped accumulation mode, a wrong coordinate, unnormalised or
shifted windowed-sinc taps, a wrong WGS-84 radius of curvature, polar axis or height."""
import os
import subprocess

import pytest

import oracle
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "geoloc_oracle.c")

MUTANTS = {
    "doppler_sign": ("*f = -(1.0 / lambda) *", "*f = (1.0 / lambda) *"),
    "tdoa_sign": ("*D = (tau_j - tau_i) * fs;", "*D = (tau_i - tau_j) * fs;"),
    "fdoa_sign": ("*nu = f_j - f_i;", "*nu = f_i - f_j;"),
    "lerp_weights_swapped": ("double ytr = (1.0 - alpha) * ar + alpha * br;", "double ytr = alpha * ar + (1.0 - alpha) * br;"),
    "missing_conjugate": ("double pr = xr * ytr + xi * yti;", "double pr = xr * ytr - xi * yti;"),
    "rotation_sign": ("double ph = 2.0 * ORC_PI * nu * t;", "double ph = -2.0 * ORC_PI * nu * t;"),
    "lag_off_by_one": ("sample_at(yj, n_samples, n + d0, &ar, &ai);", "sample_at(yj, n_samples, n + d0 + 1, &ar, &ai);"),
    "zero_padding_drops_last_sample": ("if (m < 0 || m >= n_samples)", "if (m < 0 || m >= n_samples - 1)"),
    "power_and_magnitude_swapped": ("(accum_mode == ORC_MAG) ? sqrt(pw) : pw", "(accum_mode == ORC_MAG) ? pw : sqrt(pw)"),
    "ecef_coordinate": ("xyz[3 * p + 1] = r * cos(lat[p]) * sin(lon[p]);", "xyz[3 * p + 1] = r * sin(lat[p]) * sin(lon[p]);"),
    "round_is_floor": ("*d0 = (int64_t)round(D);", "*d0 = (int64_t)floor(D);"),
    "step_sum_range": ("for (int64_t n = k * step_len; n < (k + 1) * step_len; ++n) {",
                       "for (int64_t n = k * step_len; n + 1 < (k + 1) * step_len; ++n) {"),
    "sinc_taps_unnormalised": ("for (int i = 0; i < 2 * ORC_SINC_HALF; ++i) w[i] /= sum;",
                               "for (int i = 0; i < 2 * ORC_SINC_HALF; ++i) w[i] /= 1.0;"),
    "sinc_tap_offset": ("sample_at(yj, n_samples, n + d0 + t, &cr, &ci);",
                        "sample_at(yj, n_samples, n + d0 + t + 1, &cr, &ci);"),
    "wgs84_prime_vertical_radius": ("double N = a / sqrt(1.0 - e2 * sl * sl);", "double N = a / sqrt(1.0 - e2 * cl * cl);"),
    "wgs84_z_without_eccentricity": ("xyz[3 * p + 2] = (N * (1.0 - e2) + h[p]) * sl;", "xyz[3 * p + 2] = (N + h[p]) * sl;"),
    "wgs84_height_not_along_normal": ("xyz[3 * p + 0] = (N + h[p]) * cl * cos(lon[p]);",
                                      "xyz[3 * p + 0] = (N * cl + h[p]) * cos(lon[p]);"),
}

PINS = [getattr(pins, n) for n in dir(pins) if n.startswith("test_") and n != "test_peaks_rules"]


def _run_pins():
    """Names of the pins that fail."""
    failed = []
    for f in PINS:
        kwargs = {}
        if f.__name__ == "test_p14_brute_force_tiny":
            kwargs = {"mode": oracle.LINEAR, "accum": oracle.POWER}
        try:
            f(**kwargs)
        except (AssertionError, ValueError, FloatingPointError):
            failed.append(f.__name__)
    return failed


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_every_planted_mistake_fails_a_pin(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", str(mut),
                    "-o", str(lib), "-lm"], check=True)
    with oracle.use_library(str(lib)):
        failed = _run_pins()
    assert failed, f"no pin catches the planted mistake {name!r}"
