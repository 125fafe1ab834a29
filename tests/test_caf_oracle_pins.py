"""Pins of the FP64 CAF-table oracle off the Doppler bins, and planted mistakes in it.

The CAF-table oracle (Sec. I's cross-ambiguity function, Eq. (11) evaluated on a grid of
integer lags and Doppler bins, then read back per point by interpolation) judges the MFMA
path at its own approximation, so its off-bin reading must be fixed by something other
than itself:

* an affine table: a table that is affine in (lag, Doppler) is reproduced exactly by
  bilinear interpolation, at any off-bin point, and a table constant in lag by any lag
  taps that sum to one (the eight-tap windowed sinc);
* numpy's piecewise-linear ``interp``: between two bins the table reading equals the
  linear interpolation, in Doppler, of the direct oracle's correlations at the two
  neighbouring bins (the direct oracle is the independent C code; the lag part of the
  reading is exact for every delay mode because Eq. (11) is linear in the delayed
  samples);
* maps whose every (point, step) falls on a bin: the CAF-table map equals the direct
  map, which pins the bin spacing and the bin index of ``caf_map_points``.

The planted mistakes (Doppler weights swapped, bin spacing over M instead of M - 1,
the bin index rounded instead of floored, ...) are applied to a copy of the oracle's
source on the CPU; each must fail one of these pins.
"""
import importlib.util
import math
import os

import numpy as np
import pytest

import oracle
from oracle import caf as caf_oracle

C = 299_792_458.0
R_E = 6371.0e3
FC = 1575.42e6
LAM = C / FC


def _rng(seed):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))


def _cn(rng, n):
    return ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) / math.sqrt(2)).astype(np.complex64)


# ------------------------------------------------------------------------ pins (take the module)

def pin_affine_table(cafm):
    """Bilinear reading of an affine table is exact at every off-bin point."""
    rng = _rng(301)
    lag_lo, n_lags = -7, 20
    nu_lo, dnu, M = -1234.5, 37.25, 40
    lags = lag_lo + np.arange(n_lags, dtype=np.float64)
    nus = nu_lo + dnu * np.arange(M, dtype=np.float64)
    A, B, G = 0.3 - 1.1j, 0.7 + 0.25j, -0.013 + 0.021j
    T = A + B * lags[:, None] + G * nus[None, :]
    D = rng.uniform(lag_lo + 0.01, lag_lo + n_lags - 2.01, 300)
    nu = rng.uniform(nu_lo + 0.01, nus[-1] - 0.01, 300)
    # the last lag and the last bin themselves are inside the window
    D = np.r_[D, lags[-1], lags[0] + 0.5]
    nu = np.r_[nu, nus[-1], nus[0]]
    scale = np.max(np.abs(T))
    c = cafm.interp(T, lag_lo, nu_lo, dnu, D, nu, oracle.LINEAR)
    assert np.max(np.abs(c - (A + B * D + G * nu))) <= 1e-12 * scale
    # ROUND reads the nearest lag (the random delays hold no exact halves)
    Dr = D[:-1]
    c = cafm.interp(T, lag_lo, nu_lo, dnu, Dr, nu[:-1], oracle.ROUND)
    assert np.max(np.abs(c - (A + B * np.rint(Dr) + G * nu[:-1]))) <= 1e-12 * scale
    # SINC: eight lag taps summing to one reproduce a table constant in lag
    Ts = A + G * np.broadcast_to(nus[None, :], (n_lags, M))
    Ds = rng.uniform(lag_lo + 3.01, lag_lo + n_lags - 5.01, 50)
    c = cafm.interp(Ts, lag_lo, nu_lo, dnu, Ds, nu[:50], oracle.SINC)
    assert np.max(np.abs(c - (A + G * nu[:50]))) <= 1e-12 * scale


def pin_between_bins_is_linear_in_doppler(cafm):
    """Off-bin reading = numpy's linear interpolation, over the bins, of the direct
    correlations (independent C oracle) at those bins; all three delay modes."""
    rng = _rng(302)
    N, L, fs = 3000, 1000, 1.0e6
    yi, yj = _cn(rng, N), _cn(rng, N)
    nu_b = cafm.bins(-900.0, 600.0, 13)
    lag_lo, n_lags = -12, 30
    for mode in (oracle.LINEAR, oracle.ROUND, oracle.SINC):
        for k in range(3):
            T = cafm.table(yi, yj, k, L, fs, lag_lo, n_lags, nu_b)
            for D in (3.37, -5.81, 0.5, 7.0):
                nus = rng.uniform(nu_b[0] + 1.0, nu_b[-1] - 1.0, 4)
                c_tab = cafm.interp(T, lag_lo, nu_b[0], nu_b[1] - nu_b[0], np.full(4, D), nus, mode)
                c_dir = np.array([oracle.corr(yi, yj, k, L, D, f, fs, mode) for f in nu_b])
                ref = np.interp(nus, nu_b, c_dir.real) + 1j * np.interp(nus, nu_b, c_dir.imag)
                assert np.max(np.abs(c_tab - ref)) <= 1e-9 * np.max(np.abs(c_dir)), (mode, k, D)


def _static_pair_states(K, q0, rng):
    """Two receivers 550 km up, 50 km apart, at rest: zero Doppler at every point."""
    up = q0 / np.linalg.norm(q0)
    east = np.cross([0.0, 0.0, 1.0], up)
    east /= np.linalg.norm(east)
    base = q0 + 550e3 * up
    st = np.zeros((K, 2, 6))
    for k in range(K):
        st[k, 0, :3] = base - 25e3 * east + rng.uniform(-10.0, 10.0, 3)
        st[k, 1, :3] = base + 25e3 * east + rng.uniform(-10.0, 10.0, 3)
    return st


def pin_map_on_bins_equals_direct(cafm):
    """Every (point, step) on a bin: the CAF-table map equals the direct map."""
    rng = _rng(303)
    fs, L, K = 2.0e6, 800, 3
    N = L * K
    lat = np.deg2rad(np.linspace(10.0, 10.2, 5))
    lon = np.deg2rad(np.linspace(20.0, 20.3, 4))
    la, lo = (a.ravel() for a in np.meshgrid(lat, lon, indexing="ij"))
    q0 = oracle.grid_ecef(lat[2:3], lon[1:2], R_E)[0]
    caps = np.stack([_cn(rng, N), _cn(rng, N)])
    # (1) receivers at rest: nu = 0 at every point and step, bin 3 of 11
    st = _static_pair_states(K, q0, rng)
    xyz = oracle.grid_ecef(la, lo, R_E)
    D, nu = oracle.geometry(xyz, st, (0, 1), fs, FC)
    assert np.all(nu == 0.0)
    lag_lo = int(np.floor(D.min())) - 4
    n_lags = int(np.floor(D.max())) - lag_lo + 6
    dnu = 61.5
    for mode in (oracle.LINEAR, oracle.ROUND):
        Jc = cafm.caf_map_points(la, lo, caps, st, L, fs, FC, [(0, 1)], lag_lo, n_lags, -3 * dnu, 7 * dnu, 11,
                                 radius=R_E, delay_mode=mode)
        Jd = oracle.map_points(la, lo, caps, st, L, fs, FC, pairs=[(0, 1)], radius=R_E, delay_mode=mode)
        assert np.max(np.abs(Jc - Jd)) <= 1e-9 * np.max(Jd), mode
    # (2) one point; receiver j moves along its line of sight at a speed per step that puts
    # the FDOA on bin m_k of a window whose spacing is (hi - lo) / (M - 1)
    nu_lo, nu_hi, M = -2000.0, 1500.0, 15
    dnu = (nu_hi - nu_lo) / (M - 1)
    m_k = [2, 11, 6]
    for k in range(K):
        r = st[k, 1, :3] - q0
        st[k, 1, 3:] = (-LAM * (nu_lo + m_k[k] * dnu)) * r / np.linalg.norm(r)
    la1, lo1 = lat[2:3], lon[1:2]
    D1, nu1 = oracle.geometry(oracle.grid_ecef(la1, lo1, R_E), st, (0, 1), fs, FC)
    assert np.allclose(nu1[:, 0], nu_lo + np.array(m_k) * dnu, rtol=0, atol=1e-8)
    lag_lo = int(np.floor(D1.min())) - 4
    n_lags = int(np.floor(D1.max())) - lag_lo + 6
    Jc = cafm.caf_map_points(la1, lo1, caps, st, L, fs, FC, [(0, 1)], lag_lo, n_lags, nu_lo, nu_hi, M, radius=R_E)
    Jd = oracle.map_points(la1, lo1, caps, st, L, fs, FC, pairs=[(0, 1)], radius=R_E)
    assert abs(Jc[0] - Jd[0]) <= 1e-9 * Jd[0]


PINS = [pin_affine_table, pin_between_bins_is_linear_in_doppler, pin_map_on_bins_equals_direct]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_caf_oracle_pin(pin):
    pin(caf_oracle)


# ------------------------------------------------------------------------ planted mistakes

SRC = os.path.join(os.path.dirname(oracle.__file__), "caf.py")

MUTANTS = {
    "doppler_weights_swapped": (
        "return ((1 - a) * (1 - b) * T[r0, m0] + a * (1 - b) * T[r0 + 1, m0]\n"
        "            + (1 - a) * b * T[r0, m0 + 1] + a * b * T[r0 + 1, m0 + 1])",
        "return ((1 - a) * b * T[r0, m0] + a * b * T[r0 + 1, m0]\n"
        "            + (1 - a) * (1 - b) * T[r0, m0 + 1] + a * (1 - b) * T[r0 + 1, m0 + 1])"),
    "lag_weights_swapped": (
        "return ((1 - a) * (1 - b) * T[r0, m0] + a * (1 - b) * T[r0 + 1, m0]\n"
        "            + (1 - a) * b * T[r0, m0 + 1] + a * b * T[r0 + 1, m0 + 1])",
        "return (a * (1 - b) * T[r0, m0] + (1 - a) * (1 - b) * T[r0 + 1, m0]\n"
        "            + a * b * T[r0, m0 + 1] + (1 - a) * b * T[r0 + 1, m0 + 1])"),
    "sinc_doppler_weights_swapped": (
        "((1 - b.flat[p]) * T[r, m0.flat[p]] + b.flat[p] * T[r, m0.flat[p] + 1])",
        "(b.flat[p] * T[r, m0.flat[p]] + (1 - b.flat[p]) * T[r, m0.flat[p] + 1])"),
    "map_bin_spacing_over_M": ("dnu = (nu_hi - nu_lo) / (n_bins - 1)", "dnu = (nu_hi - nu_lo) / n_bins"),
    "bins_spacing_over_M": ("return nu_lo + (nu_hi - nu_lo) / (n_bins - 1) * np.arange(n_bins)",
                            "return nu_lo + (nu_hi - nu_lo) / n_bins * np.arange(n_bins)"),
    "bin_index_rounded": ("m0f = np.floor(u)", "m0f = np.round(u)"),
    "bin_offset_dropped": ("u = (nu - nu_lo) / dnu", "u = nu / dnu"),
    "lag_index_off_by_one": ("r0 = d0 - lag_lo\n", "r0 = d0 - lag_lo - 1\n"),
    "table_time_from_step_start": ("t = (n - k * step_len - (step_len - 1) / 2.0) / fs", "t = (n - k * step_len) / fs"),
    "table_lag_conjugate_dropped": ("Lk[r] = x * np.conj(v)", "Lk[r] = x * v"),
}


def _load_mutant(src_text, tmp_path, name):
    path = tmp_path / f"caf_{name}.py"
    path.write_text(src_text)
    spec = importlib.util.spec_from_file_location(f"oracle.caf_{name}", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_mutation_sites_are_unique():
    src = open(SRC).read()
    for name, (old, _) in MUTANTS.items():
        assert src.count(old) >= 1, name


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_every_planted_caf_mistake_fails_a_pin(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert old in src, f"mutation site for {name} not found"
    mod = _load_mutant(src.replace(old, new), tmp_path, name)
    failed = []
    for pin in PINS:
        try:
            pin(mod)
        except (AssertionError, ValueError, IndexError, FloatingPointError):
            failed.append(pin.__name__)
    # the inverse-FFT pin of the table (P10) also judges the table's time origin
    import test_oracle_pins as pins
    saved = pins.caf
    pins.caf = mod
    try:
        pins.test_p10_caf_table_with_dft_bins_is_inverse_fft()
    except (AssertionError, ValueError, IndexError):
        failed.append("p10")
    finally:
        pins.caf = saved
    assert failed, f"no pin catches the planted mistake {name!r}"
