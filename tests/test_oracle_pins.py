"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these retypes the oracle's formula: each checks it against a closed form,
an invariant, a library routine, an exact construction or an independent brute
force, chosen so that a dropped term, a flipped sign, a wrong index or a swapped
operand anywhere in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute, caf, peaks
from paper_2508_06672_amd import configs, sim

C = 299_792_458.0
R_E = 6371.0e3
FC = configs.GPS_L1_HZ
LAM = C / FC


def _rng(seed):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))


def _cn(rng, n, scale=1.0):
    return (scale * (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / math.sqrt(2)).astype(np.complex64)


# ------------------------------------------------------------------------ P1: grid -> ECEF

def test_p1_ecef_closed_forms():
    lat = np.array([0.0, math.pi / 2, 0.0, -math.pi / 2, 0.0])
    lon = np.array([0.0, 1.234, math.pi / 2, 0.3, math.pi])
    xyz = oracle.grid_ecef(lat, lon, R_E, 0.0)
    exp = np.array([[R_E, 0, 0], [0, 0, R_E], [0, R_E, 0], [0, 0, -R_E], [-R_E, 0, 0]])
    assert np.max(np.abs(xyz - exp)) < 1e-9 * R_E
    rng = _rng(1)
    la, lo = rng.uniform(-1.5, 1.5, 1000), rng.uniform(-3.1, 3.1, 1000)
    for h in (0.0, 1234.5):
        p = oracle.grid_ecef(la, lo, R_E, h)
        assert np.max(np.abs(np.linalg.norm(p, axis=1) - (R_E + h))) < 1e-6
        # latitude / longitude recovered by the inverse transformation
        assert np.allclose(np.arcsin(p[:, 2] / (R_E + h)), la, atol=1e-12)
        assert np.allclose(np.arctan2(p[:, 1], p[:, 0]), lo, atol=1e-12)


# ------------------------------------------------------------------------ P2-P4: geometry

def _states(*rx):
    """states [1][n_rx][6] from (position, velocity) tuples."""
    return np.array([[np.r_[p, v] for (p, v) in rx]], dtype=np.float64)


def test_p2_delay_exact_distances():
    q = np.array([[R_E, 0.0, 0.0]])
    # 3-4-5 and 0-0-6 right triangles: rho_i = 500 km, rho_j = 600 km exactly
    si = (q[0] + [300e3, 400e3, 0.0], [0, 0, 0])
    sj = (q[0] + [0.0, 0.0, 600e3], [0, 0, 0])
    D, nu = oracle.geometry(q, _states(si, sj), (0, 1), 2e6, FC)
    assert abs(D[0, 0] - (100e3 / C) * 2e6) < 1e-9
    assert nu[0, 0] == 0.0
    # nadir: receiver 550 km straight above, the other at the point itself -> rho = altitude
    sj2 = (q[0] * (1 + 550e3 / R_E), [0, 0, 0])
    si2 = (q[0] + [1e-3, 0, 0], [0, 0, 0])
    D2, _ = oracle.geometry(q, _states(si2, sj2), (0, 1), 1.0, FC)
    assert abs(D2[0, 0] * C - (550e3 - 1e-3)) < 1e-6


def test_p3_doppler_sign_and_perpendicular():
    q = np.array([[R_E, 0.0, 0.0]])
    still = (q[0] + [0, 0, 1e5], [0, 0, 0])
    # receiver receding from q along the line of sight at 7 km/s -> f = -v / lambda
    away = (q[0] + [500e3, 0, 0], [7e3, 0, 0])
    _, nu = oracle.geometry(q, _states(still, away), (0, 1), 1.0, FC)
    assert abs(nu[0, 0] - (-7e3 / LAM)) < 1e-6 * 7e3 / LAM
    # moving perpendicular to the line of sight -> zero Doppler
    perp = (q[0] + [500e3, 0, 0], [0, 7e3, 3e3])
    _, nu = oracle.geometry(q, _states(still, perp), (0, 1), 1.0, FC)
    assert abs(nu[0, 0]) < 1e-9


def test_p3_doppler_matches_range_rate_finite_difference():
    """f = -(1/lambda) d(rho)/dt along the analytic circular orbit (pins the sign of Eq. (6))."""
    wl = configs.SMALL
    rng = _rng(7)
    for trial in range(5):
        u_mid = rng.uniform(0, 2 * math.pi)
        lat, lon = sim.make_grid(wl, u_mid)
        la, lo = lat[rng.integers(lat.size)], lon[rng.integers(lon.size)]
        q = oracle.grid_ecef([la], [lo], R_E)
        h = 1e-3
        st = sim.receiver_states(wl, u_mid, np.array([-h, 0.0, h]))          # [3][2][6]
        rho = np.linalg.norm(st[:, 1, 0:3] - q[0], axis=1)
        f_fd = -(rho[2] - rho[0]) / (2 * h) / LAM
        # reference receiver frozen in place with zero velocity -> nu = f_j
        fixed = np.r_[st[1, 0, 0:3], 0, 0, 0]
        states = np.array([[fixed, st[1, 1]]])
        _, nu = oracle.geometry(q, states, (0, 1), 1.0, FC)
        assert abs(nu[0, 0] - f_fd) < 1e-6 * max(1.0, abs(f_fd)), (nu[0, 0], f_fd)


def test_p3_nadir_of_circular_orbit_has_zero_doppler():
    wl = configs.SMALL
    r = wl.earth_radius_m + wl.orbit_alt_m
    st = sim.receiver_states(wl, 0.7, np.array([0.0]))
    p = st[0, 1, 0:3]
    q = (p / np.linalg.norm(p) * R_E)[None, :]
    still = np.r_[q[0] + [0, 0, 1e5], 0, 0, 0]
    D, nu = oracle.geometry(q, np.array([[still, st[0, 1]]]), (0, 1), 1.0, FC)
    assert abs(nu[0, 0]) < 1e-6
    assert abs(np.linalg.norm(p - q[0]) - (r - R_E)) < 1e-6


def test_p4_symmetric_pair_has_zero_tdoa():
    rng = _rng(3)
    q = np.array([[R_E, 0.0, 0.0]])
    for _ in range(20):
        a, b, c = rng.uniform(-1e6, 1e6, 3)
        si = (q[0] + [a, b, c], [0, 0, 0])
        sj = (q[0] + [a, -b, c], [0, 0, 0])
        D, _ = oracle.geometry(q, _states(si, sj), (0, 1), 10e6, FC)
        assert D[0, 0] == 0.0
    # swapping the pair flips the sign of both TDOA and FDOA (Eq. (7)-(8))
    si = (q[0] + [1e5, 2e5, 5e5], [100.0, 7000.0, 0])
    sj = (q[0] + [-3e5, 1e5, 5e5], [0.0, 7000.0, 200.0])
    D1, n1 = oracle.geometry(q, _states(si, sj), (0, 1), 10e6, FC)
    D2, n2 = oracle.geometry(q, _states(si, sj), (1, 0), 10e6, FC)
    assert D1[0, 0] == -D2[0, 0] and n1[0, 0] == -n2[0, 0]


# ------------------------------------------------------------------------ P5: zero delay / Doppler

def test_p5_identical_receivers_give_flat_map():
    rng = _rng(5)
    N, L = 3000, 1000
    y = np.stack([_cn(rng, N), _cn(rng, N)])
    s = np.r_[7e6, 1e5, 2e5, 0, 0, 0]
    states = np.array([[s, s]] * (N // L))
    lat = np.linspace(-0.1, 0.1, 4)
    lon = np.linspace(0.2, 0.3, 5)
    J = oracle.map_rect(lat, lon, y, states, L, 2e6, FC)
    yd = y.astype(np.complex128)
    expect = sum(abs(np.sum(yd[0, k * L:(k + 1) * L] * np.conj(yd[1, k * L:(k + 1) * L]))) ** 2 for k in range(N // L))
    assert np.max(np.abs(J - expect)) <= 1e-12 * expect


# ------------------------------------------------------------------------ P6: linear delay

def test_p6_linear_delay_is_linear_in_alpha_and_round_mode():
    rng = _rng(6)
    N, L = 4096, 1024
    yi, yj = _cn(rng, N), _cn(rng, N)
    for k in range(N // L):
        for _ in range(4):
            d0 = int(rng.integers(-40, 40))
            a = float(rng.uniform(0.01, 0.99))
            nu = float(rng.uniform(-3e4, 3e4))
            c = oracle.corr(yi, yj, k, L, d0 + a, nu, 2e6)
            c0 = oracle.corr(yi, yj, k, L, d0, nu, 2e6)
            c1 = oracle.corr(yi, yj, k, L, d0 + 1, nu, 2e6)
            assert abs(c - ((1 - a) * c0 + a * c1)) <= 1e-12 * (abs(c0) + abs(c1))
            # ROUND (the paper's integer delay) equals the integer correlation at round(D)
            D = d0 + a
            r = oracle.corr(yi, yj, k, L, D, nu, 2e6, oracle.ROUND)
            assert r == oracle.corr(yi, yj, k, L, float(round(D)), nu, 2e6)
    # half-way delays round away from zero
    assert oracle.corr(yi, yj, 1, L, 2.5, 0.0, 2e6, oracle.ROUND) == oracle.corr(yi, yj, 1, L, 3.0, 0.0, 2e6)
    assert oracle.corr(yi, yj, 1, L, -2.5, 0.0, 2e6, oracle.ROUND) == oracle.corr(yi, yj, 1, L, -3.0, 0.0, 2e6)


# ------------------------------------------------------------------------ P7: tone closed form

def test_p7_tone_dirichlet_and_scalloping():
    fs, N, L = 2e6, 6000, 2000
    n = np.arange(N)
    for f0 in (0.0, 123456.0, -700e3):
        y = np.exp(2j * np.pi * f0 * n / fs).astype(np.complex64)
        y64 = y.astype(np.complex128)
        for (D, nu) in [(0.0, 0.0), (17.0, 250.0), (-33.25, -1234.5), (5.5, 3333.0), (12.8, 0.3)]:
            c = oracle.corr(y, y, 1, L, D, nu, fs)
            d0 = math.floor(D)
            a = D - d0
            # with the exact complex64 samples the tone has a slowly varying amplitude error;
            # use the float32 values of y to form the closed form's per-sample phase step
            dirich = abs(math.sin(math.pi * nu * L / fs) / math.sin(math.pi * nu / fs)) if nu else float(L)
            scal = abs((1 - a) + a * np.exp(2j * np.pi * f0 / fs))
            assert abs(abs(c) - dirich * scal) <= 2e-6 * L, (f0, D, nu, abs(c), dirich * scal)
        # exactly, with the samples' own values: |C| at nu = 0 equals |sum x conj(ytilde)|
        c = oracle.corr(y, y, 1, L, 3.0, 0.0, fs)
        ex = np.sum(y64[L:2 * L] * np.conj(y64[L + 3:2 * L + 3]))
        assert abs(c - ex) <= 1e-12 * L


# ------------------------------------------------------------------------ P8: Cauchy-Schwarz, exact peak

def test_p8_model_exact_pair_peaks_with_equality():
    rng = _rng(8)
    fs, N, L = 2e6, 3000, 1000
    yi = _cn(rng, N, 2.0)
    for k in range(N // L):
        d_star, nu_star = int(rng.integers(-20, 20)), float(rng.uniform(-5e3, 5e3))
        yj = np.zeros(N, dtype=np.complex128)
        n = np.arange(k * L, (k + 1) * L)
        t = (n - k * L - (L - 1) / 2) / fs
        m = n + d_star
        ok = (m >= 0) & (m < N)
        yj[m[ok]] = yi[n[ok]].astype(np.complex128) * np.exp(2j * np.pi * nu_star * t[ok])
        yj = yj.astype(np.complex64)
        e_i = float(np.sum(np.abs(yi[n[ok]].astype(np.complex128)) ** 2))
        c = oracle.corr(yi, yj, k, L, d_star, nu_star, fs)
        assert abs(c.real - e_i) < 1e-5 * e_i and abs(c.imag) < 1e-5 * e_i
        # Cauchy-Schwarz bound everywhere else
        ei_full = float(np.sum(np.abs(yi[k * L:(k + 1) * L].astype(np.complex128)) ** 2))
        for _ in range(30):
            D = d_star + rng.uniform(-5, 5)
            nu = nu_star + rng.uniform(-3e3, 3e3)
            d0 = math.floor(D)
            a = D - d0
            yd = yj.astype(np.complex128)
            idx = n + d0
            tap = lambda q: np.where((q >= 0) & (q < N), yd[np.clip(q, 0, N - 1)], 0)
            yt = (1 - a) * tap(idx) + a * tap(idx + 1)
            bound = math.sqrt(ei_full * float(np.sum(np.abs(yt) ** 2)))
            assert abs(oracle.corr(yi, yj, k, L, D, nu, fs)) <= bound * (1 + 1e-12)


# ------------------------------------------------------------------------ P9: library cross-correlation

def test_p9_zero_doppler_integer_delay_is_numpy_correlate():
    rng = _rng(9)
    N, L = 1500, 500
    yi, yj = _cn(rng, N), _cn(rng, N)
    a, b = yi.astype(np.complex128), yj.astype(np.complex128)
    for k in range(N // L):
        x = a[k * L:(k + 1) * L]
        # numpy.correlate(v, x, 'full')[s] = sum_n v[n + s - (L-1)] conj(x[n]) over the overlap
        full = np.correlate(b, x, mode="full")       # length N + L - 1
        for d in (-L - 3, -(k * L) - 1, -7, 0, 1, 250, N - k * L - 1, N):
            c = oracle.corr(yi, yj, k, L, float(d), 0.0, 1e6, oracle.ROUND)
            s = k * L + d + (L - 1)
            ref = np.conj(full[s]) if 0 <= s < full.size else 0.0
            assert abs(c - ref) <= 1e-12 * max(1.0, abs(ref)), (k, d)


# ------------------------------------------------------------------------ P10: CAF table vs FFT

def test_p10_caf_table_with_dft_bins_is_inverse_fft():
    rng = _rng(10)
    fs, N, L = 1e6, 1024, 256
    yi, yj = _cn(rng, N), _cn(rng, N)
    nu = np.arange(L) * fs / L
    k, lag_lo, n_lags = 2, -5, 11
    T = caf.table(yi, yj, k, L, fs, lag_lo, n_lags, nu)
    a, b = yi.astype(np.complex128), yj.astype(np.complex128)
    n = np.arange(k * L, (k + 1) * L)
    m = np.arange(L)
    phase = np.exp(-1j * np.pi * m * (L - 1) / L)
    for r in range(n_lags):
        q = n + lag_lo + r
        row = a[n] * np.conj(np.where((q >= 0) & (q < N), b[np.clip(q, 0, N - 1)], 0))
        ref = L * np.fft.ifft(row) * phase
        assert np.max(np.abs(T[r] - ref)) <= 1e-10 * np.max(np.abs(ref))
    # on-bin points: the CAF-table map equals the direct correlation (Eq. (11), linear delay)
    for (D, f) in [(-2.3, nu[5]), (3.0, nu[17]), (4.999, nu[200])]:
        c_tab = caf.interp(T, lag_lo, 0.0, fs / L, np.array([D]), np.array([f]))[0]
        c_dir = oracle.corr(yi, yj, k, L, D, f, fs)
        assert abs(c_tab - c_dir) <= 1e-9 * abs(c_dir)


# ------------------------------------------------------------------------ P11, P12: invariants

def _mirror_points(wl, lat, lon, rng, n):
    la = rng.choice(lat, n)
    lo = rng.choice(lon, n)
    ml = np.array([sim.mirror_latlon(wl, a, b) for a, b in zip(la, lo)])
    return np.r_[la, ml[:, 0]], np.r_[lo, ml[:, 1]]


def test_p11_orbital_plane_mirror_symmetry():
    wl = configs.SMALL
    scn = sim.make_scenario(wl, 11)
    rng = _rng(11)
    la, lo = _mirror_points(wl, scn.lat, scn.lon, rng, 40)
    J = oracle.map_points(la, lo, scn.captures, scn.states, wl.step_len, wl.fs_hz, wl.fc_hz)
    assert np.max(np.abs(J[:40] - J[40:])) <= 1e-9 * np.max(J)


def test_p12_scaling():
    wl = configs.SMALL.with_(n_samples=8000, step_len=4000)
    scn = sim.make_scenario(wl, 12)
    la, lo = sim.points_of(scn)
    sel = slice(0, None, 97)
    J1 = oracle.map_points(la[sel], lo[sel], scn.captures, scn.states, wl.step_len, wl.fs_hz, wl.fc_hz)
    a = 2.0 ** 0.5 * np.exp(0.7j)
    J2 = oracle.map_points(la[sel], lo[sel], (scn.captures * np.complex64(a)).astype(np.complex64),
                           scn.states, wl.step_len, wl.fs_hz, wl.fc_hz)
    assert np.max(np.abs(J2 - abs(a) ** 4 * J1)) <= 1e-5 * np.max(J2)   # complex64 rounding of a*y
    J3 = oracle.map_points(la[sel], lo[sel], (scn.captures * 2).astype(np.complex64), scn.states,
                           wl.step_len, wl.fs_hz, wl.fc_hz)
    assert np.max(np.abs(J3 - 16 * J1)) <= 1e-12 * np.max(J3)           # exact power-of-two scaling
    Jm = oracle.map_points(la[sel], lo[sel], (scn.captures * 2).astype(np.complex64), scn.states,
                           wl.step_len, wl.fs_hz, wl.fc_hz, accum_mode=oracle.MAG)
    Jm1 = oracle.map_points(la[sel], lo[sel], scn.captures, scn.states, wl.step_len, wl.fs_hz, wl.fc_hz,
                            accum_mode=oracle.MAG)
    assert np.max(np.abs(Jm - 4 * Jm1)) <= 1e-12 * np.max(Jm)


# ------------------------------------------------------------------------ P13: end-to-end physics

def test_p13_noiseless_emitter_peaks_at_true_cell_three_receivers():
    """A receiver displaced across track breaks the along-track ridge; the noiseless
    physical capture must peak within one cell of the true cell."""
    wl = configs.SMALL.with_(
        name="p13", rx_along_track_m=(-25e3, 25e3, 0.0), rx_cross_track_m=(0.0, 0.0, 40e3),
        pairs=((0, 1), (0, 2), (1, 2)), n_rows=31, n_cols=31, spacing_m=500.0,
        fs_hz=4e6, n_samples=16000, step_len=4000, waveform="gauss", gauss_bw_hz=3e6)
    for seed in range(3):
        scn = sim.make_scenario(wl, seed, noiseless=True)
        J = oracle.map_scenario(scn)
        i, _ = peaks.argmax(J)
        r, c = divmod(i, wl.n_cols)
        tr = scn.true_cells[0]
        assert max(abs(r - tr[0]), abs(c - tr[1])) <= 1, (seed, (r, c), tr)


def test_p13_along_track_pair_peak_lies_on_the_true_ridge():
    wl = configs.SMALL.with_(name="p13b", n_samples=8000, step_len=4000)
    for seed in range(3):
        scn = sim.make_scenario(wl, seed, noiseless=True)
        J = oracle.map_scenario(scn)
        i, _ = peaks.argmax(J)
        r, c = divmod(i, wl.n_cols)
        tr = scn.true_cells[0]
        xyz = oracle.grid_ecef([scn.lat[r], scn.emitters[0].lat], [scn.lon[c], scn.emitters[0].lon], R_E)
        D, nu = oracle.geometry(xyz, scn.states, (0, 1), wl.fs_hz, wl.fc_hz)
        assert np.all(np.abs(D[:, 0] - D[:, 1]) <= 0.6), (seed, D)     # within the delay resolution
        assert np.all(np.abs(nu[:, 0] - nu[:, 1]) <= wl.fs_hz / wl.step_len)


def test_p13_doppler_sign_long_step_tone():
    """A pure tone is located by Doppler alone (a streak); with one 50 ms step the
    Doppler resolution (20 Hz) is far finer than the footprint's FDOA span."""
    wl = configs.SMALL.with_(name="p13c", n_rows=41, n_cols=41, spacing_m=5000.0, n_samples=100_000,
                             step_len=100_000, waveform="tone")
    scn = sim.make_scenario(wl, 4, noiseless=True)
    J = oracle.map_scenario(scn)
    i, jmax = peaks.argmax(J)
    xyz = oracle.grid_ecef([scn.lat[i // 41], scn.emitters[0].lat], [scn.lon[i % 41], scn.emitters[0].lon], R_E)
    _, nu = oracle.geometry(xyz, scn.states, (0, 1), wl.fs_hz, wl.fc_hz)
    assert abs(nu[0, 0] - nu[0, 1]) < 10.0
    # the peak approaches the coherent maximum N^2 (unit tone on both receivers); the
    # nearest 5 km cell is a few Hz off the true FDOA, which costs up to ~20 %
    assert jmax > 0.7 * wl.n_samples ** 2


# ------------------------------------------------------------------------ P14: brute force

@pytest.mark.parametrize("mode", [oracle.LINEAR, oracle.ROUND, oracle.SINC])
@pytest.mark.parametrize("accum", [oracle.POWER, oracle.MAG])
def test_p14_brute_force_tiny(mode, accum):
    wl = configs.SMALL.with_(name="tiny", rx_along_track_m=(-25e3, 25e3, 5e3), pairs=((0, 1), (2, 0), (1, 2)),
                             n_rows=3, n_cols=4, n_samples=300, step_len=100)
    scn = sim.make_scenario(wl, 14)
    la, lo = sim.points_of(scn)
    for pairs in ([(0, 1)], list(wl.pairs)):
        J = oracle.map_points(la, lo, scn.captures, scn.states, wl.step_len, wl.fs_hz, wl.fc_hz, pairs=pairs,
                              delay_mode=mode, accum_mode=accum)
        Jb = brute.brute_map(la, lo, scn.captures, scn.states, wl.step_len, wl.fs_hz, wl.fc_hz, pairs,
                             delay_mode=mode, accum_mode=accum)
        assert np.max(np.abs(J - Jb)) <= 1e-12 * np.max(np.abs(Jb))


# ------------------------------------------------------------------------ P15: paper's qualitative shapes

def test_p15_repeated_chirp_gives_equal_peaks_one_period_apart():
    """A chirp repeated with period T correlates equally at delays one period apart
    (the several equal peaks of a chirp jammer's single-snapshot grid)."""
    fs, N, L = 4e6, 8000, 2000
    T = 10e-6                                   # 40 samples
    t = np.arange(N) / fs
    x = sim.chirp(t, 1e6, T).astype(np.complex64)
    shift = 13
    yj = np.zeros(N, dtype=np.complex64)
    yj[shift:] = x[:N - shift]
    k = 2
    vals = [abs(oracle.corr(x, yj, k, L, shift + m * 40, 0.0, fs)) for m in (-2, -1, 0, 1, 2)]
    assert np.max(vals) - np.min(vals) <= 1e-5 * np.max(vals)
    off = abs(oracle.corr(x, yj, k, L, shift + 20, 0.0, fs))
    assert off < 0.2 * vals[2]


# ------------------------------------------------------------------------ peaks

def test_peaks_rules():
    J = np.array([1.0, 3.0, 3.0, 2.0])
    assert peaks.argmax(J) == (1, 3.0)
    with pytest.raises(ValueError):
        peaks.argmax(np.array([1.0, np.nan]))
    M = np.zeros((6, 7))
    M[1, 1], M[1, 2], M[4, 5] = 5.0, 4.9, 4.0
    out = peaks.topk(M.ravel(), 6, 7, 2, 2)
    assert [o[0] for o in out] == [1 * 7 + 1, 4 * 7 + 5]


# ------------------------------------------------------------------------ P16: windowed-sinc delay

def test_p16_sinc_taps_library_and_integer_delay():
    """The SINC weights are numpy's sinc times a Kaiser window built from numpy's I0,
    normalised to unit sum; at a whole-sample delay they are a unit impulse at tap 0, so
    SINC equals ROUND there."""
    for a in (0.0, 0.125, 0.3, 0.5, 0.77, 0.999):
        x = np.arange(-3, 5) - a
        g = np.sinc(x) * np.i0(6.0 * np.sqrt(np.clip(1 - (x / 4) ** 2, 0, None))) / np.i0(6.0)
        g[np.abs(x) >= 4] = 0.0
        assert np.max(np.abs(oracle.sinc_taps(a) - g / g.sum())) < 1e-14
    w = oracle.sinc_taps(0.0)
    assert abs(w[3] - 1.0) < 1e-15 and np.max(np.abs(np.delete(w, 3))) < 1e-15
    rng = _rng(16)
    y = _cn(rng, 600)
    for D in (-7.0, 0.0, 3.0, 41.0):
        cs = oracle.corr(y, y, 0, 600, D, 300.0, 1e6, oracle.SINC)
        cr = oracle.corr(y, y, 0, 600, D, 300.0, 1e6, oracle.ROUND)
        assert abs(cs - cr) <= 1e-12 * abs(cr)


def test_p16_sinc_delay_recovers_a_fractionally_delayed_band_limited_signal():
    """A sum of tones below a quarter of the sample rate, delayed by a fractional number of
    samples (built exactly from the tones' phases): SINC correlates it with its undelayed
    self to within 1e-3 of the full coherence, where LINEAR loses the closed-form
    |(1 - a) + a exp(j 2 pi f / fs)| per tone (about -2.7 dB at f = 0.24 fs, a = 1/2)."""
    fs, N = 1.0e6, 4000
    n = np.arange(N)
    freqs = np.array([-0.22, -0.13, 0.04, 0.11, 0.24]) * fs
    amps = np.array([1.0, 0.7, 1.3, 0.9, 1.1])
    for D in (2.5, -6.3, 0.75):
        yi = (amps[None, :] * np.exp(2j * np.pi * freqs[None, :] * n[:, None] / fs)).sum(1)
        yj = (amps[None, :] * np.exp(2j * np.pi * freqs[None, :] * (n[:, None] - D) / fs)).sum(1)
        # y_j[n + D] = y_i[n]: the delayed copy read back at the true delay
        full = float(np.sum(np.abs(yi) ** 2))
        s0, s1 = 16, N - 16                      # stay clear of the capture ends
        yi_w = np.zeros(N, complex)
        yi_w[s0:s1] = yi[s0:s1]
        c_sinc = oracle.corr(yi_w, yj, 0, N, D, 0.0, fs, oracle.SINC)
        c_lin = oracle.corr(yi_w, yj, 0, N, D, 0.0, fs, oracle.LINEAR)
        ref = float(np.sum(np.abs(yi_w) ** 2))
        assert abs(abs(c_sinc) / ref - 1.0) < 1e-3, (D, abs(c_sinc) / ref)
        # LINEAR reads each tone through G_f = exp(-j 2 pi f a / fs) ((1 - a) + a exp(j 2 pi f / fs))
        a = D - np.floor(D)
        G = np.exp(-2j * np.pi * freqs * a / fs) * ((1 - a) + a * np.exp(2j * np.pi * freqs / fs))
        lin_pred = abs(np.sum(amps ** 2 * np.conj(G))) * (s1 - s0)
        assert abs(abs(c_lin) - lin_pred) <= 2e-2 * ref, (D, abs(c_lin), lin_pred)
        if abs(a - 0.5) < 1e-9:
            assert np.min(np.abs(G)) < 0.74          # about -2.7 dB at 0.24 of the sample rate
        assert full > 0


def test_p16_sinc_caf_on_bin_equals_direct():
    """Eq. (11) with the windowed-sinc delay is linear in y_j, so the CAF table read with the
    same eight taps reproduces the direct SINC correlation whenever nu falls on a bin."""
    rng = _rng(161)
    N, L, fs = 3000, 1000, 1.0e6
    yi, yj = _cn(rng, N), _cn(rng, N)
    nu_b = caf.bins(-900.0, 600.0, 16)
    lag_lo, n_lags = -12, 30
    for k in range(3):
        T = caf.table(yi, yj, k, L, fs, lag_lo, n_lags, nu_b)
        for D, m in ((3.37, 4), (-5.81, 11), (0.5, 0), (7.0, 15)):
            c_dir = oracle.corr(yi, yj, k, L, D, nu_b[m], fs, oracle.SINC)
            dnu = nu_b[1] - nu_b[0]
            c_caf = caf.interp(T, lag_lo, nu_b[0], dnu, np.array([D]), np.array([nu_b[m]]), oracle.SINC)[0]
            assert abs(c_caf - c_dir) <= 1e-9 * max(1.0, abs(c_dir)), (k, D, m)


# WGS-84 ellipsoid (the grid -> ECEF step with a terrain height per point)
WGS_A = 6378137.0
WGS_F = 1.0 / 298.257223563
WGS_B = WGS_A * (1.0 - WGS_F)


def test_p17_wgs84_closed_forms():
    """Equator, 90 deg east and the poles land on the semi-axes, plus the height."""
    for h in (0.0, 1234.5, -80.0):
        x = oracle.ecef_wgs84([0.0, 0.0, math.pi / 2, -math.pi / 2], [0.0, math.pi / 2, 0.3, -1.1], h)
        assert np.allclose(x[0], [WGS_A + h, 0, 0], rtol=0, atol=1e-6)
        assert np.allclose(x[1], [0, WGS_A + h, 0], rtol=0, atol=1e-6)
        assert np.allclose(x[2], [0, 0, WGS_B + h], rtol=0, atol=1e-6)
        assert np.allclose(x[3], [0, 0, -(WGS_B + h)], rtol=0, atol=1e-6)


def test_p17_wgs84_surface_normal_and_height():
    """h = 0 lies on the ellipsoid x^2/a^2 + y^2/a^2 + z^2/b^2 = 1; the surface normal there
    (the gradient of that form) points along (cos lat cos lon, cos lat sin lon, sin lat), the
    definition of geodetic latitude; a height h moves the point h metres along it."""
    rng = _rng(17)
    lat = rng.uniform(-1.5, 1.5, 200)
    lon = rng.uniform(-math.pi, math.pi, 200)
    x0 = oracle.ecef_wgs84(lat, lon, 0.0)
    q = (x0[:, 0] ** 2 + x0[:, 1] ** 2) / WGS_A ** 2 + x0[:, 2] ** 2 / WGS_B ** 2
    assert np.max(np.abs(q - 1.0)) < 1e-14
    n = np.stack([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)], axis=1)
    g = np.stack([x0[:, 0] / WGS_A ** 2, x0[:, 1] / WGS_A ** 2, x0[:, 2] / WGS_B ** 2], axis=1)
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    assert np.max(np.abs(g - n)) < 1e-13
    h = rng.uniform(-400.0, 8800.0, 200)
    xh = oracle.ecef_wgs84(lat, lon, h)
    assert np.max(np.abs(xh - x0 - h[:, None] * n)) < 1e-7


def test_p17_wgs84_inverse_by_iteration_recovers_the_input():
    """An independent inverse (fixed-point iteration on latitude and height) returns the
    geodetic coordinates the forward map started from."""
    rng = _rng(18)
    lat = rng.uniform(-1.55, 1.55, 300)
    lon = rng.uniform(-math.pi, math.pi, 300)
    h = rng.uniform(-400.0, 9000.0, 300)
    x = oracle.ecef_wgs84(lat, lon, h)
    e2 = WGS_F * (2 - WGS_F)
    p = np.hypot(x[:, 0], x[:, 1])
    lo = np.arctan2(x[:, 1], x[:, 0])
    la = np.arctan2(x[:, 2], p * (1 - e2))
    hh = np.zeros_like(p)
    for _ in range(30):
        N = WGS_A / np.sqrt(1 - e2 * np.sin(la) ** 2)
        hh = p / np.cos(la) - N
        la = np.arctan2(x[:, 2], p * (1 - e2 * N / (N + hh)))
    assert np.max(np.abs(la - lat)) < 1e-12
    assert np.max(np.abs(np.angle(np.exp(1j * (lo - lon))))) < 1e-12
    assert np.max(np.abs(hh - h)) < 1e-6


def test_p17_map_at_ecef_points_equals_map_at_grid_points():
    """The ECEF-input map at the sphere's own ECEF points is the grid map."""
    wl = configs.SMALL.with_(n_rows=5, n_cols=6, n_samples=4000, step_len=2000)
    scn = sim.make_scenario(wl, 2)
    la, lo = sim.points_of(scn)
    Jg = oracle.map_points(la, lo, scn.captures, scn.states, wl.step_len, wl.fs_hz, wl.fc_hz,
                           pairs=list(wl.pairs), radius=wl.earth_radius_m)
    Jx = oracle.map_xyz(oracle.grid_ecef(la, lo, wl.earth_radius_m), scn.captures, scn.states, wl.step_len,
                        wl.fs_hz, wl.fc_hz, pairs=list(wl.pairs))
    assert np.array_equal(Jg, Jx)
