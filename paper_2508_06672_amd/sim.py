"""Seeded scenario simulator: receivers in LEO, one or more ground emitters, raw captures.

This module only generates inputs. It computes the physics of the capture
(orbits, the true propagation delay and carrier phase of each emitter at each
receiver, receiver noise) and the lat/lon grid to search. It holds none of the
method's arithmetic: no candidate-point geometry, no correlation, no map.

Signal model (Sec. II-A, Eq. (1)-(2); exact form): the sample received by
receiver i at time t_n = n / f_s is

    y_i[n] = sum_e x_e(t_n - tau_ie(t_n)) * exp(-j 2 pi f_c tau_ie(t_n)) + w_i[n]

with tau_ie(t) = |p_i(t) - p_e| / c at the reception time (exact for a static
emitter in a non-rotating frame). The time-varying delay contains the Doppler
shift of Eq. (6) implicitly: -f_c d(tau)/dt = -(1/lambda) d(rho)/dt.

Waveforms (Sec. IV-A): pure tone, the chirp of Eq. (12) repeated with its
period, the sawtooth (chirp followed by its conjugate), and band-limited complex
Gaussian noise evaluated at arbitrary times with a windowed-sinc interpolator.

Orbits: circular, inclination 53 deg, ascending node on the +x axis, the
receivers spaced along track by arc length (optionally displaced along the
orbit normal by a constant offset); the Earth is a non-rotating sphere,
so ECEF and inertial axes coincide.  Receiver states handed to the method are
the exact orbit states at each step's centre time t_0 + (kL + (L-1)/2) / f_s.

Random numbers: numpy PCG64 seeded by SeedSequence(seed), spawned in the fixed
order [geometry, emitter, waveform, noise rx0, noise rx1, noise rx2, ...].
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Tuple

import numpy as np

from .configs import Workload

C_LIGHT = 299_792_458.0
MU_EARTH = 3.986004418e14


@dataclass
class Emitter:
    lat: float
    lon: float
    waveform: str
    tone_hz: float = 0.0
    power: float = 1.0
    bw_hz: float = 0.0          # chirp / sawtooth sweep (0: the workload's)
    period_s: float = 0.0       # chirp / sawtooth period (0: the workload's)
    code_seed: int = 0          # bpsk: seed of its spreading and data bits
    ecef: Optional[Tuple[float, float, float]] = None   # position (m); None: on the sphere at (lat, lon)


@dataclass
class Scenario:
    workload: Workload
    seed: int
    lat: np.ndarray            # [n_rows] radians
    lon: np.ndarray            # [n_cols] radians
    states: np.ndarray         # [K][n_rx][6] float64, ECEF position (m) and velocity (m/s)
    captures: np.ndarray       # [n_rx][N] complex64
    emitters: List[Emitter]
    true_cells: List[Tuple[int, int]]
    mirror_cells: List[Tuple[int, int]]
    noise_var: float
    snr_db: float
    u_mid: float

    @property
    def n_points(self) -> int:
        return self.lat.size * self.lon.size


# ----------------------------------------------------------------------------- orbits

def _orbit_frame(inc: float):
    node = np.array([1.0, 0.0, 0.0])
    inplane = np.array([0.0, math.cos(inc), math.sin(inc)])
    normal = np.cross(node, inplane)
    return node, inplane, normal


def receiver_states(wl: Workload, u_mid: float, t_rel: np.ndarray) -> np.ndarray:
    """Exact circular-orbit states at times t_rel (s, relative to mid-capture).

    Returns [len(t_rel)][n_rx][6]."""
    r = wl.earth_radius_m + wl.orbit_alt_m
    v = math.sqrt(MU_EARTH / r)
    w = v / r
    node, inplane, normal = _orbit_frame(math.radians(wl.inclination_deg))
    t_rel = np.asarray(t_rel, dtype=np.float64)
    out = np.empty((t_rel.size, wl.n_rx, 6))
    cross = wl.rx_cross_track_m or (0.0,) * wl.n_rx
    for i, s in enumerate(wl.rx_along_track_m):
        u = u_mid + s / r + w * t_rel
        cu, su = np.cos(u), np.sin(u)
        out[:, i, 0:3] = r * (cu[:, None] * node + su[:, None] * inplane) + cross[i] * normal
        out[:, i, 3:6] = v * (-su[:, None] * node + cu[:, None] * inplane)
    return out


def step_centre_times(wl: Workload) -> np.ndarray:
    """Step reference instants relative to mid-capture (centre of each step)."""
    k = np.arange(wl.n_steps, dtype=np.float64)
    t_abs = (k * wl.step_len + (wl.step_len - 1) / 2.0) / wl.fs_hz
    return t_abs - (wl.n_samples - 1) / (2.0 * wl.fs_hz)


def _latlon_of(p: np.ndarray) -> Tuple[float, float]:
    return math.asin(p[2] / np.linalg.norm(p)), math.atan2(p[1], p[0])


def _surface(lat: float, lon: float, radius: float) -> np.ndarray:
    return radius * np.array([math.cos(lat) * math.cos(lon), math.cos(lat) * math.sin(lon), math.sin(lat)])


# ----------------------------------------------------------------------------- grid

def make_grid(wl: Workload, u_mid: float):
    """Rectilinear lat/lon grid centred on the sub-satellite point of the formation
    midpoint at mid-capture; spacing is exact in km at the centre latitude."""
    r = wl.earth_radius_m + wl.orbit_alt_m
    node, inplane, _ = _orbit_frame(math.radians(wl.inclination_deg))
    p_mid = r * (math.cos(u_mid) * node + math.sin(u_mid) * inplane)
    lat_c, lon_c = _latlon_of(p_mid)
    dlat = wl.spacing_m / wl.earth_radius_m
    dlon = wl.spacing_m / (wl.earth_radius_m * math.cos(lat_c))
    lat = lat_c + (np.arange(wl.n_rows) - (wl.n_rows - 1) / 2.0) * dlat
    lon = lon_c + (np.arange(wl.n_cols) - (wl.n_cols - 1) / 2.0) * dlon
    return lat, lon


def nearest_cell(lat: np.ndarray, lon: np.ndarray, la: float, lo: float) -> Tuple[int, int]:
    dlat = lat[1] - lat[0] if lat.size > 1 else 1.0
    dlon = lon[1] - lon[0] if lon.size > 1 else 1.0
    row = int(np.clip(round((la - lat[0]) / dlat), 0, lat.size - 1))
    col = int(np.clip(round((lo - lon[0]) / dlon), 0, lon.size - 1))
    return row, col


def mirror_latlon(wl: Workload, la: float, lo: float) -> Tuple[float, float]:
    """Reflection of a surface point through the receivers' orbital plane."""
    _, _, n = _orbit_frame(math.radians(wl.inclination_deg))
    p = _surface(la, lo, wl.earth_radius_m)
    m = p - 2.0 * np.dot(p, n) * n
    return _latlon_of(m)


# ----------------------------------------------------------------------------- waveforms

def chirp(t: np.ndarray, bw: float, period: float) -> np.ndarray:
    """Eq. (12) repeated with period T: sweeps -B/2 -> +B/2 over each period."""
    tp = np.mod(t, period)
    ph = (bw / (2.0 * period)) * tp * tp - 0.5 * bw * tp          # cycles
    return np.exp(2j * np.pi * np.mod(ph, 1.0))


def sawtooth(t: np.ndarray, bw: float, period: float) -> np.ndarray:
    """Chirp followed by its complex conjugate; full period 2T."""
    tp = np.mod(t, 2.0 * period)
    up = tp < period
    out = chirp(np.where(up, tp, tp - period), bw, period)
    return np.where(up, out, np.conj(out))


def tone(t: np.ndarray, f0: float) -> np.ndarray:
    return np.exp(2j * np.pi * np.mod(f0 * t, 1.0))


def bpsk(t: np.ndarray, seed: int, chip_rate: float = 1.023e6, n_chips: int = 1023, bit_rate: float = 50.0,
         n_bits: int = 1500) -> np.ndarray:
    """Spread-spectrum stand-in for a GPS L1 C/A-like signal (Sec. IV-A): a seeded random
    +-1 code of n_chips chips at chip_rate, repeating every n_chips / chip_rate seconds,
    times seeded random +-1 data bits at bit_rate (n_bits of them, then repeating). The
    published C/A Gold codes are not used."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    code = rng.choice(np.array([-1.0, 1.0]), n_chips)
    data = rng.choice(np.array([-1.0, 1.0]), n_bits)
    t = np.asarray(t, dtype=np.float64)
    ci = np.mod(np.floor(t * chip_rate).astype(np.int64), n_chips)
    bi = np.mod(np.floor(t * bit_rate).astype(np.int64), n_bits)
    return (code[ci] * data[bi]).astype(np.complex128)


class BandlimitedGaussian:
    """Complex Gaussian noise of unit power, band-limited to |f| < bw/2, defined on
    continuous time through a 32-tap Kaiser-windowed sinc interpolator."""

    HALF = 16
    BETA = 9.0

    def __init__(self, rng: np.random.Generator, fs: float, m_lo: int, m_hi: int, bw: float = 0.0):
        self.fs = fs
        self.m_lo = m_lo - self.HALF - 1
        n = (m_hi + self.HALF + 1) - self.m_lo + 1
        g = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / math.sqrt(2.0)
        if bw and bw < fs:
            spec = np.fft.fft(g)
            f = np.fft.fftfreq(n, d=1.0 / fs)
            spec[np.abs(f) >= bw / 2.0] = 0.0
            g = np.fft.ifft(spec)
            g /= math.sqrt(np.mean(np.abs(g) ** 2))
        self.g = g

    # the Kaiser window w(z) = I0(beta sqrt(1 - (z / HALF)^2)) / I0(beta), tabulated every
    # 1/8192 sample and read by linear interpolation (error below 1e-9, under the complex64
    # rounding of the samples)
    _TABLE_STEP = 8192
    _window = None

    @classmethod
    def _window_table(cls) -> np.ndarray:
        if cls._window is None:
            z = np.arange(-cls.HALF * cls._TABLE_STEP, cls.HALF * cls._TABLE_STEP + 2) / cls._TABLE_STEP
            a = np.clip(1.0 - (z / cls.HALF) ** 2, 0.0, None)
            cls._window = np.i0(cls.BETA * np.sqrt(a)) / np.i0(cls.BETA)
        return cls._window

    def __call__(self, t: np.ndarray, chunk: int = 1 << 18) -> np.ndarray:
        u = np.asarray(t, dtype=np.float64) * self.fs
        out = np.empty(u.shape, dtype=np.complex128)
        tab = self._window_table()
        for s in range(0, u.size, chunk):
            uu = u[s:s + chunk]
            base = np.floor(uu).astype(np.int64)
            fr = uu - base
            # sinc(fr - q) = (-1)^q sin(pi fr) / (pi (fr - q)): one sine per sample for all taps;
            # sin(pi fr) is taken as sin(pi (1 - fr)) above one half, where 1 - fr is exact, so it
            # keeps its relative accuracy as fr approaches 1
            sn = np.sin(np.pi * np.where(fr > 0.5, 1.0 - fr, fr))
            acc = np.zeros(uu.shape, dtype=np.complex128)
            for q in range(-self.HALF + 1, self.HALF + 1):
                z = fr - q
                with np.errstate(divide="ignore", invalid="ignore"):
                    sc = np.where(z == 0.0, 1.0, (-1.0 if q & 1 else 1.0) * sn / (np.pi * z))
                x = (z + self.HALF) * self._TABLE_STEP
                i = np.floor(x).astype(np.int64)
                f = x - i
                w = tab[i] + f * (tab[i + 1] - tab[i])
                acc += self.g[base + q - self.m_lo] * (sc * w)
            out[s:s + chunk] = acc
        return out


# ----------------------------------------------------------------------------- scenario

def _pick_waveform(wl: Workload, rng: np.random.Generator) -> str:
    if "|" in wl.waveform:
        opts = wl.waveform.split("|")
        return opts[int(rng.integers(len(opts)))]
    return wl.waveform


def make_scenario(wl: Workload, seed: int, snr_db: Optional[float] = None, noiseless: bool = False,
                  emitter_latlon: Optional[List[Tuple[float, float]]] = None,
                  waveform: Optional[str] = None, t_offset_s: float = 0.0, stream: int = 0,
                  emitters: Optional[List[Emitter]] = None) -> Scenario:
    """One capture of n_samples centred t_offset_s after the reference instant of the
    seed's geometry. Geometry, emitter and SNR come from the seed alone; `stream` > 0
    draws the waveform and the receiver noise from a stream of their own (the separate
    snapshots of one scenario). `emitters` replaces the drawn emitters by given ones."""
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(3 + max(3, wl.n_rx))
    rng_geo, rng_em, rng_wave = (np.random.Generator(np.random.PCG64(k)) for k in kids[:3])
    rng_noise = [np.random.Generator(np.random.PCG64(k)) for k in kids[3:3 + wl.n_rx]]
    if stream:
        sk = np.random.SeedSequence(seed, spawn_key=(1_000_000 + int(stream),)).spawn(1 + wl.n_rx)
        rng_wave = np.random.Generator(np.random.PCG64(sk[0]))
        rng_noise = [np.random.Generator(np.random.PCG64(k)) for k in sk[1:]]

    u_mid = float(rng_geo.uniform(0.0, 2.0 * math.pi))
    lat, lon = make_grid(wl, u_mid)
    dlat = lat[1] - lat[0] if lat.size > 1 else 0.0
    dlon = lon[1] - lon[0] if lon.size > 1 else 0.0

    if snr_db is None:
        snr_db = float(rng_em.uniform(*wl.snr_db_range)) if wl.snr_db_range else wl.snr_db

    drawn: List[Emitter] = []
    for e in range(wl.n_emitters):
        if emitter_latlon is not None:
            la, lo = emitter_latlon[e]
        else:
            la = lat[0] + dlat * rng_em.uniform(1.0, max(1.0, lat.size - 2.0))
            lo = lon[0] + dlon * rng_em.uniform(1.0, max(1.0, lon.size - 2.0))
        wf = waveform or _pick_waveform(wl, rng_em)
        f0 = float(rng_em.uniform(-wl.tone_offset_max_hz, wl.tone_offset_max_hz)) if wl.tone_offset_max_hz else 0.0
        power = 2.0 if wf == "chirp+gauss" else 1.0
        drawn.append(Emitter(la, lo, wf, f0, power))
    if emitters is not None:
        emitters = list(emitters)
    else:
        emitters = drawn

    N, fs = wl.n_samples, wl.fs_hz
    t_abs = t_offset_s + np.arange(N, dtype=np.float64) / fs
    t_rel = t_abs - (N - 1) / (2.0 * fs)
    st = receiver_states(wl, u_mid, t_rel)                        # [N][R][6]

    y = np.zeros((wl.n_rx, N), dtype=np.complex128)
    for e, em in enumerate(emitters):
        pe = np.asarray(em.ecef, dtype=np.float64) if em.ecef is not None else _surface(em.lat, em.lon, wl.earth_radius_m)
        taus = [np.linalg.norm(st[:, i, 0:3] - pe, axis=1) / C_LIGHT for i in range(wl.n_rx)]
        gauss = None
        if "gauss" in em.waveform:
            lo_t = min(float(np.min(t_abs - tau)) for tau in taus)
            hi_t = max(float(np.max(t_abs - tau)) for tau in taus)
            gauss = BandlimitedGaussian(rng_wave, fs, int(math.floor(lo_t * fs)), int(math.ceil(hi_t * fs)),
                                        wl.gauss_bw_hz)
        for i in range(wl.n_rx):
            te = t_abs - taus[i]                                  # emission time of what arrives at t_n
            bw = em.bw_hz or wl.chirp_bw_hz
            period = em.period_s or wl.chirp_period_s
            if em.waveform == "tone":
                x = tone(te, em.tone_hz)
            elif em.waveform == "chirp":
                x = chirp(te, bw, period)
            elif em.waveform == "sawtooth":
                x = sawtooth(te, bw, period)
            elif em.waveform == "bpsk":
                x = bpsk(te, em.code_seed)
            elif em.waveform == "gauss":
                x = gauss(te)
            elif em.waveform == "chirp+gauss":
                x = chirp(te, wl.chirp_bw_hz, wl.chirp_period_s) + gauss(te)
            else:
                raise ValueError(f"unknown waveform {em.waveform!r}")
            carrier = np.exp(-2j * np.pi * np.mod(wl.fc_hz * taus[i], 1.0))
            y[i] += x * carrier

    p_ref = emitters[0].power
    noise_var = 0.0 if noiseless else p_ref * 10.0 ** (-snr_db / 10.0)
    if noise_var > 0:
        sd = math.sqrt(noise_var / 2.0)
        for i in range(wl.n_rx):
            g = rng_noise[i]
            y[i] += sd * (g.standard_normal(N) + 1j * g.standard_normal(N))

    states = receiver_states(wl, u_mid, t_offset_s + step_centre_times(wl))
    true_cells = [nearest_cell(lat, lon, em.lat, em.lon) for em in emitters]
    mirror_cells = [nearest_cell(lat, lon, *mirror_latlon(wl, em.lat, em.lon)) for em in emitters]
    return Scenario(wl, seed, lat, lon, states, np.ascontiguousarray(y.astype(np.complex64)),
                    emitters, true_cells, mirror_cells, noise_var, snr_db, u_mid)


def reference_grid(wl: Workload, seed: int):
    """(lat, lon, u_mid) of a seed's scenario without simulating it (the geometry stream's
    first draw, as in make_scenario)."""
    kids = np.random.SeedSequence(seed).spawn(3 + max(3, wl.n_rx))
    u_mid = float(np.random.Generator(np.random.PCG64(kids[0])).uniform(0.0, 2.0 * math.pi))
    lat, lon = make_grid(wl, u_mid)
    return lat, lon, u_mid


def paper_formation(wl: Workload, seed: int, d_rows: float = 100.4, d_cols: float = 250.3) -> List[Emitter]:
    """Four emitters at the corners of a rectangle centred on the grid (Sec. IV-B): a
    spread-spectrum stand-in for the L1 C/A spoofer, a tone at the carrier, a chirp of
    2 MHz and 20 us, and a sawtooth of 200 kHz and 5 ms, at equal power. Offsets in cells,
    deliberately off the grid nodes."""
    lat, lon, _ = reference_grid(wl, seed)
    dlat, dlon = lat[1] - lat[0], lon[1] - lon[0]
    r0, c0 = (lat.size - 1) / 2.0, (lon.size - 1) / 2.0
    spec = [("bpsk", -1, -1, 0.0, 0.0), ("tone", -1, 1, 0.0, 0.0), ("chirp", 1, -1, 2.0e6, 20e-6),
            ("sawtooth", 1, 1, 200e3, 5e-3)]
    out = []
    for i, (wf, sr, sc, bw, per) in enumerate(spec):
        out.append(Emitter(lat[0] + dlat * (r0 + sr * d_rows), lon[0] + dlon * (c0 + sc * d_cols), wf, 0.0, 1.0,
                           bw, per, code_seed=seed * 16 + i))
    return out


def snapshot_offsets(wl: Workload) -> np.ndarray:
    """Centre times of the snapshots relative to the reference instant, symmetric."""
    s = np.arange(wl.n_snapshots, dtype=np.float64)
    return (s - (wl.n_snapshots - 1) / 2.0) * wl.snapshot_spacing_s


def make_snapshots(wl: Workload, seed: int, **kw) -> List[Scenario]:
    """The wl.n_snapshots separate captures of one scenario (same grid, emitter and SNR;
    own waveform and noise draws, receivers further along their orbits). One snapshot
    is exactly make_scenario(wl, seed)."""
    if wl.n_snapshots == 1:
        return [make_scenario(wl, seed, **kw)]
    return [make_scenario(wl, seed, t_offset_s=float(t), stream=i + 1, **kw)
            for i, t in enumerate(snapshot_offsets(wl))]


def points_of(scn: Scenario) -> Tuple[np.ndarray, np.ndarray]:
    """Flattened (row-major, rows = latitude) lat/lon of every grid node."""
    la, lo = np.meshgrid(scn.lat, scn.lon, indexing="ij")
    return la.ravel().copy(), lo.ravel().copy()


def random_captures(n_rx: int, n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Independent CN(0, scale^2) captures, for tests that need arbitrary data."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    y = scale * (rng.standard_normal((n_rx, n)) + 1j * rng.standard_normal((n_rx, n))) / math.sqrt(2.0)
    return y.astype(np.complex64)
