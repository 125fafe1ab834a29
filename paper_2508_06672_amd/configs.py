"""Workload descriptions for direct geolocation of an interference emitter from LEO.

Each workload is a frozen dataclass naming the orbit, the grid, the capture and
the emitter waveform. The scenario simulator (``sim.py``) turns a workload and
a seed into synthetic inputs; nothing here computes any part of the method.

The paper's own scenario (Sec. IV-B: two LEO receivers, 5 MHz complex captures
at the GPS L1 carrier, chirp / tone / sawtooth / C/A emitters) is the model for
the structure of these inputs; its exact orbits and SNR are not printed, so the
sizes below are the ones this library is measured on.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Tuple

GPS_L1_HZ = 1575.42e6          # carrier used throughout the paper (Sec. IV-B)


@dataclass(frozen=True)
class Workload:
    name: str
    # orbit (circular, non-rotating spherical Earth)
    earth_radius_m: float = 6371.0e3
    orbit_alt_m: float = 550.0e3
    inclination_deg: float = 53.0
    rx_along_track_m: Tuple[float, ...] = (-25.0e3, 25.0e3)   # arc offsets from the formation midpoint
    rx_cross_track_m: Tuple[float, ...] | None = None           # offsets along the orbit normal (None -> 0)
    # grid (rectilinear lat/lon centred on the mid-capture sub-satellite point)
    n_rows: int = 101
    n_cols: int = 101
    spacing_m: float = 1000.0
    # capture
    fs_hz: float = 2.0e6
    fc_hz: float = GPS_L1_HZ
    n_samples: int = 20000
    step_len: int = 4000
    # emitter
    waveform: str = "chirp+gauss"      # tone | chirp | chirp+gauss | gauss | tone|chirp | sawtooth
    chirp_bw_hz: float = 1.0e6
    chirp_period_s: float = 10e-6
    tone_offset_max_hz: float = 0.0
    gauss_bw_hz: float = 0.0           # 0 -> full band (fs)
    snr_db: float = -5.0
    snr_db_range: Tuple[float, float] | None = None
    n_emitters: int = 1
    pairs: Tuple[Tuple[int, int], ...] = ((0, 1),)
    # separate captures (snapshots) of n_samples each, their centres spaced in time; the
    # map of a scenario accumulates over them (Sec. IV-B: 58 captures 1 s apart)
    n_snapshots: int = 1
    snapshot_spacing_s: float = 0.0

    @property
    def n_steps(self) -> int:
        return self.n_samples // self.step_len

    @property
    def n_points(self) -> int:
        return self.n_rows * self.n_cols

    @property
    def n_rx(self) -> int:
        return len(self.rx_along_track_m)

    @property
    def units(self) -> int:
        """grid-point x sample correlations in one full map (all snapshots)."""
        return self.n_points * self.n_samples * len(self.pairs) * self.n_snapshots

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# 101 x 101 grid at 1 km, 2 MHz, 10 ms in 5 steps; chirp (1 MHz / 10 us) plus unit
# Gaussian at -5 dB per receiver.  Small enough for the FP64 oracle in seconds.
SMALL = Workload(name="small_101x101_2MHz_20k")

# 1000 x 1000 grid at 0.5 km (1e6 points), 10 MHz, 100 ms in 100 steps of 10,000;
# tone at a random offset in +-500 kHz or a chirp, 50/50 by seed, at -15 dB.
MAP_1E6 = Workload(
    name="map_1000x1000_10MHz_1e6",
    n_rows=1000, n_cols=1000, spacing_m=500.0,
    fs_hz=10.0e6, n_samples=1_000_000, step_len=10_000,
    waveform="tone|chirp", tone_offset_max_hz=500e3, snr_db=-15.0,
)

# CAF-table comparison on the small scenario re-cut into 2 steps of 10,000 samples
# (512 lags x 256 Doppler bins per step).
CAF_SMALL = SMALL.with_(name="caf_small_101x101_2x10k", step_len=10_000)
CAF_LAGS = 512
CAF_BINS = 256
CAF_LITERAL_WINDOW_HZ = (-40e3, 40e3)

# Learned proposal: 1024 x 1024 fine grid at 0.5 km, 64 x 64 coarse cells of 8 km; 10 separate
# 10 ms captures (one coherent step each) 4 s apart, so that the changing geometry turns the
# single-capture delay / Doppler ridges into a peak (Sec. IV-B accumulates 58 captures 1 s apart).
PROPOSAL = MAP_1E6.with_(
    name="proposal_1024x1024_10MHz_10x10ms",
    n_rows=1024, n_cols=1024, waveform="tone|chirp|gauss",
    snr_db=-10.0, snr_db_range=(-20.0, 0.0),
    n_samples=100_000, step_len=100_000, n_snapshots=10, snapshot_spacing_s=4.0,
)
# The learned-proposal workload exactly as first specified: one contiguous 100 ms capture of
# the 1e6-point map's kind (100 coherent steps of 1 ms) on the 1024 x 1024 grid. Its map is a
# delay ridge whose maximum along the ridge is set by the noise, so it is evaluated beside
# PROPOSAL (whose network was trained on PROPOSAL), not trained on.
PROPOSAL_C4 = MAP_1E6.with_(
    name="proposal_c4_1024x1024_10MHz_1x100ms",
    n_rows=1024, n_cols=1024, waveform="tone|chirp|gauss",
    snr_db=-10.0, snr_db_range=(-20.0, 0.0),
)
PROPOSAL_COARSE = 64
PROPOSAL_TILE = 16
PROPOSAL_TOPK = 16

# Continental footprint: 4000 x 4000 at 0.5 km, 3 receivers 40 km apart, 20 MHz,
# 200 ms in 200 steps, chirp (10 MHz / 10 us) plus 10 MHz Gaussian, -20 dB.
CONTINENTAL = Workload(
    name="continental_4000x4000_20MHz_4e6",
    rx_along_track_m=(-40.0e3, 0.0, 40.0e3),
    n_rows=4000, n_cols=4000, spacing_m=500.0,
    fs_hz=20.0e6, n_samples=4_000_000, step_len=20_000,
    waveform="chirp+gauss", chirp_bw_hz=10e6, gauss_bw_hz=10e6, snr_db=-20.0,
    n_emitters=2, pairs=((0, 1), (0, 2), (1, 2)),
)

# The multi-capture scenario of Sec. IV-B: 58 captures of 50 ms at 5 MHz, 1 s apart, each
# correlated coherently as one step and accumulated; four emitters in a rectangle (a
# spread-spectrum stand-in for the L1 C/A spoofer, a tone at the carrier, a 2 MHz / 20 us
# chirp and a 200 kHz / 5 ms sawtooth, equal power; see sim.paper_formation). The receivers
# fly 50 km apart along track with a 30 km cross-track offset (two neighbouring orbital
# planes), which removes the exact mirror twin of every peak; 1000 x 450 cells at 1 km.
PAPER_IVB = Workload(
    name="paper_58x50ms_5MHz",
    rx_along_track_m=(-25.0e3, 25.0e3), rx_cross_track_m=(0.0, 30.0e3),
    n_rows=450, n_cols=1000, spacing_m=1000.0,
    fs_hz=5.0e6, n_samples=250_000, step_len=250_000, n_snapshots=58, snapshot_spacing_s=1.0,
    waveform="tone", snr_db=-10.0, n_emitters=4,
)

ALL = {w.name: w for w in (SMALL, MAP_1E6, CAF_SMALL, PROPOSAL, CONTINENTAL, PAPER_IVB)}
