"""FP64 CPU oracle of the position-domain correlation map -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It shares no code with the GPU library
(``paper_2508_06672_amd``) and never imports it.

Contents
  * ``geoloc_oracle.c`` (built to ``liboracle.so`` with gcc, -O2 -fopenmp
    -ffp-contract=off): grid -> ECEF (sphere, or the WGS-84 ellipsoid with a
    height per point), geometry (Eq. (3)-(9)), one correlation
    (Eq. (11)) with a ROUND, LINEAR or eight-tap windowed-sinc delay, the full map
    (Algorithm 1, accumulated over steps and pairs).
  * ``caf.py``: the FP64 CAF-table form of Eq. (11) (lag-product matrix times a
    Doppler phasor matrix, then bilinear interpolation in lag and Doppler).
  * ``brute.py``: Eq. (11) written as literal Python loops, for tiny inputs.
  * ``peaks.py``: argmax / top-k with non-maximum suppression.
  * ``cfar.py``: cell-averaging CFAR detection of several emitters.
  * ``cnn.py``: FP64 forward / backward / Adam of the tile-proposal CNN.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

LINEAR, ROUND, SINC = 0, 1, 2
POWER, MAG = 0, 1

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from .build import build
            build()
        lib = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        ip = ctypes.POINTER(ctypes.c_int32)
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.oracle_grid_ecef.argtypes = [i64, dp, dp, f64, f64, dp]
        lib.oracle_geometry.argtypes = [i64, dp, i32, i32, dp, i32, i32, f64, f64, dp, dp]
        lib.oracle_corr.argtypes = [fp, fp, i64, i64, i64, f64, f64, f64, i32, dp, dp]
        lib.oracle_map.argtypes = [i64, dp, dp, f64, f64, i32, i64, i64, fp, dp, i32, ip, f64, f64, i32, i32, dp]
        lib.oracle_sinc_taps.argtypes = [f64, dp]
        lib.oracle_ecef_wgs84.argtypes = [i64, dp, dp, dp, dp]
        lib.oracle_map_xyz.argtypes = [i64, dp, i32, i64, i64, fp, dp, i32, ip, f64, f64, i32, i32, dp]
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


class use_library:
    """Context manager that points every oracle call at another build of geoloc_oracle.c
    (used by the tests that plant mistakes in the oracle to show that the pins catch them)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self._saved = _load()
        _lib = None
        saved_path = globals()["LIB_PATH"]
        globals()["LIB_PATH"] = self.path
        try:
            _load()
        finally:
            globals()["LIB_PATH"] = saved_path
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fptr(a: np.ndarray):
    assert a.dtype == np.float32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def sinc_taps(alpha: float) -> np.ndarray:
    """The eight SINC-mode weights for fractional delay alpha (taps -3 .. 4 around floor(D))."""
    w = np.empty(8)
    _load().oracle_sinc_taps(float(alpha), _dptr(w))
    return w


def grid_ecef(lat, lon, radius: float = 6371.0e3, alt: float = 0.0) -> np.ndarray:
    lat = np.ascontiguousarray(lat, dtype=np.float64).ravel()
    lon = np.ascontiguousarray(lon, dtype=np.float64).ravel()
    out = np.empty((lat.size, 3))
    _load().oracle_grid_ecef(lat.size, _dptr(lat), _dptr(lon), radius, alt, _dptr(out))
    return out


def ecef_wgs84(lat, lon, h) -> np.ndarray:
    """Geodetic latitude / longitude (radians) and height above the WGS-84 ellipsoid (m,
    one per point or a scalar) to ECEF [n][3]."""
    lat = np.ascontiguousarray(lat, dtype=np.float64).ravel()
    lon = np.ascontiguousarray(lon, dtype=np.float64).ravel()
    h = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), lat.shape))
    out = np.empty((lat.size, 3))
    _load().oracle_ecef_wgs84(lat.size, _dptr(lat), _dptr(lon), _dptr(h), _dptr(out))
    return out


def map_xyz(xyz, captures: np.ndarray, states: np.ndarray, step_len: int, fs: float, fc: float,
            pairs: Optional[Sequence[Tuple[int, int]]] = None, delay_mode: int = LINEAR,
            accum_mode: int = POWER) -> np.ndarray:
    """J at candidate points given in ECEF (m)."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    caps = np.ascontiguousarray(captures, dtype=np.complex64)
    R, N = caps.shape
    if pairs is None:
        pairs = [(i, j) for i in range(R) for j in range(i + 1, R)]
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    st = np.ascontiguousarray(states, dtype=np.float64)
    assert st.shape == (N // step_len, R, 6)
    J = np.empty(xyz.shape[0])
    _load().oracle_map_xyz(xyz.shape[0], _dptr(xyz), R, N, step_len, _fptr(caps.view(np.float32)), _dptr(st),
                           pr.shape[0], pr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), fs, fc, delay_mode,
                           accum_mode, _dptr(J))
    return J


def geometry(xyz: np.ndarray, states: np.ndarray, pair: Tuple[int, int], fs: float, fc: float):
    """(D [K][P] in samples, nu [K][P] in Hz) for one pair."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    states = np.ascontiguousarray(states, dtype=np.float64)
    K, R, _ = states.shape
    P = xyz.shape[0]
    D = np.empty((K, P))
    nu = np.empty((K, P))
    _load().oracle_geometry(P, _dptr(xyz), K, R, _dptr(states), int(pair[0]), int(pair[1]), fs, fc,
                            _dptr(D), _dptr(nu))
    return D, nu


def _c64_as_f32(y: np.ndarray) -> np.ndarray:
    y = np.ascontiguousarray(y, dtype=np.complex64)
    return y.view(np.float32)


def corr(yi: np.ndarray, yj: np.ndarray, k: int, step_len: int, D: float, nu: float, fs: float,
         delay_mode: int = LINEAR) -> complex:
    """One correlation C_k (Eq. (11)) for a given delay D (samples) and FDOA nu (Hz)."""
    a, b = _c64_as_f32(yi), _c64_as_f32(yj)
    assert yi.size == yj.size
    cr, ci = ctypes.c_double(), ctypes.c_double()
    _load().oracle_corr(_fptr(a), _fptr(b), yi.size, k, step_len, float(D), float(nu), fs, delay_mode,
                        ctypes.byref(cr), ctypes.byref(ci))
    return complex(cr.value, ci.value)


def map_points(lat_p, lon_p, captures: np.ndarray, states: np.ndarray, step_len: int, fs: float, fc: float,
               pairs: Optional[Sequence[Tuple[int, int]]] = None, radius: float = 6371.0e3, alt: float = 0.0,
               delay_mode: int = LINEAR, accum_mode: int = POWER) -> np.ndarray:
    """J at an explicit list of points (lat_p, lon_p radians). Returns float64 [P]."""
    lat_p = np.ascontiguousarray(lat_p, dtype=np.float64).ravel()
    lon_p = np.ascontiguousarray(lon_p, dtype=np.float64).ravel()
    caps = np.ascontiguousarray(captures, dtype=np.complex64)
    R, N = caps.shape
    if pairs is None:
        pairs = [(i, j) for i in range(R) for j in range(i + 1, R)]
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    st = np.ascontiguousarray(states, dtype=np.float64)
    assert st.shape == (N // step_len, R, 6)
    J = np.empty(lat_p.size)
    _load().oracle_map(lat_p.size, _dptr(lat_p), _dptr(lon_p), radius, alt, R, N, step_len,
                       _fptr(caps.view(np.float32)), _dptr(st), pr.shape[0],
                       pr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), fs, fc, delay_mode, accum_mode, _dptr(J))
    return J


def map_rect(lat, lon, captures, states, step_len, fs, fc, **kw) -> np.ndarray:
    """J on a rectilinear grid, flat index row * n_cols + col (rows = latitude)."""
    la, lo = np.meshgrid(np.asarray(lat, dtype=np.float64), np.asarray(lon, dtype=np.float64), indexing="ij")
    return map_points(la.ravel(), lo.ravel(), captures, states, step_len, fs, fc, **kw)


def map_scenario(scn, **kw) -> np.ndarray:
    wl = scn.workload
    return map_rect(scn.lat, scn.lon, scn.captures, scn.states, wl.step_len, wl.fs_hz, wl.fc_hz,
                    pairs=list(wl.pairs), radius=wl.earth_radius_m, **kw)
