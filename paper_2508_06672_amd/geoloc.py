"""ctypes binding of libgeoloc.so -- argument marshalling only.

The functions named ``geoloc_*`` mirror the C ABI in ``include/geoloc.h`` one to
one; ``Plan`` wraps them for torch device buffers (PyTorch provides device memory
and the stream; every step of the computation runs in the library's kernels).
If the library is not built, importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgeoloc.so")

ABI_VERSION = 4

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENAN, EUNSUPPORTED, ELAUNCH = 0, -1, -2, -3, -4, -5, -6, -7
DIRECT_FP32, CAF_BF16, CAF_FP16, DIRECT_FP32_POINTWISE = 0, 1, 2, 3
DELAY_LINEAR, DELAY_ROUND, DELAY_SINC = 0, 1, 2
ACC_POWER, ACC_MAG = 0, 1
GRID_RECT, GRID_POINTS = 0, 1
EARTH_SPHERE, EARTH_WGS84 = 0, 1
ACCUMULATE = 1


class GeolocError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (status {status})")
        self.status = status


_vp = ctypes.c_void_p


class geoloc_desc(ctypes.Structure):
    _fields_ = [
        ("n_rx", ctypes.c_int32), ("n_pairs", ctypes.c_int32), ("pairs", ctypes.POINTER(ctypes.c_int32)),
        ("n_samples", ctypes.c_int64), ("step_len", ctypes.c_int64),
        ("fs_hz", ctypes.c_double), ("fc_hz", ctypes.c_double),
        ("grid_kind", ctypes.c_int32), ("_pad0", ctypes.c_int32),
        ("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64),
        ("lat", ctypes.POINTER(ctypes.c_double)), ("lon", ctypes.POINTER(ctypes.c_double)),
        ("earth_radius_m", ctypes.c_double), ("alt_m", ctypes.c_double),
        ("method", ctypes.c_int32), ("delay_mode", ctypes.c_int32), ("accum_mode", ctypes.c_int32),
        ("caf_lags", ctypes.c_int32), ("caf_bins", ctypes.c_int32),
        ("caf_lag_lo_set", ctypes.c_int32), ("caf_lag_lo", ctypes.c_int32), ("_pad1", ctypes.c_int32),
        ("caf_nu_lo_hz", ctypes.c_double), ("caf_nu_hi_hz", ctypes.c_double),
        ("earth_model", ctypes.c_int32), ("_pad2", ctypes.c_int32), ("alt_grid", ctypes.POINTER(ctypes.c_double)),
    ]


class geoloc_inputs(ctypes.Structure):
    _fields_ = [("captures", _vp), ("rx_state", ctypes.POINTER(ctypes.c_double)), ("stream", _vp)]


class geoloc_plan_info(ctypes.Structure):
    _fields_ = [
        ("n_points", ctypes.c_int64), ("n_steps", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
        ("n_samples", ctypes.c_int64), ("step_len", ctypes.c_int64),
        ("method", ctypes.c_int32), ("delay_mode", ctypes.c_int32),
        ("caf_lag_lo", ctypes.c_int32), ("caf_lags", ctypes.c_int32), ("caf_bins", ctypes.c_int32),
        ("_pad", ctypes.c_int32),
        ("caf_nu_lo_hz", ctypes.c_double), ("caf_nu_hi_hz", ctypes.c_double),
        ("device_bytes", ctypes.c_int64), ("timed_maps", ctypes.c_int64), ("correlate_launches", ctypes.c_int64),
        ("geometry_ms", ctypes.c_double), ("correlate_ms", ctypes.c_double), ("interp_ms", ctypes.c_double),
        ("map_ms", ctypes.c_double),
        ("tile_rows", ctypes.c_int32), ("tile_cols", ctypes.c_int32), ("tile_shear", ctypes.c_int32),
        ("tile_transpose", ctypes.c_int32), ("step_segments", ctypes.c_int32), ("segment_len", ctypes.c_int32),
        ("taylor_block", ctypes.c_int32), ("_pad3", ctypes.c_int32),
    ]


class geoloc_cnn_desc(ctypes.Structure):
    _fields_ = [("in_ch", ctypes.c_int32), ("hidden", ctypes.c_int32), ("layers", ctypes.c_int32),
                ("height", ctypes.c_int32), ("width", ctypes.c_int32), ("max_batch", ctypes.c_int32)]


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.geoloc_abi_version.restype = ctypes.c_int
    lib.geoloc_plan.argtypes = [P(geoloc_desc), P(_vp)]
    lib.geoloc_set_timing.argtypes = [_vp, ctypes.c_int]
    lib.geoloc_set_grid.argtypes = [_vp, P(ctypes.c_double), P(ctypes.c_double)]
    lib.geoloc_map.argtypes = [_vp, P(geoloc_inputs), _vp, ctypes.c_uint32]
    lib.geoloc_geometry.argtypes = [_vp, P(geoloc_inputs), ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _vp, _vp]
    lib.geoloc_caf_table.argtypes = [_vp, P(geoloc_inputs), ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _vp,
                                     ctypes.c_int64]
    lib.geoloc_argmax.argtypes = [_vp, _vp, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_int64), P(ctypes.c_float), _vp]
    lib.geoloc_detect.argtypes = [_vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                  ctypes.c_int32, P(ctypes.c_int64), P(ctypes.c_float), P(ctypes.c_float),
                                  P(ctypes.c_int32), _vp]
    lib.geoloc_set_tiling.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.geoloc_set_taylor_block.argtypes = [_vp, ctypes.c_int32]
    lib.geoloc_set_points_from_tiles.argtypes = [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                                 P(ctypes.c_int32), ctypes.c_int32, _vp]
    lib.geoloc_info.argtypes = [_vp, P(geoloc_plan_info)]
    lib.geoloc_destroy.argtypes = [_vp]
    lib.geoloc_strerror.argtypes = [ctypes.c_int]
    lib.geoloc_strerror.restype = ctypes.c_char_p
    lib.geoloc_last_error.restype = ctypes.c_char_p
    lib.geoloc_subbands.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _vp, _vp]
    lib.geoloc_cfar_scale.argtypes = [ctypes.c_double, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_double)]
    lib.geoloc_argmax_noalloc.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_int32, P(ctypes.c_int64), P(ctypes.c_float), _vp]
    lib.geoloc_fma_probe.argtypes = [ctypes.c_int32, ctypes.c_int32, _vp, P(ctypes.c_int64), _vp]
    for name in ("geoloc_plan", "geoloc_set_timing", "geoloc_set_grid", "geoloc_map", "geoloc_geometry", "geoloc_caf_table", "geoloc_argmax",
                 "geoloc_detect", "geoloc_set_tiling", "geoloc_set_taylor_block", "geoloc_set_points_from_tiles", "geoloc_info", "geoloc_destroy",
                 "geoloc_subbands", "geoloc_cfar_scale", "geoloc_argmax_noalloc", "geoloc_fma_probe"):
        getattr(lib, name).restype = ctypes.c_int
    i32, i64, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    lib.geoloc_cnn_create.argtypes = [P(geoloc_cnn_desc), P(_vp)]
    lib.geoloc_cnn_param_count.argtypes = [_vp, P(i64)]
    lib.geoloc_cnn_set_params.argtypes = [_vp, P(f32), i64]
    lib.geoloc_cnn_get_params.argtypes = [_vp, i32, P(f32), i64]
    lib.geoloc_cnn_prepare.argtypes = [_vp, _vp, _vp, _vp, i32, _vp, _vp]
    lib.geoloc_cnn_forward.argtypes = [_vp, _vp, i32, _vp, _vp]
    lib.geoloc_cnn_loss.argtypes = [_vp, _vp, _vp, i32, _vp, _vp, _vp]
    lib.geoloc_cnn_backward.argtypes = [_vp, _vp, i32, _vp]
    lib.geoloc_cnn_adam_step.argtypes = [_vp, f32, f32, f32, f32, _vp]
    lib.geoloc_cnn_topk.argtypes = [_vp, _vp, i32, i32, P(i32), P(f32), _vp]
    lib.geoloc_cnn_destroy.argtypes = [_vp]
    for name in ("geoloc_cnn_create", "geoloc_cnn_param_count", "geoloc_cnn_set_params", "geoloc_cnn_get_params",
                 "geoloc_cnn_prepare", "geoloc_cnn_forward", "geoloc_cnn_loss", "geoloc_cnn_backward",
                 "geoloc_cnn_adam_step", "geoloc_cnn_topk", "geoloc_cnn_destroy"):
        getattr(lib, name).restype = ctypes.c_int
    if lib.geoloc_abi_version() != ABI_VERSION:
        raise ImportError(f"libgeoloc ABI {lib.geoloc_abi_version()} != binding ABI {ABI_VERSION}")
    _lib = lib
    return lib


def _check(status: int, where: str) -> None:
    if status != OK:
        raise GeolocError(status, where, geoloc_last_error())


# --------------------------------------------------------------------------- one-to-one calls

def geoloc_abi_version() -> int:
    return load().geoloc_abi_version()


def geoloc_strerror(status: int) -> str:
    return load().geoloc_strerror(status).decode()


def geoloc_last_error() -> str:
    return load().geoloc_last_error().decode()


def geoloc_plan(desc: geoloc_desc) -> int:
    h = _vp()
    _check(load().geoloc_plan(ctypes.byref(desc), ctypes.byref(h)), "geoloc_plan")
    return h.value


def geoloc_set_timing(plan: int, enable: bool) -> None:
    _check(load().geoloc_set_timing(plan, int(bool(enable))), "geoloc_set_timing")


def geoloc_set_grid(plan: int, lat: np.ndarray, lon: np.ndarray) -> None:
    la = np.ascontiguousarray(lat, dtype=np.float64)
    lo = np.ascontiguousarray(lon, dtype=np.float64)
    _check(load().geoloc_set_grid(plan, la.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  lo.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "geoloc_set_grid")


def geoloc_map(plan: int, inputs: geoloc_inputs, J_dev: int, flags: int = 0) -> None:
    _check(load().geoloc_map(plan, ctypes.byref(inputs), J_dev, flags), "geoloc_map")


def geoloc_geometry(plan: int, inputs: geoloc_inputs, pair_index: int, step_lo: int, n_steps: int,
                    D_dev: int, nu_dev: int) -> None:
    _check(load().geoloc_geometry(plan, ctypes.byref(inputs), pair_index, step_lo, n_steps, D_dev, nu_dev),
           "geoloc_geometry")


def geoloc_caf_table(plan: int, inputs: geoloc_inputs, pair_index: int, step_lo: int, n_steps: int, T_dev: int,
                     T_capacity: int) -> None:
    _check(load().geoloc_caf_table(plan, ctypes.byref(inputs), pair_index, step_lo, n_steps, T_dev, T_capacity),
           "geoloc_caf_table")


def geoloc_argmax(plan: int, J_dev: int, top_k: int, nms_radius: int, stream: int) -> Tuple[np.ndarray, np.ndarray]:
    idx = np.empty(top_k, dtype=np.int64)
    val = np.empty(top_k, dtype=np.float32)
    _check(load().geoloc_argmax(plan, J_dev, top_k, nms_radius,
                                idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                val.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), stream), "geoloc_argmax")
    return idx, val


def geoloc_argmax_noalloc(J_dev: int, grid_kind: int, n_rows: int, n_cols: int, top_k: int, nms_radius: int,
                          stream: int) -> Tuple[np.ndarray, np.ndarray]:
    idx = np.empty(top_k, dtype=np.int64)
    val = np.empty(top_k, dtype=np.float32)
    _check(load().geoloc_argmax_noalloc(J_dev, grid_kind, n_rows, n_cols, top_k, nms_radius,
                                        idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        val.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), stream),
           "geoloc_argmax_noalloc")
    return idx, val


def geoloc_detect(plan: int, J_dev: int, guard: int, train: int, scale: float, max_detections: int, nms_radius: int,
                  stream: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    idx = np.empty(max_detections, dtype=np.int64)
    val = np.empty(max_detections, dtype=np.float32)
    noise = np.empty(max_detections, dtype=np.float32)
    n = ctypes.c_int32(0)
    _check(load().geoloc_detect(plan, J_dev, guard, train, float(scale), max_detections, nms_radius,
                                idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                val.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                noise.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(n),
                                stream), "geoloc_detect")
    return idx[:n.value], val[:n.value], noise[:n.value]


def geoloc_cfar_scale(pfa: float, n_train: int, looks: int = 1) -> float:
    out = ctypes.c_double(0.0)
    _check(load().geoloc_cfar_scale(float(pfa), int(n_train), int(looks), ctypes.byref(out)), "geoloc_cfar_scale")
    return out.value


def geoloc_fma_probe(n_blocks: int, iters: int, out_ptr: int, stream: int = 0) -> int:
    """Launch the library's FP32 FMA issue-rate probe; returns the FMAs each lane runs."""
    n = ctypes.c_int64(0)
    _check(load().geoloc_fma_probe(int(n_blocks), int(iters), ctypes.c_void_p(out_ptr), ctypes.byref(n),
                                   ctypes.c_void_p(stream)), "geoloc_fma_probe")
    return n.value


def cfar_scale(pfa: float, n_train: int, looks: int = 1) -> float:
    """CFAR threshold scale for false-alarm probability pfa with n_train training cells of
    independent Gamma(looks) noise (computed by the library, geoloc_cfar_scale)."""
    return geoloc_cfar_scale(pfa, n_train, looks)


def cfar_training_cells(guard: int, train: int) -> int:
    """Training cells of an interior grid cell."""
    return (2 * train + 1) ** 2 - (2 * guard + 1) ** 2


def geoloc_info(plan: int) -> geoloc_plan_info:
    out = geoloc_plan_info()
    _check(load().geoloc_info(plan, ctypes.byref(out)), "geoloc_info")
    return out


def geoloc_destroy(plan: int) -> None:
    _check(load().geoloc_destroy(plan), "geoloc_destroy")


def geoloc_subbands(captures_dev: int, n_ch: int, n_samples: int, n_bands: int, half_taps: int, out_dev: int,
                    stream: int) -> None:
    _check(load().geoloc_subbands(captures_dev, n_ch, n_samples, n_bands, half_taps, out_dev, stream),
           "geoloc_subbands")


# --------------------------------------------------------------------------- torch-facing wrapper

def _stream_handle(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def subbands(captures, n_bands: int, half_taps: int, out=None, stream=None):
    """Sub-band split of complex64 CUDA captures [n_ch][N] -> [n_bands * n_ch][N / n_bands]
    (band-major: band b of channel c is row b * n_ch + c)."""
    import torch
    if captures.dtype != torch.complex64 or not captures.is_cuda or not captures.is_contiguous():
        raise ValueError("captures must be a contiguous complex64 CUDA tensor")
    C, N = captures.shape
    if out is None:
        out = torch.empty((n_bands * C, N // n_bands), dtype=torch.complex64, device=captures.device)
    elif (tuple(out.shape) != (n_bands * C, N // n_bands) or out.dtype != torch.complex64
          or not out.is_contiguous()):
        raise ValueError("out must be a contiguous complex64 tensor [n_bands * n_ch][N / n_bands]")
    geoloc_subbands(captures.data_ptr(), C, N, n_bands, half_taps, out.data_ptr(), _stream_handle(stream))
    return out


class Plan:
    """A plan over one grid and capture shape; maps take torch complex64 captures on the GPU."""

    def __init__(self, *, n_rx: int, n_samples: int, step_len: int, fs_hz: float, fc_hz: float,
                 lat, lon, grid_kind: int = GRID_RECT, n_rows: Optional[int] = None, n_cols: Optional[int] = None,
                 pairs: Optional[Sequence[Tuple[int, int]]] = None, earth_radius_m: float = 6371.0e3,
                 alt_m: float = 0.0, method: int = DIRECT_FP32, delay_mode: int = DELAY_LINEAR,
                 accum_mode: int = ACC_POWER, caf_lags: int = 0, caf_bins: int = 0,
                 caf_lag_lo: Optional[int] = None, caf_nu_lo_hz: float = math.nan, caf_nu_hi_hz: float = math.nan,
                 earth_model: int = EARTH_SPHERE, alt_grid=None):
        self._lat = np.ascontiguousarray(lat, dtype=np.float64).ravel()
        self._lon = np.ascontiguousarray(lon, dtype=np.float64).ravel()
        if grid_kind == GRID_RECT:
            n_rows, n_cols = self._lat.size, self._lon.size
        else:
            if n_rows is None:
                n_rows, n_cols = 1, self._lat.size
        pr = np.ascontiguousarray(np.asarray(pairs if pairs else [], dtype=np.int32).reshape(-1, 2))
        self._pairs = pr
        d = geoloc_desc()
        d.n_rx, d.n_pairs = n_rx, pr.shape[0]
        d.pairs = pr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if pr.size else None
        d.n_samples, d.step_len = n_samples, step_len
        d.fs_hz, d.fc_hz = fs_hz, fc_hz
        d.grid_kind, d.n_rows, d.n_cols = grid_kind, n_rows, n_cols
        d.lat = self._lat.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.lon = self._lon.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.earth_radius_m, d.alt_m = earth_radius_m, alt_m
        d.method, d.delay_mode, d.accum_mode = method, delay_mode, accum_mode
        d.caf_lags, d.caf_bins = caf_lags, caf_bins
        d.caf_lag_lo_set = 0 if caf_lag_lo is None else 1
        d.caf_lag_lo = 0 if caf_lag_lo is None else int(caf_lag_lo)
        d.caf_nu_lo_hz, d.caf_nu_hi_hz = caf_nu_lo_hz, caf_nu_hi_hz
        d.earth_model = earth_model
        self._alt = None
        if alt_grid is not None:
            self._alt = np.ascontiguousarray(alt_grid, dtype=np.float64).ravel()
            if self._alt.size != n_rows * n_cols:
                raise ValueError(f"alt_grid has {self._alt.size} entries for {n_rows * n_cols} points")
            d.alt_grid = self._alt.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.n_rx, self.n_samples, self.step_len = n_rx, n_samples, step_len
        self.n_steps = n_samples // step_len
        self.n_rows, self.n_cols = n_rows, n_cols
        self.n_points = n_rows * n_cols
        self.grid_kind = grid_kind
        self.handle = geoloc_plan(d)

    @classmethod
    def for_scenario(cls, scn, **kw) -> "Plan":
        wl = scn.workload
        return cls(n_rx=wl.n_rx, n_samples=wl.n_samples, step_len=wl.step_len, fs_hz=wl.fs_hz, fc_hz=wl.fc_hz,
                   lat=scn.lat, lon=scn.lon, pairs=list(wl.pairs), earth_radius_m=wl.earth_radius_m, **kw)

    def _inputs(self, captures, states: np.ndarray, stream) -> Tuple[geoloc_inputs, np.ndarray]:
        st = np.ascontiguousarray(states, dtype=np.float64)
        if st.shape != (self.n_steps, self.n_rx, 6):
            raise ValueError(f"states shape {st.shape} != {(self.n_steps, self.n_rx, 6)}")
        inp = geoloc_inputs()
        if captures is not None:
            import torch
            if captures.dtype != torch.complex64 or not captures.is_cuda or not captures.is_contiguous():
                raise ValueError("captures must be a contiguous complex64 CUDA tensor")
            if tuple(captures.shape) != (self.n_rx, self.n_samples):
                raise ValueError(f"captures shape {tuple(captures.shape)} != {(self.n_rx, self.n_samples)}")
            inp.captures = captures.data_ptr()
        inp.rx_state = st.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        inp.stream = _stream_handle(stream)
        return inp, st

    def map(self, captures, states: np.ndarray, J=None, accumulate: bool = False, stream=None):
        import torch
        if J is None:
            J = torch.empty(self.n_points, dtype=torch.float32, device=captures.device)
        if J.dtype != torch.float32 or not J.is_contiguous() or J.numel() != self.n_points:
            raise ValueError("J must be a contiguous float32 tensor of n_points")
        inp, _keep = self._inputs(captures, states, stream)
        geoloc_map(self.handle, inp, J.data_ptr(), ACCUMULATE if accumulate else 0)
        return J

    def geometry(self, states: np.ndarray, pair_index: int = 0, step_lo: int = 0, n_steps: Optional[int] = None,
                 device="cuda", stream=None):
        import torch
        n = self.n_steps - step_lo if n_steps is None else n_steps
        D = torch.empty((n, self.n_points), dtype=torch.float64, device=device)
        nu = torch.empty_like(D)
        inp, _keep = self._inputs(None, states, stream)
        geoloc_geometry(self.handle, inp, pair_index, step_lo, n, D.data_ptr(), nu.data_ptr())
        return D, nu

    def caf_table(self, captures, states: np.ndarray, pair_index: int = 0, step_lo: int = 0,
                  n_steps: Optional[int] = None, max_entries: Optional[int] = None, stream=None):
        """CAF tables [n_steps][lags][bins] complex64 (the window is reported by info())."""
        import torch
        n = self.n_steps - step_lo if n_steps is None else n_steps
        cap = max_entries if max_entries is not None else n * (1 << 22)
        T = torch.empty(cap, dtype=torch.complex64, device=captures.device)
        inp, _keep = self._inputs(captures, states, stream)
        geoloc_caf_table(self.handle, inp, pair_index, step_lo, n, T.data_ptr(), cap)
        i = geoloc_info(self.handle)
        return T[: n * i.caf_lags * i.caf_bins].view(n, i.caf_lags, i.caf_bins)

    def argmax(self, J, top_k: int = 1, nms_radius: int = 0, stream=None):
        return geoloc_argmax(self.handle, J.data_ptr(), top_k, nms_radius, _stream_handle(stream))

    def set_tiling(self, tile_w: int = 0, tile_h: int = 0, shear: int = 0, transpose: int = 0) -> None:
        """Fix the factored kernel's tiling (shear in 1/256 column per row); tile_w = 0 returns
        to the per-map choice."""
        _check(load().geoloc_set_tiling(self.handle, tile_w, tile_h, shear, transpose), "geoloc_set_tiling")

    def set_taylor_block(self, samples: int = 0) -> None:
        """Fix the factored kernel's Taylor block length (64 or 256 samples); 0 returns to
        the per-map choice."""
        _check(load().geoloc_set_taylor_block(self.handle, samples), "geoloc_set_taylor_block")

    def detect(self, J, guard: int, train: int, scale: float, max_detections: int = 16, nms_radius: int = 0,
               stream=None):
        """CFAR detections of a RECT map: (flat indices, J values, noise means), largest first."""
        return geoloc_detect(self.handle, J.data_ptr(), guard, train, scale, max_detections, nms_radius,
                             _stream_handle(stream))

    def set_grid(self, lat, lon) -> None:
        lat = np.ascontiguousarray(lat, dtype=np.float64).ravel()
        lon = np.ascontiguousarray(lon, dtype=np.float64).ravel()
        want = (self.n_rows, self.n_cols) if self.grid_kind == GRID_RECT else (self.n_points, self.n_points)
        if (lat.size, lon.size) != want:
            raise ValueError(f"grid coordinates {(lat.size, lon.size)} != {want}")
        geoloc_set_grid(self.handle, lat, lon)
        self._lat, self._lon = lat, lon

    def set_points_from_tiles(self, lat_dev, lon_dev, tile: int, tiles, stream=None) -> None:
        """Points = the cells of whole tiles (tile index = tile row x n_cols / tile + tile column)
        of the grid lat_dev x lon_dev (device float64 tensors), tile by tile, set on the device."""
        t = np.ascontiguousarray(np.asarray(tiles, dtype=np.int32).ravel())
        self._tiles = t                     # the host tile list stays alive past the copy
        _check(load().geoloc_set_points_from_tiles(self.handle, lat_dev.data_ptr(), lon_dev.data_ptr(),
                                                   lat_dev.numel(), lon_dev.numel(), tile,
                                                   t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), t.size,
                                                   _stream_handle(stream)), "geoloc_set_points_from_tiles")

    def set_timing(self, enable: bool = True) -> None:
        geoloc_set_timing(self.handle, enable)

    def info(self) -> dict:
        i = geoloc_info(self.handle)
        return {f: getattr(i, f) for f, _ in geoloc_plan_info._fields_ if not f.startswith("_")}

    def close(self) -> None:
        if getattr(self, "handle", None):
            geoloc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# --------------------------------------------------------------------------- learned tile proposal

def geoloc_cnn_create(desc: geoloc_cnn_desc) -> int:
    h = _vp()
    _check(load().geoloc_cnn_create(ctypes.byref(desc), ctypes.byref(h)), "geoloc_cnn_create")
    return h.value


def geoloc_cnn_param_count(cnn: int) -> int:
    n = ctypes.c_int64()
    _check(load().geoloc_cnn_param_count(cnn, ctypes.byref(n)), "geoloc_cnn_param_count")
    return n.value


def geoloc_cnn_set_params(cnn: int, theta: np.ndarray) -> None:
    t = np.ascontiguousarray(theta, dtype=np.float32)
    _check(load().geoloc_cnn_set_params(cnn, t.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), t.size),
           "geoloc_cnn_set_params")


def geoloc_cnn_get_params(cnn: int, which: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float32)
    _check(load().geoloc_cnn_get_params(cnn, which, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n),
           "geoloc_cnn_get_params")
    return out


def geoloc_cnn_prepare(cnn: int, J_dev: int, D_dev: int, nu_dev: int, batch: int, x_dev: int, stream: int) -> None:
    _check(load().geoloc_cnn_prepare(cnn, J_dev, D_dev, nu_dev, batch, x_dev, stream), "geoloc_cnn_prepare")


def geoloc_cnn_forward(cnn: int, x_dev: int, batch: int, logits_dev: int, stream: int) -> None:
    _check(load().geoloc_cnn_forward(cnn, x_dev, batch, logits_dev, stream), "geoloc_cnn_forward")


def geoloc_cnn_loss(cnn: int, logits_dev: int, label_dev: int, batch: int, dlogits_dev: int, loss_dev: int,
                    stream: int) -> None:
    _check(load().geoloc_cnn_loss(cnn, logits_dev, label_dev, batch, dlogits_dev, loss_dev, stream), "geoloc_cnn_loss")


def geoloc_cnn_backward(cnn: int, dlogits_dev: int, batch: int, stream: int) -> None:
    _check(load().geoloc_cnn_backward(cnn, dlogits_dev, batch, stream), "geoloc_cnn_backward")


def geoloc_cnn_adam_step(cnn: int, lr: float, beta1: float, beta2: float, eps: float, stream: int) -> None:
    _check(load().geoloc_cnn_adam_step(cnn, lr, beta1, beta2, eps, stream), "geoloc_cnn_adam_step")


def geoloc_cnn_topk(cnn: int, logits_dev: int, batch: int, k: int, stream: int) -> Tuple[np.ndarray, np.ndarray]:
    tiles = np.empty((batch, k), dtype=np.int32)
    probs = np.empty((batch, k), dtype=np.float32)
    _check(load().geoloc_cnn_topk(cnn, logits_dev, batch, k, tiles.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  probs.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), stream), "geoloc_cnn_topk")
    return tiles, probs


def geoloc_cnn_destroy(cnn: int) -> None:
    _check(load().geoloc_cnn_destroy(cnn), "geoloc_cnn_destroy")


class CNN:
    """Tile-proposal network on the device; tensors are torch CUDA float32 NCHW."""

    def __init__(self, in_ch: int = 3, hidden: int = 32, layers: int = 4, height: int = 64, width: int = 64,
                 max_batch: int = 64):
        d = geoloc_cnn_desc(in_ch, hidden, layers, height, width, max_batch)
        self.in_ch, self.hidden, self.layers, self.height, self.width, self.max_batch = (
            in_ch, hidden, layers, height, width, max_batch)
        self.handle = geoloc_cnn_create(d)
        self.n_params = geoloc_cnn_param_count(self.handle)

    def set_params(self, theta: np.ndarray) -> None:
        geoloc_cnn_set_params(self.handle, theta)

    def params(self, which: int = 0) -> np.ndarray:
        return geoloc_cnn_get_params(self.handle, which, self.n_params)

    def prepare(self, J, D, nu, stream=None):
        import torch
        B = J.shape[0]
        x = torch.empty((B, 3, self.height, self.width), dtype=torch.float32, device=J.device)
        geoloc_cnn_prepare(self.handle, J.data_ptr(), D.data_ptr(), nu.data_ptr(), B, x.data_ptr(),
                           _stream_handle(stream))
        return x

    def forward(self, x, stream=None):
        import torch
        B = x.shape[0]
        z = torch.empty((B, self.height, self.width), dtype=torch.float32, device=x.device)
        geoloc_cnn_forward(self.handle, x.data_ptr(), B, z.data_ptr(), _stream_handle(stream))
        return z

    def loss(self, z, label, stream=None):
        import torch
        B = z.shape[0]
        dz = torch.empty_like(z)
        loss = torch.empty(B, dtype=torch.float32, device=z.device)
        geoloc_cnn_loss(self.handle, z.data_ptr(), label.data_ptr(), B, dz.data_ptr(), loss.data_ptr(),
                        _stream_handle(stream))
        return loss, dz

    def backward(self, dz, stream=None) -> None:
        geoloc_cnn_backward(self.handle, dz.data_ptr(), dz.shape[0], _stream_handle(stream))

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None) -> None:
        geoloc_cnn_adam_step(self.handle, lr, beta1, beta2, eps, _stream_handle(stream))

    def topk(self, z, k: int, stream=None):
        return geoloc_cnn_topk(self.handle, z.data_ptr(), z.shape[0], k, _stream_handle(stream))

    def close(self) -> None:
        if getattr(self, "handle", None):
            geoloc_cnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
