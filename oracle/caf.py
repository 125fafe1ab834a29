"""FP64 CAF-table form of the position-domain correlation -- TEST INFRASTRUCTURE.

Eq. (11) for every integer lag d of a window and every Doppler bin nu_m of a
uniform grid is a cross-ambiguity (CAF) table of step k:

    T_k[d, m] = sum_{n in step k} y_i[n] * conj(y_j[n + d]) * exp(+j 2 pi nu_m t_n)

with t_n measured from the step centre and y_j = 0 outside the capture. It is
the product of the lag-product matrix L_k[d, n] = y_i[n] conj(y_j[n + d]) with
the phasor matrix F[n, m] = exp(j 2 pi nu_m t_n) (a library matmul).

A candidate point with delay D = d0 + alpha (samples) and FDOA nu reads the
table by bilinear interpolation of the complex values:

    u = (nu - nu_0) / dnu,  m0 = floor(u), beta = u - m0
    C = (1-a)(1-b) T[d0, m0] + a(1-b) T[d0+1, m0] + (1-a) b T[d0, m0+1] + a b T[d0+1, m0+1]

With the two-tap linear fractional delay the lag interpolation is exact, so the
table reproduces the direct correlation whenever nu falls on a bin.
The map is then accumulated as in Algorithm 1.
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple

import numpy as np

from . import geometry, grid_ecef, sinc_taps, LINEAR, ROUND, SINC, POWER, MAG


def bins(nu_lo: float, nu_hi: float, n_bins: int) -> np.ndarray:
    """Doppler bin centres nu_m = nu_lo + m * dnu, m = 0..M-1, both ends included."""
    return nu_lo + (nu_hi - nu_lo) / (n_bins - 1) * np.arange(n_bins)


def table(yi: np.ndarray, yj: np.ndarray, k: int, step_len: int, fs: float, lag_lo: int, n_lags: int,
          nu: np.ndarray) -> np.ndarray:
    """T_k [n_lags][M] complex128 for lags lag_lo .. lag_lo + n_lags - 1."""
    N = yi.size
    n = np.arange(k * step_len, (k + 1) * step_len)
    x = yi[n].astype(np.complex128)
    Lk = np.zeros((n_lags, step_len), dtype=np.complex128)
    for r in range(n_lags):
        m = n + lag_lo + r
        ok = (m >= 0) & (m < N)
        v = np.zeros(step_len, dtype=np.complex128)
        v[ok] = yj[m[ok]]
        Lk[r] = x * np.conj(v)
    t = (n - k * step_len - (step_len - 1) / 2.0) / fs
    F = np.exp(2j * math.pi * np.outer(t, nu))
    return Lk @ F


def interp(T: np.ndarray, lag_lo: int, nu_lo: float, dnu: float, D: np.ndarray, nu: np.ndarray,
           delay_mode: int = LINEAR) -> np.ndarray:
    """Complex interpolation of one step's table at (D, nu) per point: linear in Doppler,
    and in lag linear (LINEAR), nearest (ROUND) or the eight windowed-sinc taps (SINC)."""
    if delay_mode == ROUND:
        d0 = np.where(D >= 0, np.floor(np.abs(D) + 0.5), -np.floor(np.abs(D) + 0.5)).astype(np.int64)
        a = np.zeros_like(D)
    else:
        f = np.floor(D)
        d0 = f.astype(np.int64)
        a = D - f
    u = (nu - nu_lo) / dnu
    m0f = np.floor(u)
    m0 = m0f.astype(np.int64)
    b = u - m0f
    nl, M = T.shape
    r0 = d0 - lag_lo
    # a point exactly on the last bin / lag reads the cell below with weight 1
    top = (m0 == M - 1) & (b == 0.0)
    m0 = np.where(top, M - 2, m0)
    b = np.where(top, 1.0, b)
    if delay_mode == SINC:
        # eight lag taps (d0 - 3 .. d0 + 4), each interpolated linearly in Doppler
        if np.any(r0 - 3 < 0) or np.any(r0 + 4 >= nl) or np.any(m0 < 0) or np.any(m0 + 1 >= M):
            raise ValueError("CAF window does not cover every point")
        out = np.zeros(D.shape, dtype=np.complex128)
        for p in range(D.size):
            w = sinc_taps(float(a.flat[p]))
            for t in range(8):
                r = r0.flat[p] - 3 + t
                out.flat[p] += w[t] * ((1 - b.flat[p]) * T[r, m0.flat[p]] + b.flat[p] * T[r, m0.flat[p] + 1])
        return out
    topd = (r0 == nl - 1) & (a == 0.0)
    r0 = np.where(topd, nl - 2, r0)
    a = np.where(topd, 1.0, a)
    if np.any(r0 < 0) or np.any(r0 + 1 >= nl) or np.any(m0 < 0) or np.any(m0 + 1 >= M):
        raise ValueError("CAF window does not cover every point")
    return ((1 - a) * (1 - b) * T[r0, m0] + a * (1 - b) * T[r0 + 1, m0]
            + (1 - a) * b * T[r0, m0 + 1] + a * b * T[r0 + 1, m0 + 1])


def caf_map_points(lat_p, lon_p, captures: np.ndarray, states: np.ndarray, step_len: int, fs: float, fc: float,
                   pairs: Sequence[Tuple[int, int]], lag_lo: int, n_lags: int, nu_lo: float, nu_hi: float,
                   n_bins: int, radius: float = 6371.0e3, delay_mode: int = LINEAR,
                   accum_mode: int = POWER) -> np.ndarray:
    """FP64 CAF-table map at explicit points. lag window / Doppler bins are per pair
    (the same window is used for every pair and step here)."""
    xyz = grid_ecef(lat_p, lon_p, radius)
    R, N = captures.shape
    K = N // step_len
    nu_b = bins(nu_lo, nu_hi, n_bins)
    dnu = (nu_hi - nu_lo) / (n_bins - 1)
    J = np.zeros(xyz.shape[0])
    for (i, j) in pairs:
        D, nu = geometry(xyz, states, (i, j), fs, fc)
        for k in range(K):
            T = table(captures[i], captures[j], k, step_len, fs, lag_lo, n_lags, nu_b)
            c = interp(T, lag_lo, nu_lo, dnu, D[k], nu[k], delay_mode)
            pw = np.abs(c) ** 2
            J += np.sqrt(pw) if accum_mode == MAG else pw
    return J
