"""FP64 sub-band split of the captures -- TEST INFRASTRUCTURE.

The coarse map of the learned tile proposal is computed from the captures split into
M frequency bands, each decimated by M, so that the cross-correlation peak of a
wideband emitter is as wide as a coarse cell instead of one 10 MHz sample (a coarse
grid sampled at cell centres would otherwise miss the narrow delay ridge). This is an
addition to the paper's method, not a step of it; the definition is the textbook
DFT filter bank (mix each band to zero frequency, low-pass, keep every M-th sample):

    z_b[m] = sum_{t=-h}^{h} g[t] x[m M - t] exp(-j 2 pi f_b (m M - t)),   f_b = (b - M/2) / M

in cycles per sample, with x = 0 outside the capture. Because f_b M is an integer the
first factor of the exponential is 1 and

    z_b[m] = sum_{t=-h}^{h} g[t] exp(+j 2 pi (b - M/2) t / M) x[m M - t].

g is the Blackman-windowed ideal low-pass with cut-off 1/(2M) cycles per sample,
scaled to unit gain at zero frequency:

    g0[t] = sin(pi t / M) / (pi t)   (1/M at t = 0),
    w[t]  = 0.42 + 0.5 cos(pi t / h) + 0.08 cos(2 pi t / h),
    g[t]  = g0[t] w[t] / sum_s g0[s] w[s].

Output layout: [M][n_channels][N / M], band-major, so that band b of channel c is row
b * n_channels + c of a capture array of M * n_channels receivers.
"""
from __future__ import annotations

import numpy as np


def prototype(n_bands: int, half_taps: int) -> np.ndarray:
    """The 2 h + 1 low-pass taps g[-h..h] (float64)."""
    M, h = int(n_bands), int(half_taps)
    t = np.arange(-h, h + 1, dtype=np.float64)
    g0 = np.empty_like(t)
    nz = t != 0
    g0[nz] = np.sin(np.pi * t[nz] / M) / (np.pi * t[nz])
    g0[~nz] = 1.0 / M
    w = 0.42 + 0.5 * np.cos(np.pi * t / h) + 0.08 * np.cos(2.0 * np.pi * t / h)
    g = g0 * w
    return g / g.sum()


def subbands(x: np.ndarray, n_bands: int, half_taps: int) -> np.ndarray:
    """z [M][C][N / M] complex128 of captures x [C][N] (N divisible by M)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.complex128))
    C, N = x.shape
    M, h = int(n_bands), int(half_taps)
    assert N % M == 0
    g = prototype(M, h)
    t = np.arange(-h, h + 1)
    n_out = N // M
    out = np.zeros((M, C, n_out), dtype=np.complex128)
    # x padded by h zeros on both sides: x[m M - t] = xp[m M - t + h]
    xp = np.zeros((C, N + 2 * h), dtype=np.complex128)
    xp[:, h:h + N] = x
    # rows m, columns t: the samples each output reads
    idx = (np.arange(n_out)[:, None] * M - t[None, :]) + h
    for b in range(M):
        taps = g * np.exp(2j * np.pi * (b - M // 2) * t / M)
        for c in range(C):
            out[b, c] = xp[c][idx] @ taps
    return out


def states_for_bands(states: np.ndarray, n_bands: int) -> np.ndarray:
    """Receiver states [K][M * R][6] for the band-major capture layout (band b of
    receiver r is receiver b * R + r)."""
    st = np.asarray(states, dtype=np.float64)
    return np.ascontiguousarray(np.tile(st, (1, int(n_bands), 1)))


def pairs_for_bands(pairs, n_rx: int, n_bands: int):
    """Every pair (i, j) repeated within each band: (b R + i, b R + j)."""
    return [(b * n_rx + i, b * n_rx + j) for b in range(int(n_bands)) for (i, j) in pairs]
