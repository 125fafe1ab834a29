"""Eq. (11) as literal Python loops over candidates, steps and samples -- for tiny inputs.

Test infrastructure (see the package docstring). Independent of the C oracle: it
recomputes the geometry of Sec. II-B with Python floats and evaluates the
correlation one sample at a time with ``cmath.exp``.
"""
from __future__ import annotations

import cmath
import math
from typing import Sequence, Tuple

import numpy as np

C = 299_792_458.0


def _ecef(lat: float, lon: float, radius: float) -> Tuple[float, float, float]:
    return (radius * math.cos(lat) * math.cos(lon), radius * math.cos(lat) * math.sin(lon), radius * math.sin(lat))


def _tau_f(q, s, lam):
    r = [s[0] - q[0], s[1] - q[1], s[2] - q[2]]
    rho = math.sqrt(r[0] ** 2 + r[1] ** 2 + r[2] ** 2)
    f = -(r[0] * s[3] + r[1] * s[4] + r[2] * s[5]) / (rho * lam)
    return rho / C, f


def _sinc_weights(a: float):
    """Eight weights of the windowed-sinc delay (taps -3 .. 4), from numpy's sinc and I0."""
    x = np.arange(-3, 5) - a
    g = np.where(np.abs(x) < 4.0, np.sinc(x) * np.i0(6.0 * np.sqrt(np.clip(1.0 - (x / 4.0) ** 2, 0.0, None)))
                 / np.i0(6.0), 0.0)
    return [float(v) for v in g / g.sum()]


def brute_map(lat_p: Sequence[float], lon_p: Sequence[float], captures: np.ndarray, states: np.ndarray,
              step_len: int, fs: float, fc: float, pairs: Sequence[Tuple[int, int]], radius: float = 6371.0e3,
              delay_mode: int = 0, accum_mode: int = 0) -> np.ndarray:
    lam = C / fc
    R, N = captures.shape
    K = N // step_len
    y = [[complex(v) for v in captures[i]] for i in range(R)]

    def sample(i, m):
        return y[i][m] if 0 <= m < N else 0j

    J = np.zeros(len(lat_p))
    for p in range(len(lat_p)):
        q = _ecef(lat_p[p], lon_p[p], radius)
        for (i, j) in pairs:
            for k in range(K):
                ti, fi = _tau_f(q, states[k][i], lam)
                tj, fj = _tau_f(q, states[k][j], lam)
                D = (tj - ti) * fs
                nu = fj - fi
                if delay_mode == 1:
                    d0 = int(math.floor(abs(D) + 0.5)) * (1 if D >= 0 else -1)
                    a = 0.0
                else:
                    d0 = math.floor(D)
                    a = D - d0
                w = _sinc_weights(a) if delay_mode == 2 else None
                s = 0j
                for n in range(k * step_len, (k + 1) * step_len):
                    if w is None:
                        yt = (1 - a) * sample(j, n + d0) + a * sample(j, n + d0 + 1)
                    else:
                        yt = sum(w[t + 3] * sample(j, n + d0 + t) for t in range(-3, 5))
                    t = (n - k * step_len - (step_len - 1) / 2) / fs
                    s += sample(i, n) * yt.conjugate() * cmath.exp(2j * math.pi * nu * t)
                J[p] += abs(s) if accum_mode == 1 else abs(s) ** 2
    return J
