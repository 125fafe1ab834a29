"""Threshold detection of several emitters on a RECT map -- TEST INFRASTRUCTURE.

Algorithm 1 ends with a threshold that detects emitters, and the paper states no rule for
it. The reading taken here is cell-averaging CFAR (constant false-alarm rate): the noise
level at a cell is the mean of J over its training window -- the (2t+1) x (2t+1) cells
around it, clipped to the grid, less the (2g+1) x (2g+1) guard window around the cell --
and the cell is a detection when J exceeds `scale` times that mean. Detections are then
reported as peaks: the largest first, each excluding a (2r+1) x (2r+1) window around it
(the same rule as the top-k of `peaks`), up to k of them.

`scale_for_pfa` gives the scale for a false-alarm probability when the noise-only cells
are independent Gamma(L, theta) variables (L noncoherent looks; L = 1 is exponential,
the |C|^2 of one complex Gaussian correlation): a cell x and the training sum z of N
cells give x / (x + z) ~ Beta(L, N L), so P(x > a z / N) = 1 - I_{a / (N + a)}(L, N L).

Plain loops and slices, float64 throughout.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from . import peaks


def noise_estimate(J: np.ndarray, guard: int, train: int) -> Tuple[np.ndarray, np.ndarray]:
    """Mean of J over each cell's training window, and the number of training cells."""
    J = np.asarray(J, dtype=np.float64)
    R, C = J.shape
    noise = np.zeros((R, C))
    count = np.zeros((R, C), dtype=np.int64)
    for r in range(R):
        for c in range(C):
            r0, r1 = max(0, r - train), min(R - 1, r + train)
            c0, c1 = max(0, c - train), min(C - 1, c + train)
            g0, g1 = max(0, r - guard), min(R - 1, r + guard)
            h0, h1 = max(0, c - guard), min(C - 1, c + guard)
            s = J[r0:r1 + 1, c0:c1 + 1].sum() - J[g0:g1 + 1, h0:h1 + 1].sum()
            n = (r1 - r0 + 1) * (c1 - c0 + 1) - (g1 - g0 + 1) * (h1 - h0 + 1)
            count[r, c] = n
            noise[r, c] = s / n if n > 0 else 0.0
    return noise, count


def detect(J: np.ndarray, guard: int, train: int, scale: float, k: int,
           radius: int) -> List[Tuple[int, float, float]]:
    """Detections (flat index, J, noise mean), largest first, at most k."""
    J = np.asarray(J, dtype=np.float64)
    R, C = J.shape
    noise, count = noise_estimate(J, guard, train)
    hit = (count > 0) & (J > scale * noise)
    masked = np.where(hit, J, -np.inf)
    out = []
    for i, v in peaks.topk(masked, R, C, k, radius):
        out.append((i, v, float(noise.ravel()[i])))
    return out


def scale_for_pfa(pfa: float, n_train: int, looks: int = 1) -> float:
    """Scale a with P(x > a mean(training)) = pfa for independent Gamma(looks) noise. The
    Beta quantile is taken from the upper tail itself (inverse of 1 - I_b), not as the
    (1 - pfa) quantile, so that 1 - pfa does not round away the digits of a small pfa."""
    from scipy.special import betainccinv
    b = float(betainccinv(looks, n_train * looks, pfa))
    return n_train * b / (1.0 - b)
