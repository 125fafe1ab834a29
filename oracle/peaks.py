"""Peak extraction from a map -- TEST INFRASTRUCTURE.

Algorithm 1 ends by thresholding the summed grid to detect emitters; the single
emitter estimate is the maximum of J (the maximum-likelihood point, Sec. III).
Rules: ties go to the lowest flat index; a NaN anywhere is an error; top-k
repeats the argmax after masking a (2r+1) x (2r+1) window around each peak found.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def argmax(J: np.ndarray) -> Tuple[int, float]:
    J = np.asarray(J).ravel()
    if np.isnan(J).any():
        raise ValueError("NaN in map")
    i = int(np.argmax(J))            # numpy returns the first maximal index
    return i, float(J[i])


def topk(J: np.ndarray, n_rows: int, n_cols: int, k: int, radius: int) -> List[Tuple[int, float]]:
    J = np.asarray(J, dtype=np.float64).reshape(n_rows, n_cols).copy()
    if np.isnan(J).any():
        raise ValueError("NaN in map")
    out = []
    masked = np.zeros(J.shape, dtype=bool)
    for _ in range(k):
        cand = np.where(masked, -np.inf, J)
        i = int(np.argmax(cand))
        if not np.isfinite(cand.ravel()[i]):
            break
        out.append((i, float(J.ravel()[i])))
        r, c = divmod(i, n_cols)
        masked[max(0, r - radius):r + radius + 1, max(0, c - radius):c + radius + 1] = True
    return out
