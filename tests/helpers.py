"""Shared comparison rules for GPU-vs-oracle tests.

Tolerance: err_J = max_p |J_gpu(p) - J_orc(p)| / max_p J_orc(p).
Argmax: exact agreement is required when the oracle's best point beats every other
point by more than twice the tolerance (then any error within tolerance cannot move
the peak); otherwise the GPU's peak must be tol-optimal, J_orc(a_gpu) >= (1 - 2 tol)
J_orc(a_orc), because near-ties (mirror symmetry through the orbital plane, tone
ridges, chirp ambiguity peaks) make the exact argmax ill-posed.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

DIRECT_TOL = 1e-4


def log(msg: str) -> None:
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    return torch


def err_J(Jg: np.ndarray, Jo: np.ndarray) -> float:
    Jg = np.asarray(Jg, dtype=np.float64).ravel()
    Jo = np.asarray(Jo, dtype=np.float64).ravel()
    return float(np.max(np.abs(Jg - Jo)) / np.max(np.abs(Jo)))


def check_argmax(Jg: np.ndarray, Jo: np.ndarray, tol: float) -> str:
    Jg = np.asarray(Jg, dtype=np.float64).ravel()
    Jo = np.asarray(Jo, dtype=np.float64).ravel()
    ao, ag = int(np.argmax(Jo)), int(np.argmax(Jg))
    top = Jo[ao]
    second = np.max(np.delete(Jo, ao)) if Jo.size > 1 else -np.inf
    gap = (top - second) / top
    if gap > 2 * tol:
        assert ag == ao, f"argmax {ag} != oracle {ao} with gap {gap:.3g}"
        return "exact"
    assert Jo[ag] >= (1 - 2 * tol) * top, f"argmax {ag} not tol-optimal: {Jo[ag] / top:.6f}"
    return "exact" if ag == ao else "tol-optimal"
