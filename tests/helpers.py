"""Shared comparison rules for GPU-vs-oracle tests.

Tolerance: err_J = max_p |J_gpu(p) - J_orc(p)| / max_p J_orc(p).
Argmax: exact agreement is required when the oracle's best point beats every other
point by more than twice the tolerance (then any error within tolerance cannot move
the peak); otherwise the GPU's peak must be tol-optimal, J_orc(a_gpu) >= (1 - tol)
J_orc(a_orc), because near-ties (mirror symmetry through the orbital plane, tone
ridges, chirp ambiguity peaks) make the exact argmax ill-posed. The accelerated forms
(CAF table, learned proposal) are held to the cell rule of
paper_2508_06672_amd.agreement (within one cell of the reference peak or its mirror
where the margin exceeds 2 tol, tol-optimal otherwise).
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
    assert Jo[ag] >= (1 - tol) * top, f"argmax {ag} not tol-optimal: {Jo[ag] / top:.6f}"
    return "exact" if ag == ao else "tol-optimal"


def check_cells(J_ref: np.ndarray, n_cols: int, a_test: int, a_ref: int, tol: float, mirror=None) -> dict:
    """Peak a_test against the reference map's peak a_ref: within one cell (of a_ref or its
    mirror) on a well-conditioned map (margin > 2 tol), tol-optimal on any other."""
    from paper_2508_06672_amd import agreement
    c = agreement.classify(J_ref, n_cols, a_test, a_ref, tol, mirror)
    log(f"  peak {a_test} vs {a_ref}: margin {c['margin']:.3g}, {c['cell_dist']} cells, "
        f"tol-optimal {c['eps_optimal']}")
    if c["well_conditioned"]:
        assert c["within_one"], c
    else:
        assert c["eps_optimal"], c
    return c
