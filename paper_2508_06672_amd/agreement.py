"""Agreement of a map's peak with a reference map's peak (the rule the accelerated forms
are judged by against the plain map, and the GPU against the oracle).

Exact near-ties are built into direct geolocation: with every receiver in one orbital
plane and a non-rotating Earth the map is symmetric through that plane (J(p) = J(M p)),
a tone has no delay resolution (its map is a ridge along a line of equal Doppler, whose
maximum along the ridge is set by the noise), and a repeated chirp has ambiguity peaks
one period apart. An exact argmax is therefore well-posed only when the reference peak
stands clear of everything outside its own neighbourhood:

  margin m = (J_max - max over q outside N1(a) and N1(M a) of J(q)) / J_max,

with a the reference peak, M a its mirror cell and N1 the 3 x 3 neighbourhood. A scenario
is well-conditioned at tolerance eps when m > 2 eps (then no error within eps of the
peak can move it out of N1); there a peak must lie within one cell of a or of M a. On
every scenario the peak is also classed eps-optimal when J_ref(peak) >= (1 - eps) J_max.
"""
from __future__ import annotations

from typing import Optional

import numpy as np


def cell_dist(a: int, b: int, n_cols: int) -> int:
    """Chebyshev distance in cells between two flat indices of a RECT grid."""
    ra, ca = divmod(int(a), n_cols)
    rb, cb = divmod(int(b), n_cols)
    return max(abs(ra - rb), abs(ca - cb))


def mirror_cell(wl, lat: np.ndarray, lon: np.ndarray, a: int) -> int:
    """Grid cell nearest to the reflection of cell a through the receivers' orbital plane."""
    from . import sim
    r, c = divmod(int(a), lon.size)
    mr, mc = sim.nearest_cell(lat, lon, *sim.mirror_latlon(wl, lat[r], lon[c]))
    return mr * lon.size + mc


def margin(J: np.ndarray, n_cols: int, a: int, mirror: Optional[int] = None) -> float:
    """Relative gap between J[a] and the largest value outside N1(a) and N1(mirror)."""
    J = np.asarray(J, dtype=np.float64).ravel()
    n_rows = J.size // n_cols
    G = J.reshape(n_rows, n_cols)
    keep = np.ones_like(G, dtype=bool)
    for cell in (a, mirror):
        if cell is None:
            continue
        r, c = divmod(int(cell), n_cols)
        keep[max(0, r - 1):r + 2, max(0, c - 1):c + 2] = False
    rest = G[keep]
    top = J[int(a)]
    if rest.size == 0 or not top > 0:
        return float("inf") if rest.size == 0 else 0.0
    return float((top - rest.max()) / top)


def classify(J_ref: np.ndarray, n_cols: int, a_test: int, a_ref: int, eps: float,
             mirror: Optional[int] = None) -> dict:
    """Rule above for one scenario: margin, well-conditioned, within one cell of the
    reference peak or its mirror, eps-optimal on the reference map."""
    J_ref = np.asarray(J_ref, dtype=np.float64).ravel()
    m = margin(J_ref, n_cols, a_ref, mirror)
    d = cell_dist(a_test, a_ref, n_cols)
    if mirror is not None:
        d = min(d, cell_dist(a_test, mirror, n_cols))
    return {"margin": m, "well_conditioned": bool(m > 2 * eps), "cell_dist": int(d), "within_one": bool(d <= 1),
            "eps_optimal": bool(J_ref[int(a_test)] >= (1.0 - eps) * J_ref[int(a_ref)])}


def summarise(records, eps: float) -> dict:
    """Rates over a list of classify() results."""
    n = len(records)
    wc = [r for r in records if r["well_conditioned"]]
    return {"n_scenarios": n, "eps": eps,
            "well_conditioned_fraction": len(wc) / n if n else None,
            "within_one_cell_well_conditioned": (sum(r["within_one"] for r in wc) / len(wc)) if wc else None,
            "within_one_cell_all": sum(r["within_one"] for r in records) / n if n else None,
            "eps_optimal_all": sum(r["eps_optimal"] for r in records) / n if n else None,
            "within_one_or_eps_optimal_all": sum(r["within_one"] or r["eps_optimal"] for r in records) / n
            if n else None}
