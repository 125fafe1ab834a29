"""Pins of the CFAR detection oracle (threshold step of Algorithm 1, read as cell-averaging
CFAR): brute force over the window cells, the window counts at edges and corners, the
exponential closed form of the scale, the false-alarm rate it gives on Gamma noise maps
(one look and eight), planted peaks, and constant maps."""
import numpy as np
import pytest

from oracle import cfar


def _brute_noise(J, g, t):
    R, C = J.shape
    out = np.zeros((R, C))
    cnt = np.zeros((R, C), dtype=int)
    for r in range(R):
        for c in range(C):
            s = 0.0
            n = 0
            for rr in range(R):
                for cc in range(C):
                    d = max(abs(rr - r), abs(cc - c))   # Chebyshev distance
                    if g < d <= t:
                        s += J[rr, cc]
                        n += 1
            cnt[r, c] = n
            out[r, c] = s / n if n else 0.0
    return out, cnt


@pytest.mark.parametrize("g,t", [(0, 1), (1, 3), (2, 4)])
def test_noise_estimate_matches_brute_force(g, t):
    rng = np.random.Generator(np.random.PCG64(5))
    J = rng.exponential(size=(9, 11))
    nz, n = cfar.noise_estimate(J, g, t)
    bz, bn = _brute_noise(J, g, t)
    assert np.array_equal(n, bn)
    assert np.allclose(nz, bz, rtol=1e-13, atol=0)


def test_window_counts_at_edges_and_corners():
    J = np.ones((20, 30))
    _, n = cfar.noise_estimate(J, 1, 3)
    assert n[10, 15] == 7 * 7 - 3 * 3           # interior
    assert n[0, 0] == 4 * 4 - 2 * 2              # corner: rows 0..3, cols 0..3, guard 0..1
    assert n[0, 15] == 4 * 7 - 2 * 3             # top edge
    assert n[10, 29] == 7 * 4 - 3 * 2            # right edge


def test_exponential_closed_form_of_the_scale():
    for N in (8, 24, 48, 120):
        for pfa in (1e-2, 1e-4, 1e-6, 1e-9):
            a = cfar.scale_for_pfa(pfa, N, 1)
            assert a == pytest.approx(N * (pfa ** (-1.0 / N) - 1.0), rel=1e-9)
            assert (1.0 + a / N) ** (-N) == pytest.approx(pfa, rel=1e-9)


@pytest.mark.parametrize("looks", [1, 8])
def test_false_alarm_rate_on_gamma_noise(looks):
    """Interior cells of noise-only maps: the measured rate of J > a * mean matches the
    requested 2e-3 within five binomial standard deviations."""
    g, t, pfa = 1, 4, 2e-3
    N = (2 * t + 1) ** 2 - (2 * g + 1) ** 2
    a = cfar.scale_for_pfa(pfa, N, looks)
    rng = np.random.Generator(np.random.PCG64(11 + looks))
    hits = trials = 0
    for _ in range(3):
        J = rng.gamma(looks, 2.5, size=(140, 140))
        nz, _ = cfar.noise_estimate(J, g, t)
        inner = (slice(t, -t), slice(t, -t))
        hits += int(np.sum(J[inner] > a * nz[inner]))
        trials += J[inner].size
    rate = hits / trials
    sd = np.sqrt(pfa * (1 - pfa) / trials)
    assert abs(rate - pfa) <= 5 * sd, (rate, pfa, sd)


def test_planted_peaks_are_the_detections():
    rng = np.random.Generator(np.random.PCG64(3))
    R, C = 60, 80
    J = rng.exponential(1.0, size=(R, C))
    rows, cols = np.mgrid[0:R, 0:C]
    centres = [(12, 15, 400.0), (40, 60, 250.0), (30, 30, 120.0)]
    for (r, c, h) in centres:
        J += h * np.exp(-((rows - r) ** 2 + (cols - c) ** 2) / 2.0)
    det = cfar.detect(J, guard=3, train=8, scale=cfar.scale_for_pfa(1e-6, 17 * 17 - 7 * 7), k=10, radius=4)
    assert [divmod(i, C) for i, _, _ in det] == [(r, c) for r, c, _ in centres]
    vals = [v for _, v, _ in det]
    assert vals == sorted(vals, reverse=True)
    for i, v, nz in det:
        assert v > 20 * nz


def test_constant_map_has_no_detection():
    J = np.full((15, 15), 3.0)
    assert cfar.detect(J, 1, 3, 1.0, 5, 1) == []
    J[7, 7] = 3.5
    det = cfar.detect(J, 1, 3, 1.1, 5, 1)
    assert len(det) == 1 and det[0][0] == 7 * 15 + 7 and det[0][2] == pytest.approx(3.0)


CFAR_MUTANTS = {
    "guard_not_excluded": ("s = J[r0:r1 + 1, c0:c1 + 1].sum() - J[g0:g1 + 1, h0:h1 + 1].sum()",
                           "s = J[r0:r1 + 1, c0:c1 + 1].sum()"),
    "window_one_short": ("r0, r1 = max(0, r - train), min(R - 1, r + train)",
                         "r0, r1 = max(0, r - train), min(R - 1, r + train - 1)"),
    "count_ignores_clipping": ("n = (r1 - r0 + 1) * (c1 - c0 + 1) - (g1 - g0 + 1) * (h1 - h0 + 1)",
                               "n = (2 * train + 1) ** 2 - (g1 - g0 + 1) * (h1 - h0 + 1)"),
    "threshold_on_sum": ("hit = (count > 0) & (J > scale * noise)", "hit = (count > 0) & (J > scale * noise * count)"),
    "scale_looks_ignored": ("b = float(betainccinv(looks, n_train * looks, pfa))",
                            "b = float(betainccinv(1, n_train, pfa))"),
    "scale_lower_tail": ("b = float(betainccinv(looks, n_train * looks, pfa))",
                         "b = float(betainccinv(looks, n_train * looks, 1.0 - pfa))"),
}


@pytest.mark.parametrize("name", sorted(CFAR_MUTANTS))
def test_every_planted_cfar_mistake_fails_a_pin(name, tmp_path, monkeypatch):
    import importlib.util
    import sys
    old, new = CFAR_MUTANTS[name]
    src = open(cfar.__file__).read()
    assert src.count(old) == 1, name
    path = tmp_path / "cfar_mutant.py"
    path.write_text(src.replace(old, new).replace("from . import peaks", "from oracle import peaks"))
    spec = importlib.util.spec_from_file_location("cfar_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    monkeypatch.setattr(sys.modules[__name__], "cfar", mod)
    pins = [lambda: test_noise_estimate_matches_brute_force(1, 3), test_window_counts_at_edges_and_corners,
            test_exponential_closed_form_of_the_scale, lambda: test_false_alarm_rate_on_gamma_noise(8),
            test_planted_peaks_are_the_detections, test_constant_map_has_no_detection]
    failed = 0
    for f in pins:
        try:
            f()
        except AssertionError:
            failed += 1
    assert failed > 0, f"mutant {name} passed every pin"
