"""Pins of the FP64 sub-band split (the coarse-map input of the learned tile proposal)
against a library filter design, the textbook mix / filter / decimate chain, a tone at
each band centre, shift invariance and literal loops on a tiny input."""
import math

import numpy as np
import pytest
import scipy.signal

from oracle import subband


def _rng(seed):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))


def _cn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2)


@pytest.mark.parametrize("M,h", [(16, 64), (8, 32), (4, 9)])
def test_prototype_is_scipy_blackman_firwin(M, h):
    """Windowed-sinc design with a symmetric Blackman window and unit DC gain is what
    scipy's firwin builds for a cut-off of 1/M of Nyquist."""
    ref = scipy.signal.firwin(2 * h + 1, 1.0 / M, window="blackman", scale=True)
    g = subband.prototype(M, h)
    assert np.max(np.abs(g - ref)) < 1e-15
    assert abs(g.sum() - 1.0) < 1e-14 and np.allclose(g, g[::-1], atol=0, rtol=0)


@pytest.mark.parametrize("M,h", [(16, 64), (4, 9)])
def test_equals_mix_filter_decimate_chain(M, h):
    """Band b = mix the capture down by f_b, convolve with g (numpy), keep n = m M."""
    rng = _rng(1)
    C, N = 2, 40 * M
    x = _cn(rng, (C, N))
    z = subband.subbands(x, M, h)
    g = subband.prototype(M, h)
    n = np.arange(N)
    for b in range(M):
        fb = (b - M // 2) / M
        for c in range(C):
            full = np.convolve(x[c] * np.exp(-2j * np.pi * fb * n), g)       # full[n'] = sum g[k] x[n' - k]
            ref = full[np.arange(N // M) * M + h]
            assert np.max(np.abs(z[b, c] - ref)) < 1e-12, (b, c)


def test_tone_at_band_centre_passes_unit_gain_and_nowhere_else():
    """A tone at f_b leaves band b with modulus 1 and phase exp(j 2 pi f_b m M) away from
    the capture ends; every other band holds less than the Blackman design's stop-band
    level (about -74 dB; 3e-4 allowed)."""
    M, h = 16, 64
    N = 200 * M
    n = np.arange(N)
    interior = slice(h // M + 1, N // M - h // M - 1)
    for b in (0, 3, 8, 13):
        fb = (b - M // 2) / M
        x = np.exp(2j * np.pi * fb * n)
        z = subband.subbands(x, M, h)[:, 0, :]
        m = np.arange(N // M)
        assert np.max(np.abs(z[b, interior] - np.exp(2j * np.pi * fb * m * M)[interior])) < 1e-12
        others = np.delete(np.abs(z[:, interior]), b, axis=0)
        assert others.max() < 3e-4, (b, others.max())


def test_shift_by_m_samples_shifts_output_by_one():
    M, h = 8, 32
    rng = _rng(2)
    N = 64 * M
    x = _cn(rng, N)
    xs = np.zeros_like(x)
    xs[M:] = x[:-M]
    z = subband.subbands(x, M, h)[:, 0]
    zs = subband.subbands(xs, M, h)[:, 0]
    keep = N // M - h // M - 1          # outputs whose taps stay inside the shorter capture
    assert np.max(np.abs(zs[:, 1:keep] - z[:, :keep - 1])) < 1e-12


def test_literal_loops_tiny():
    M, h = 4, 6
    rng = _rng(3)
    x = _cn(rng, (2, 5 * M))
    g = subband.prototype(M, h)
    z = subband.subbands(x, M, h)
    for b in range(M):
        for c in range(2):
            for m in range(5):
                acc = 0j
                for t in range(-h, h + 1):
                    i = m * M - t
                    if 0 <= i < x.shape[1]:
                        acc += g[t + h] * x[c, i] * complex(math.cos(2 * math.pi * (b - M / 2) * t / M),
                                                            math.sin(2 * math.pi * (b - M / 2) * t / M))
                assert abs(z[b, c, m] - acc) < 1e-13


def test_band_layout_helpers():
    st = np.arange(2 * 3 * 6, dtype=np.float64).reshape(2, 3, 6)
    sb = subband.states_for_bands(st, 4)
    assert sb.shape == (2, 12, 6)
    for b in range(4):
        assert np.array_equal(sb[:, 3 * b:3 * b + 3], st)
    assert subband.pairs_for_bands([(0, 1), (2, 0)], 3, 2) == [(0, 1), (2, 0), (3, 4), (5, 3)]
