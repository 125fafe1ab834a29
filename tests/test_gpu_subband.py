"""Parity of the gfx950 sub-band split (geoloc_subbands) with the FP64 oracle, and of the
coarse map computed from its output with the oracle's map of the oracle's bands."""
import math

import numpy as np
import pytest

import oracle
from oracle import subband as osub
from helpers import DIRECT_TOL, err_J, log, require_gpu
from paper_2508_06672_amd import configs, sim

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def G():
    from paper_2508_06672_amd import geoloc
    geoloc.load()
    return geoloc


def _rng(seed):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))


def _tol(M, h, x):
    """FP32 bound: each output sums 2h+1 products of taps (sum |g| < 1.2) and samples; allow
    4 unit roundoffs per term of the worst case."""
    return 4.0 * (2 * h + 1) * 2.0 ** -24 * 1.2 * float(np.max(np.abs(x)))


@pytest.mark.parametrize("C,N,M,h", [(2, 16 * 1000, 16, 64), (3, 8 * 333, 8, 32), (1, 32 * 70, 32, 63),
                                     (2, 4 * 17, 4, 9), (2, 640, 1, 5), (1, 16 * 64, 16, 127)])
def test_subbands_match_oracle(torch, G, C, N, M, h):
    """Ragged output counts (not multiples of the 64-output workgroup), inputs shorter than
    the filter span, one band (the low-pass is then the identity), the largest tap table."""
    rng = _rng(C * N + M)
    x = ((rng.standard_normal((C, N)) + 1j * rng.standard_normal((C, N))) / math.sqrt(2)).astype(np.complex64)
    log(f"subbands C={C} N={N} M={M} h={h}")
    z = G.subbands(torch.from_numpy(x).cuda(), M, h)
    torch.cuda.synchronize()
    zg = z.cpu().numpy().reshape(M, C, N // M)
    zo = osub.subbands(x, M, h)
    e = float(np.max(np.abs(zg - zo)))
    assert e <= _tol(M, h, x), (e, _tol(M, h, x))
    if M == 1:
        assert np.max(np.abs(zg[0] - x)) <= 1e-6


def test_subbands_full_capture_and_stream(torch, G):
    """The proposal's split (16 bands, 129 taps) of a full 1e6-sample, 2-receiver scenario
    on a side stream, into a caller-provided buffer."""
    wl = configs.PROPOSAL
    scn = sim.make_scenario(wl, 5)
    M, h = 16, 64
    caps = torch.from_numpy(scn.captures).cuda()
    out = torch.empty((M * wl.n_rx, wl.n_samples // M), dtype=torch.complex64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        G.subbands(caps, M, h, out=out, stream=s)
    s.synchronize()
    zg = out.cpu().numpy().reshape(M, wl.n_rx, -1)
    log("subbands full: oracle")
    zo = osub.subbands(scn.captures, M, h)
    assert float(np.max(np.abs(zg - zo))) <= _tol(M, h, scn.captures)


def test_coarse_subband_map_matches_oracle(torch, G):
    """Coarse map over the 16 decimated bands (band-major receivers, one pair per band),
    as the learned proposal computes it, against the oracle's map of the oracle's bands."""
    wl = configs.PROPOSAL.with_(n_rows=64, n_cols=64, n_samples=200_000)
    scn = sim.make_scenario(wl, 6)
    M, h = 16, 64
    lat = scn.lat[8::16][:16]
    lon = scn.lon[8::16][:16]
    st = osub.states_for_bands(scn.states, M)
    pairs = osub.pairs_for_bands(list(wl.pairs), wl.n_rx, M)
    zo = osub.subbands(scn.captures, M, h).reshape(M * wl.n_rx, -1).astype(np.complex64)
    log("coarse subband map: oracle")
    Jo = oracle.map_rect(lat, lon, zo, st, wl.step_len // M, wl.fs_hz / M, wl.fc_hz, pairs=pairs,
                         radius=wl.earth_radius_m)
    caps = torch.from_numpy(scn.captures).cuda()
    z = G.subbands(caps, M, h)
    with G.Plan(n_rx=M * wl.n_rx, n_samples=wl.n_samples // M, step_len=wl.step_len // M, fs_hz=wl.fs_hz / M,
                fc_hz=wl.fc_hz, lat=lat, lon=lon, pairs=pairs, earth_radius_m=wl.earth_radius_m) as plan:
        J = plan.map(z, st)
        torch.cuda.synchronize()
        Jg = J.cpu().numpy().astype(np.float64)
    e = err_J(Jg, Jo)
    log(f"  err_J = {e:.3g}")
    assert e <= DIRECT_TOL
