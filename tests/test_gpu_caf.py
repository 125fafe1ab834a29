"""Parity of the MFMA CAF-table path with the FP64 CAF-table oracle (same lag window,
Doppler bins and bilinear interpolation), called through the C ABI."""
import numpy as np
import pytest

import oracle
from oracle import caf as ocaf
from helpers import check_argmax, check_cells, err_J, log, require_gpu
from paper_2508_06672_amd import agreement, configs, sim

pytestmark = pytest.mark.gpu

CAF_TOL = 1e-2          # normalised max |J error| for BF16 / FP16 inputs, FP32 accumulation


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def G():
    from paper_2508_06672_amd import geoloc
    geoloc.load()
    return geoloc


def _window(info):
    return info["caf_lag_lo"], info["caf_lags"], info["caf_nu_lo_hz"], info["caf_nu_hi_hz"], info["caf_bins"]


@pytest.mark.parametrize("method", ["bf16", "fp16"])
def test_caf_table_matches_fp64_table(torch, G, method):
    wl = configs.CAF_SMALL
    scn = sim.make_scenario(wl, 1)
    m = G.CAF_BF16 if method == "bf16" else G.CAF_FP16
    caps = torch.from_numpy(scn.captures).cuda()
    with G.Plan.for_scenario(scn, method=m, caf_lags=configs.CAF_LAGS, caf_bins=configs.CAF_BINS) as plan:
        T = plan.caf_table(caps, scn.states).cpu().numpy()
        lag_lo, n_lags, lo, hi, M = _window(plan.info())
    assert n_lags == configs.CAF_LAGS and M == configs.CAF_BINS
    nu = ocaf.bins(lo, hi, M)
    for k in range(wl.n_steps):
        log(f"caf table {method} step {k}")
        To = ocaf.table(scn.captures[0], scn.captures[1], k, wl.step_len, wl.fs_hz, lag_lo, n_lags, nu)
        e = np.max(np.abs(T[k] - To)) / np.max(np.abs(To))
        log(f"  max |T err| / max |T| = {e:.3g}")
        assert e <= (1e-2 if method == "bf16" else 2e-3)


@pytest.mark.parametrize("method", ["bf16", "fp16"])
@pytest.mark.parametrize("seed", [0, 3])
def test_caf_map_matches_caf_oracle(torch, G, method, seed):
    wl = configs.CAF_SMALL
    scn = sim.make_scenario(wl, seed)
    m = G.CAF_BF16 if method == "bf16" else G.CAF_FP16
    caps = torch.from_numpy(scn.captures).cuda()
    with G.Plan.for_scenario(scn, method=m, caf_lags=configs.CAF_LAGS, caf_bins=configs.CAF_BINS) as plan:
        Jg = plan.map(caps, scn.states).cpu().numpy().astype(np.float64)
        lag_lo, n_lags, lo, hi, M = _window(plan.info())
    la, lo_ = sim.points_of(scn)
    Jo = ocaf.caf_map_points(la, lo_, scn.captures, scn.states, wl.step_len, wl.fs_hz, wl.fc_hz, list(wl.pairs),
                             lag_lo, n_lags, lo, hi, M)
    e = err_J(Jg, Jo)
    Jd = oracle.map_scenario(scn)
    log(f"caf map {method} seed {seed}: err vs CAF oracle {e:.3g}, CAF oracle vs direct oracle {err_J(Jo, Jd):.3g}")
    assert e <= CAF_TOL
    ag, ao = int(np.argmax(Jg)), int(np.argmax(Jo))
    check_cells(Jo, wl.n_cols, ag, ao, CAF_TOL, agreement.mirror_cell(wl, scn.lat, scn.lon, ao))


def test_caf_literal_window_and_round_mode(torch, G):
    """The literal +-40 kHz, 256-bin window (bins wider than the Doppler main lobe) still
    matches the FP64 CAF oracle with the same window; ROUND delay and MAG accumulation too."""
    wl = configs.CAF_SMALL
    scn = sim.make_scenario(wl, 2)
    caps = torch.from_numpy(scn.captures).cuda()
    lo, hi = configs.CAF_LITERAL_WINDOW_HZ
    with G.Plan.for_scenario(scn, method=G.CAF_BF16, caf_lags=configs.CAF_LAGS, caf_bins=configs.CAF_BINS,
                             caf_nu_lo_hz=lo, caf_nu_hi_hz=hi, delay_mode=G.DELAY_ROUND,
                             accum_mode=G.ACC_MAG) as plan:
        Jg = plan.map(caps, scn.states).cpu().numpy().astype(np.float64)
        lag_lo, n_lags, lo2, hi2, M = _window(plan.info())
    assert (lo2, hi2) == (lo, hi)
    la, lo_ = sim.points_of(scn)
    Jo = ocaf.caf_map_points(la, lo_, scn.captures, scn.states, wl.step_len, wl.fs_hz, wl.fc_hz, list(wl.pairs),
                             lag_lo, n_lags, lo, hi, M, delay_mode=oracle.ROUND, accum_mode=oracle.MAG)
    assert err_J(Jg, Jo) <= CAF_TOL


def test_caf_three_pairs_and_fitted_window(torch, G):
    wl = configs.SMALL.with_(rx_along_track_m=(-25e3, 25e3, 0.0), rx_cross_track_m=(0.0, 0.0, 30e3),
                             pairs=((0, 1), (0, 2), (1, 2)), n_rows=40, n_cols=33, n_samples=16000, step_len=8000)
    scn = sim.make_scenario(wl, 4)
    caps = torch.from_numpy(scn.captures).cuda()
    with G.Plan.for_scenario(scn, method=G.CAF_BF16) as plan:
        Jg = plan.map(caps, scn.states).cpu().numpy().astype(np.float64)
        lag_lo, n_lags, lo, hi, M = _window(plan.info())
    la, lo_ = sim.points_of(scn)
    Jo = ocaf.caf_map_points(la, lo_, scn.captures, scn.states, wl.step_len, wl.fs_hz, wl.fc_hz, list(wl.pairs),
                             lag_lo, n_lags, lo, hi, M)
    Jd = oracle.map_scenario(scn)
    log(f"fitted window lags [{lag_lo}, +{n_lags}) bins [{lo:.1f}, {hi:.1f}] x {M}: err {err_J(Jg, Jo):.3g}, "
        f"vs direct {err_J(Jg, Jd):.3g}")
    assert err_J(Jg, Jo) <= CAF_TOL
    # with a fitted window the CAF map is also close to the direct map itself
    assert err_J(Jg, Jd) <= 2 * CAF_TOL


def test_caf_window_validation(torch, G):
    wl = configs.CAF_SMALL
    scn = sim.make_scenario(wl, 0)
    caps = torch.from_numpy(scn.captures).cuda()
    with G.Plan.for_scenario(scn, method=G.CAF_BF16, caf_lags=8) as plan:
        with pytest.raises(G.GeolocError) as ei:
            plan.map(caps, scn.states)
        assert ei.value.status == G.EINVAL
    with G.Plan.for_scenario(scn, method=G.CAF_BF16, caf_nu_lo_hz=0.0, caf_nu_hi_hz=100.0) as plan:
        with pytest.raises(G.GeolocError) as ei:
            plan.map(caps, scn.states)
        assert ei.value.status == G.EINVAL


def test_caf_1e6_map_agrees_with_direct(torch, G):
    """At the full 1000 x 1000, 1e6-sample size: the BF16 CAF map's peak is within one cell
    of the direct FP32 map's peak or its mirror when that peak is well-conditioned, and
    tol-optimal on the direct map otherwise."""
    wl = configs.MAP_1E6
    scn = sim.make_scenario(wl, 0)
    caps = torch.from_numpy(scn.captures).cuda()
    with G.Plan.for_scenario(scn) as pd:
        Jd = pd.map(caps, scn.states)
        ad = int(pd.argmax(Jd)[0][0])
        Jd = Jd.cpu().numpy().astype(np.float64)
    with G.Plan.for_scenario(scn, method=G.CAF_BF16) as pc:
        Jc = pc.map(caps, scn.states)
        ac = int(pc.argmax(Jc)[0][0])
        Jc = Jc.cpu().numpy().astype(np.float64)
        info = pc.info()
    e = err_J(Jc, Jd)
    log(f"1e6 CAF window lags {info['caf_lags']} bins {info['caf_bins']}: err vs direct {e:.3g}, "
        f"argmax {ac} vs {ad}")
    check_cells(Jd, wl.n_cols, ac, ad, CAF_TOL, agreement.mirror_cell(wl, scn.lat, scn.lon, ad))
    assert e <= 5e-2


def test_caf_sinc_delay(torch, G):
    """The CAF map read with the eight windowed-sinc lag taps (BF16 and FP16) against the
    FP64 CAF oracle with the same window and taps, and the FP32 direct SINC map."""
    wl = configs.CAF_SMALL
    scn = sim.make_scenario(wl, 5)
    caps = torch.from_numpy(scn.captures).cuda()
    la, lo_ = sim.points_of(scn)
    Jd = oracle.map_scenario(scn, delay_mode=oracle.SINC)
    for m in (G.CAF_BF16, G.CAF_FP16):
        with G.Plan.for_scenario(scn, method=m, delay_mode=G.DELAY_SINC) as plan:
            Jg = plan.map(caps, scn.states).cpu().numpy().astype(np.float64)
            lag_lo, n_lags, lo, hi, M = _window(plan.info())
        Jo = ocaf.caf_map_points(la, lo_, scn.captures, scn.states, wl.step_len, wl.fs_hz, wl.fc_hz, list(wl.pairs),
                                 lag_lo, n_lags, lo, hi, M, delay_mode=oracle.SINC)
        log(f"caf sinc method {m}: err vs CAF oracle {err_J(Jg, Jo):.3g}, vs direct {err_J(Jg, Jd):.3g}")
        assert err_J(Jg, Jo) <= CAF_TOL
        assert err_J(Jo, Jd) <= 1e-2
