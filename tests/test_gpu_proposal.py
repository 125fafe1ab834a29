"""The learned-proposal pipeline on the GPU: refine/fallback plumbing on a small grid,
and (when trained weights are present) what the trained network gains over choosing
tiles from the coarse map alone."""
import os

import numpy as np
import pytest

from helpers import err_J, log, require_gpu
from paper_2508_06672_amd import configs, sim

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def P():
    from paper_2508_06672_amd import geoloc, proposal
    geoloc.load()
    return proposal


SMALL_WL = configs.PROPOSAL.with_(name="proposal_small", n_rows=128, n_cols=160, n_samples=40_000,
                                  step_len=10_000, n_snapshots=3, waveform="chirp")


def _scenario(P, wl, seed):
    snaps = sim.make_snapshots(wl, seed)
    caps, states, _ = P.stack_snapshots(snaps, wl.pairs)
    return snaps[0], caps, states


def test_zero_weight_network_falls_back_to_the_full_map(torch, P):
    from paper_2508_06672_amd import geoloc
    wl = SMALL_WL
    net = geoloc.CNN(3, 32, 4, wl.n_rows // P.TILE, wl.n_cols // P.TILE, max_batch=4)
    prop = P.Proposer(wl, net)
    scn, capn, states = _scenario(P, wl, 1)
    caps = torch.from_numpy(capn).cuda()
    prop.set_grid(scn.lat, scn.lon)
    r = prop.run(caps, states)
    a_full, v_full, _ = prop.full_map(caps, states)
    assert r["fallback"] and abs(r["score"] - P.TOPK / (8 * 10)) < 1e-5
    assert r["idx"] == a_full and r["val"] == v_full
    prop.close()
    net.close()


def test_top_two_peaks_of_refined_tiles(torch, P):
    """run_top with no fallback: the k best cells of the chosen tiles' map, each more than the
    exclusion radius from the ones before, read off the full map at those cells (the refine
    map equals it to FP32 rounding); with a zero-weight network it falls back to the full
    map's own top-k."""
    from paper_2508_06672_amd import geoloc
    wl = SMALL_WL
    net = geoloc.CNN(3, 32, 4, wl.n_rows // P.TILE, wl.n_cols // P.TILE, max_batch=4)
    scn, capn, states = _scenario(P, wl, 3)
    caps = torch.from_numpy(capn).cuda()
    for threshold, fallback in ((0.0, False), (1.0, True)):
        prop = P.Proposer(wl, net, threshold=threshold)
        prop.set_grid(scn.lat, scn.lon)
        r = prop.run_top(caps, states, k=2, radius=3)
        _, _, Jf = prop.full_map(caps, states)
        Jf = Jf.cpu().numpy().astype(np.float64)
        assert r["fallback"] == fallback and len(r["idx"]) == 2
        if fallback:
            i, v = prop.full.argmax(prop.full.map(caps, states), top_k=2, nms_radius=3)
            assert list(r["idx"]) == [int(t) for t in i]
        else:
            # the same cells on the full map: the refined tiles' best two, 3 cells apart
            _, _, flat = P.tile_points(scn.lat, scn.lon, r["tiles"])
            Js = Jf[flat]
            a, b = r["idx"]
            assert Jf[a] >= (1 - 2e-5) * Js.max()
            ra, ca = divmod(a, wl.n_cols)
            far = [f for f in flat if max(abs(f // wl.n_cols - ra), abs(f % wl.n_cols - ca)) > 3]
            assert max(abs(b // wl.n_cols - ra), abs(b % wl.n_cols - ca)) > 3
            assert Jf[b] >= (1 - 2e-5) * Jf[far].max()
        prop.close()
    net.close()


def test_refined_tiles_reproduce_the_full_map(torch, P):
    """The refine map (a POINTS grid of whole tiles) at the chosen tiles' cells equals the
    full-grid map at those cells to FP32 rounding (the full grid may use sheared tiles, so
    the sums group differently), as does the per-point kernel; the same points set on the
    device from the tile list give the same map bit for bit (and within rounding with 256-sample
    Taylor blocks), a tile index outside the grid
    gives NaN, and bad sizes are rejected. When the chosen tiles contain the full map's peak
    the refined peak is that peak."""
    from paper_2508_06672_amd import geoloc
    wl = SMALL_WL
    net = geoloc.CNN(3, 32, 4, wl.n_rows // P.TILE, wl.n_cols // P.TILE, max_batch=4)
    prop = P.Proposer(wl, net)
    scn, capn, states = _scenario(P, wl, 2)
    caps = torch.from_numpy(capn).cuda()
    prop.set_grid(scn.lat, scn.lon)
    a_full, v_full, Jf = prop.full_map(caps, states)
    Jf = Jf.cpu().numpy()
    with geoloc.Plan(n_rx=prop.n_vrx, n_samples=wl.n_samples, step_len=wl.step_len, fs_hz=wl.fs_hz,
                     fc_hz=wl.fc_hz, lat=scn.lat, lon=scn.lon, pairs=prop.vpairs, earth_radius_m=wl.earth_radius_m,
                     method=geoloc.DIRECT_FP32_POINTWISE) as pw:
        Jp = pw.map(caps, states).cpu().numpy()
    assert err_J(Jf.astype(np.float64), Jp.astype(np.float64)) <= 2e-5
    tile_of = (a_full // wl.n_cols // P.TILE) * (wl.n_cols // P.TILE) + (a_full % wl.n_cols) // P.TILE
    tiles = [tile_of] + [t for t in range(P.TOPK) if t != tile_of][: P.TOPK - 1]
    plat, plon, idx = P.tile_points(scn.lat, scn.lon, tiles)
    prop.refine.set_grid(plat, plon)
    Jr = prop.refine.map(caps, states).cpu().numpy()
    assert float(np.max(np.abs(Jr.astype(np.float64) - Jf[idx]))) <= 2e-5 * float(Jf.max())
    # the same points set on the device from the tile list give the same map, bit for bit
    lat_d = torch.from_numpy(np.ascontiguousarray(scn.lat)).cuda()
    lon_d = torch.from_numpy(np.ascontiguousarray(scn.lon)).cuda()
    prop.refine.set_points_from_tiles(lat_d, lon_d, P.TILE, tiles)
    Jd = prop.refine.map(caps, states).cpu().numpy()
    assert np.array_equal(Jd, Jr)
    # a POINTS plan takes a fixed Taylor block length too
    prop.refine.set_taylor_block(256)
    J256 = prop.refine.map(caps, states).cpu().numpy().astype(np.float64)
    assert prop.refine.info()["taylor_block"] == 256
    assert float(np.max(np.abs(J256 - Jf[idx]))) <= 2e-5 * float(Jf.max())
    prop.refine.set_taylor_block(0)
    assert np.array_equal(prop.refine.map(caps, states).cpu().numpy(), Jr)
    assert prop.refine.info()["taylor_block"] == 64
    bad = list(tiles)
    bad[3] = (wl.n_rows // P.TILE) * (wl.n_cols // P.TILE)      # one past the last tile
    prop.refine.set_points_from_tiles(lat_d, lon_d, P.TILE, bad)
    with pytest.raises(geoloc.GeolocError) as ei:
        prop.refine.argmax(prop.refine.map(caps, states))
    assert ei.value.status == geoloc.ENAN
    for args in [(lat_d, lon_d, P.TILE, tiles[:-1]), (lat_d, lon_d, 7, tiles)]:
        with pytest.raises(geoloc.GeolocError) as ei:
            prop.refine.set_points_from_tiles(*args)
        assert ei.value.status == geoloc.EINVAL
    with pytest.raises(geoloc.GeolocError) as ei:
        prop.full.set_points_from_tiles(lat_d, lon_d, P.TILE, tiles)
    assert ei.value.status == geoloc.EINVAL
    i, v = prop.refine_tiles(caps, states, tiles)
    assert Jf[i] >= (1 - 4e-5) * v_full and abs(v - v_full) <= 2e-5 * v_full
    prop.close()
    net.close()


@pytest.mark.skipif(not os.path.exists(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                                    "paper_2508_06672_amd", "weights", "proposal_cnn.npz")),
                    reason="no trained proposal weights in the tree")
def test_trained_network_beats_coarse_map_tiles(torch, P):
    """On 100 held-out seeds the trained network's 16 tiles (no fallback: the tile choice
    itself) find the full map's peak, by the agreement rule, strictly more often than the
    16 best tiles of the coarse map itself: what the network adds to the method."""
    from paper_2508_06672_amd import geoloc
    theta, meta = P.load_weights()
    net = P.make_net(geoloc, meta, max_batch=64)
    net.set_params(theta)
    wl = P.TRAIN_WL
    prop = P.Proposer(wl, net, threshold=0.0)
    seeds = list(range(P.SEED_TEST, P.SEED_TEST + 100))
    try:
        res = P.evaluate(prop, wl, seeds, None)
    finally:
        prop.close()
        net.close()
    L, A = res["learned"], res["coarse_top16_ablation"]
    log(f"learned {L['agree_rate']:.3f} {L['rule']} | ablation {A['agree_rate']:.3f} {A['rule']}")
    assert L["agree_rate"] > A["agree_rate"]
