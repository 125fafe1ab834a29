"""Parity of the gfx950 direct path (geometry, FP32 correlation, sum, argmax) with the
FP64 oracle, called through the C ABI."""
import math

import numpy as np
import pytest

import oracle
from oracle import peaks as opeaks
from helpers import DIRECT_TOL, check_argmax, err_J, log, require_gpu
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


def _gpu_map(torch, G, scn, **kw):
    caps = torch.from_numpy(scn.captures).cuda()
    with G.Plan.for_scenario(scn, **kw) as plan:
        J = plan.map(caps, scn.states)
        torch.cuda.synchronize()
        return J.cpu().numpy().astype(np.float64)


def test_geometry_parity(torch, G):
    for wl in (configs.SMALL, configs.MAP_1E6.with_(n_rows=37, n_cols=29, n_samples=50_000, step_len=10_000)):
        scn = sim.make_scenario(wl, 3)
        log(f"geometry {wl.name}")
        xyz = oracle.grid_ecef(*sim.points_of(scn), wl.earth_radius_m)
        Do, nuo = oracle.geometry(xyz, scn.states, (0, 1), wl.fs_hz, wl.fc_hz)
        with G.Plan.for_scenario(scn) as plan:
            D, nu = plan.geometry(scn.states)
            D1, nu1 = plan.geometry(scn.states, step_lo=1, n_steps=2)
            torch.cuda.synchronize()
            D, nu, D1, nu1 = (t.cpu().numpy() for t in (D, nu, D1, nu1))
        assert np.max(np.abs(D - Do)) <= 1e-8, np.max(np.abs(D - Do))
        assert np.max(np.abs(nu - nuo)) <= 1e-8, np.max(np.abs(nu - nuo))
        assert np.array_equal(D1, D[1:3]) and np.array_equal(nu1, nu[1:3])


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_direct_parity_small(torch, G, seed):
    scn = sim.make_scenario(configs.SMALL, seed)
    log(f"direct small seed {seed}")
    Jo = oracle.map_scenario(scn)
    Jg = _gpu_map(torch, G, scn)
    e = err_J(Jg, Jo)
    log(f"  err_J = {e:.3g}")
    assert e <= DIRECT_TOL
    check_argmax(Jg, Jo, DIRECT_TOL)


@pytest.mark.parametrize("delay,accum", [(1, 0), (0, 1), (1, 1)])
def test_direct_modes(torch, G, delay, accum):
    scn = sim.make_scenario(configs.SMALL.with_(n_samples=12000), 5)
    log(f"direct modes delay={delay} accum={accum}")
    Jo = oracle.map_scenario(scn, delay_mode=delay, accum_mode=accum)
    Jg = _gpu_map(torch, G, scn, delay_mode=delay, accum_mode=accum)
    assert err_J(Jg, Jo) <= DIRECT_TOL
    check_argmax(Jg, Jo, DIRECT_TOL)


def test_direct_three_receivers_three_pairs(torch, G):
    wl = configs.SMALL.with_(rx_along_track_m=(-25e3, 25e3, 0.0), rx_cross_track_m=(0.0, 0.0, 30e3),
                             pairs=((0, 1), (2, 0), (1, 2)), n_rows=45, n_cols=38, n_samples=8000)
    scn = sim.make_scenario(wl, 6)
    log("direct three pairs")
    Jo = oracle.map_scenario(scn)
    Jg = _gpu_map(torch, G, scn)
    assert err_J(Jg, Jo) <= DIRECT_TOL
    check_argmax(Jg, Jo, DIRECT_TOL)


def test_direct_point_list_wide_lag_spread(torch, G):
    """Random points over a 500 km footprint at 10 MHz: a 256-point tile spans more lags
    than the LDS halo holds, which exercises the global-memory tap path."""
    wl = configs.MAP_1E6.with_(n_samples=20_000, step_len=10_000)
    scn = sim.make_scenario(wl, 7)
    la, lo = sim.points_of(scn)
    rng = np.random.Generator(np.random.PCG64(7))
    sel = rng.choice(la.size, 1500, replace=False)
    lat_p, lon_p = la[sel], lo[sel]
    log("direct point list")
    Jo = oracle.map_points(lat_p, lon_p, scn.captures, scn.states, wl.step_len, wl.fs_hz, wl.fc_hz)
    caps = torch.from_numpy(scn.captures).cuda()
    with G.Plan(n_rx=2, n_samples=wl.n_samples, step_len=wl.step_len, fs_hz=wl.fs_hz, fc_hz=wl.fc_hz,
                lat=lat_p, lon=lon_p, grid_kind=G.GRID_POINTS) as plan:
        D, _ = plan.geometry(scn.states)
        spread = D.floor().cpu().numpy()
        assert np.max(spread[:, :256].max(1) - spread[:, :256].min(1)) > 512
        J = plan.map(caps, scn.states)
        torch.cuda.synchronize()
        Jg = J.cpu().numpy()
    assert err_J(Jg, Jo) <= DIRECT_TOL


def test_direct_ragged_shapes(torch, G):
    """Step length that is not a multiple of the 16-sample block nor of the LDS tile,
    grid edges that cut 16 x 16 tiles, and delays reaching past the capture ends."""
    wl = configs.SMALL.with_(n_rows=19, n_cols=23, n_samples=3 * 1301, step_len=1301)
    scn = sim.make_scenario(wl, 8)
    log("direct ragged")
    Jo = oracle.map_scenario(scn)
    Jg = _gpu_map(torch, G, scn)
    assert err_J(Jg, Jo) <= DIRECT_TOL
    # one point, one step
    wl1 = configs.SMALL.with_(n_rows=1, n_cols=1, n_samples=999, step_len=999)
    scn1 = sim.make_scenario(wl1, 9)
    Jo1 = oracle.map_scenario(scn1)
    Jg1 = _gpu_map(torch, G, scn1)
    assert abs(Jg1[0] - Jo1[0]) <= DIRECT_TOL * Jo1[0]


def test_accumulate_and_determinism(torch, G):
    scn = sim.make_scenario(configs.SMALL.with_(n_samples=8000), 10)
    caps = torch.from_numpy(scn.captures).cuda()
    with G.Plan.for_scenario(scn) as plan:
        J1 = plan.map(caps, scn.states).clone()
        J2 = plan.map(caps, scn.states).clone()
        J3 = plan.map(caps, scn.states, J=J2.clone(), accumulate=True)
        torch.cuda.synchronize()
    assert torch.equal(J1, J2)
    assert torch.allclose(J3, 2 * J1, rtol=1e-6, atol=0)


def test_argmax_rules(torch, G):
    scn = sim.make_scenario(configs.SMALL, 0)
    rng = np.random.Generator(np.random.PCG64(11))
    with G.Plan.for_scenario(scn) as plan:
        P = plan.n_points
        for trial in range(4):
            J = rng.integers(0, 50, P).astype(np.float32)         # many exact ties
            idx, val = plan.argmax(torch.from_numpy(J).cuda())
            i, v = opeaks.argmax(J)
            assert idx[0] == i and val[0] == v
            idx, val = plan.argmax(torch.from_numpy(J).cuda(), top_k=3, nms_radius=2)
            ref = opeaks.topk(J, plan.n_rows, plan.n_cols, 3, 2)
            assert list(idx) == [r[0] for r in ref]
        J = np.ones(P, dtype=np.float32)
        J[1234] = np.nan
        with pytest.raises(G.GeolocError) as ei:
            plan.argmax(torch.from_numpy(J).cuda())
        assert ei.value.status == G.ENAN


def test_map_1e6_sampled_points(torch, G):
    """The full 1000 x 1000-point, 1e6-sample map in the benchmark's launch
    configuration, checked at sampled points (random + a window around the peak)."""
    wl = configs.MAP_1E6
    scn = sim.make_scenario(wl, 0)
    log("1e6 map: gpu")
    Jg = _gpu_map(torch, G, scn)
    ag = int(np.argmax(Jg))
    rng = np.random.Generator(np.random.PCG64(12))
    r0, c0 = divmod(ag, wl.n_cols)
    win = [(r, c) for r in range(max(0, r0 - 5), min(wl.n_rows, r0 + 6))
           for c in range(max(0, c0 - 5), min(wl.n_cols, c0 + 6))]
    idx = np.unique(np.r_[rng.choice(wl.n_points, 256, replace=False), [r * wl.n_cols + c for r, c in win]])
    rows, cols = np.divmod(idx, wl.n_cols)
    log(f"1e6 map: oracle at {idx.size} points")
    Jo = oracle.map_points(scn.lat[rows], scn.lon[cols], scn.captures, scn.states, wl.step_len, wl.fs_hz, wl.fc_hz)
    e = float(np.max(np.abs(Jg[idx] - Jo)) / np.max(Jo))
    log(f"1e6 map: err_J = {e:.3g}")
    assert e <= DIRECT_TOL
    # the peak of the sampled window is the GPU's peak within tolerance
    assert Jo[np.searchsorted(idx, ag)] >= (1 - DIRECT_TOL) * np.max(Jo)


def test_factored_and_pointwise_kernels_agree_at_1e6(torch, G):
    """The tile-factored kernel (default on RECT grids) and the per-point kernel compute
    the same 1e6-point map to FP32 rounding."""
    wl = configs.MAP_1E6
    scn = sim.make_scenario(wl, 1)
    log("1e6 map: factored vs pointwise")
    Jf = _gpu_map(torch, G, scn)
    Jp = _gpu_map(torch, G, scn, method=G.DIRECT_FP32_POINTWISE)
    e = err_J(Jf, Jp)
    log(f"  factored vs pointwise err_J = {e:.3g}")
    assert e <= 2e-5
    check_argmax(Jf, Jp, 2e-5)


def test_factored_kernel_defers_wide_tiles(torch, G):
    """8 km cells at 10 MHz: a 16 x 16 tile spans hundreds of lags, so the factored kernel
    hands every step to the per-point kernel; a 0.5 km grid next to it is factored. Both
    match the oracle, in LINEAR and ROUND delay."""
    for spacing, name in ((8000.0, "wide"), (500.0, "narrow")):
        wl = configs.MAP_1E6.with_(n_rows=37, n_cols=41, spacing_m=spacing, n_samples=30_000)
        scn = sim.make_scenario(wl, 11)
        for delay in (0, 1):
            log(f"factored {name} delay={delay}")
            Jo = oracle.map_scenario(scn, delay_mode=delay)
            Jg = _gpu_map(torch, G, scn, delay_mode=delay)
            assert err_J(Jg, Jo) <= DIRECT_TOL, (name, delay)
            check_argmax(Jg, Jo, DIRECT_TOL)


def test_sheared_tiles_match_oracle(torch, G):
    """On a 0.5 km grid the plan picks slanted (sheared) tiles of 256 to 1024 cells that
    follow the lines of equal delay, at a slope of whole or fractional columns per row;
    which slope depends on the geometry, so two seeds with opposite gradient signs are
    mapped, LINEAR and SINC. All agree with the oracle over the whole grid."""
    shears = set()
    cells = set()
    for seed, delay in ((0, 0), (3, 0), (3, 2)):
        wl = configs.MAP_1E6.with_(n_rows=150, n_cols=170, n_samples=30_000)
        scn = sim.make_scenario(wl, seed)
        log(f"sheared tiles seed {seed} delay {delay}")
        Jo = oracle.map_scenario(scn, delay_mode=delay)
        caps = torch.from_numpy(scn.captures).cuda()
        with G.Plan.for_scenario(scn, delay_mode=delay) as plan:
            Jg = plan.map(caps, scn.states).cpu().numpy().astype(np.float64)
            info = plan.info()
        shears.add((info["tile_shear"], info["tile_transpose"]))
        cells.add(info["tile_rows"] * info["tile_cols"])
        log(f"  tile {info['tile_rows']}x{info['tile_cols']} shear {info['tile_shear'] / 256:+.3f} "
            f"transpose {info['tile_transpose']}")
        e = err_J(Jg, Jo)
        log(f"  err_J = {e:.3g}")
        assert e <= DIRECT_TOL
        check_argmax(Jg, Jo, DIRECT_TOL)
    assert cells <= {256, 512, 1024}
    assert any(sh != 0 for sh, _ in shears) and len({s for s, _ in shears}) >= 2


@pytest.mark.parametrize("accum", [0, 1])
def test_sinc_delay_factored_and_pointwise(torch, G, accum):
    """The eight-tap windowed-sinc delay on the small workload (tile-factored kernel) and
    on the same grid with the per-point kernel, against the oracle in SINC mode."""
    scn = sim.make_scenario(configs.SMALL.with_(n_samples=12000), 21)
    log(f"sinc delay accum={accum}")
    Jo = oracle.map_scenario(scn, delay_mode=oracle.SINC, accum_mode=accum)
    for method in (G.DIRECT_FP32, G.DIRECT_FP32_POINTWISE):
        Jg = _gpu_map(torch, G, scn, delay_mode=G.DELAY_SINC, accum_mode=accum, method=method)
        e = err_J(Jg, Jo)
        log(f"  method {method}: err_J = {e:.3g}")
        assert e <= DIRECT_TOL
        check_argmax(Jg, Jo, DIRECT_TOL)


def test_sinc_delay_wide_tiles_and_point_list(torch, G):
    """SINC on 8 km cells (every tile-step deferred to the per-point SINC kernel) and on a
    scattered point list at 10 MHz, against the oracle."""
    wl = configs.MAP_1E6.with_(n_rows=37, n_cols=41, spacing_m=8000.0, n_samples=30_000)
    scn = sim.make_scenario(wl, 22)
    log("sinc wide tiles")
    Jo = oracle.map_scenario(scn, delay_mode=oracle.SINC)
    Jg = _gpu_map(torch, G, scn, delay_mode=G.DELAY_SINC)
    assert err_J(Jg, Jo) <= DIRECT_TOL
    wl = configs.MAP_1E6.with_(n_samples=20_000, step_len=10_000)
    scn = sim.make_scenario(wl, 23)
    la, lo = sim.points_of(scn)
    rng = np.random.Generator(np.random.PCG64(23))
    sel = rng.choice(la.size, 700, replace=False)
    log("sinc point list")
    Jo = oracle.map_points(la[sel], lo[sel], scn.captures, scn.states, wl.step_len, wl.fs_hz, wl.fc_hz,
                           delay_mode=oracle.SINC)
    caps = torch.from_numpy(scn.captures).cuda()
    with G.Plan(n_rx=2, n_samples=wl.n_samples, step_len=wl.step_len, fs_hz=wl.fs_hz, fc_hz=wl.fc_hz,
                lat=la[sel], lon=lo[sel], grid_kind=G.GRID_POINTS, delay_mode=G.DELAY_SINC) as plan:
        Jg = plan.map(caps, scn.states).cpu().numpy()
    assert err_J(Jg, Jo) <= DIRECT_TOL


@pytest.mark.parametrize("delay,accum,spacing", [(0, 0, 500.0), (2, 1, 500.0), (1, 0, 500.0), (0, 0, 8000.0)])
def test_step_segments(torch, G, delay, accum, spacing):
    """A small grid with long steps: the factored kernel splits each 41,000-sample step into
    coherent segments (the last one 40 samples long) and adds their complex partial sums
    before |C|^2 (or |C|). On 8 km cells part of the tile-steps also go to the per-point pass
    after the segment reduction."""
    wl = configs.MAP_1E6.with_(n_rows=30, n_cols=41, spacing_m=spacing, n_samples=123_000, step_len=41_000)
    scn = sim.make_scenario(wl, 40 + delay)
    log(f"step segments delay={delay} accum={accum} spacing={spacing}")
    Jo = oracle.map_scenario(scn, delay_mode=delay, accum_mode=accum)
    caps = torch.from_numpy(scn.captures).cuda()
    with G.Plan.for_scenario(scn, delay_mode=delay, accum_mode=accum) as plan:
        Jg = plan.map(caps, scn.states).cpu().numpy().astype(np.float64)
        info = plan.info()
    log(f"  {info['step_segments']} segments of {info['segment_len']}, err_J = {err_J(Jg, Jo):.3g}")
    assert info["step_segments"] == 11 and info["segment_len"] == 4096
    assert err_J(Jg, Jo) <= DIRECT_TOL
    check_argmax(Jg, Jo, DIRECT_TOL)


@pytest.mark.parametrize("w,h,shear,tr,spacing,delay", [(16, 32, 0, 0, 8000.0, 0), (8, 64, 333, 1, 500.0, 0),
                                                        (4, 128, -700, 0, 500.0, 1), (32, 16, 150, 1, 8000.0, 1),
                                                        (4, 64, -100, 0, 500.0, 2), (16, 16, 1024, 1, 2000.0, 2),
                                                        (8, 128, -318, 0, 500.0, 0), (32, 32, 200, 1, 2000.0, 1),
                                                        (16, 64, 0, 0, 8000.0, 0), (8, 64, -318, 0, 500.0, 2),
                                                        (16, 64, -318, 0, 500.0, 2), (32, 32, 200, 1, 2000.0, 2)])
def test_fixed_tilings_match_oracle(torch, G, w, h, shear, tr, spacing, delay):
    """Tilings the plan would not pick, fixed through geoloc_set_tiling: 512- and 1024-cell
    tiles on 8 km cells (most tile-steps deferred to the second factored pass and the
    per-point kernel in 256-cell parts), 1024-cell tiles (four cells per thread) in all three delay modes, steep and
    fractional shears, both orientations, SINC on 256- to 1024-cell tiles; all match the oracle.
    Returning to the per-map choice works, and bad tilings are rejected."""
    wl = configs.MAP_1E6.with_(n_rows=45, n_cols=52, spacing_m=spacing, n_samples=30_000)
    scn = sim.make_scenario(wl, 60 + w + h + delay)
    log(f"fixed tiling {w}x{h} shear {shear} transpose {tr} spacing {spacing} delay {delay}")
    Jo = oracle.map_scenario(scn, delay_mode=delay)
    caps = torch.from_numpy(scn.captures).cuda()
    with G.Plan.for_scenario(scn, delay_mode=delay) as plan:
        plan.set_tiling(w, h, shear, tr)
        plan.set_timing(True)
        Jg = plan.map(caps, scn.states).cpu().numpy().astype(np.float64)
        info = plan.info()
        assert (info["tile_cols"], info["tile_rows"], info["tile_shear"], info["tile_transpose"]) == (w, h, shear, tr)
        log(f"  err_J = {err_J(Jg, Jo):.3g}, per-point pass {info['interp_ms']:.3f} ms")
        assert err_J(Jg, Jo) <= DIRECT_TOL
        check_argmax(Jg, Jo, DIRECT_TOL)
        plan.set_tiling(0)
        J2 = plan.map(caps, scn.states).cpu().numpy().astype(np.float64)
        assert err_J(J2, Jo) <= DIRECT_TOL
        for bad in [(10, 10, 0, 0), (16, 16, 1025, 0), (16, 16, 0, 2), (32, 64, 0, 0)]:
            with pytest.raises(G.GeolocError) as ei:
                plan.set_tiling(*bad)
            assert ei.value.status == G.EINVAL, bad


@pytest.mark.parametrize("block,delay,spacing,step", [(64, 0, 500.0, 10_000), (256, 0, 500.0, 10_000),
                                                     (256, 1, 2000.0, 10_000), (256, 2, 500.0, 10_000),
                                                     (256, 0, 8000.0, 7_000), (256, 0, 500.0, 41_000)])
def test_taylor_blocks_match_oracle(torch, G, block, delay, spacing, step):
    """The factored kernel with Taylor blocks of 64 samples and of 256 (four 64-sample blocks
    moved to the long block's centre and summed across a lane quad), fixed through
    geoloc_set_taylor_block: steps of 10,000 samples end in a partial long block, 8 km cells
    need more Taylor terms (part of the tile-steps go to the per-point pass), 41,000-sample
    steps are split into segments. All match the oracle; bad lengths are rejected."""
    wl = configs.MAP_1E6.with_(n_rows=37, n_cols=58, spacing_m=spacing, n_samples=3 * step, step_len=step)
    scn = sim.make_scenario(wl, 90 + delay + block)
    log(f"taylor block {block} delay {delay} spacing {spacing} step {step}")
    Jo = oracle.map_scenario(scn, delay_mode=delay)
    caps = torch.from_numpy(scn.captures).cuda()
    with G.Plan.for_scenario(scn, delay_mode=delay) as plan:
        plan.set_taylor_block(block)
        plan.set_timing(True)
        Jg = plan.map(caps, scn.states).cpu().numpy().astype(np.float64)
        info = plan.info()
        log(f"  tile {info['tile_cols']}x{info['tile_rows']} segments {info['step_segments']} "
            f"err_J = {err_J(Jg, Jo):.3g}, per-point pass {info['interp_ms']:.3f} ms")
        assert info["taylor_block"] == block
        assert err_J(Jg, Jo) <= DIRECT_TOL
        check_argmax(Jg, Jo, DIRECT_TOL)
        for bad in (1, 128, 512, -64):
            with pytest.raises(G.GeolocError) as ei:
                plan.set_taylor_block(bad)
            assert ei.value.status == G.EINVAL, bad
        plan.set_taylor_block(0)
        J2 = plan.map(caps, scn.states).cpu().numpy().astype(np.float64)
        assert plan.info()["taylor_block"] in (64, 256)
        assert err_J(J2, Jo) <= DIRECT_TOL


@pytest.mark.parametrize("w,h,delay,step", [(16, 16, 0, 10_000), (16, 32, 1, 7_000), (16, 64, 0, 10_000),
                                          (32, 32, 1, 10_000), (8, 32, 2, 7_000), (16, 64, 0, 41_000),
                                          (16, 64, 2, 10_000)])
def test_deferred_pairs_second_factored_pass(torch, G, w, h, delay, step):
    """8 km cells with 256-sample Taylor blocks defer many (tile, step) pairs; a second
    factored pass takes them again in 256-cell parts of the tile with 64-sample blocks and
    the per-point kernel adds the parts it defers again. With 256- to 1024-cell tiles, item
    groups or (41,000-sample steps) segments, the map matches the oracle and the map made
    with 64-sample blocks throughout."""
    wl = configs.MAP_1E6.with_(n_rows=47, n_cols=61, spacing_m=8000.0, n_samples=3 * step, step_len=step)
    scn = sim.make_scenario(wl, 700 + w + h + delay)
    log(f"second pass: tile {w}x{h} delay {delay} step {step}")
    Jo = oracle.map_scenario(scn, delay_mode=delay)
    caps = torch.from_numpy(scn.captures).cuda()
    with G.Plan.for_scenario(scn, delay_mode=delay) as plan:
        plan.set_tiling(w, h, 0, 0)
        plan.set_taylor_block(256)
        plan.set_timing(True)
        J256 = plan.map(caps, scn.states).cpu().numpy().astype(np.float64)
        info = plan.info()
        plan.set_taylor_block(64)
        J64 = plan.map(caps, scn.states).cpu().numpy().astype(np.float64)
    log(f"  segments {info['step_segments']}: err_J {err_J(J256, Jo):.3g} "
        f"(64-sample blocks {err_J(J64, Jo):.3g}), deferred passes {info['interp_ms']:.3f} ms")
    assert info["taylor_block"] == 256
    assert err_J(J256, Jo) <= DIRECT_TOL
    assert err_J(J64, Jo) <= DIRECT_TOL
    assert err_J(J256, J64) <= DIRECT_TOL
    check_argmax(J256, Jo, DIRECT_TOL)


@pytest.mark.parametrize("seed,n_cases,shapes", [
    (77, 20, [(16, 16), (8, 32), (4, 64), (32, 8), (64, 4), (16, 32), (8, 64), (4, 128), (32, 16), (128, 4)]),
    (78, 10, [(32, 32), (16, 64), (64, 16), (8, 128), (128, 8), (4, 256), (256, 4)])])
def test_random_tilings_on_ragged_grids(torch, G, seed, n_cases, shapes):
    """Seeded random tilings (shape, shear in 1/256 column per row, orientation) on grids of
    odd sizes, some narrower than a tile, with one or two cells per thread, and with four
    (1024-cell tiles): every cell is covered exactly once and the map matches the oracle."""
    rng = np.random.Generator(np.random.PCG64(seed))
    wl0 = configs.MAP_1E6.with_(n_samples=20_000, step_len=10_000)
    for case in range(n_cases):
        rows, cols = int(rng.integers(3, 70)), int(rng.integers(3, 70))
        w, h = shapes[int(rng.integers(len(shapes)))]
        shear = int(rng.integers(-1024, 1025))
        tr = int(rng.integers(2))
        wl = wl0.with_(n_rows=rows, n_cols=cols, spacing_m=float(rng.choice([500.0, 2000.0])))
        scn = sim.make_scenario(wl, 500 + case + 100 * (seed - 77))
        Jo = oracle.map_scenario(scn)
        caps = torch.from_numpy(scn.captures).cuda()
        with G.Plan.for_scenario(scn) as plan:
            plan.set_tiling(w, h, shear, tr)
            Jg = plan.map(caps, scn.states).cpu().numpy().astype(np.float64)
        e = err_J(Jg, Jo)
        log(f"  case {case}: {rows}x{cols} tile {w}x{h} shear {shear} transpose {tr}: err_J {e:.3g}")
        assert e <= DIRECT_TOL, (case, rows, cols, w, h, shear, tr)
