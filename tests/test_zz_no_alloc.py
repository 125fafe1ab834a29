"""geoloc_argmax_noalloc (no plan, no device allocation: its scratch is a static device array)
against geoloc_argmax on plans of the same grids, through the C ABI: bit-exact peaks and
values, two calls in a row with the second on a smaller map, top-k with the exclusion
window, a POINTS list, NaN and the argument errors."""
import numpy as np
import pytest

from helpers import log, require_gpu
from oracle import peaks as opeaks
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


def _maps(rng, P):
    yield rng.integers(0, 50, P).astype(np.float32)              # many exact ties
    yield rng.standard_normal(P).astype(np.float32) ** 2
    J = np.zeros(P, dtype=np.float32)
    J[P - 1] = 1.0                                                 # the last point alone
    yield J


def _compare(torch, G, plan, J, stream, top_k, radius):
    Jd = torch.from_numpy(J).cuda()
    a_idx, a_val = plan.argmax(Jd, top_k=top_k, nms_radius=radius)
    b_idx, b_val = G.geoloc_argmax_noalloc(Jd.data_ptr(), plan.grid_kind, plan.n_rows, plan.n_cols, top_k, radius,
                                           stream)
    assert list(b_idx) == list(a_idx)
    assert np.array_equal(b_val.view(np.uint32), a_val.view(np.uint32))
    return b_idx


def test_noalloc_argmax_matches_plan_argmax(torch, G):
    rng = np.random.Generator(np.random.PCG64(21))
    stream = torch.cuda.current_stream().cuda_stream
    big = sim.make_scenario(configs.SMALL, 0)                      # 101 x 101
    small = sim.make_scenario(configs.SMALL.with_(name="small", n_rows=33, n_cols=35, n_samples=8000,
                                                  step_len=4000), 0)
    for scn in (big, small):                                       # the second call is on a smaller map
        with G.Plan.for_scenario(scn) as plan:
            log(f"noalloc argmax on {plan.n_rows} x {plan.n_cols}")
            for J in _maps(rng, plan.n_points):
                idx = _compare(torch, G, plan, J, stream, 1, 0)
                assert idx[0] == opeaks.argmax(J)[0]
                idx = _compare(torch, G, plan, J, stream, 5, 2)
                assert list(idx) == [r[0] for r in opeaks.topk(J, plan.n_rows, plan.n_cols, 5, 2)]
            # more peaks asked for than the window leaves: idx -1, val -inf in both
            J = np.zeros(plan.n_points, dtype=np.float32)
            J[0] = 1.0
            idx = _compare(torch, G, plan, J, stream, 64, max(plan.n_rows, plan.n_cols))
            assert idx[0] == 0 and (idx[1:] == -1).all()


def test_noalloc_argmax_points_and_errors(torch, G):
    rng = np.random.Generator(np.random.PCG64(22))
    stream = torch.cuda.current_stream().cuda_stream
    scn = sim.make_scenario(configs.SMALL, 1)
    lat = np.repeat(scn.lat[:40], 7)[:257]
    lon = np.tile(scn.lon[:7], 40)[:257]
    wl = scn.workload
    with G.Plan(n_rx=wl.n_rx, n_samples=wl.n_samples, step_len=wl.step_len, fs_hz=wl.fs_hz, fc_hz=wl.fc_hz,
                lat=lat, lon=lon, grid_kind=G.GRID_POINTS, pairs=list(wl.pairs)) as plan:
        for J in _maps(rng, plan.n_points):
            _compare(torch, G, plan, J, stream, 3, 0)
    J = np.ones(1000, dtype=np.float32)
    J[777] = np.nan
    Jd = torch.from_numpy(J).cuda()
    with pytest.raises(G.GeolocError) as ei:
        G.geoloc_argmax_noalloc(Jd.data_ptr(), G.GRID_RECT, 10, 100, 1, 0, stream)
    assert ei.value.status == G.ENAN
    for args in [(G.GRID_RECT, 10, 100, 65, 0), (G.GRID_RECT, 10, 100, 0, 0), (G.GRID_POINTS, 1, 1000, 1, 1),
                 (G.GRID_RECT, 0, 100, 1, 0), (7, 10, 100, 1, 0), (G.GRID_RECT, 10, 100, 1, -1)]:
        with pytest.raises(G.GeolocError) as ei:
            G.geoloc_argmax_noalloc(Jd.data_ptr(), *args, stream)
        assert ei.value.status == G.EINVAL
    # a valid call after the errors still works on the same scratch
    J = rng.standard_normal(1000).astype(np.float32)
    idx, val = G.geoloc_argmax_noalloc(torch.from_numpy(J).cuda().data_ptr(), G.GRID_RECT, 10, 100, 1, 0, stream)
    assert idx[0] == int(np.argmax(J)) and val[0] == J.max()
