"""The multi-capture scenario of Sec. IV-B on the GPU: 58 separate 50 ms captures, 1 s
apart, of four emitters (spread-spectrum stand-in, tone, chirp, sawtooth), accumulated in
one map call over 116 virtual receivers. After accumulation the four largest peaks are
the four emitters, CFAR detection on the map finds all four (and matches the oracle's
detection on the same map), and the map matches the oracle at sampled cells and around
each peak. Mapped one capture at a time, the same scenario shows why the grids are summed:
the emitters' peaks persist from capture to capture while sidelobes as strong as they are
move, and only the accumulated map puts every emitter above every sidelobe."""
import time

import numpy as np
import pytest

import oracle
from oracle import cfar as ocfar
from helpers import DIRECT_TOL, log, require_gpu
from paper_2508_06672_amd import configs, sim

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def scenario():
    wl = configs.PAPER_IVB
    seed = 7
    t0 = time.time()
    em = sim.paper_formation(wl, seed)
    snaps = sim.make_snapshots(wl, seed, emitters=em)
    log(f"paper scenario: {len(snaps)} captures simulated in {time.time() - t0:.0f} s")
    return wl, em, snaps


def test_58_captures_find_the_four_emitters(torch, scenario):
    from paper_2508_06672_amd import geoloc
    from paper_2508_06672_amd import proposal as P
    wl, em, snaps = scenario
    capn, states, vpairs = P.stack_snapshots(snaps, wl.pairs)
    s0 = snaps[0]
    caps = torch.from_numpy(capn).cuda()
    with geoloc.Plan(n_rx=capn.shape[0], n_samples=wl.n_samples, step_len=wl.step_len, fs_hz=wl.fs_hz,
                     fc_hz=wl.fc_hz, lat=s0.lat, lon=s0.lon, pairs=vpairs, earth_radius_m=wl.earth_radius_m) as plan:
        J = plan.map(caps, states)
        torch.cuda.synchronize()
        t0 = time.time()
        J = plan.map(caps, states, J=J)
        torch.cuda.synchronize()
        t_map = time.time() - t0
        pk, pv = plan.argmax(J, top_k=4, nms_radius=15)
        # CFAR detection on the accumulated map (58 noncoherent looks per cell)
        guard, train = 6, 16
        scale = geoloc.cfar_scale(1e-6, geoloc.cfar_training_cells(guard, train), looks=len(snaps))
        dk, dv, dn = plan.detect(J, guard, train, scale, max_detections=16, nms_radius=15)
        Jg = J.cpu().numpy().astype(np.float64)
    log(f"  map {t_map * 1e3:.1f} ms ({wl.units / t_map:.3g} correlations/s); peaks {list(pk)}")
    cells = [tuple(divmod(int(p), wl.n_cols)) for p in pk]
    for (r, c), e in zip(s0.true_cells, em):
        d = min(max(abs(r - pr), abs(c - pc)) for pr, pc in cells)
        log(f"  {e.waveform:8s} true cell {(r, c)}: nearest peak {d} cells away")
        assert d <= 2, (e.waveform, (r, c), cells)

    dcells = [tuple(divmod(int(p), wl.n_cols)) for p in dk]
    log(f"  CFAR scale {scale:.3f}: {len(dk)} detections {dcells}, J / noise {[round(float(v / n), 2) for v, n in zip(dv, dn)]}")
    for (r, c), e in zip(s0.true_cells, em):
        d = min((max(abs(r - pr), abs(c - pc)) for pr, pc in dcells), default=10 ** 9)
        assert d <= 2, ("CFAR missed", e.waveform, (r, c), dcells)
    Jd = Jg.reshape(wl.n_rows, wl.n_cols)
    scale_o = ocfar.scale_for_pfa(1e-6, (2 * train + 1) ** 2 - (2 * guard + 1) ** 2, len(snaps))
    assert abs(scale - scale_o) <= 1e-9 * scale_o
    do = ocfar.detect(Jd, guard, train, scale_o, 16, 15)
    assert [i for i, _, _ in do] == [int(p) for p in dk]

    rng = np.random.Generator(np.random.PCG64(33))
    idx = [rng.choice(wl.n_points, 128, replace=False)]
    for p in pk:
        r0, c0 = divmod(int(p), wl.n_cols)
        idx.append(np.array([rr * wl.n_cols + cc for rr in range(max(0, r0 - 2), min(wl.n_rows, r0 + 3))
                             for cc in range(max(0, c0 - 2), min(wl.n_cols, c0 + 3))]))
    idx = np.unique(np.concatenate(idx))
    rows, cols = np.divmod(idx, wl.n_cols)
    log(f"  oracle at {idx.size} points")
    Jo = oracle.map_points(s0.lat[rows], s0.lon[cols], capn, states, wl.step_len, wl.fs_hz, wl.fc_hz, pairs=vpairs,
                           radius=wl.earth_radius_m)
    e = float(np.max(np.abs(Jg[idx] - Jo)) / np.max(Jo))
    log(f"  err_J = {e:.3g}")
    assert e <= DIRECT_TOL


def _peaks_outside(G, k, radius, exclude, exclude_radius):
    """The k largest values of G at least `radius` cells apart, none within exclude_radius
    cells of an excluded cell: [(row, col, value)]."""
    G = G.copy()
    for a, b in exclude:
        G[max(0, a - exclude_radius):a + exclude_radius + 1, max(0, b - exclude_radius):b + exclude_radius + 1] = -np.inf
    out = []
    for _ in range(k):
        i = int(np.argmax(G))
        a, b = divmod(i, G.shape[1])
        out.append((a, b, float(G[a, b])))
        G[max(0, a - radius):a + radius + 1, max(0, b - radius):b + radius + 1] = -np.inf
    return out


def test_peaks_persist_and_sidelobes_move(torch, scenario):
    """Sec. IV-B's account of why the grids of separate captures are summed: in each capture
    the emitters' peaks are there but so are sidelobes as strong as they are; the geometry
    changes from capture to capture, so the sidelobes move while the emitters stay, and
    only the accumulated map leaves the true peaks on top. Each capture is mapped on its
    own through the C ABI:
      * every emitter's cell (within 2 cells) holds most of its capture's maximum in most
        captures (median over captures of local max / capture max >= 0.5);
      * the strongest sidelobes of a capture (outside 15 cells of every emitter) do not
        recur: at their cells the other captures' maps are small (median <= 0.05 of their
        maximum) and they are almost never among another capture's five strongest sidelobes;
      * in most single captures some sidelobe beats the weakest emitter (contrast > 1),
        while after accumulation every emitter beats every sidelobe (contrast < 1) and the
        contrast of the accumulated map is below that of every single capture."""
    from paper_2508_06672_amd import geoloc
    wl, em, snaps = scenario
    s0 = snaps[0]
    R = s0.captures.shape[0]
    maps = []
    with geoloc.Plan(n_rx=R, n_samples=wl.n_samples, step_len=wl.step_len, fs_hz=wl.fs_hz, fc_hz=wl.fc_hz,
                     lat=s0.lat, lon=s0.lon, pairs=list(wl.pairs), earth_radius_m=wl.earth_radius_m) as plan:
        for sc in snaps:
            J = plan.map(torch.from_numpy(sc.captures).cuda(), sc.states)
            maps.append(J.cpu().numpy().astype(np.float64).reshape(wl.n_rows, wl.n_cols))
    M = np.stack(maps)
    S = len(M)
    norm = M / M.reshape(S, -1).max(axis=1)[:, None, None]
    cells = list(s0.true_cells)
    for (r, c), e in zip(cells, em):
        loc = norm[:, max(0, r - 2):r + 3, max(0, c - 2):c + 3].reshape(S, -1).max(axis=1)
        log(f"  {e.waveform:8s}: local max / capture max median {np.median(loc):.3f}, min {loc.min():.3f}")
        assert np.median(loc) >= 0.5, e.waveform
    side = [_peaks_outside(norm[s], 5, 15, cells, 15) for s in range(S)]
    others, recur = [], []
    for s in range(S):
        for a, b, _ in side[s][:3]:
            others.append(np.median([norm[t, a, b] for t in range(S) if t != s]))
            recur.append(np.mean([any(max(abs(a - x), abs(b - y)) <= 2 for x, y, _ in side[t])
                                  for t in range(S) if t != s]))
    log(f"  sidelobes: value at their cells in other captures median {np.median(others):.4f}, "
        f"recurring among other captures' top 5: mean {np.mean(recur):.4f}")
    assert np.median(others) <= 0.05
    assert np.mean(recur) <= 0.05

    def contrast(G):
        weakest = min(G[max(0, r - 2):r + 3, max(0, c - 2):c + 3].max() for r, c in cells)
        return _peaks_outside(G, 1, 15, cells, 15)[0][2] / weakest

    single = np.array([contrast(M[s]) for s in range(S)])
    acc = contrast(M.sum(axis=0))
    log(f"  contrast (strongest sidelobe / weakest emitter): single captures median {np.median(single):.3f}, "
        f"min {single.min():.3f}; accumulated {acc:.3f}")
    assert np.median(single) > 1.0
    assert acc < 1.0 and acc < single.min()

