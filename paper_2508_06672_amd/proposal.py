"""Learned tile proposal over the direct position-domain map.

This is an addition to the method (the paper has no learned part). Pipeline for one
scenario, every step through libgeoloc on the GPU:
  1. coarse map: the captures are split into 16 frequency bands, each decimated by 16
     (geoloc_subbands), and the plain direct map of every band (one receiver pair per
     band, summed into one J) is evaluated at the centres of the 64 x 64 tiles (16 x 16
     fine cells each) of the fine grid. At 1/16 of the sample rate the delay peak of a
     wideband emitter is 16 samples wide, about one coarse cell, so the coarse grid does
     not miss it between its points, and a narrowband emitter keeps its band;
  2. features [log-compressed coarse map, TDOA (decimated samples) and FDOA of the
     middle step] -> CNN -> tile logits -> softmax -> the 16 most likely tiles;
  3. refine: the plain direct map at the 16 x 256 fine cells of those tiles, argmax;
  4. fallback: when the softmax mass of the chosen tiles is below 0.5 (or, with
     rule="top1", the top tile's probability), the plain map over the full grid.
Training labels come from the plain full-grid map: every tile holding a cell within
1 % of the map's maximum (orbital-plane mirror ties and flat ridges make it a set),
uniformly weighted. Network: 4 convolutions 3 -> 32 -> 32 -> 32 -> 1, FP16 weights,
FP32 accumulation, trained with Adam by the library's own kernels; PyTorch only holds
the device buffers.

CLI:  python -m paper_2508_06672_amd.proposal train --n-train 4000 --out <weights.npz>
      python -m paper_2508_06672_amd.proposal calibrate --n-val 1000 --target 0.995
      python -m paper_2508_06672_amd.proposal evaluate --weights <weights.npz> --n-test 200
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import agreement, configs, sim

COARSE = configs.PROPOSAL_COARSE
TILE = configs.PROPOSAL_TILE
TOPK = configs.PROPOSAL_TOPK
BANDS, BAND_HALF_TAPS = 16, 64          # coarse-map sub-bands: 16 bands, 129-tap low-pass
LABEL_EPS = 1e-2
IN_CH, HIDDEN, LAYERS = 3, 32, 4
TRAIN_WL = configs.PROPOSAL
WORKLOADS = {"proposal": configs.PROPOSAL, "single_capture": configs.PROPOSAL_C4}
WEIGHTS_SINGLE_CAPTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "proposal_cnn_c4.npz")
SEED_TRAIN, SEED_VAL, SEED_TEST = 1_000_000, 1_020_000, 1_030_000
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "proposal_cnn.npz")


def log(msg: str) -> None:
    print(f"[proposal {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


# --------------------------------------------------------------------------- grid helpers

def coarse_axes(lat: np.ndarray, lon: np.ndarray, tile: int = TILE):
    """Latitudes / longitudes of the tile centres of a rectilinear fine grid."""
    def centres(a):
        n = a.size // tile
        i0 = tile * np.arange(n) + tile // 2 - 1
        return 0.5 * (a[i0] + a[i0 + 1])
    return centres(np.asarray(lat)), centres(np.asarray(lon))


def tile_points(lat: np.ndarray, lon: np.ndarray, tiles: Sequence[int], tile: int = TILE):
    """Fine-grid points (lat, lon, flat index) of the given tiles, tile by tile."""
    n_tile_cols = lon.size // tile
    idx = []
    for t in tiles:
        R, C = divmod(int(t), n_tile_cols)
        rr, cc = np.meshgrid(np.arange(R * tile, (R + 1) * tile), np.arange(C * tile, (C + 1) * tile), indexing="ij")
        idx.append((rr * lon.size + cc).ravel())
    idx = np.concatenate(idx)
    return lat[idx // lon.size], lon[idx % lon.size], idx


def tile_label(J: np.ndarray, n_rows: int, n_cols: int, tile: int = TILE, eps: float = LABEL_EPS) -> np.ndarray:
    """Uniform distribution over the tiles holding a cell with J >= (1 - eps) max J."""
    Jt = np.asarray(J, dtype=np.float64).reshape(n_rows // tile, tile, n_cols // tile, tile).max(axis=(1, 3))
    mask = Jt >= (1.0 - eps) * Jt.max()
    return (mask / mask.sum()).ravel().astype(np.float32)


def stack_snapshots(snaps, pairs):
    """Separate captures as virtual receivers of one map call: receiver r of snapshot s is
    receiver s * R + r, with that snapshot's states, and each pair is repeated within each
    snapshot. Returns (captures [S*R][N], states [K][S*R][6], pairs)."""
    R = snaps[0].captures.shape[0]
    caps = np.ascontiguousarray(np.concatenate([sc.captures for sc in snaps], axis=0))
    states = np.ascontiguousarray(np.concatenate([sc.states for sc in snaps], axis=1))
    vpairs = [(s * R + i, s * R + j) for s in range(len(snaps)) for (i, j) in pairs]
    return caps, states, vpairs


def band_states(states: np.ndarray, n_bands: int = BANDS) -> np.ndarray:
    """Receiver states for the band-major sub-band captures: band b of receiver r is
    receiver b * R + r, at the same position and velocity."""
    st = np.asarray(states, dtype=np.float64)
    return np.ascontiguousarray(np.tile(st, (1, n_bands, 1)))


def band_pairs(pairs, n_rx: int, n_bands: int = BANDS):
    """Each receiver pair within each band."""
    return [(b * n_rx + i, b * n_rx + j) for b in range(n_bands) for (i, j) in pairs]


def he_init(seed: int, hidden: int = HIDDEN, layers: int = LAYERS) -> np.ndarray:
    """He-normal convolution weights, zero biases, in the library's flat parameter order."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    chans = [IN_CH] + [hidden] * (layers - 1) + [1]
    out = []
    for ci, co in zip(chans[:-1], chans[1:]):
        out += [rng.standard_normal(co * ci * 9) * math.sqrt(2.0 / (ci * 9)), np.zeros(co)]
    return np.concatenate(out).astype(np.float32)


def save_weights(path: str, theta: np.ndarray, meta: dict) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, theta=np.asarray(theta, dtype=np.float32), meta=np.frombuffer(json.dumps(meta).encode(), np.uint8))


def make_net(geoloc, meta: Optional[dict] = None, max_batch: int = 64, height: int = COARSE, width: int = COARSE):
    """The proposal CNN in the shape the weights' metadata names (the defaults otherwise), on
    a coarse grid of height x width tiles (the network is fully convolutional, so weights
    trained on 64 x 64 tiles apply to any coarse grid)."""
    meta = meta or {}
    return geoloc.CNN(int(meta.get("in_ch", IN_CH)), int(meta.get("hidden", HIDDEN)), int(meta.get("layers", LAYERS)),
                      height, width, max_batch=max_batch)


def load_weights(path: str = WEIGHTS):
    z = np.load(path, allow_pickle=False)
    return z["theta"], json.loads(bytes(z["meta"]).decode())


# --------------------------------------------------------------------------- the proposer

class Proposer:
    """Plans and network for one fine-grid shape; set_grid() retargets a scenario. Maps take
    the scenario's snapshots stacked as virtual receivers (stack_snapshots)."""

    def __init__(self, wl, net, topk: int = TOPK, threshold: float = 0.5, rule: str = "mass",
                 fallback_method: Optional[int] = None):
        """fallback_method: the method of the full-grid map the proposal falls back to
        (geoloc.DIRECT_FP32 when None; geoloc.CAF_BF16 gives the combined form)."""
        from . import geoloc
        self.G = geoloc
        self.wl, self.net, self.topk, self.threshold, self.rule = wl, net, topk, threshold, rule
        lat0, lon0 = sim.make_grid(wl, 0.0)
        clat, clon = coarse_axes(lat0, lon0)
        # every snapshot's receivers as virtual receivers of one map call
        self.n_vrx = wl.n_snapshots * wl.n_rx
        self.vpairs = [(s * wl.n_rx + i, s * wl.n_rx + j) for s in range(wl.n_snapshots) for (i, j) in wl.pairs]
        kw = dict(n_rx=self.n_vrx, n_samples=wl.n_samples, step_len=wl.step_len, fs_hz=wl.fs_hz, fc_hz=wl.fc_hz,
                  pairs=self.vpairs, earth_radius_m=wl.earth_radius_m)
        if wl.n_samples % BANDS or wl.step_len % BANDS:
            raise ValueError(f"capture and step lengths must be multiples of {BANDS}")
        self.coarse = geoloc.Plan(n_rx=BANDS * self.n_vrx, n_samples=wl.n_samples // BANDS,
                                  step_len=wl.step_len // BANDS, fs_hz=wl.fs_hz / BANDS, fc_hz=wl.fc_hz,
                                  pairs=band_pairs(self.vpairs, self.n_vrx), earth_radius_m=wl.earth_radius_m,
                                  lat=clat, lon=clon)
        self._bands = None
        plat, plon, _ = tile_points(lat0, lon0, range(topk))
        self.refine = geoloc.Plan(lat=plat, lon=plon, grid_kind=geoloc.GRID_POINTS, **kw)
        self.full = geoloc.Plan(lat=lat0, lon=lon0, **kw)
        self.fallback = self.full
        if fallback_method is not None and fallback_method != geoloc.DIRECT_FP32:
            self.fallback = geoloc.Plan(lat=lat0, lon=lon0, method=fallback_method, **kw)
        self.lat, self.lon = lat0, lon0
        self._lat_dev = self._lon_dev = None      # the fine grid's axes on the device
        self.n_tile_rows, self.n_tile_cols = wl.n_rows // TILE, wl.n_cols // TILE

    def set_grid(self, lat: np.ndarray, lon: np.ndarray) -> None:
        self.lat, self.lon = np.asarray(lat), np.asarray(lon)
        self._lat_dev = self._lon_dev = None
        self.coarse.set_grid(*coarse_axes(lat, lon))
        self.full.set_grid(lat, lon)
        if self.fallback is not self.full:
            self.fallback.set_grid(lat, lon)

    def coarse_features(self, caps, states):
        """(coarse map [tile rows * tile cols], CNN input [1, 3, tile rows, tile cols])."""
        import torch
        if self._bands is None:
            self._bands = torch.empty((BANDS * self.n_vrx, self.wl.n_samples // BANDS), dtype=torch.complex64,
                                      device=caps.device)
        z = self.G.subbands(caps, BANDS, BAND_HALF_TAPS, out=self._bands)
        st = band_states(states)
        Jc = self.coarse.map(z, st)
        # TDOA / FDOA features: the first pair of the middle snapshot, band 0, middle step
        mid = (self.wl.n_snapshots // 2) * len(self.wl.pairs)
        D, nu = self.coarse.geometry(st, mid, self.wl.n_steps // 2, 1)
        x = self.net.prepare(Jc.view(1, -1), D, nu)
        return Jc, x

    def refine_tiles(self, caps, states, tiles):
        """Map the cells of the given tiles (set on the device from the tile list) and return
        the best one's flat index on the fine grid and its value."""
        import torch
        if self._lat_dev is None:
            self._lat_dev = torch.from_numpy(np.ascontiguousarray(self.lat, dtype=np.float64)).to(caps.device)
            self._lon_dev = torch.from_numpy(np.ascontiguousarray(self.lon, dtype=np.float64)).to(caps.device)
        tiles = np.asarray(tiles, dtype=np.int64)
        self.refine.set_points_from_tiles(self._lat_dev, self._lon_dev, TILE, tiles)
        J = self.refine.map(caps, states)
        i, v = self.refine.argmax(J)
        t, w = divmod(int(i[0]), TILE * TILE)
        R, C = divmod(int(tiles[t]), self.lon.size // TILE)
        r, c = R * TILE + w // TILE, C * TILE + w % TILE
        return r * self.lon.size + c, float(v[0])

    def refine_peaks(self, caps, states, tiles, k: int, radius: int):
        """The k largest cells of the given tiles' map, each more than `radius` cells
        (Chebyshev distance on the fine grid) from the ones before: (flat indices, values)."""
        if self._lat_dev is None:
            import torch
            self._lat_dev = torch.from_numpy(np.ascontiguousarray(self.lat, dtype=np.float64)).to(caps.device)
            self._lon_dev = torch.from_numpy(np.ascontiguousarray(self.lon, dtype=np.float64)).to(caps.device)
        tiles = np.asarray(tiles, dtype=np.int64)
        self.refine.set_points_from_tiles(self._lat_dev, self._lon_dev, TILE, tiles)
        J = self.refine.map(caps, states).cpu().numpy().astype(np.float64)
        _, _, flat = tile_points(self.lat, self.lon, tiles)
        rows, cols = np.divmod(flat, self.lon.size)
        order = np.argsort(-J, kind="stable")
        out_i, out_v = [], []
        for o in order:
            if all(max(abs(rows[o] - rows[p]), abs(cols[o] - cols[p])) > radius for p in out_i):
                out_i.append(int(o))
                out_v.append(float(J[o]))
                if len(out_i) == k:
                    break
        return [int(flat[o]) for o in out_i], out_v

    def full_map(self, caps, states):
        J = self.full.map(caps, states)
        i, v = self.full.argmax(J)
        return int(i[0]), float(v[0]), J

    def run_top(self, caps, states, k: int = 2, radius: int = 8) -> Dict:
        """The learned proposal for k emitters: the CNN's tiles refined at full resolution and
        the k best separated cells there; below the confidence threshold the fallback plan's
        full-grid map and its top k (the combined form when that plan is the CAF table)."""
        Jc, x = self.coarse_features(caps, states)
        z = self.net.forward(x)
        tiles, probs = self.net.topk(z, self.topk)
        tiles, probs = tiles[0], probs[0]
        score = float(probs[0]) if self.rule == "top1" else float(probs.sum())
        if score < self.threshold:
            J = self.fallback.map(caps, states)
            i, v = self.fallback.argmax(J, top_k=k, nms_radius=radius)
            return {"idx": [int(t) for t in i], "val": [float(t) for t in v], "fallback": True, "tiles": tiles,
                    "score": score}
        i, v = self.refine_peaks(caps, states, tiles, k, radius)
        return {"idx": i, "val": v, "fallback": False, "tiles": tiles, "score": score}

    def run(self, caps, states, selector: str = "cnn") -> Dict:
        """selector: 'cnn' (learned) or 'coarse' (ablation: top tiles of the coarse map itself)."""
        import torch
        Jc, x = self.coarse_features(caps, states)
        if selector == "cnn":
            z = self.net.forward(x)
            tiles, probs = self.net.topk(z, self.topk)
            tiles, probs = tiles[0], probs[0]
            score = float(probs[0]) if self.rule == "top1" else float(probs.sum())
        else:
            jc = Jc.cpu().numpy()
            tiles = np.argsort(-jc, kind="stable")[: self.topk]
            score = float("inf")                      # the ablation never falls back
        if score < self.threshold:
            i, v, _ = self.full_map(caps, states)
            return {"idx": i, "val": v, "fallback": True, "tiles": tiles, "score": score}
        i, v = self.refine_tiles(caps, states, tiles)
        return {"idx": i, "val": v, "fallback": False, "tiles": tiles, "score": score}

    def close(self) -> None:
        for p in (self.coarse, self.refine, self.full):
            p.close()
        if self.fallback is not self.full:
            self.fallback.close()


# --------------------------------------------------------------------------- data

def _simulate(args):
    wl, seed = args
    snaps = sim.make_snapshots(wl, seed)
    caps, states, _ = stack_snapshots(snaps, wl.pairs)
    s = snaps[0]
    return seed, s.lat, s.lon, states, caps, s.emitters[0].waveform, s.snr_db


def scenario_stream(wl, seeds: Sequence[int], pool=None):
    """Simulated scenarios in seed order: in CPU worker processes (a pool forked before the
    GPU was touched), or in this process when pool is None."""
    jobs = [(wl, s) for s in seeds]
    it = pool.imap(_simulate, jobs, chunksize=4) if pool is not None else map(_simulate, jobs)
    for rec in it:
        yield rec


def build_dataset(prop: Proposer, wl, seeds, pool):
    """Features [n, 3, 64, 64] and labels [n, 4096] on the GPU."""
    import torch
    n = len(seeds)
    X = torch.empty((n, IN_CH, prop.n_tile_rows, prop.n_tile_cols), dtype=torch.float32, device="cuda")
    Y = torch.empty((n, prop.n_tile_rows * prop.n_tile_cols), dtype=torch.float32, device="cuda")
    t0 = time.time()
    for k, (seed, lat, lon, states, capn, wf, snr) in enumerate(scenario_stream(wl, seeds, pool)):
        caps = torch.from_numpy(capn).cuda()
        prop.set_grid(lat, lon)
        _, x = prop.coarse_features(caps, states)
        X[k] = x[0]
        _, _, J = prop.full_map(caps, states)
        Y[k] = torch.from_numpy(tile_label(J.cpu().numpy(), wl.n_rows, wl.n_cols)).cuda()
        if (k + 1) % 250 == 0 or k + 1 == n:
            log(f"  dataset {k + 1}/{n} ({time.time() - t0:.0f} s)")
    return X, Y


def train(net, X, Y, Xv, Yv, epochs: int, batch: int = 64, lr: float = 1e-3, seed: int = 0) -> List[dict]:
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    n = X.shape[0]
    hist = []
    step = 0
    total = epochs * (n // batch)
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        tl = 0.0
        for b in range(n // batch):
            sel = perm[b * batch:(b + 1) * batch]
            z = net.forward(X[sel])
            loss, dz = net.loss(z, Y[sel])
            net.backward(dz)
            lr_t = lr * 0.5 * (1 + math.cos(math.pi * step / total))
            net.adam_step(lr_t)
            tl += float(loss.sum())
            step += 1
        vl, vh = validate(net, Xv, Yv)
        hist.append({"epoch": ep, "train_loss": tl / (n // batch * batch), "val_loss": vl, "val_top16_hit": vh})
        log(f"  epoch {ep}: train {hist[-1]['train_loss']:.4f} val {vl:.4f} top-16 hit {vh:.3f}")
    return hist


def validate(net, Xv, Yv, batch: int = 64, scores: bool = False):
    """Mean loss and the fraction of samples whose top tiles hit the label set; with
    scores=True also per-sample (top-tile mass, top-1 probability, hit)."""
    import torch
    n = Xv.shape[0]
    tl, hits, rec = 0.0, 0, []
    for b in range(0, n, batch):
        x, y = Xv[b:b + batch], Yv[b:b + batch]
        z = net.forward(x)
        loss, _ = net.loss(z, y)
        tl += float(loss.sum())
        tiles, probs = net.topk(z, TOPK)
        yh = y.cpu().numpy()
        for i in range(tiles.shape[0]):
            h = bool(np.any(yh[i, tiles[i]] > 0))
            hits += h
            rec.append((float(probs[i].sum()), float(probs[i, 0]), h))
    return (tl / n, hits / n, rec) if scores else (tl / n, hits / n)


def calibrate(rec, target: float = 0.99, rule: str = "mass") -> dict:
    """Smallest threshold on the confidence score whose accepted samples hit the label set
    at rate >= target (the rest fall back to the full map)."""
    sc = np.array([r[0] if rule == "mass" else r[1] for r in rec])
    hit = np.array([r[2] for r in rec])
    best = float(np.inf)
    for t in np.unique(sc)[::-1]:
        acc = sc >= t
        if hit[acc].mean() >= target:
            best = float(t)
        else:
            break
    acc = sc >= best
    return {"rule": rule, "threshold": best, "target": target, "accept_rate": float(acc.mean()),
            "accepted_hit_rate": float(hit[acc].mean()) if acc.any() else None}


def calibrate_overall(scores, ok, target: float = 0.99) -> dict:
    """Smallest threshold on the confidence score for which the whole pipeline (the refined
    peak where the score reaches the threshold, the full map's own peak where it falls back)
    agrees with the full map on at least `target` of the scenarios."""
    sc = np.asarray(scores, dtype=np.float64)
    ok = np.asarray(ok, dtype=bool)
    best = float(np.inf)
    for t in np.unique(sc):
        if np.mean(ok | (sc < t)) >= target:
            best = float(t)
            break
    acc = sc >= best
    return {"rule": "mass", "threshold": best, "target": target, "criterion": "overall agreement",
            "accept_rate": float(acc.mean()), "overall_agreement": float(np.mean(ok | ~acc)),
            "accepted_agreement": float(ok[acc].mean()) if acc.any() else None}


# --------------------------------------------------------------------------- evaluation

AGREE_EPS = 1e-4      # the refine map is the full map's own FP32 values at the chosen cells


def _agrees(wl, lat, lon, a: int, a_full: int, J_full: np.ndarray, eps: float = AGREE_EPS) -> dict:
    """The peak a against the full plain map's peak (agreement.classify): margin of the full
    map, within one cell of its peak or of that peak's orbital-plane mirror, eps-optimal;
    'ok' is within one cell on a well-conditioned map and eps-optimal on any other."""
    c = agreement.classify(J_full, wl.n_cols, a, a_full, eps, agreement.mirror_cell(wl, lat, lon, a_full))
    c["ok"] = c["within_one"] if c["well_conditioned"] else (c["within_one"] or c["eps_optimal"])
    return c


def evaluate(prop: Proposer, wl, seeds, pool) -> dict:
    import torch
    recs = []
    for seed, lat, lon, states, capn, wf, snr in scenario_stream(wl, seeds, pool):
        caps = torch.from_numpy(capn).cuda()
        prop.set_grid(lat, lon)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a_full, _, J = prop.full_map(caps, states)
        torch.cuda.synchronize()
        t_full = time.perf_counter() - t0
        Jh = J.cpu().numpy()
        out = {"seed": seed, "waveform": wf, "snr_db": snr, "t_full_ms": t_full * 1e3}
        for sel in ("cnn", "coarse"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = prop.run(caps, states, selector=sel)
            torch.cuda.synchronize()
            t_ms = (time.perf_counter() - t0) * 1e3
            c = _agrees(wl, lat, lon, r["idx"], a_full, Jh)
            out[sel] = {"ok": c["ok"], "rule": c, "fallback": r["fallback"], "score": r["score"], "t_ms": t_ms}
        recs.append(out)
        log(f"  seed {seed} {wf:5s} {snr:6.1f} dB: cnn ok={out['cnn']['ok']} fb={out['cnn']['fallback']} "
            f"score={out['cnn']['score']:.2f} | coarse ok={out['coarse']['ok']}")
    n = len(recs)

    def summ(sel):
        ok = [r[sel]["ok"] for r in recs]
        fb = [r[sel]["fallback"] for r in recs]
        t = [r[sel]["t_ms"] for r in recs]
        by_wf = {}
        for wf in sorted({r["waveform"] for r in recs}):
            sub = [r for r in recs if r["waveform"] == wf]
            by_wf[wf] = {"n": len(sub), "agree_rate": float(np.mean([r[sel]["ok"] for r in sub])),
                         "fallback_rate": float(np.mean([r[sel]["fallback"] for r in sub]))}
        return {"agree_rate": float(np.mean(ok)), "fallback_rate": float(np.mean(fb)),
                "rule": agreement.summarise([r[sel]["rule"] for r in recs], AGREE_EPS),
                "median_ms": float(np.median(t)), "mean_ms": float(np.mean(t)),
                "speedup_vs_full_median": float(np.median([r["t_full_ms"] / r[sel]["t_ms"] for r in recs])),
                "speedup_vs_full_mean": float(np.mean([r["t_full_ms"] for r in recs]) / np.mean(t)),
                "by_waveform": by_wf}
    return {"scenarios": n, "seeds": f"{seeds[0]}..{seeds[-1]}", "workload": wl.name,
            "full_map_median_ms": float(np.median([r["t_full_ms"] for r in recs])),
            "learned": summ("cnn"), "coarse_top16_ablation": summ("coarse"), "records": recs}


# --------------------------------------------------------------------------- CLI

def _workload_of(name, meta):
    """The named workload, else the one the weights were trained on."""
    if name:
        return WORKLOADS[name]
    for w in WORKLOADS.values():
        if w.name == meta.get("train_workload"):
            return w
    return TRAIN_WL


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--n-train", type=int, default=6000)
    t.add_argument("--n-val", type=int, default=200)
    t.add_argument("--epochs", type=int, default=20)
    t.add_argument("--hidden", type=int, default=HIDDEN, help="channels of the hidden layers (at most 32)")
    t.add_argument("--layers", type=int, default=LAYERS, help="3 x 3 convolutions")
    t.add_argument("--workload", choices=sorted(WORKLOADS), default="proposal")
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--workers", type=int, default=16)
    t.add_argument("--out", default=WEIGHTS)
    c = sub.add_parser("calibrate", help="set the fallback threshold from the full pipeline's agreement on "
                                          "validation scenarios")
    c.add_argument("--weights", default=WEIGHTS)
    c.add_argument("--n-val", type=int, default=1000)
    c.add_argument("--target", type=float, default=0.995, help="agreement of the whole pipeline on validation")
    c.add_argument("--workers", type=int, default=16)
    c.add_argument("--out", default=None, help="where to write the re-calibrated weights (default: in place)")
    c.add_argument("--workload", choices=sorted(WORKLOADS), default=None,
                   help="default: the workload the weights were trained on")
    e = sub.add_parser("evaluate")
    e.add_argument("--weights", default=WEIGHTS)
    e.add_argument("--n-test", type=int, default=200)
    e.add_argument("--samples", type=int, default=0, help="capture length (default: the workload's)")
    e.add_argument("--workers", type=int, default=16)
    e.add_argument("--out", default=None)
    e.add_argument("--threshold", type=float, default=None, help="override the calibrated threshold")
    e.add_argument("--workload", choices=sorted(WORKLOADS), default=None,
                   help="default: the workload the weights were trained on")
    args = ap.parse_args(argv)

    # simulator workers are forked before anything touches the GPU
    pool = mp.get_context("fork").Pool(args.workers)
    import torch
    from . import geoloc
    assert torch.cuda.is_available()
    meta0 = load_weights(args.weights)[1] if args.cmd != "train" else {"hidden": args.hidden, "layers": args.layers}
    net = make_net(geoloc, meta0, max_batch=64)
    try:
        if args.cmd == "train":
            wl = WORKLOADS[args.workload]
            prop = Proposer(wl, net)
            log(f"building {args.n_train} training + {args.n_val} validation scenarios ({wl.name})")
            X, Y = build_dataset(prop, wl, list(range(SEED_TRAIN, SEED_TRAIN + args.n_train)), pool)
            Xv, Yv = build_dataset(prop, wl, list(range(SEED_VAL, SEED_VAL + args.n_val)), pool)
            net.set_params(he_init(0, args.hidden, args.layers))
            hist = train(net, X, Y, Xv, Yv, args.epochs, lr=args.lr)
            _, _, rec = validate(net, Xv, Yv, scores=True)
            cal = calibrate(rec)
            log(f"calibration on the validation set: {cal}")
            meta = {"in_ch": IN_CH, "hidden": args.hidden, "layers": args.layers, "n_params": net.n_params,
                    "calibration": cal, "threshold": cal["threshold"], "rule": cal["rule"],
                    "train_workload": wl.name, "n_train": args.n_train, "n_val": args.n_val,
                    "seeds_train": [SEED_TRAIN, SEED_TRAIN + args.n_train], "epochs": args.epochs, "lr": args.lr,
                    "label_eps": LABEL_EPS, "history": hist}
            save_weights(args.out, net.params(0), meta)
            log(f"saved {args.out} ({net.n_params} parameters)")
            prop.close()
        elif args.cmd == "calibrate":
            # the threshold on the chosen tiles' softmax mass above which the refined peak
            # agrees with the full map's (agreement rule) at rate >= target on validation
            # scenarios, every one of them run through the whole pipeline without fallback
            theta, meta = load_weights(args.weights)
            net.set_params(theta)
            wl = _workload_of(args.workload, meta)
            prop = Proposer(wl, net, threshold=0.0, rule="mass")
            seeds = list(range(SEED_VAL, SEED_VAL + args.n_val))
            res = evaluate(prop, wl, seeds, pool)
            prop.close()
            cal = calibrate_overall([r["cnn"]["score"] for r in res["records"]],
                                    [bool(r["cnn"]["ok"]) for r in res["records"]], target=args.target)
            rec = res["records"]
            cal.update({"on": "agreement of the refined peak with the full map", "n_val": len(rec),
                        "seeds": [seeds[0], seeds[-1] + 1]})
            log(f"calibration on the agreement of {len(rec)} validation scenarios: {cal}")
            meta["calibration_label_hits"] = meta.get("calibration")
            meta["calibration"] = cal
            meta["threshold"] = cal["threshold"]
            meta["rule"] = "mass"
            save_weights(args.out or args.weights, theta, meta)
        else:
            theta, meta = load_weights(args.weights)
            net.set_params(theta)
            wl = _workload_of(args.workload, meta)
            if args.samples:
                wl = wl.with_(n_samples=args.samples)
            thr = args.threshold if args.threshold is not None else meta.get("threshold", 0.5)
            prop = Proposer(wl, net, threshold=thr, rule=meta.get("rule", "mass"))
            log(f"threshold {thr} ({meta.get('rule', 'mass')})")
            res = evaluate(prop, wl, list(range(SEED_TEST, SEED_TEST + args.n_test)), pool)
            res["weights"] = os.path.basename(args.weights)
            res["threshold"] = thr
            summary = {k: v for k, v in res.items() if k != "records"}
            print(json.dumps(summary), flush=True)
            if args.out:
                with open(args.out, "w") as fh:
                    json.dump(res, fh)
            prop.close()
    finally:
        pool.terminate()
        net.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
