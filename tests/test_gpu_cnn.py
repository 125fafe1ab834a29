"""The tile-proposal CNN kernels against the FP64 CNN oracle (given the same FP16-rounded
parameters), through the C ABI: forward, softmax cross-entropy, backward, Adam, top-k,
input features, and the zero-weight fallback case."""
import numpy as np
import pytest

from oracle import cnn as ocnn
from helpers import log, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def G():
    from paper_2508_06672_amd import geoloc
    geoloc.load()
    return geoloc


def _rng(s):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(s)))


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _setup(torch, G, in_ch, hidden, layers, H, W, B, seed):
    net = G.CNN(in_ch, hidden, layers, H, W, max_batch=B)
    rng = _rng(seed)
    theta = ocnn.he_init(in_ch, hidden, layers, seed) + 0.01 * rng.standard_normal(net.n_params)
    net.set_params(theta)
    th16 = net.params(1).astype(np.float64)                     # the FP16 working copy, widened
    x = rng.standard_normal((B, in_ch, H, W)).astype(np.float32)
    q = rng.random((B, H, W))
    q /= q.sum(axis=(1, 2), keepdims=True)
    return net, th16, x, q.astype(np.float32)


@pytest.mark.parametrize("shape", [(3, 8, 4, 13, 17, 3), (3, 32, 4, 64, 64, 4)])
def test_forward_loss_backward_match_oracle(torch, G, shape):
    in_ch, hidden, layers, H, W, B = shape
    net, th16, x, q = _setup(torch, G, in_ch, hidden, layers, H, W, B, 1)
    assert np.max(np.abs(th16 - net.params(0))) <= 1e-3 * np.max(np.abs(th16))   # FP16 rounding only
    xd = torch.from_numpy(x).cuda()
    z = net.forward(xd)
    loss, dz = net.loss(z, torch.from_numpy(q).cuda())
    net.backward(dz)
    torch.cuda.synchronize()
    g = net.params(2)
    zo, cache = ocnn.forward(th16, x.astype(np.float64), in_ch, hidden, layers)
    lo, dzo, _ = ocnn.softmax_ce(zo, q.astype(np.float64))
    go = ocnn.backward(th16, cache, dzo, in_ch, hidden, layers)
    ez, el, eg = _rel(z.cpu().numpy(), zo), abs(float(loss.sum().cpu()) / B - lo) / abs(lo), _rel(g, go)
    log(f"cnn {shape}: logits {ez:.2e} loss {el:.2e} grad {eg:.2e}")
    assert ez <= 1e-4 and el <= 1e-5 and eg <= 1e-3
    # per-layer gradient blocks too (a wrong layer would hide in the total)
    o = 0
    for ci, co in ocnn.layer_shapes(in_ch, hidden, layers):
        n = co * ci * 9 + co
        assert _rel(g[o:o + n], go[o:o + n]) <= 2e-3
        o += n


def test_adam_step_matches_oracle(torch, G):
    net, th16, x, q = _setup(torch, G, 3, 8, 4, 12, 12, 2, 2)
    master0 = net.params(0).astype(np.float64)
    xd = torch.from_numpy(x).cuda()
    qd = torch.from_numpy(q).cuda()
    m = np.zeros(net.n_params)
    v = np.zeros(net.n_params)
    th = master0.copy()
    for t in range(1, 4):
        z = net.forward(xd)
        _, dz = net.loss(z, qd)
        net.backward(dz)
        g = net.params(2).astype(np.float64)
        net.adam_step(1e-3)
        th, m, v = ocnn.adam(th, m, v, g, t, 1e-3)
        assert np.max(np.abs(net.params(0) - th)) <= 1e-6 * max(1.0, np.max(np.abs(th)))


def test_topk_prepare_and_zero_weights(torch, G):
    B, H, W = 3, 64, 64
    net = G.CNN(3, 32, 4, H, W, max_batch=B)
    rng = _rng(3)
    z = rng.standard_normal((B, H, W)).astype(np.float32)
    z[1, 5, 5] = z[1, 5, 6] = 9.0                                  # a tie: lower index first
    tiles, probs = net.topk(torch.from_numpy(z).cuda(), 16)
    zf = z.reshape(B, -1).astype(np.float64)
    p = np.exp(zf - zf.max(1, keepdims=True))
    p /= p.sum(1, keepdims=True)
    for b in range(B):
        order = np.lexsort((np.arange(H * W), -zf[b]))[:16]
        assert list(tiles[b]) == list(order)
        assert np.allclose(probs[b], p[b, order], rtol=1e-5)
    # input features
    J = (rng.random((B, H * W)) * 10 + 1e-3).astype(np.float32)
    J[0, 0] = 0.0
    D = rng.uniform(-300, 300, (B, H * W))
    nu = rng.uniform(-3400, -2300, (B, H * W))
    x = net.prepare(torch.from_numpy(J).cuda(), torch.from_numpy(D).cuda(), torch.from_numpy(nu).cuda()).cpu().numpy()
    mj = J.astype(np.float64).mean(1, keepdims=True)
    lj = np.where(J > 0, np.log(np.maximum(J, 1e-30) / mj), -8.0).clip(-8, 8)
    assert np.allclose(x[:, 0].reshape(B, -1), lj, atol=1e-5)
    assert np.allclose(x[:, 1].reshape(B, -1), D / 64, rtol=1e-6)
    assert np.allclose(x[:, 2].reshape(B, -1), (nu - nu.mean(1, keepdims=True)) / 256, atol=1e-4)
    # a fresh network has zero weights: every tile has probability 1/4096 < 0.5
    zz = net.forward(torch.from_numpy(x).cuda())
    _, pr = net.topk(zz, 1)
    assert np.allclose(pr, 1.0 / (H * W))
