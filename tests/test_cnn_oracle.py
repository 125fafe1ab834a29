"""Pins of the FP64 CNN oracle: a library convolution, central finite differences of
the loss, the zero-weight special case, softmax-CE closed forms and Adam's first step."""
import pytest
import numpy as np
import scipy.signal

from oracle import cnn

IN, HID, LAY = 3, 4, 4


def _rng(s):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(s)))


def test_conv_matches_scipy_correlate2d():
    rng = _rng(1)
    x = rng.standard_normal((2, 3, 7, 9))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = cnn.conv3x3(x, W, b)
    for bi in range(2):
        for o in range(4):
            ref = b[o] + sum(scipy.signal.correlate2d(x[bi, c], W[o, c], mode="same", boundary="fill")
                             for c in range(3))
            assert np.allclose(y[bi, o], ref, atol=1e-12)


def test_param_count_and_layout():
    assert cnn.n_params(3, 32, 4) == 3 * 32 * 9 + 32 + 2 * (32 * 32 * 9 + 32) + 32 * 9 + 1
    theta = np.arange(cnn.n_params(IN, HID, LAY), dtype=np.float64)
    p = cnn.unpack(theta, IN, HID, LAY)
    assert p[0][0].shape == (HID, IN, 3, 3) and p[-1][0].shape == (1, HID, 3, 3)
    assert p[0][1][0] == HID * IN * 9


def test_zero_weights_give_uniform_softmax():
    theta = np.zeros(cnn.n_params(IN, HID, LAY))
    x = _rng(2).standard_normal((2, IN, 8, 8))
    z, _ = cnn.forward(theta, x, IN, HID, LAY)
    _, _, p = cnn.softmax_ce(z, np.full((2, 8, 8), 1 / 64))
    assert np.allclose(p, 1 / 64) and p.max() < 0.5


def test_softmax_ce_closed_forms():
    z = _rng(3).standard_normal((3, 4, 5))
    q = np.zeros_like(z)
    q[:, 1, 2] = 1.0
    loss, dz, p = cnn.softmax_ce(z, q)
    zf = z.reshape(3, -1)
    ref = -np.mean(zf[:, 7] - np.log(np.exp(zf).sum(1)))
    assert abs(loss - ref) < 1e-12
    assert np.allclose(dz.reshape(3, -1).sum(1), 0.0, atol=1e-15)          # softmax and label both sum to 1
    assert np.allclose(p.reshape(3, -1).sum(1), 1.0)


def test_gradient_matches_central_differences():
    rng = _rng(4)
    theta = cnn.he_init(IN, HID, LAY, 5) + 0.05 * rng.standard_normal(cnn.n_params(IN, HID, LAY))
    x = rng.standard_normal((2, IN, 6, 7))
    q = rng.random((2, 6, 7))
    q /= q.sum(axis=(1, 2), keepdims=True)

    def loss_of(t):
        z, _ = cnn.forward(t, x, IN, HID, LAY)
        return cnn.softmax_ce(z, q)[0]

    z, cache = cnn.forward(theta, x, IN, HID, LAY)
    _, dz, _ = cnn.softmax_ce(z, q)
    g = cnn.backward(theta, cache, dz, IN, HID, LAY)
    h = 1e-6
    idx = rng.choice(theta.size, 60, replace=False)
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (loss_of(theta + e) - loss_of(theta - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])


def test_adam_first_step_is_sign_step():
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = cnn.adam(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, lr=0.01)
    # after one step m_hat = g and v_hat = g^2, so the update is -lr * g / (|g| + eps)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8))


def test_adam_constant_gradient_takes_equal_steps():
    """With a constant gradient the moments are m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2,
    so the bias-corrected update is -lr g / (|g| + eps) at every step, not only the first:
    this fixes both bias corrections at t = 2 and 3, where b^t differs from b."""
    g = np.array([0.3, -2.0, 1e-3, 7.5])
    th, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    step = -0.01 * g / (np.abs(g) + 1e-8)
    for t in (1, 2, 3):
        th, m, v = cnn.adam(th, m, v, g, t, lr=0.01)
        assert np.allclose(th, t * step, rtol=1e-12, atol=0), t


def test_adam_second_step_with_a_new_gradient():
    """Two steps with gradients g1 then g2, against the moments written out for t = 2:
    m = (1 - b1)(b1 g1 + g2), v = (1 - b2)(b2 g1^2 + g2^2), bias factors 1 - b^2."""
    b1, b2, lr, eps = 0.9, 0.999, 0.05, 1e-8
    g1, g2 = np.array([0.5, -1.0, 2.0]), np.array([-0.25, -3.0, 2.0])
    th, m, v = cnn.adam(np.zeros(3), np.zeros(3), np.zeros(3), g1, 1, lr=lr)
    th, m, v = cnn.adam(th, m, v, g2, 2, lr=lr)
    mh = (1 - b1) * (b1 * g1 + g2) / (1 - b1 ** 2)
    vh = (1 - b2) * (b2 * g1 ** 2 + g2 ** 2) / (1 - b2 ** 2)
    ref = -lr * g1 / (np.abs(g1) + eps) - lr * mh / (np.sqrt(vh) + eps)
    assert np.allclose(th, ref, rtol=1e-12, atol=1e-15)


ADAM_MUTANTS = {
    "first_bias_correction_fixed_at_t1": ("mh = m / (1 - b1 ** t)", "mh = m / (1 - b1)"),
    "second_bias_correction_fixed_at_t1": ("vh = v / (1 - b2 ** t)", "vh = v / (1 - b2)"),
    "no_square_root": ("np.sqrt(vh) + eps", "vh + eps"),
    "first_moment_weights_swapped": ("m = b1 * m + (1 - b1) * g", "m = (1 - b1) * m + b1 * g"),
}


@pytest.mark.parametrize("name", sorted(ADAM_MUTANTS))
def test_every_planted_adam_mistake_fails_a_pin(name, tmp_path):
    import importlib.util
    import os
    global cnn
    old, new = ADAM_MUTANTS[name]
    src = open(os.path.join(os.path.dirname(cnn.__file__), "cnn.py")).read()
    assert src.count(old) == 1, name
    path = tmp_path / f"cnn_{name}.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"oracle.cnn_{name}", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    saved, failed = cnn, []
    cnn = mod
    try:
        for pin in (test_adam_first_step_is_sign_step, test_adam_constant_gradient_takes_equal_steps,
                    test_adam_second_step_with_a_new_gradient):
            try:
                pin()
            except AssertionError:
                failed.append(pin.__name__)
    finally:
        cnn = saved
    assert failed, f"no pin catches the planted mistake {name!r}"
