"""Pins of the float64 network reference: every parameter gradient against
central finite differences of the loss, the periodic convolution against a
brute-force site loop, and the shape bookkeeping of the skips."""
import numpy as np
import pytest

from oracle import unet


def small_problem(seed=0, shape=(8, 4, 4)):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(2,) + shape)
    t = rng.normal(size=(1,) + shape)
    p = unet.init_params(seed)
    for k in p:                                    # non-zero biases exercise db
        if k.endswith(".b"):
            p[k] = rng.normal(scale=0.1, size=p[k].shape)
    return p, x, t


def test_parameter_count():
    assert unet.param_count() == 73137


def test_conv_matches_site_loop():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(3, 4, 6, 4))
    w = rng.normal(size=(27, 3, 2))
    b = rng.normal(size=2)
    out = unet.conv(x, w, b)
    C, Z, Y, X = x.shape
    ref = np.zeros((2, Z, Y, X))
    for z in range(Z):
        for y in range(Y):
            for xx in range(X):
                for t, (dz, dy, dx) in enumerate(unet.TAPS):
                    ref[:, z, y, xx] += x[:, (z + dz) % Z, (y + dy) % Y, (xx + dx) % X] @ w[t]
                ref[:, z, y, xx] += b
    assert np.allclose(out, ref, rtol=1e-12, atol=1e-12)


def test_gradients_match_finite_differences():
    p, x, t = small_problem()
    out, cache = unet.forward(p, x)
    g = unet.backward(p, cache, out, t)
    rng = np.random.default_rng(7)
    h = 1e-6
    for k in p:
        idx = [tuple(rng.integers(0, n) for n in p[k].shape) for _ in range(3)]
        for i in idx:
            old = p[k][i]
            p[k][i] = old + h
            lp = unet.loss(unet.forward(p, x)[0], t)
            p[k][i] = old - h
            lm = unet.loss(unet.forward(p, x)[0], t)
            p[k][i] = old
            fd = (lp - lm) / (2 * h)
            assert g[k][i] == pytest.approx(fd, rel=1e-5, abs=1e-10), (k, i)


def test_adam_moves_against_gradient_and_reduces_loss():
    p, x, t = small_problem(3)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(w) for k, w in p.items()}
    losses = []
    for it in range(1, 30):
        out, c = unet.forward(p, x)
        losses.append(unet.loss(out, t))
        unet.adam_step(p, unet.backward(p, c, out, t), m, v, it, 1e-2)
    assert losses[-1] < 0.5 * losses[0]


def test_flatten_roundtrip():
    p = unet.init_params(5)
    q = unet.unflatten(unet.flatten(p))
    for k in p:
        assert np.array_equal(p[k], q[k])
