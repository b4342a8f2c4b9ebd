"""GPU parity of the warm-start network (bfloat16 activations on the matrix
cores, float32 accumulation) against the float64 network oracle: forward
output, every parameter gradient, and Adam steps, through the C ABI.

Tolerances.  The oracle gets the same bfloat16-rounded parameters and input,
so the GPU differs only by rounding each stored activation (9 tensors in the
forward pass, 10 more in the backward pass) to bfloat16, relative error at
most 2^-9 each, and by float32 accumulation order.  Stacked through the
layers this gives a relative L2 error of at most a few 2^-9 (about 1 %) on
the output; the bound used is 2e-2.  Gradients pass through about twice as
many roundings, and a ReLU gate can flip where a rounded activation crosses
zero, so their bound is 5e-2 in relative L2 per parameter tensor, together
with a cosine similarity above 0.998.  Adam is compared on the GPU's own
gradient, so only float32 arithmetic differs (1e-5 relative).
"""
import numpy as np
import pytest

from oracle import unet as oun
from tests.parity import bf16_round, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPE = (24, 12, 16)      # (z, y, x): the quarter-resolution level has 72 sites (ragged tail)


@pytest.fixture(scope="module")
def ek():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1710_09421_amd import ek as binding
    binding.lib()
    return binding


def problem(seed, shape=SHAPE):
    rng = np.random.default_rng(seed)
    p = oun.init_params(seed)
    for k in p:
        if k.endswith(".b"):
            p[k] = rng.normal(scale=0.05, size=p[k].shape)
        p[k] = bf16_round(p[k])
    b = rng.normal(size=shape) + 0.3
    solid = (rng.uniform(size=shape) < 0.2).astype(np.uint8)
    target = rng.normal(size=shape)
    return p, b, solid, target


def oracle_input(b, solid):
    x, s = oun.network_input(b - b.mean(), solid)
    x[0] = bf16_round(x[0])
    return x, s


def to_dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def test_forward_matches_oracle(ek):
    p, b, solid, _ = problem(1)
    c_out = 0.37
    net = ek.UNet(SHAPE, training=False)
    net.set_params(oun.flatten(p), c_out)
    guess = torch.zeros(SHAPE, dtype=torch.float64, device="cuda")
    net.forward(to_dev(b), to_dev(solid, torch.uint8), guess)
    x, s = oracle_input(b, solid)
    out, _ = oun.forward(p, x)
    ref = out[0] * s * c_out
    err = rel_l2(guess.cpu().numpy(), ref)
    print("forward relative L2", err)
    assert err < 1e-2


def test_gradients_match_oracle(ek):
    p, b, solid, y = problem(2)
    c_out = 1.7
    net = ek.UNet(SHAPE, training=True)
    net.set_params(oun.flatten(p), c_out)
    x, s = oracle_input(b, solid)
    net.accumulate(to_dev(b), to_dev(solid, torch.uint8), to_dev(y * s * c_out))
    g_gpu = oun.unflatten(net.gradient())
    loss_gpu, count = net.read_loss()
    out, cache = oun.forward(p, x)
    g_ref = oun.backward(p, cache, out, y[None])
    assert count == 1
    assert loss_gpu == pytest.approx(oun.loss(out, y[None]), rel=2e-2)
    for k in p:
        e = rel_l2(g_gpu[k], g_ref[k])
        cos = float(np.dot(g_gpu[k].ravel(), g_ref[k].ravel()) /
                    (np.linalg.norm(g_gpu[k]) * np.linalg.norm(g_ref[k])))
        print(k, "relative L2", e, "cosine", cos)
        assert e < 2e-2 and cos > 0.9995, (k, e, cos)


def test_gradient_accumulates_and_clears(ek):
    p, b, solid, y = problem(3)
    net = ek.UNet(SHAPE, training=True)
    net.set_params(oun.flatten(p), 1.0)
    args = (to_dev(b), to_dev(solid, torch.uint8), to_dev(y))
    net.accumulate(*args)
    g1 = net.gradient()
    net.accumulate(*args)
    g2 = net.gradient()
    assert np.allclose(g2, 2 * g1, rtol=1e-5, atol=1e-12)   # same deterministic sum twice
    net.zero_gradient()
    assert not net.gradient().any()
    assert net.read_loss()[1] == 2


def test_adam_matches_oracle_on_the_same_gradient(ek):
    p, b, solid, y = problem(4)
    net = ek.UNet(SHAPE, training=True)
    net.set_params(oun.flatten(p), 1.0)
    args = (to_dev(b), to_dev(solid, torch.uint8), to_dev(y))
    ref = {k: v.copy() for k, v in p.items()}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(w) for k, w in p.items()}
    lr = 1e-3
    for t in (1, 2, 3):
        net.accumulate(*args)
        g = net.gradient()
        net.adam_step(lr, grad_scale=0.5)
        oun.adam_step(ref, oun.unflatten(0.5 * g.astype(np.float64)), m, v, t, lr)
        got = oun.unflatten(net.params()[0].astype(np.float64))
        for k in p:
            assert np.allclose(got[k], ref[k], rtol=1e-5, atol=2e-5 * lr), (t, k)
        assert not net.gradient().any()
