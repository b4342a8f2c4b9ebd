"""Float64 reference of the small 3-D convolutional network used as a warm
start of the Poisson solve: forward pass, loss, backward pass (explicit chain
rule, no autograd), Adam step.

The network maps the charge density (scaled by its RMS s) and the solid mask
to the potential (divided by s and by a fixed output scale c_out); with
uniform permittivity the potential is linear in the charge, so the same
network serves every salt concentration.  Layout here is channels-first,
[C, Z, Y, X]; every convolution wraps around the periodic box.

    A  conv 3x3x3  2 -> 16, bias, ReLU                       a1   (full grid)
       average pool 2x2x2                                    p1   (1/2)
    B  conv 3x3x3 16 -> 32, bias, ReLU                       a2   (1/2)
       average pool 2x2x2                                    p2   (1/4)
    C  conv 3x3x3 32 -> 64, bias, ReLU                       a3   (1/4)
    D  conv 1x1x1 64 -> 32, bias                             u3   (1/4)
       nearest upsample, add a2, ReLU                        c2   (1/2)
    E  conv 1x1x1 32 -> 16, bias                             u2   (1/2)
       nearest upsample, add a1, ReLU                        c1   (full)
    F  conv 3x3x3 16 -> 1, bias                              out  (full)

Weights of a 3x3x3 layer are [27, C_in, C_out] with tap t = (dz+1)*9 +
(dy+1)*3 + (dx+1), meaning out[:, z, y, x] sums in[:, z+dz, y+dy, x+dx]; 1x1x1
layers are [1, C_in, C_out].  Parameters are listed in the order A..F,
weights then bias.
"""
import numpy as np

LAYERS = [("A", 27, 2, 16), ("B", 27, 16, 32), ("C", 27, 32, 64), ("D", 1, 64, 32),
          ("E", 1, 32, 16), ("F", 27, 16, 1)]

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def param_shapes():
    out = []
    for name, taps, cin, cout in LAYERS:
        out.append((name + ".w", (taps, cin, cout)))
        out.append((name + ".b", (cout,)))
    return out


def param_count():
    return sum(int(np.prod(s)) for _, s in param_shapes())


def init_params(seed=0):
    """He-style initial weights (normal, std sqrt(2 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, taps, cin, cout in LAYERS:
        p[name + ".w"] = rng.normal(scale=np.sqrt(2.0 / (taps * cin)), size=(taps, cin, cout))
        p[name + ".b"] = np.zeros(cout)
    return p


def flatten(p):
    return np.concatenate([p[k].ravel() for k, _ in param_shapes()])


def unflatten(v):
    p, o = {}, 0
    for k, s in param_shapes():
        n = int(np.prod(s))
        p[k] = np.asarray(v[o:o + n], dtype=np.float64).reshape(s)
        o += n
    return p


def _shift(x, dz, dy, dx):
    """x[:, z+dz, y+dy, x+dx] on the periodic grid."""
    return np.roll(x, (-dz, -dy, -dx), axis=(1, 2, 3))


def conv(x, w, b):
    """x [Cin, Z, Y, X], w [taps, Cin, Cout], b [Cout] -> [Cout, Z, Y, X]."""
    taps = TAPS if w.shape[0] == 27 else [(0, 0, 0)]
    out = np.zeros((w.shape[2],) + x.shape[1:])
    for t, (dz, dy, dx) in enumerate(taps):
        out += np.einsum("czyx,cd->dzyx", _shift(x, dz, dy, dx), w[t])
    return out + b[:, None, None, None]


def conv_backward(x, w, dy):
    """Gradients of conv(x, w, b) given dL/dout: (dx, dw, db)."""
    taps = TAPS if w.shape[0] == 27 else [(0, 0, 0)]
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for t, (dz, dyy, dxx) in enumerate(taps):
        xs = _shift(x, dz, dyy, dxx)
        dw[t] = np.einsum("czyx,dzyx->cd", xs, dy)
        # out(r) gets x(r + d) w: the gradient flows back to x at r + d
        dx += _shift(np.einsum("dzyx,cd->czyx", dy, w[t]), -dz, -dyy, -dxx)
    return dx, dw, dy.sum(axis=(1, 2, 3))


def pool(x):
    C, Z, Y, X = x.shape
    return x.reshape(C, Z // 2, 2, Y // 2, 2, X // 2, 2).mean(axis=(2, 4, 6))


def pool_backward(dy):
    return upsample(dy) / 8.0


def upsample(x):
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def upsample_backward(dy):
    C, Z, Y, X = dy.shape
    return dy.reshape(C, Z // 2, 2, Y // 2, 2, X // 2, 2).sum(axis=(2, 4, 6))


def relu(x):
    return np.maximum(x, 0.0)


def forward(p, x):
    """x [2, Z, Y, X] -> (out [1, Z, Y, X], cache of activations)."""
    c = {}
    c["x"] = x
    c["a1"] = relu(conv(x, p["A.w"], p["A.b"]))
    c["p1"] = pool(c["a1"])
    c["a2"] = relu(conv(c["p1"], p["B.w"], p["B.b"]))
    c["p2"] = pool(c["a2"])
    c["a3"] = relu(conv(c["p2"], p["C.w"], p["C.b"]))
    c["u3"] = conv(c["a3"], p["D.w"], p["D.b"])
    c["c2"] = relu(upsample(c["u3"]) + c["a2"])
    c["u2"] = conv(c["c2"], p["E.w"], p["E.b"])
    c["c1"] = relu(upsample(c["u2"]) + c["a1"])
    out = conv(c["c1"], p["F.w"], p["F.b"])
    return out, c


def loss(out, target):
    """Mean squared error over all sites."""
    return float(np.mean((out - target) ** 2))


def backward(p, c, out, target):
    """Gradients of loss(forward(p, x), target) with respect to every parameter."""
    g = {}
    dout = 2.0 * (out - target) / out.size
    dc1, g["F.w"], g["F.b"] = conv_backward(c["c1"], p["F.w"], dout)
    dc1 = dc1 * (c["c1"] > 0)
    du2 = upsample_backward(dc1)
    da1 = dc1.copy()
    dc2, g["E.w"], g["E.b"] = conv_backward(c["c2"], p["E.w"], du2)
    dc2 = dc2 * (c["c2"] > 0)
    du3 = upsample_backward(dc2)
    da2 = dc2.copy()
    da3, g["D.w"], g["D.b"] = conv_backward(c["a3"], p["D.w"], du3)
    dpre3 = da3 * (c["a3"] > 0)
    dp2, g["C.w"], g["C.b"] = conv_backward(c["p2"], p["C.w"], dpre3)
    da2 = da2 + pool_backward(dp2)
    dpre2 = da2 * (c["a2"] > 0)
    dp1, g["B.w"], g["B.b"] = conv_backward(c["p1"], p["B.w"], dpre2)
    da1 = da1 + pool_backward(dp1)
    dpre1 = da1 * (c["a1"] > 0)
    _, g["A.w"], g["A.b"] = conv_backward(c["x"], p["A.w"], dpre1)
    return g


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) of every parameter, t counting from 1."""
    for k in p:
        m[k] = beta1 * m[k] + (1 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1 - beta2) * g[k] ** 2
        mh = m[k] / (1 - beta1 ** t)
        vh = v[k] / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def network_input(rho, solid):
    """(rho / s, solid) with s the RMS of rho; returns (x, s)."""
    s = float(np.sqrt(np.mean(rho * rho)))
    s = s if s > 0 else 1.0
    return np.stack([rho / s, solid.astype(np.float64)]), s
