"""Multilevel convolutional network of the learned preconditioner: FP64 numpy
oracle of its forward pass, parameter gradient and Adam step.  Test
infrastructure only.  Not in the paper (a builder's design).

The network N(x, alpha) maps a normalised residual x (one channel, H x W, H and
W multiples of 8) to a correction y of the same shape.  Layers, with ReLU after
every convolution but the last, 2x2 average pooling `pool` and nearest 2x
upsampling `up`:

    x0 = [x, (alpha - 1)]                     2 channels
    a0 = relu(cin(x0))                        32 channels, H x W
    a1 = relu(d1(pool a0))                    H/2
    a2 = relu(d2(pool a1))                    H/4
    a3 = relu(d3(pool a2))                    H/8
    c3 = relu(b3(a3))                         H/8
    c2 = relu(u2(a2 + up c3))                 H/4
    c1 = relu(u1(a1 + up c2))                 H/2
    c0 = relu(u0(a0 + up c1))                 H
    y  = out(c0)                              1 channel

Every convolution is 3 x 3 with zero padding, conv(x)[p, co] = b[co] +
sum_{ky,kx,ci} x[p + (ky-1, kx-1), ci] W[3 ky + kx, ci, co].  The flat
parameter vector holds, in this order, W then b of cin (W: 9 x 2 x 32), of d1,
d2, d3, b3, u2, u1, u0 (9 x 32 x 32 each) and of out (9 x 32, bias 1).

The learned preconditioner is z = B (r + s N(r / s, alpha)) with s the RMS of r
and B the inverse of the sine-basis diagonal of M; N is trained so that
r + s N(r/s) matches D e, e = M^{-1} r, D = Q diag(tau) Q^T.

Pins (tests/test_oracle_net.py): central finite differences of the loss
against the analytic gradient, pooling/upsampling adjointness, a conv layer
against an explicit loop, the Adam step against its defining formulas on a
scalar example.
"""
import numpy as np

C = 32
LAYERS = [("cin", 2, C), ("d1", C, C), ("d2", C, C), ("d3", C, C), ("b3", C, C),
          ("u2", C, C), ("u1", C, C), ("u0", C, C), ("out", C, 1)]


def param_shapes():
    return [(name, (9, ci, co), (co,)) for name, ci, co in LAYERS]


def nparams():
    return sum(9 * ci * co + co for _, ci, co in LAYERS)


def unpack(theta):
    out, o = {}, 0
    for name, ws, bs in param_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out[name] = (theta[o:o + nw].reshape(ws), theta[o + nw:o + nw + nb])
        o += nw + nb
    return out


def init_params(seed):
    """He-uniform weights, zero biases, last layer scaled by 0.1 (seeded numpy draw)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for name, ci, co in LAYERS:
        lim = np.sqrt(6.0 / (9 * ci))
        w = rng.uniform(-lim, lim, size=(9, ci, co))
        if name == "out":
            w *= 0.1
        parts += [w.ravel(), np.zeros(co)]
    return np.concatenate(parts)


def conv(x, W, b):
    """x [B, H, W, ci] -> [B, H, W, co], 3x3, zero padding (cross-correlation)."""
    Bn, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    y = np.broadcast_to(b, (Bn, H, Wd, W.shape[2])).copy()
    for ky in range(3):
        for kx in range(3):
            y += np.tensordot(xp[:, ky:ky + H, kx:kx + Wd, :], W[3 * ky + kx], axes=([3], [0]))
    return y


def conv_grads(x, W, g):
    """Given upstream g = dL/dy: (dL/dx, dL/dW, dL/db) of y = conv(x, W, b)."""
    Bn, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for ky in range(3):
        for kx in range(3):
            xs = xp[:, ky:ky + H, kx:kx + Wd, :]
            dW[3 * ky + kx] = np.tensordot(xs, g, axes=([0, 1, 2], [0, 1, 2]))
            dxp[:, ky:ky + H, kx:kx + Wd, :] += np.tensordot(g, W[3 * ky + kx], axes=([3], [1]))
    return dxp[:, 1:-1, 1:-1, :], dW, g.sum(axis=(0, 1, 2))


def pool(x):
    Bn, H, Wd, c = x.shape
    return x.reshape(Bn, H // 2, 2, Wd // 2, 2, c).mean(axis=(2, 4))


def pool_adjoint(g):
    return np.repeat(np.repeat(g, 2, axis=1), 2, axis=2) / 4.0


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_adjoint(g):
    Bn, H, Wd, c = g.shape
    return g.reshape(Bn, H // 2, 2, Wd // 2, 2, c).sum(axis=(2, 4))


def relu(x):
    return np.maximum(x, 0.0)


def forward(theta, x, alpha, keep=False):
    """x [B, H, W], alpha [B] -> y [B, H, W] (and the activations if keep)."""
    P = unpack(np.asarray(theta, dtype=np.float64))
    x = np.asarray(x, dtype=np.float64)
    al = np.asarray(alpha, dtype=np.float64).reshape(-1, 1, 1, 1)
    x0 = np.concatenate([x[..., None], np.broadcast_to(al - 1.0, x[..., None].shape)], axis=3)
    act = {"x0": x0}
    act["a0"] = relu(conv(x0, *P["cin"]))
    act["p1"] = pool(act["a0"])
    act["a1"] = relu(conv(act["p1"], *P["d1"]))
    act["p2"] = pool(act["a1"])
    act["a2"] = relu(conv(act["p2"], *P["d2"]))
    act["p3"] = pool(act["a2"])
    act["a3"] = relu(conv(act["p3"], *P["d3"]))
    act["c3"] = relu(conv(act["a3"], *P["b3"]))
    act["s2"] = act["a2"] + up(act["c3"])
    act["c2"] = relu(conv(act["s2"], *P["u2"]))
    act["s1"] = act["a1"] + up(act["c2"])
    act["c1"] = relu(conv(act["s1"], *P["u1"]))
    act["s0"] = act["a0"] + up(act["c1"])
    act["c0"] = relu(conv(act["s0"], *P["u0"]))
    y = conv(act["c0"], *P["out"])[..., 0]
    return (y, act) if keep else y


def grad(theta, x, alpha, gy):
    """Parameter gradient of sum(gy * N(x, alpha)) (reverse pass, layer by layer)."""
    P = unpack(np.asarray(theta, dtype=np.float64))
    _, A = forward(theta, x, alpha, keep=True)
    G = {}
    g = np.asarray(gy, dtype=np.float64)[..., None]
    dc0, G["out_W"], G["out_b"] = conv_grads(A["c0"], P["out"][0], g)
    ds0, G["u0_W"], G["u0_b"] = conv_grads(A["s0"], P["u0"][0], dc0 * (A["c0"] > 0))
    dc1 = up_adjoint(ds0)
    ds1, G["u1_W"], G["u1_b"] = conv_grads(A["s1"], P["u1"][0], dc1 * (A["c1"] > 0))
    dc2 = up_adjoint(ds1)
    ds2, G["u2_W"], G["u2_b"] = conv_grads(A["s2"], P["u2"][0], dc2 * (A["c2"] > 0))
    dc3 = up_adjoint(ds2)
    da3, G["b3_W"], G["b3_b"] = conv_grads(A["a3"], P["b3"][0], dc3 * (A["c3"] > 0))
    dp3, G["d3_W"], G["d3_b"] = conv_grads(A["p3"], P["d3"][0], da3 * (A["a3"] > 0))
    da2 = ds2 + pool_adjoint(dp3)
    dp2, G["d2_W"], G["d2_b"] = conv_grads(A["p2"], P["d2"][0], da2 * (A["a2"] > 0))
    da1 = ds1 + pool_adjoint(dp2)
    dp1, G["d1_W"], G["d1_b"] = conv_grads(A["p1"], P["d1"][0], da1 * (A["a1"] > 0))
    da0 = ds0 + pool_adjoint(dp1)
    _, G["cin_W"], G["cin_b"] = conv_grads(A["x0"], P["cin"][0], da0 * (A["a0"] > 0))
    return np.concatenate([np.concatenate([G[f"{n}_W"].ravel(), G[f"{n}_b"].ravel()]) for n, _, _ in LAYERS])


def loss(theta, x, alpha, t):
    """Training loss: mean over the batch of ||N(x) - t||^2 / (H W)."""
    y = forward(theta, x, alpha)
    Bn = y.shape[0]
    return float(((y - t) ** 2).sum() / (Bn * y.shape[1] * y.shape[2]))


def loss_grad(theta, x, alpha, t):
    y = forward(theta, x, alpha)
    Bn, H, Wd = y.shape
    return grad(theta, x, alpha, 2.0 * (y - t) / (Bn * H * Wd))


def adam_step(theta, g, m, v, k, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015, Algorithm 1), step number k >= 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** k)
    vh = v / (1 - b2 ** k)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
