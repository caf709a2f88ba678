"""Multilevel convolutional network of the learned preconditioner: FP64 numpy
oracle of its forward pass, parameter gradient and Adam step.  Test
infrastructure only.  Not in the paper (a builder's design).

The network N(x, alpha) maps a normalised residual x (one channel on a 2D grid
H x W or a 3D grid D x H x W, every side a multiple of 8) to a correction y of
the same shape.  Layers, with ReLU after every convolution but the last,
average pooling over 2 x 2 (x 2) blocks `pool` and nearest 2x upsampling `up`:

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

Every convolution is 3 x 3 (2D) or 3 x 3 x 3 (3D) with zero padding,
conv(x)[p, co] = b[co] + sum_{k,ci} x[p + k - 1, ci] W[t(k), ci, co], the tap
index t(k) row-major over the offsets k in {0,1,2}^d (t = 3 ky + kx in 2D,
9 kz + 3 ky + kx in 3D).  With K = 3^d taps, the flat parameter vector holds,
in this order, W then b of cin (W: K x 2 x 32), of d1, d2, d3, b3, u2, u1, u0
(K x 32 x 32 each) and of out (K x 32, bias 1).

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


def taps(d=2):
    return 3 ** d


def param_shapes(d=2):
    K = taps(d)
    return [(name, (K, ci, co), (co,)) for name, ci, co in LAYERS]


def nparams(d=2):
    return sum(taps(d) * ci * co + co for _, ci, co in LAYERS)


def unpack(theta, d=2):
    out, o = {}, 0
    for name, ws, bs in param_shapes(d):
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out[name] = (theta[o:o + nw].reshape(ws), theta[o + nw:o + nw + nb])
        o += nw + nb
    return out


def init_params(seed, d=2):
    """He-uniform weights, zero biases, last layer scaled by 0.1 (seeded numpy draw)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    K = taps(d)
    parts = []
    for name, ci, co in LAYERS:
        lim = np.sqrt(6.0 / (K * ci))
        w = rng.uniform(-lim, lim, size=(K, ci, co))
        if name == "out":
            w *= 0.1
        parts += [w.ravel(), np.zeros(co)]
    return np.concatenate(parts)


def _offsets(d):
    """Tap offsets k in {0,1,2}^d in tap-index order (row-major)."""
    return list(np.ndindex(*(3,) * d))


def _window(xp, k, S):
    return xp[(slice(None),) + tuple(slice(k[i], k[i] + S[i]) for i in range(len(S))) + (slice(None),)]


def conv(x, W, b):
    """x [B, *S, ci] -> [B, *S, co], 3^d taps, zero padding (cross-correlation)."""
    S = x.shape[1:-1]
    d = len(S)
    xp = np.pad(x, ((0, 0),) + ((1, 1),) * d + ((0, 0),))
    y = np.broadcast_to(b, x.shape[:-1] + (W.shape[2],)).copy()
    for t, k in enumerate(_offsets(d)):
        y += np.tensordot(_window(xp, k, S), W[t], axes=([d + 1], [0]))
    return y


def conv_grads(x, W, g):
    """Given upstream g = dL/dy: (dL/dx, dL/dW, dL/db) of y = conv(x, W, b)."""
    S = x.shape[1:-1]
    d = len(S)
    xp = np.pad(x, ((0, 0),) + ((1, 1),) * d + ((0, 0),))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    ax = list(range(d + 1))
    for t, k in enumerate(_offsets(d)):
        dW[t] = np.tensordot(_window(xp, k, S), g, axes=(ax, ax))
        _window(dxp, k, S)[...] += np.tensordot(g, W[t], axes=([d + 1], [1]))
    inner = (slice(None),) + (slice(1, -1),) * d + (slice(None),)
    return dxp[inner], dW, g.sum(axis=tuple(ax))


def _blocks(x):
    """[B, *S, c] -> [B, S_0/2, 2, S_1/2, 2, ..., c] and the axes of the 2s."""
    S = x.shape[1:-1]
    shp = [x.shape[0]]
    for v in S:
        shp += [v // 2, 2]
    return x.reshape(shp + [x.shape[-1]]), tuple(2 + 2 * i for i in range(len(S)))


def pool(x):
    xb, ax = _blocks(x)
    return xb.mean(axis=ax)


def up(x):
    for i in range(x.ndim - 2):
        x = np.repeat(x, 2, axis=1 + i)
    return x


def pool_adjoint(g):
    return up(g) / 2.0 ** (g.ndim - 2)


def up_adjoint(g):
    gb, ax = _blocks(g)
    return gb.sum(axis=ax)


def relu(x):
    return np.maximum(x, 0.0)


def forward(theta, x, alpha, keep=False):
    """x [B, *S], alpha [B] -> y [B, *S] (and the activations if keep); d = len(S)."""
    x = np.asarray(x, dtype=np.float64)
    d = x.ndim - 1
    P = unpack(np.asarray(theta, dtype=np.float64), d)
    al = np.asarray(alpha, dtype=np.float64).reshape((-1,) + (1,) * (d + 1))
    x0 = np.concatenate([x[..., None], np.broadcast_to(al - 1.0, x[..., None].shape)], axis=d + 1)
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
    P = unpack(np.asarray(theta, dtype=np.float64), np.ndim(x) - 1)
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
    """Training loss: mean over the batch of ||N(x) - t||^2 / (number of grid points)."""
    y = forward(theta, x, alpha)
    return float(((y - t) ** 2).sum() / y.size)


def loss_grad(theta, x, alpha, t):
    y = forward(theta, x, alpha)
    return grad(theta, x, alpha, 2.0 * (y - t) / y.size)


def adam_step(theta, g, m, v, k, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015, Algorithm 1), step number k >= 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** k)
    vh = v / (1 - b2 ** k)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
