"""Pins of the network oracle (oracle/net.py)."""
import numpy as np
import pytest

from oracle import net as NN


def _batch(seed, B=2, H=16, W=8):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((B, H, W)), rng.uniform(0.2, 1.9, size=B), rng.standard_normal((B, H, W))


def test_param_count_and_layout():
    assert NN.nparams() == 9 * 2 * 32 + 32 + 7 * (9 * 32 * 32 + 32) + 9 * 32 + 1
    th = NN.init_params(0)
    P = NN.unpack(th)
    assert P["cin"][0].shape == (9, 2, 32) and P["out"][0].shape == (9, 32, 1)
    assert np.all(P["u0"][1] == 0)


def test_conv_against_explicit_loop():
    rng = np.random.Generator(np.random.PCG64(1))
    x = rng.standard_normal((1, 5, 4, 3))
    W = rng.standard_normal((9, 3, 2))
    b = rng.standard_normal(2)
    y = NN.conv(x, W, b)
    for i in range(5):
        for j in range(4):
            for co in range(2):
                s = b[co]
                for ky in range(3):
                    for kx in range(3):
                        ii, jj = i + ky - 1, j + kx - 1
                        if 0 <= ii < 5 and 0 <= jj < 4:
                            s += x[0, ii, jj, :] @ W[3 * ky + kx, :, co]
                assert abs(y[0, i, j, co] - s) < 1e-12


def test_pool_up_adjoints():
    rng = np.random.Generator(np.random.PCG64(2))
    a = rng.standard_normal((2, 8, 6, 3))
    c = rng.standard_normal((2, 4, 3, 3))
    assert np.isclose((NN.pool(a) * c).sum(), (a * NN.pool_adjoint(c)).sum(), rtol=1e-13)
    assert np.isclose((NN.up(c) * a).sum(), (c * NN.up_adjoint(a)).sum(), rtol=1e-13)


def test_conv_input_gradient_is_adjoint():
    rng = np.random.Generator(np.random.PCG64(3))
    x = rng.standard_normal((1, 6, 5, 4))
    W = rng.standard_normal((9, 4, 3))
    g = rng.standard_normal((1, 6, 5, 3))
    dx, _, _ = NN.conv_grads(x, W, g)
    assert np.isclose((NN.conv(x, W, np.zeros(3)) * g).sum(), (x * dx).sum(), rtol=1e-12)


def test_gradient_by_finite_differences():
    x, al, t = _batch(4)
    th = NN.init_params(7)
    th = th + 0.05 * np.random.Generator(np.random.PCG64(8)).standard_normal(th.shape)  # nonzero biases
    g = NN.loss_grad(th, x, al, t)
    rng = np.random.Generator(np.random.PCG64(9))
    # sample coordinates in every layer (weights and biases)
    offs, o = [], 0
    for _, ci, co in NN.LAYERS:
        nw = 9 * ci * co
        offs += list(o + rng.integers(0, nw, 4)) + list(o + nw + rng.integers(0, co, 2))
        o += nw + co
    for i in offs:
        e = np.zeros_like(th)
        e[i] = 1e-6
        fd = (NN.loss(th + e, x, al, t) - NN.loss(th - e, x, al, t)) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g).max()), (i, fd, g[i])


def test_adam_step_scalar():
    th, m, v = np.array([1.0]), np.zeros(1), np.zeros(1)
    th1, m1, v1 = NN.adam_step(th, np.array([0.5]), m, v, 1, 0.1)
    # first step of Adam moves by lr * sign(g) (bias-corrected moments equal g and g^2)
    assert np.isclose(th1[0], 1.0 - 0.1 * 0.5 / (0.5 + 1e-8))
    assert np.isclose(m1[0], 0.05) and np.isclose(v1[0], 0.001 * 0.25)


def test_zero_last_layer_gives_zero_correction():
    x, al, _ = _batch(5)
    th = NN.init_params(3)
    P = NN.unpack(th)
    P["out"][0][:] = 0.0
    assert np.all(NN.forward(th, x, al) == 0.0)


# ---------------------------------------------------------------------------
# 3D form (3 x 3 x 3 kernels, 2 x 2 x 2 pooling)
# ---------------------------------------------------------------------------
def test_param_count_and_layout_3d():
    assert NN.nparams(3) == 27 * 2 * 32 + 32 + 7 * (27 * 32 * 32 + 32) + 27 * 32 + 1
    P = NN.unpack(NN.init_params(0, 3), 3)
    assert P["cin"][0].shape == (27, 2, 32) and P["d3"][0].shape == (27, 32, 32) and P["out"][0].shape == (27, 32, 1)


def test_conv3d_against_explicit_loop():
    rng = np.random.Generator(np.random.PCG64(11))
    x = rng.standard_normal((1, 3, 4, 5, 2))
    W = rng.standard_normal((27, 2, 3))
    b = rng.standard_normal(3)
    y = NN.conv(x, W, b)
    for i in range(3):
        for j in range(4):
            for k in range(5):
                for co in range(3):
                    s = b[co]
                    for kz in range(3):
                        for ky in range(3):
                            for kx in range(3):
                                ii, jj, kk = i + kz - 1, j + ky - 1, k + kx - 1
                                if 0 <= ii < 3 and 0 <= jj < 4 and 0 <= kk < 5:
                                    s += x[0, ii, jj, kk, :] @ W[9 * kz + 3 * ky + kx, :, co]
                    assert abs(y[0, i, j, k, co] - s) < 1e-12


def test_conv3d_with_planar_kernel_is_2d_conv_per_slice():
    # a 3 x 3 x 3 kernel that vanishes off its middle plane acts slice by slice
    rng = np.random.Generator(np.random.PCG64(12))
    x = rng.standard_normal((2, 4, 6, 5, 3))
    W2 = rng.standard_normal((9, 3, 4))
    b = rng.standard_normal(4)
    W3 = np.zeros((27, 3, 4))
    W3[9:18] = W2
    y3 = NN.conv(x, W3, b)
    for z in range(4):
        assert np.allclose(y3[:, z], NN.conv(x[:, z], W2, b), rtol=1e-13, atol=1e-13)


def test_pool_up_adjoints_3d():
    rng = np.random.Generator(np.random.PCG64(13))
    a = rng.standard_normal((2, 4, 8, 6, 3))
    c = rng.standard_normal((2, 2, 4, 3, 3))
    assert np.isclose((NN.pool(a) * c).sum(), (a * NN.pool_adjoint(c)).sum(), rtol=1e-13)
    assert np.isclose((NN.up(c) * a).sum(), (c * NN.up_adjoint(a)).sum(), rtol=1e-13)
    # pool of a constant field is that constant; up then pool is the identity
    assert np.allclose(NN.pool(np.full((1, 4, 4, 4, 1), 2.5)), 2.5)
    assert np.allclose(NN.pool(NN.up(c)), c, rtol=1e-14)


def test_conv3d_input_gradient_is_adjoint():
    rng = np.random.Generator(np.random.PCG64(14))
    x = rng.standard_normal((1, 4, 5, 3, 4))
    W = rng.standard_normal((27, 4, 3))
    g = rng.standard_normal((1, 4, 5, 3, 3))
    dx, _, _ = NN.conv_grads(x, W, g)
    assert np.isclose((NN.conv(x, W, np.zeros(3)) * g).sum(), (x * dx).sum(), rtol=1e-12)


def test_gradient_by_finite_differences_3d():
    rng = np.random.Generator(np.random.PCG64(15))
    x, t = rng.standard_normal((1, 8, 8, 8)), rng.standard_normal((1, 8, 8, 8))
    al = np.array([1.4])
    th = NN.init_params(16, 3)
    th = th + 0.05 * np.random.Generator(np.random.PCG64(17)).standard_normal(th.shape)
    g = NN.loss_grad(th, x, al, t)
    offs, o = [], 0
    for _, ci, co in NN.LAYERS:
        nw = 27 * ci * co
        offs += list(o + rng.integers(0, nw, 3)) + list(o + nw + rng.integers(0, co, 1))
        o += nw + co
    for i in offs:
        e = np.zeros_like(th)
        e[i] = 1e-6
        fd = (NN.loss(th + e, x, al, t) - NN.loss(th - e, x, al, t)) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g).max()), (i, fd, g[i])
