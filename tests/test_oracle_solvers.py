"""Pins of the oracle's preconditioner, Krylov solvers and time stepping."""
import os

import numpy as np
import pytest
from scipy import linalg

from oracle import krylov as KR
from oracle import operator as O
from oracle import precond as PC

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n", [(7,), (5, 6), (3, 4, 5)])
@pytest.mark.parametrize("shift", [(0.0, 1.0), (1.0, 0.3)])
def test_sine_inverse_equals_dense_fd_solve(n, shift):
    rng = np.random.default_rng(3)
    r = rng.standard_normal(n)
    scale = 2.7
    z = PC.apply_inverse(r, scale, *shift)
    A = PC.fd_matrix(n, scale, *shift)
    ref = np.linalg.solve(A, r.ravel()).reshape(n)
    assert np.abs(z - ref).max() <= 1e-12 * np.abs(ref).max()


def test_sine_inverse_1d_equals_thomas():
    n, scale = 50, 0.9
    r = np.random.default_rng(4).standard_normal(n)
    ab = np.zeros((3, n))
    ab[0, 1:] = -scale
    ab[1, :] = 2 * scale
    ab[2, :-1] = -scale
    ref = linalg.solve_banded((1, 1), ab, r)
    assert np.allclose(PC.apply_inverse(r, scale), ref, rtol=1e-12, atol=1e-13)


def test_fd_preconditioner_is_the_laplacian_part_of_m():
    # M = C h^d (K + L): the nearest-neighbour coupling of M minus that of K is the FD part.
    d, alpha, h, n = 2, 1.4, 0.05, (5, 4)
    op = O.Operator(d, alpha, h, n)
    C, B = op.C, op.B
    # nearest-neighbour weight w_e = C h^{-alpha}(-1 + B); K contributes -C h^{-alpha}
    assert op.w[1, 0] == pytest.approx(C * h**-alpha * (-1 + B), rel=1e-14)
    assert PC.pc_scale(d, alpha, h) == pytest.approx(C * abs(B) * h**-alpha, rel=1e-14)


@pytest.mark.parametrize("n", [(20,), (8, 9), (4, 5, 3)])
def test_pcg_matches_cholesky(n):
    d, alpha, h = len(n), 1.3, 0.06
    op = O.Operator(d, alpha, h, n)
    M = op.dense()
    f = np.random.default_rng(5).standard_normal(n)
    ref = linalg.cho_solve(linalg.cho_factor(M), f.ravel()).reshape(n)
    sc = PC.pc_scale(d, alpha, h)
    for pc in (None, lambda r: PC.apply_inverse(r, sc)):
        x, it, rr, _ = KR.pcg(op.apply, f, pc, tol=1e-14, maxit=500)
        assert np.abs(x - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.slow
@pytest.mark.parametrize("row", [0, 2])
def test_table_2dcg_pcg_iterations(row):
    N, alpha, p6, p9 = np.loadtxt(os.path.join(GOLDEN, "tab_2dcg.txt"), comments="#")[row]
    n = int(N)
    h = 1.0 / (n + 1)
    op = O.Operator(2, alpha, h, (n, n))
    f = np.ones((n, n))
    sc = PC.pc_scale(2, alpha, h)
    pc = lambda r: PC.apply_inverse(r, sc)
    it6 = KR.pcg(op.apply, f, pc, tol=1e-6)[1]
    it9 = KR.pcg(op.apply, f, pc, tol=1e-9)[1]
    assert abs(it6 - p6) <= 2 and abs(it9 - p9) <= 3, (it6, it9, p6, p9)


def test_fcg_with_fixed_preconditioner_equals_pcg():
    n, alpha, h = (10, 9), 1.5, 0.05
    op = O.Operator(2, alpha, h, n)
    f = np.random.default_rng(6).standard_normal(n)
    sc = PC.pc_scale(2, alpha, h)
    pc = lambda r: PC.apply_inverse(r, sc)
    x1, it1, _, h1 = KR.pcg(op.apply, f, pc, tol=1e-12)
    x2, it2, _, h2 = KR.fcg(op.apply, f, pc, tol=1e-12)
    assert abs(it1 - it2) <= 1
    m = min(len(h1), len(h2)) - 2
    assert np.allclose(h1[:m], h2[:m], rtol=1e-6)
    assert np.abs(x1 - x2).max() <= 1e-10 * np.abs(x1).max()


@pytest.mark.parametrize("theta", [0.5, 1.0])
@pytest.mark.parametrize("n", [(12, 12), (5, 4, 6)])
def test_theta_steps_equal_exact_propagator(theta, n):
    d, alpha, h, dt, K = len(n), 1.2, 0.08, 0.01, 6
    op = O.Operator(d, alpha, h, n)
    M = op.dense()
    u0 = np.random.default_rng(7).standard_normal(n)
    sc = PC.pc_scale(d, alpha, h)
    pc = lambda r: PC.apply_inverse(r, sc, 1.0, theta * dt)
    u = u0.copy()
    norms = [np.linalg.norm(u)]
    for _ in range(K):
        u, it = KR.theta_step(op.apply, pc, u, dt, theta, tol=1e-14)
        norms.append(np.linalg.norm(u))
    ref = KR.exact_propagator(M, dt, theta, K, u0).reshape(n)
    assert np.abs(u - ref).max() <= 1e-11 * np.abs(ref).max()
    # with f = 0 the scheme is a contraction (M is SPD, |g| < 1)
    assert all(norms[i + 1] <= norms[i] for i in range(K))


def test_theta_step_is_linear_solve():
    n, alpha, h, dt = (9, 8), 0.7, 0.1, 0.05
    op = O.Operator(2, alpha, h, n)
    M = op.dense()
    u = np.random.default_rng(8).standard_normal(n)
    f1 = np.random.default_rng(9).standard_normal(n)
    x, _ = KR.theta_step(op.apply, None, u, dt, 1.0, tol=1e-14, f_k1=f1)
    A = np.eye(M.shape[0]) + dt * M
    ref = np.linalg.solve(A, u.ravel() + dt * f1.ravel()).reshape(n)
    assert np.abs(x - ref).max() <= 1e-11 * np.abs(ref).max()


def test_planted_sign_error_is_caught():
    # A plausible mistake in the stencil (omega_e = -1 - B instead of -1 + B) must break
    # the 1D table pin: recompute e_app for N = 511, alpha = 1.25 with the sign flipped.
    import math
    from scipy import special
    from oracle import constants as Kc
    N, alpha = 511, 1.25
    x, h = O.grid_points(N)
    w = O.weights_folded(1, alpha, h, (N,))
    B = Kc.b_const(1, alpha)
    w_bad = w.copy()
    w_bad[1] = Kc.c_alpha(alpha, 1) * h**-alpha * (-1 - B)
    Kq = 2**alpha * math.gamma(3 + alpha / 2) * math.gamma((1 + alpha) / 2) / (2 * math.sqrt(math.pi))
    f = special.hyp2f1((1 + alpha) / 2, -2, 0.5, x**2)
    ut = (1 - x**2) ** (2 + alpha / 2) / Kq
    good = np.linalg.norm(O.apply_dense(w, ut) - f) / np.linalg.norm(f)
    bad = np.linalg.norm(O.apply_dense(w_bad, ut) - f) / np.linalg.norm(f)
    assert good < 4e-6 < 1e-3 < bad
