"""Pins of the oracle's sine-basis diagonal preconditioner (oracle/spectral.py)."""
import math

import numpy as np
import pytest

from oracle import krylov as KR
from oracle import operator as O
from oracle import precond as PC
from oracle import spectral as SP
from workloads import white_noise


@pytest.mark.parametrize("n", [1, 2, 5, 12, 33])
def test_sine_correlation_closed_form(n):
    assert np.allclose(SP.sine_correlation(n), SP.sine_correlation_direct(n), atol=1e-13, rtol=0)


@pytest.mark.parametrize("n", [(9,), (7, 8), (4, 5, 3)])
def test_fd_laplacian_is_in_the_algebra(n):
    # T's folded stencil: 2d at the centre, -1 at the unit lags; its sine
    # diagonal must be its exact eigenvalues
    d = len(n)
    st = np.zeros(n)
    st[(0,) * d] = 2.0 * d
    for a in range(d):
        idx = [0] * d
        idx[a] = 1
        if n[a] > 1:
            st[tuple(idx)] = -1.0
    got = SP.diagonal_from_weights(st)
    assert np.allclose(got, PC.fd_eigenvalues(n), atol=1e-13, rtol=0)


@pytest.mark.parametrize("n,alpha", [((11,), 0.7), ((6, 7), 1.3), ((5, 4, 6), 1.8), ((8, 8), 0.3)])
def test_tau_matches_bruteforce_diagonal(n, alpha):
    d = len(n)
    h = 2.0 / (max(n) + 1)
    op = O.Operator(d, alpha, h, n)
    Om = op.dense() / (op.C * h ** -alpha)
    want = SP.dst_diagonal_dense(Om, n)
    got = SP.tau_eigenvalues(d, alpha, n)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-13)
    assert np.all(got > 0)  # diagonal of an SPD matrix in an orthonormal basis


def test_tau_inverse_is_the_dense_inverse_of_its_matrix():
    n, alpha = (6, 5), 1.1
    m = SP.tau_eigenvalues(2, alpha, n)
    Q = np.kron(PC.sine_matrix(6) * math.sqrt(2 / 7), PC.sine_matrix(5) * math.sqrt(2 / 6))
    A = Q @ np.diag((0.3 + 2.0 * m).ravel()) @ Q.T
    r = white_noise(n, 2)
    z = SP.apply_tau_inverse(r, m, 2.0, shift0=0.3)
    assert np.allclose(z.ravel(), np.linalg.solve(A, r.ravel()), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("alpha", [0.5, 1.0, 1.5])
def test_tau_pcg_iterations_are_few_and_grid_independent(alpha):
    # the point of the preconditioner: few iterations at every grid size,
    # where the FD Laplacian needs many more (Table 2dcg of the paper)
    its = []
    for n in (16, 32):
        h = 2.0 / (n + 1)
        op = O.Operator(2, alpha, h, (n, n))
        M = op.dense()
        m = SP.tau_eigenvalues(2, alpha, (n, n))
        sc = op.C * h ** -alpha
        f = white_noise((n, n), 3)
        _, it, rel, _ = KR.pcg(lambda v: (M @ v.ravel()).reshape(v.shape), f,
                               lambda r: SP.apply_tau_inverse(r, m, sc), tol=1e-10)
        _, it_fd, _, _ = KR.pcg(lambda v: (M @ v.ravel()).reshape(v.shape), f,
                                lambda r: PC.apply_inverse(r, PC.pc_scale(2, alpha, h)), tol=1e-10)
        assert rel <= 1e-10
        assert it < it_fd
        its.append(it)
    assert max(its) <= 14
    assert abs(its[1] - its[0]) <= 2
