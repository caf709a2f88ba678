"""The CPU baseline with a library FFT (oracle/cpu_fft.py) against the
oracle's explicit-DFT application, dense matrices and sine-matrix
preconditioner."""
import numpy as np
import pytest

from oracle import cpu_fft as CF
from oracle import operator as O
from oracle import precond as PC


@pytest.mark.parametrize("n", [(13,), (9, 11), (5, 6, 7)])
def test_apply_matches_dense(n):
    rng = np.random.default_rng(len(n) + 40)
    d, alpha, h = len(n), 1.2, 0.1
    s = CF.FFTSolver(d, alpha, h, n)
    u = rng.standard_normal(n)
    want = O.apply_dense(O.weights_folded(d, alpha, h, n), u)
    assert np.abs(s.apply(u) - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("n", [(13,), (9, 11), (5, 6, 7)])
@pytest.mark.parametrize("shift", [(0.0, 1.0), (1.0, 0.03)])
def test_precond_matches_sine_matrices(n, shift):
    rng = np.random.default_rng(len(n) + 41)
    d, alpha, h = len(n), 1.6, 0.1
    s = CF.FFTSolver(d, alpha, h, n)
    r = rng.standard_normal(n)
    want = PC.apply_inverse(r, PC.pc_scale(d, alpha, h), *shift)
    assert np.abs(s.precond(r, *shift) - want).max() <= 1e-12 * np.abs(want).max()


def test_solve_matches_dense_solution():
    n, alpha, h = (20, 17), 1.5, 0.08
    s = CF.FFTSolver(2, alpha, h, n)
    f = np.random.default_rng(3).standard_normal(n)
    x, it, res, _ = s.solve(f, tol=1e-12)
    M = O.Operator(2, alpha, h, n).dense()
    xs = np.linalg.solve(M, f.ravel()).reshape(n)
    assert res <= 1e-12 and np.abs(x - xs).max() <= 1e-9 * np.abs(xs).max()
