"""Sine-basis diagonal ("symbol-matched") preconditioner: FP64 oracle, test infrastructure only.

This preconditioner is not in the paper.  The paper preconditions with the
finite-difference Laplacian T (Sec. 3.1), which the type-I sine transform
diagonalises.  Here the same sine basis is kept but the eigenvalues are
replaced by the diagonal of the operator itself in that basis,

    m_k = (Q^T Omega Q)_{kk},   Q = Q_1 x ... x Q_d,  (Q_a)_{jk} = sqrt(2/(n_a+1)) sin(pi j k/(n_a+1)),

where Omega is the dimensionless operator (M = C h^{-alpha} Omega, the
weights omega_m of Sec. 3.1).  Q diag(m) Q^T is the best approximation of
Omega, in the Frobenius norm, among matrices the sine transform diagonalises
(the tau algebra of Bini and Di Benedetto).  Because Omega is a symmetric
multilevel Toeplitz matrix, the diagonal separates:

    m_k = sum_{m >= 0} omega_m prod_a G_a(k_a, m_a),
    G(k, m) = c_m sum_{i=1}^{n-m} q_k(i) q_k(i+m),  c_0 = 1, c_m = 2 (m > 0),

with the closed form (theta = pi k/(n+1), cos((n+1) theta) = (-1)^k)

    sum_{i=1}^{n-m} sin(i theta) sin((i+m) theta) = ((n-m) cos(m theta) - (-1)^k sin((n-m) theta)/sin(theta)) / 2.

Pins (tests/test_oracle_spectral.py): the brute-force diagonal of Q^T Omega Q
on tiny grids; the closed form of G against its defining sum; the FD
Laplacian, which lies in the algebra, giving back its exact eigenvalues
sum_a 4 sin^2(pi k_a/(2(n_a+1))); positivity; bounded PCG iteration counts.
"""
import math

import numpy as np

from . import operator as O
from .precond import sine_matrix


def sine_correlation_direct(n):
    """G(k, m), k = 1..n (row k-1), m = 0..n-1, by the defining sum (O(n^3))."""
    Q = sine_matrix(n) * math.sqrt(2.0 / (n + 1))  # Q[j-1, k-1]
    G = np.zeros((n, n))
    for m in range(n):
        G[:, m] = (Q[: n - m, :] * Q[m:, :]).sum(axis=0) * (1.0 if m == 0 else 2.0)
    return G


def sine_correlation(n):
    """G(k, m) by the closed form above (O(n^2))."""
    k = np.arange(1, n + 1, dtype=np.float64)[:, None]
    m = np.arange(n, dtype=np.float64)[None, :]
    th = math.pi * k / (n + 1)
    sgn = np.where(np.arange(1, n + 1) % 2 == 0, 1.0, -1.0)[:, None]
    s = 0.5 * ((n - m) * np.cos(m * th) - sgn * np.sin((n - m) * th) / np.sin(th))
    c = np.where(m == 0, 1.0, 2.0)
    return (2.0 / (n + 1)) * s * c


def diagonal_from_weights(om):
    """sum_m om_m prod_a G_a(k_a, m_a) for folded weights om of shape n (m_a < n_a)."""
    x = np.asarray(om, dtype=np.float64)
    for a in range(x.ndim):
        G = sine_correlation(x.shape[a])
        x = np.moveaxis(np.tensordot(G, x, axes=([1], [a])), 0, a)
    return x


def tau_eigenvalues(d, alpha, n, c=20.0):
    """Dimensionless m_k of Omega on the grid n (array of shape n, index k_a - 1)."""
    return diagonal_from_weights(O.omega_folded(d, alpha, n, c))


def dst_diagonal_dense(A, n):
    """diag(Q^T A Q) for a dense A on the grid n, by brute force (tiny grids)."""
    Q = np.ones((1, 1))
    for v in n:
        Q = np.kron(Q, sine_matrix(v) * math.sqrt(2.0 / (v + 1)))
    return np.einsum("jk,jl,lk->k", Q, A, Q).reshape(n)


def apply_tau_inverse(r, m, scale, shift0=0.0, shift1=1.0):
    """z = Q diag(1/(shift0 + shift1 scale m)) Q^T r with dense sine matrices."""
    x = np.asarray(r, dtype=np.float64)
    n = x.shape

    def sine_axes(v):
        for a in range(v.ndim):
            S = sine_matrix(v.shape[a])
            v = np.moveaxis(np.tensordot(S, v, axes=([1], [a])), 0, a)
        return v

    y = sine_axes(x) / (shift0 + shift1 * scale * m)
    return sine_axes(y) * np.prod([2.0 / (v + 1) for v in n])
