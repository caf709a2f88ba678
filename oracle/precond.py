"""Finite-difference Laplacian preconditioner (FP64 oracle; test infrastructure only).

Paper Sec. 3.1 ("Preconditioning: Laplacian pattern and fast Poisson solver"):
M = C h^d (K + L) where L = (A_2 + A_3) L_FD is, up to the positive factor
-(A_2 + A_3), the standard finite-difference negative Laplacian with
homogeneous Dirichlet data.  In dimensionless form

    Pc = C h^d L = C |B| h^{-alpha} T,   T = sum_a I x ... x tridiag(-1, 2, -1) x ... x I,

on the box.  For time steps (Sec. 3.2) the preconditioner is I + theta dt Pc
(the paper: I + (dt/2) C h^d L for Crank-Nicolson), written here as
shift0 I + shift1 Pc.  T is diagonalised by the type-I sine transform:
eigenvectors prod_a sin(pi j_a k_a/(n_a+1)), eigenvalues
sum_a 4 sin^2(pi k_a / (2 (n_a + 1))), k_a = 1..n_a.  Its inverse is
applied here with dense sine matrices (S^2 = (n+1)/2 I per axis).
"""
import math

import numpy as np

from . import constants as K


def sine_matrix(n):
    """S_{jk} = sin(pi j k / (n+1)), j, k = 1..n."""
    j = np.arange(1, n + 1)
    return np.sin(math.pi * np.outer(j, j) / (n + 1))


def fd_eigenvalues(n):
    """Eigenvalues of T on the grid n (array of shape n), k_a = 1..n_a."""
    lam = 0.0
    for a, v in enumerate(n):
        e = 4.0 * np.sin(math.pi * np.arange(1, v + 1) / (2.0 * (v + 1))) ** 2
        shape = [1] * len(n)
        shape[a] = v
        lam = lam + e.reshape(shape)
    return lam


def pc_scale(d, alpha, h, c=20.0):
    """C |B| h^{-alpha}: the factor in front of T."""
    return K.c_alpha(alpha, d) * abs(K.b_const(d, alpha, c)) * h ** (-alpha)


def _sine_axes(x):
    for a in range(x.ndim):
        S = sine_matrix(x.shape[a])
        x = np.moveaxis(np.tensordot(S, x, axes=([1], [a])), 0, a)
    return x


def apply_inverse(r, scale, shift0=0.0, shift1=1.0):
    """z = (shift0 I + shift1 scale T)^{-1} r by dense sine transforms."""
    n = r.shape
    rh = _sine_axes(np.asarray(r, dtype=np.float64))
    rh = rh / (shift0 + shift1 * scale * fd_eigenvalues(n))
    z = _sine_axes(rh)
    return z * np.prod([2.0 / (v + 1) for v in n])


def fd_matrix(n, scale, shift0=0.0, shift1=1.0):
    """Dense shift0 I + shift1 scale T assembled as a Kronecker sum (used to pin apply_inverse)."""
    N = int(np.prod(n))
    A = np.zeros((N, N))
    for a, v in enumerate(n):
        t = 2.0 * np.eye(v) - np.eye(v, k=1) - np.eye(v, k=-1)
        ops = [np.eye(m) for m in n]
        ops[a] = t
        kr = ops[0]
        for o in ops[1:]:
            kr = np.kron(kr, o)
        A += kr
    return shift0 * np.eye(N) + shift1 * scale * A


# ---------------------------------------------------------------------------
# Occluded domains (Sec. 3.1 "Preconditioning" and Sec. 4.4): on a grid
# domain Omega inside the box the preconditioner is the same FD Laplacian
# with homogeneous Dirichlet data outside Omega, i.e. the principal submatrix
# L_Omega of the box matrix on the points of Omega.  The paper applies its
# inverse with a sparse Cholesky factorisation; here a sparse LU of the
# submatrix (scipy), the same exact inverse.
# ---------------------------------------------------------------------------
def fd_matrix_sparse(n, scale, shift0=0.0, shift1=1.0):
    """shift0 I + shift1 scale T as a scipy sparse matrix (Kronecker sum)."""
    import scipy.sparse as sp
    N = int(np.prod(n))
    A = sp.csr_matrix((N, N))
    for a, v in enumerate(n):
        t = sp.diags([-np.ones(v - 1), 2.0 * np.ones(v), -np.ones(v - 1)], [-1, 0, 1])
        kr = None
        for b, m in enumerate(n):
            o = t if b == a else sp.identity(m)
            kr = o if kr is None else sp.kron(kr, o)
        A = A + kr
    return (shift0 * sp.identity(N) + shift1 * scale * A).tocsc()


def apply_inverse_masked(r, mask, scale, shift0=0.0, shift1=1.0):
    """z = (shift0 I + shift1 scale T)_Omega^{-1} r on Omega (mask 1), z = 0 off it."""
    import scipy.sparse.linalg as spl
    n = r.shape
    m = np.asarray(mask).reshape(-1).astype(bool)
    A = fd_matrix_sparse(n, scale, shift0, shift1)[m][:, m]
    z = np.zeros(int(np.prod(n)))
    z[m] = spl.splu(A.tocsc()).solve(np.asarray(r, dtype=np.float64).reshape(-1)[m])
    return z.reshape(n)


# ---------------------------------------------------------------------------
# M~ (Sec. 3.1, the alternative preconditioner): M restricted to the sparsity
# pattern of L, M~_ij = M_ij where L_ij != 0 (i = j or |i - j|_1 = 1), else 0.
# With the weights of M, omega_0 = Z - 2dB and omega_{e_k} = -1 + B, and the
# shift sum S = 2d I - T of the stencil, M~ = C h^-alpha (omega_0 I +
# omega_e S) = q0 I + q1 T with q0 = C h^-alpha (Z - 2d), q1 = C h^-alpha (1 - B).
# ---------------------------------------------------------------------------
def mtilde_matrix(M, n):
    """M~ from a dense M on the grid n: entries off the FD pattern set to 0."""
    pattern = fd_matrix(n, 1.0) != 0.0
    return np.where(pattern, M, 0.0)


def mtilde_parts(d, alpha, h, c=20.0):
    """(q0, q1) with M~ = q0 I + q1 T on the box."""
    Ch = K.c_alpha(alpha, d) * h ** (-alpha)
    return Ch * (K.lattice_zeta(d, alpha) - 2.0 * d), Ch * (1.0 - K.b_const(d, alpha, c))


def apply_mtilde_inverse(r, d, alpha, h, shift0=0.0, shift1=1.0, mask=None, c=20.0):
    """z = (shift0 I + shift1 M~)^{-1} r on the box (dense sine transforms) or,
    with a mask, on Omega (sparse LU of the submatrix)."""
    q0, q1 = mtilde_parts(d, alpha, h, c)
    if mask is not None:
        return apply_inverse_masked(r, mask, q1, shift0 + shift1 * q0, shift1)
    return apply_inverse(r, q1, shift0 + shift1 * q0, shift1)
