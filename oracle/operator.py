"""The discrete operator M (FP64 oracle; test infrastructure only).

Paper Sec. 3.1, eqs. (linearelliptic) and (matelliptic): on the grid index
set J = [n_1] x ... x [n_d] with spacing h,

  (M u)_i = C h^d [ A_1 u_i - sum_{j in J, j != i} u_j / |y_i - y_j|^{d+alpha}
                    + (A_2 + A_3) L_FD u_i ],

with L_FD the (2d+1)-point Laplacian (Sec. 2.6).  The printed stencil centre
"-2^d u_i" is read as "-2d u_i" (the two agree for d <= 2; only 2d is a
consistent Laplacian in 3D).  In dimensionless weights, with s = d + alpha,

  M_ij = C h^{-alpha} omega_{i-j},   omega_0 = Z - 2 d B,
  omega_{+-e_k} = -1 + B,            omega_m = -|m|^{-s} otherwise,

which is the splitting M = C h^d (K + L) of Sec. 3.1 ("Preconditioning").
M is translation invariant (block Toeplitz with Toeplitz blocks), hence its
generating array w_m = C h^{-alpha} omega_m on the folded octant m >= 0 says
everything about it.

Circulant embedding (Sec. 3.1, "Forward operator and application with FFT";
the paper only says "FFT"): per axis the Toeplitz block is embedded in a
circulant of even length P_a >= 2 n_a (smallest 2^a 3^b 5^c), with
c_m = w_|m| when every |m_a| <= n_a - 1 and c_m = 0 at all other lags.  The
symbol lambda = DFT(c) is real and even; it is kept on the folded octant
k in [0, P_a/2]^d.  Lags of size >= n_a never reach the cropped product, so
the application M u = crop(IDFT(lambda * DFT(pad(u)))) is exact whatever
those lags hold.
"""
import itertools
import math

import numpy as np

from . import constants as K


def padded_length(n):
    """Smallest even P >= 2n whose prime factors are all in {2, 3, 5}."""
    P = 2 * n
    while True:
        m = P // 2
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            return P
        P += 2


def omega_folded(d, alpha, n, c=20.0):
    """Dimensionless weights omega_m on m in [0, n_1-1] x ... x [0, n_d-1]."""
    n = tuple(int(v) for v in n)
    s = d + alpha
    Z = K.lattice_zeta(d, alpha)
    B = K.b_const(d, alpha, c)
    grids = np.meshgrid(*[np.arange(v, dtype=np.float64) for v in n], indexing="ij")
    r2 = sum(g * g for g in grids)
    with np.errstate(divide="ignore"):
        om = -(r2 ** (-0.5 * s))
    om[(0,) * d] = Z - 2.0 * d * B
    for k in range(d):
        idx = [0] * d
        idx[k] = 1
        if n[k] > 1:
            om[tuple(idx)] = -1.0 + B
    return om


def weights_folded(d, alpha, h, n, c=20.0):
    """w_m = C h^{-alpha} omega_m on the folded octant [0, n_a - 1]."""
    return K.c_alpha(alpha, d) * h ** (-alpha) * omega_folded(d, alpha, n, c)


def dense_matrix(w):
    """The N x N matrix M_ij = w_{|i-j|} (row-major flattening, last axis fastest)."""
    n = w.shape
    d = len(n)
    idx = np.stack(np.meshgrid(*[np.arange(v) for v in n], indexing="ij"), -1).reshape(-1, d)
    diff = np.abs(idx[:, None, :] - idx[None, :, :])
    return w[tuple(diff[..., a] for a in range(d))]


def apply_dense(w, u):
    """(M u)_i = sum_{j in J} w_{|i-j|} u_j by direct summation (the definition)."""
    M = dense_matrix(w)
    return (M @ u.reshape(-1)).reshape(u.shape)


def apply_at(w, u, points):
    """(M u)_i for a list of multi-indices i, each by direct summation over all j."""
    n = u.shape
    d = len(n)
    out = np.empty(len(points))
    grids = np.meshgrid(*[np.arange(v) for v in n], indexing="ij")
    for t, i in enumerate(points):
        lag = tuple(np.abs(grids[a] - i[a]) for a in range(d))
        out[t] = math.fsum((w[lag] * u).ravel())
    return out


def circulant_folded(w, P):
    """Folded circulant generator c_m, m in [0, P_a/2]: w_m where m_a < n_a, else 0."""
    n = w.shape
    cf = np.zeros(tuple(p // 2 + 1 for p in P))
    cf[tuple(slice(0, min(v, p // 2 + 1)) for v, p in zip(n, P))] = \
        w[tuple(slice(0, min(v, p // 2 + 1)) for v, p in zip(n, P))]
    return cf


def _unfold(cf, P):
    """Even extension of a folded array to the full periodic array of shape P."""
    full = cf
    for a, p in enumerate(P):
        idx = np.array([min(k, p - k) for k in range(p)])
        full = np.take(full, idx, axis=a)
    return full


def dft_matrix(P, sign=-1):
    """Explicit DFT matrix F_{kj} = exp(sign 2 pi i k j / P)."""
    k = np.arange(P)
    return np.exp(sign * 2j * math.pi * np.outer(k, k) / P)


def _dft_axes(x, sign):
    for a in range(x.ndim):
        F = dft_matrix(x.shape[a], sign)
        x = np.moveaxis(np.tensordot(F, x, axes=([1], [a])), 0, a)
    return x


def symbol_full(w, P=None):
    """lambda = DFT of the circulant embedding, full P^d array (real part; imaginary ~ 0)."""
    if P is None:
        P = tuple(padded_length(v) for v in w.shape)
    lam = _dft_axes(_unfold(circulant_folded(w, P), P).astype(np.complex128), -1)
    return lam.real, float(np.max(np.abs(lam.imag)))


def symbol_folded(w, P=None):
    """lambda on the folded octant k in [0, P_a/2]^d."""
    if P is None:
        P = tuple(padded_length(v) for v in w.shape)
    lam, _ = symbol_full(w, P)
    return lam[tuple(slice(0, p // 2 + 1) for p in P)]


def apply_dft(lam_full, u):
    """M u = crop(IDFT(lambda * DFT(zero-pad(u)))) with explicit DFT matrices (no FFT)."""
    P = lam_full.shape
    n = u.shape
    x = np.zeros(P, dtype=np.complex128)
    x[tuple(slice(0, v) for v in n)] = u
    X = _dft_axes(x, -1) * lam_full
    y = _dft_axes(X, +1) / float(np.prod(P))
    return y[tuple(slice(0, v) for v in n)].real


def apply_fft(lam_full, u):
    """The same product as apply_dft with numpy's FFT (a library transform)
    in place of the explicit DFT matrices; for long sequences of
    applications (many time steps) where the matrix form is too slow."""
    P = lam_full.shape
    n = u.shape
    x = np.zeros(P)
    x[tuple(slice(0, v) for v in n)] = u
    y = np.fft.ifftn(np.fft.fftn(x) * lam_full)
    return y[tuple(slice(0, v) for v in n)].real


class Operator:
    """Bundle of the oracle's M for one (d, alpha, h, n): weights, symbol, apply."""

    def __init__(self, d, alpha, h, n, c=20.0, masked=None):
        self.d, self.alpha, self.h, self.n, self.c = d, alpha, h, tuple(n), c
        self.C = K.c_alpha(alpha, d)
        self.B = K.b_const(d, alpha, c)
        self.w = weights_folded(d, alpha, h, self.n, c)
        self.P = tuple(padded_length(v) for v in self.n)
        self._lam = None
        self.mask = masked

    @property
    def lam_full(self):
        if self._lam is None:
            self._lam, _ = symbol_full(self.w, self.P)
        return self._lam

    def apply(self, u, method="auto"):
        u = np.asarray(u, dtype=np.float64)
        if self.mask is not None:
            u = u * self.mask
        N = int(np.prod(self.n))
        if method == "dense" or (method == "auto" and N <= 4096):
            y = apply_dense(self.w, u)
        elif method == "fft":
            y = apply_fft(self.lam_full, u)
        else:
            y = apply_dft(self.lam_full, u)
        if self.mask is not None:
            y = y * self.mask
        return y

    def dense(self):
        M = dense_matrix(self.w)
        if self.mask is not None:
            m = self.mask.reshape(-1).astype(bool)
            return M[np.ix_(m, m)]
        return M


def grid_points(n, lo=-1.0, hi=1.0):
    """Interior points x_j = lo + j h, j = 1..n, h = (hi - lo)/(n + 1) (Sec. 3.1 grid, read as n interior points)."""
    h = (hi - lo) / (n + 1)
    return lo + h * np.arange(1, n + 1), h


def all_lags(n):
    return list(itertools.product(*[range(v) for v in n]))


def apply_line(w, u, lead):
    """(M u)_i for every i on one line of the last axis, the leading indices
    fixed at `lead`, by direct summation over all j (the definition,
    reordered): with m the lag along the last axis,

        A[m, j_last] = sum_{j_lead} w[|lead - j_lead|, m] u[j_lead, j_last],
        (M u)_{lead, i} = sum_{j_last} A[|i - j_last|, j_last].

    The inner sum over the leading axes is one matrix product."""
    n = u.shape
    d = len(n)
    lead = tuple(int(v) for v in lead)
    if len(lead) != d - 1:
        raise ValueError("lead must fix every axis but the last")
    lags = np.meshgrid(*[np.abs(np.arange(n[a]) - lead[a]) for a in range(d - 1)], indexing="ij")
    G = w[tuple(lags)] if d > 1 else w[None, :]          # [n_0..n_{d-2}, n_last] (lag m last)
    G2 = G.reshape(-1, n[-1])
    U2 = np.asarray(u, dtype=np.float64).reshape(-1, n[-1])
    A = G2.T @ U2                                        # [m, j_last]
    i = np.arange(n[-1])
    return A[np.abs(i[:, None] - i[None, :]), i[None, :]].sum(axis=1)
