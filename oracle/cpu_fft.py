"""The paper's solver as it runs on a CPU, with a library FFT (a CPU baseline
for timing; test infrastructure only, like the rest of this package).

Sec. 3.1: M is applied as a zero-padded FFT convolution with the symbol of
its circulant embedding, and the FD-Laplacian preconditioner
(C h^d L)^{-1} = (C |B| h^{-alpha} T)^{-1} is applied with type-I sine
transforms (a fast Poisson solver); the solve is PCG with the relative
residual test of Sec. 4.  This is the same method the paper times in MATLAB,
here with scipy.fft (FP64, `workers` threads) for every transform; it is a
baseline to time beside the GPU, not a reference for parity (the explicit-DFT
oracle in operator.py and precond.py is that).
"""
import math

import numpy as np
import scipy.fft as sfft

from . import constants as K
from . import krylov as KR
from . import operator as O


class FFTSolver:
    """M, its FD preconditioner and PCG for one (d, alpha, h, n) on the box."""

    def __init__(self, d, alpha, h, n, c=20.0, workers=None):
        self.d, self.alpha, self.h, self.n = d, alpha, h, tuple(int(v) for v in n)
        self.workers = workers
        w = O.weights_folded(d, alpha, h, self.n, c)
        self.P = tuple(O.padded_length(v) for v in self.n)
        # symbol: DFT of the even circulant embedding (real); rfftn keeps the half spectrum
        full = O.circulant_folded(w, self.P)
        for a, p in enumerate(self.P):
            idx = np.array([min(k, p - k) for k in range(p)])
            full = np.take(full, idx, axis=a)
        self.lam = sfft.rfftn(full, workers=workers).real
        self.scale = K.c_alpha(alpha, d) * abs(K.b_const(d, alpha, c)) * h ** (-alpha)
        ev = 0.0
        for a, v in enumerate(self.n):
            e = 4.0 * np.sin(math.pi * np.arange(1, v + 1) / (2.0 * (v + 1))) ** 2
            sh = [1] * d
            sh[a] = v
            ev = ev + e.reshape(sh)
        self.ev = ev

    def apply(self, u):
        X = sfft.rfftn(u, s=self.P, workers=self.workers)
        y = sfft.irfftn(X * self.lam, s=self.P, workers=self.workers)
        return y[tuple(slice(0, v) for v in self.n)]

    def precond(self, r, shift0=0.0, shift1=1.0):
        # DST-I per axis; scipy's unnormalised type-I transform is 2 S with
        # S_jk = sin(pi j k / (n + 1)), and S^2 = (n + 1)/2 I
        rh = sfft.dstn(r, type=1, workers=self.workers)
        rh = rh / (shift0 + shift1 * self.scale * self.ev)
        z = sfft.dstn(rh, type=1, workers=self.workers)
        return z / np.prod([2.0 * (v + 1) for v in self.n])

    def solve(self, f, tol=1e-8, maxit=None):
        maxit = maxit or max(1000, int(10 * math.sqrt(np.prod(self.n))))
        return KR.pcg(self.apply, f, self.precond, tol=tol, maxit=maxit)
