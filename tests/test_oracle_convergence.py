"""Observed convergence of the oracle's discretisation against the paper's
grid-refinement tables (Sec. 4.2, 4.5): the Richardson rate estimate of
eq. (rich) on nested grids of [0,1]^2, and single-step iteration counts.

Readings: the 2D apply rates of the paper (Table 2drich, f columns) lie 0.09
to 0.13 below the rate 4 - alpha that the quadrature's symbol error gives for
the smooth g_1 (the paper evaluates the lattice sum A_1 by Chebyshev
far-field compression, this build exactly); the solution rates, limited by
the boundary behaviour of u, match the printed two digits.  The single-step
table's right-hand side is "random": i.i.d. N(0,1), seed 0; PCG counts match,
plain-CG counts depend on the draw (about 15% above the printed ones).
"""
import math
import os

import numpy as np
import pytest

from oracle import krylov as KR
from oracle import operator as O
from oracle import precond as PC

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _g1(n, d):
    x = np.arange(1, n + 1) / (n + 1)
    g = 0.25 * (1.0 + np.cos(2.0 * math.pi * x - math.pi)) ** 2
    out = g
    for _ in range(d - 1):
        out = np.multiply.outer(out, g)
    return out


def _coarse(v, level):
    s = 2 ** level
    return v[tuple(slice(s - 1, None, s) for _ in range(v.ndim))]


def _rate(c, m, f, p):
    nrm = (lambda x: np.abs(x).max()) if p == np.inf else (lambda x: np.linalg.norm(x.ravel()))
    return (math.log(nrm(f - m)) - math.log(nrm(m - c))) / math.log(0.5)


@pytest.mark.slow
def test_2d_richardson_rates_alpha_1_5():
    alpha = 1.5
    row = [r for r in np.loadtxt(os.path.join(GOLDEN, "tab_2drich.txt"), comments="#") if r[0] == alpha][0]
    fs, us = [], []
    for level, n in enumerate((255, 511, 1023)):
        h = 1.0 / (n + 1)
        op = O.Operator(2, alpha, h, (n, n))
        fs.append(_coarse(op.apply(_g1(n, 2), method="fft"), level))
        sc = PC.pc_scale(2, alpha, h)
        x, _, _, _ = KR.pcg(lambda v: op.apply(v, method="fft"), np.ones((n, n)),
                            lambda r: PC.apply_inverse(r, sc), tol=1e-12)
        us.append(_coarse(x, level))
    uR2, uRi = _rate(*us, 2), _rate(*us, np.inf)
    fR2, fRi = _rate(*fs, 2), _rate(*fs, np.inf)
    print("u", uR2, uRi, "f", fR2, fRi, "printed", row[1:])
    assert abs(uR2 - row[1]) <= 0.015 and abs(uRi - row[2]) <= 0.015
    assert abs(fR2 - (4 - alpha)) <= 0.05 and abs(fRi - (4 - alpha)) <= 0.05
    assert abs(fR2 - row[3]) <= 0.15 and abs(fRi - row[4]) <= 0.2


@pytest.mark.parametrize("alpha", [1.25, 1.5, 1.75])
def test_single_step_iterations_255(alpha):
    d, n = 2, 255
    rows = np.loadtxt(os.path.join(GOLDEN, "tab_td_its.txt"), comments="#")
    _, _, _, p_pcg, p_cg = [r for r in rows if r[0] == d and r[1] == n and r[2] == alpha][0]
    h = dt = 1.0 / (n + 1)
    op = O.Operator(d, alpha, h, (n, n))
    b = np.random.Generator(np.random.PCG64(0)).standard_normal((n, n))
    sc = PC.pc_scale(d, alpha, h)
    A = lambda v: v + 0.5 * dt * op.apply(v, method="fft")  # noqa: E731
    it_p = KR.pcg(A, b, lambda r: PC.apply_inverse(r, sc, 1.0, 0.5 * dt), tol=1e-9)[1]
    it_c = KR.pcg(A, b, None, tol=1e-9)[1]
    print(alpha, it_p, it_c, "printed", p_pcg, p_cg)
    assert abs(it_p - p_pcg) <= 1
    assert abs(it_c - p_cg) <= 0.25 * p_cg
