"""Pins of the oracle's scalar constants against closed forms and quadrature."""
import math

import mpmath
import numpy as np
import pytest
from scipy import integrate, special

from oracle import constants as K

ALPHAS = [0.2, 0.75, 1.0, 1.5, 1.9]


def _dirichlet_beta(x):
    # beta(x) = 4^{-x} [zeta(x, 1/4) - zeta(x, 3/4)]  (Hurwitz zeta)
    return float(mpmath.power(4, -x) * (mpmath.zeta(x, 0.25) - mpmath.zeta(x, 0.75)))


@pytest.mark.parametrize("alpha", ALPHAS)
def test_lattice_zeta_1d_is_riemann(alpha):
    # sum_{j != 0} |j|^{-(1+alpha)} = 2 zeta(1 + alpha)
    assert K.lattice_zeta(1, alpha) == pytest.approx(2.0 * float(mpmath.zeta(1 + alpha)), rel=1e-13)


@pytest.mark.parametrize("alpha", ALPHAS)
def test_lattice_zeta_2d_is_zeta_times_beta(alpha):
    # Square-lattice sum: sum |j|^{-2x} = 4 zeta(x) beta(x), x = 1 + alpha/2
    x = 1.0 + alpha / 2.0
    ref = 4.0 * float(mpmath.zeta(x)) * _dirichlet_beta(x)
    assert K.lattice_zeta(2, alpha) == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("alpha", [0.3, 1.2, 1.8])
def test_lattice_zeta_split_independent(d, alpha):
    z = [K.lattice_zeta(d, alpha, lam=lam) for lam in (0.6, 1.0, 1.7)]
    assert max(z) - min(z) <= 1e-13 * z[1]


@pytest.mark.parametrize("alpha", [0.8, 1.2, 1.8])
def test_lattice_zeta_3d_brute_force(alpha):
    # brute force over |j| <= R plus the continuum tail |S^2| R^{-alpha} / alpha
    R = 40
    ax = np.arange(-R, R + 1, dtype=np.float64)
    g = np.meshgrid(ax, ax, ax, indexing="ij")
    r2 = g[0] ** 2 + g[1] ** 2 + g[2] ** 2
    m = (r2 > 0) & (r2 <= R * R)
    brute = np.sum(r2[m] ** (-(3 + alpha) / 2))
    # tail with the lattice-point-count correction of the sphere of radius R + 1/2
    tail = 4 * math.pi * (R + 0.5) ** (-alpha) / alpha
    assert K.lattice_zeta(3, alpha) == pytest.approx(brute + tail, rel=2e-3)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("alpha", ALPHAS)
def test_c_alpha_from_gaussian_at_origin(d, alpha):
    # (-Delta)^{alpha/2} e^{-|x|^2} at x = 0 equals 2^alpha Gamma((d+alpha)/2)/Gamma(d/2) (1F1 at 0 is 1).
    # Through eq. (fl) it equals C |S^{d-1}| int_0^inf (1 - e^{-r^2}) r^{-1-alpha} dr.
    f = lambda r: (-math.expm1(-r * r)) * r ** (-1.0 - alpha)
    I = integrate.quad(f, 0, 1, limit=200)[0] + integrate.quad(f, 1, np.inf, limit=200)[0]
    lhs = K.c_alpha(alpha, d) * K.sphere_area(d) * I
    rhs = 2**alpha * math.gamma((d + alpha) / 2) / math.gamma(d / 2)
    assert lhs == pytest.approx(rhs, rel=1e-8)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("alpha", ALPHAS)
def test_a3_closed_form_against_quadrature(d, alpha):
    # h^{s-2} A_3 = -(1/2)(|S^{d-1}|/d) int_0^c r^{1-alpha} W(r/c) dr   (eq. a3 in polar form)
    c = 20.0
    I = integrate.quad(lambda r: r ** (1 - alpha) * float(K.window(r / c)), 0, c, limit=200)[0]
    assert K.a3_scaled(d, alpha, c) == pytest.approx(-0.5 * K.sphere_area(d) / d * I, rel=1e-10)


def test_a3_1d_matches_1d_definition():
    # Sec. 2.3: A_3 = -(1/2h) int w(y) |y|^{1-alpha} dy  (both half-lines) with delta = c h
    alpha, c = 1.3, 20.0
    I = 2 * integrate.quad(lambda y: float(K.window(y / c)) * y ** (1 - alpha), 0, c, limit=200)[0]
    assert K.a3_scaled(1, alpha, c) == pytest.approx(-0.5 * I, rel=1e-10)


@pytest.mark.parametrize("d", [2, 3])
def test_a2_e1_form_equals_isotropic_form(d):
    # cubic symmetry: sum W j_1^2 |j|^{-s} = (1/d) sum W |j|^{2-s}
    alpha, c = 1.1, 20.0
    R = int(c)
    ax = np.arange(-R, R + 1, dtype=np.float64)
    g = np.meshgrid(*([ax] * d), indexing="ij")
    r = np.sqrt(sum(v * v for v in g))
    m = (r > 0) & (r < c)
    iso = np.sum(K.window(r[m] / c) * r[m] ** (2 - d - alpha)) / d
    assert K.a2_sum(d, alpha, c) == pytest.approx(iso, rel=1e-12)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("alpha", ALPHAS)
def test_b_negative_and_near_mellin_limit(d, alpha):
    # B < 0 (Sec. 3.1: A_2 + A_3 < 0).  For a smooth window B -> Z_d(d+alpha-2)/(2d)
    # (analytically continued Epstein zeta) with an O(c^{-4}) gap.
    B = K.b_const(d, alpha)
    assert B < 0
    s = alpha - 1.0 + (d - 1.0)  # d + alpha - 2
    if d == 1:
        z = 2.0 * float(mpmath.zeta(s))
    elif d == 2:
        x = s / 2.0
        z = 4.0 * float(mpmath.zeta(x)) * float(
            mpmath.power(4, -x) * (mpmath.zeta(x, 0.25) - mpmath.zeta(x, 0.75)))
    else:
        # no closed form in 3D: the theta-function split continues the lattice
        # sum below s = d (exponent alpha - 2 < 0); its value must not depend
        # on the split parameter
        z = K.lattice_zeta(3, alpha - 2.0, lam=1.0)
        assert K.lattice_zeta(3, alpha - 2.0, lam=0.6) == pytest.approx(z, rel=1e-11)
    assert B == pytest.approx(z / (2 * d), rel=5e-5, abs=5e-6)


def test_window_pins():
    # W(0) = 1 and W, W', W'', W''' vanish at t = 1 (window is C^3 across the cut)
    t = 1.0
    W = K.window
    assert float(W(0.0)) == 1.0
    p = np.polynomial.Polynomial([1, 0, 0, 0, -35, 84, -70, 20])
    for k in range(4):
        assert abs(p.deriv(k)(t) if k else p(t)) < 1e-12
    assert float(W(1.0)) == 0.0
    # moment closed form
    I = integrate.quad(lambda x: x ** (1 - 0.7) * p(x), 0, 1)[0]
    assert K.window_moment(0.7) == pytest.approx(I, rel=1e-12)
