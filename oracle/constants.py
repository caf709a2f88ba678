"""Scalar constants of the discretisation (FP64 oracle; test infrastructure only).

Paper: Minden & Ying, Sec. 2 ("Spatial discretization of the fractional
Laplacian").  Dimensionless form used throughout: with y_j = h j and
delta = c h (window radius c grid points, Sec. 4.1 uses c = 20),

    A_1 = h^{-s} Z,        Z   = sum_{j != 0} |j|^{-s},            s = d + alpha
    A_2 = h^{2-s} a2 / 2,  a2  = sum_{0<|j|<c} W(|j|/c) j_1^2 |j|^{-s}
    A_3 = -h^{2-s} (|S^{d-1}|/d) c^{2-alpha} Pw(alpha) / 2
    B   = h^{s-2} (A_2 + A_3)                  (dimensionless, must be < 0)

A_1 and A_2 follow eq. (int1constants); A_3 is eq. (a3) evaluated in closed
form for the polynomial window of eq. (window) (integral of (e_1.y)^2 g(|y|)
equals (1/d) of the integral of |y|^2 g(|y|); the radial moment of W is the
polynomial Pw below).

The normalising constant C_{alpha,d} is only called "known" in Sec. 1
(eq. fl).  Reading: the standard constant whose Fourier symbol is |xi|^alpha.
"""
import math

import numpy as np
from scipy import special


def c_alpha(alpha, d):
    """Normalising constant of eq. (fl): symbol of (-Delta)^{alpha/2} is |xi|^alpha.

    C = alpha 2^{alpha-1} Gamma((d+alpha)/2) / (pi^{d/2} Gamma(1 - alpha/2)).
    """
    return (alpha * 2.0 ** (alpha - 1.0) * math.gamma((d + alpha) / 2.0)
            / (math.pi ** (d / 2.0) * math.gamma(1.0 - alpha / 2.0)))


def sphere_area(d):
    """|S^{d-1}| = 2 pi^{d/2} / Gamma(d/2)  (2 for d=1, 2 pi for d=2, 4 pi for d=3)."""
    return 2.0 * math.pi ** (d / 2.0) / math.gamma(d / 2.0)


def window(t):
    """Window of eq. (window) as a function of t = r/delta: 1-35t^4+84t^5-70t^6+20t^7 on t<1, else 0."""
    t = np.asarray(t, dtype=np.float64)
    p = 1.0 - 35.0 * t**4 + 84.0 * t**5 - 70.0 * t**6 + 20.0 * t**7
    return np.where(t < 1.0, p, 0.0)


def window_moment(alpha):
    """Pw(alpha) = integral_0^1 t^{1-alpha} W(t) dt, exact for the polynomial window."""
    return (1.0 / (2.0 - alpha) - 35.0 / (6.0 - alpha) + 84.0 / (7.0 - alpha)
            - 70.0 / (8.0 - alpha) + 20.0 / (9.0 - alpha))


def _upper_gamma(a, x):
    """Non-regularised upper incomplete gamma Gamma(a, x) for a > -1, x > 0."""
    x = np.asarray(x, dtype=np.float64)
    if a > 0:
        return special.gammaincc(a, x) * special.gamma(a)
    # Gamma(a, x) = (Gamma(a+1, x) - x^a e^{-x}) / a   for a in (-1, 0)
    return (special.gammaincc(a + 1.0, x) * special.gamma(a + 1.0)
            - x**a * np.exp(-x)) / a


def _lattice(d, R):
    """All j in [-R, R]^d except 0, as an (m, d) integer array."""
    ax = np.arange(-R, R + 1)
    g = np.stack(np.meshgrid(*([ax] * d), indexing="ij"), axis=-1).reshape(-1, d)
    return g[np.any(g != 0, axis=1)]


def lattice_zeta(d, alpha, lam=1.0, R=6):
    """Z = sum_{j in Z^d, j != 0} |j|^{-(d+alpha)}  (the A_1 lattice sum of eq. int1constants).

    The paper evaluates A_1 with Chebyshev far-field compression (Sec. 2.7);
    here the same number is computed by the theta-function (Ewald) split of the
    Mellin integral, with split parameter lam (the result must not depend on it):

      pi^{-sig} Gamma(sig) Z = sum_{j!=0} [ (pi|j|^2)^{-sig} Gamma(sig, pi lam |j|^2)
                                          + (pi|j|^2)^{alpha/2} Gamma(-alpha/2, pi|j|^2/lam) ]
                               + (2/alpha) lam^{alpha/2} - lam^{sig}/sig,      sig = (d+alpha)/2.
    """
    sig = 0.5 * (d + alpha)
    j = _lattice(d, R).astype(np.float64)
    q = math.pi * np.sum(j * j, axis=1)          # pi |j|^2
    t1 = q ** (-sig) * _upper_gamma(sig, lam * q)
    t2 = q ** (0.5 * alpha) * _upper_gamma(-0.5 * alpha, q / lam)
    # sum small-to-large for a clean FP64 result
    terms = np.sort(np.concatenate([t1, t2]))
    total = math.fsum(terms) + (2.0 / alpha) * lam ** (0.5 * alpha) - lam**sig / sig
    return total * math.pi**sig / math.gamma(sig)


def a2_sum(d, alpha, c=20.0):
    """a2 = sum_{0<|j|<c} W(|j|/c) j_1^2 |j|^{-(d+alpha)}  (h^{s-2} * 2 A_2, eq. int1constants)."""
    R = int(math.ceil(c))
    j = _lattice(d, R).astype(np.float64)
    r = np.sqrt(np.sum(j * j, axis=1))
    inside = r < c
    j, r = j[inside], r[inside]
    terms = window(r / c) * j[:, 0] ** 2 * r ** (-(d + alpha))
    return math.fsum(np.sort(terms))


def a3_scaled(d, alpha, c=20.0):
    """h^{s-2} A_3 = -(1/2) (|S^{d-1}|/d) c^{2-alpha} Pw(alpha)   (eq. a3, closed form)."""
    return -0.5 * sphere_area(d) / d * c ** (2.0 - alpha) * window_moment(alpha)


def b_const(d, alpha, c=20.0):
    """B = h^{s-2}(A_2 + A_3): coefficient of the finite-difference Laplacian (dimensionless)."""
    return 0.5 * a2_sum(d, alpha, c) + a3_scaled(d, alpha, c)


def all_constants(d, alpha, c=20.0):
    """Dictionary with C, Z, a2, B and the dimensionless stencil values omega_0, omega_e."""
    C = c_alpha(alpha, d)
    Z = lattice_zeta(d, alpha)
    B = b_const(d, alpha, c)
    return {"C": C, "Z": Z, "a2": a2_sum(d, alpha, c), "B": B,
            "omega0": Z - 2.0 * d * B, "omega_e": -1.0 + B}
