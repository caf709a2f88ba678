"""Krylov solvers and time stepping (FP64 oracle; test infrastructure only).

pcg     Conjugate gradients (Hestenes-Stiefel), optionally preconditioned,
        with the relative l2 residual stopping test of Sec. 4.1
        (||r_k|| / ||f|| <= eps_res).  The paper gives no further detail; the
        reading is x_0 = 0 (or a given warm start), the recurrence residual in
        the test, and the iteration count = number of operator applications
        inside the loop.
fcg     Flexible CG (truncated FCG(1), Notay 2000) for a preconditioner that
        may change between iterations (the learned one); not in the paper.
theta_rhs / theta_step
        The implicit scheme of Sec. 3.2, eq. (timestepping), generalised to
        theta in (0, 1]: theta = 1/2 is the paper's Crank-Nicolson,
        theta = 1 backward Euler.  The system (I + theta dt M) u^{k+1} = b is
        solved with PCG and preconditioner I + theta dt C h^d L, warm-started
        from u^k (Sec. 4.4).
"""
import math

import numpy as np


def _dot(a, b):
    return float(np.dot(a.ravel(), b.ravel()))


def pcg(apply, f, precond=None, tol=1e-10, maxit=1000, x0=None):
    """Solve M x = f.  Returns (x, iterations, recurrence relative residual, history)."""
    f = np.asarray(f, dtype=np.float64)
    nf = math.sqrt(_dot(f, f))
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    r = f - apply(x) if x0 is not None else f.copy()
    hist = [math.sqrt(_dot(r, r)) / nf]
    if hist[-1] <= tol:
        return x, 0, hist[-1], hist
    z = precond(r) if precond else r
    p = z.copy()
    rz = _dot(r, z)
    it = 0
    while it < maxit:
        q = apply(p)
        pq = _dot(p, q)
        a = rz / pq
        x = x + a * p
        r = r - a * q
        it += 1
        hist.append(math.sqrt(_dot(r, r)) / nf)
        if hist[-1] <= tol:
            break
        z = precond(r) if precond else r
        rz_new = _dot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, hist[-1], hist


def fcg(apply, f, precond, tol=1e-10, maxit=1000, x0=None):
    """Truncated flexible CG, FCG(1): beta_k = -z_{k+1}.q_k / p_k.q_k, alpha_k = p_k.r_k / p_k.q_k."""
    f = np.asarray(f, dtype=np.float64)
    nf = math.sqrt(_dot(f, f))
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    r = f - apply(x) if x0 is not None else f.copy()
    hist = [math.sqrt(_dot(r, r)) / nf]
    if hist[-1] <= tol:
        return x, 0, hist[-1], hist
    z = precond(r)
    p = z.copy()
    it = 0
    while it < maxit:
        q = apply(p)
        pq = _dot(p, q)
        a = _dot(p, r) / pq
        x = x + a * p
        r = r - a * q
        it += 1
        hist.append(math.sqrt(_dot(r, r)) / nf)
        if hist[-1] <= tol:
            break
        z = precond(r)
        beta = -_dot(z, q) / pq
        p = z + beta * p
    return x, it, hist[-1], hist


def theta_rhs(apply, u, dt, theta, f_k=None, f_k1=None):
    """b = (I - (1-theta) dt M) u^k + dt (theta f^{k+1} + (1-theta) f^k)."""
    b = np.array(u, dtype=np.float64)
    if theta < 1.0:
        b = b - (1.0 - theta) * dt * apply(u)
    if f_k1 is not None:
        b = b + dt * theta * f_k1
    if f_k is not None and theta < 1.0:
        b = b + dt * (1.0 - theta) * f_k
    return b


def theta_step(apply, precond_inv, u, dt, theta, tol=1e-12, maxit=1000, f_k=None, f_k1=None):
    """One step of eq. (timestepping) with PCG; returns (u^{k+1}, iterations)."""
    b = theta_rhs(apply, u, dt, theta, f_k, f_k1)

    def sysop(v):
        return v + theta * dt * apply(v)

    x, it, _, _ = pcg(sysop, b, precond_inv, tol=tol, maxit=maxit, x0=u)
    return x, it


def exact_propagator(Mdense, dt, theta, steps, u0):
    """u^K = V g(Lambda)^K V^T u^0 with g = (1 - (1-theta) dt lam)/(1 + theta dt lam), via eigh."""
    lam, V = np.linalg.eigh(Mdense)
    g = (1.0 - (1.0 - theta) * dt * lam) / (1.0 + theta * dt * lam)
    return V @ (g**steps * (V.T @ u0.ravel()))
