"""Grid-refinement studies of the paper (host orchestration of the C entry
points; every application, solve and time step runs in the HIP library).

Sec. 4.2-4.3, eq. (rich): with three nested grids of [0,1]^d (coarse n_c,
medium 2 n_c + 1, fine 4 n_c + 3 interior points per axis, so that coarse
point i is medium point 2 i and fine point 4 i), the grid-error rate estimate
of a discrete quantity v sampled on the common coarse grid is

    R_p = (log ||v_f - v_m||_p - log ||v_m - v_c||_p) / log(1/2).

`elliptic_rates` estimates it for the application error (v = M g_1 with the
smooth bump g_1(x) = prod_i (1 + cos(2 pi x_i - pi))^2 / 4) and for the
solution error (v = M^{-1} g_2, g_2 = 1).  `parabolic_rates` does the same for
the solution at T = 0.25 of the time-dependent problem of Sec. 4.5:
Crank-Nicolson steps (eq. timestepping) with dt = 1/(n + 1) (so that T / dt
is an integer), f = 0 and u_0(x) = prod_i (1 + cos(2 pi nu_i x_i - pi))^2 / 4,
nu = (3, 11, 2).  `single_step_iterations` counts the CG iterations of one
such step with a random right-hand side, with and without the preconditioner
(the paper's single-step table).  `smooth_errors` is the smooth 2D example of
Sec. 4.2: f = M g_1 on a fine grid (4095^2, padded to 8192 points per axis),
subsampled to coarser grids, solved there and compared with g_1.
"""
import math

import numpy as np
import torch

from . import FL_PC_AUTO, FL_PC_FD, FL_PC_NONE, Op, solve_opts


def unit_grid(n):
    """Interior points x_j = j / (n + 1), j = 1..n, of [0, 1] and h."""
    h = 1.0 / (n + 1)
    return h * np.arange(1, n + 1), h


def bump(n, d, nu=None):
    """prod_i (1 + cos(2 pi nu_i x_i - pi))^2 / 4 on the n^d grid of [0,1]^d (nu_i = 1 by default)."""
    x, _ = unit_grid(n)
    nu = nu or (1,) * d
    out = np.ones((1,) * d)
    for a in range(d):
        g = 0.25 * (1.0 + np.cos(2.0 * math.pi * nu[a] * x - math.pi)) ** 2
        sh = [1] * d
        sh[a] = n
        out = out * g.reshape(sh)
    return np.ascontiguousarray(np.broadcast_to(out, (n,) * d))


def coarse_view(v, level):
    """Values of a grid of 2^level (n_c + 1) - 1 points per axis at the coarse points."""
    step = 2 ** level
    return v[tuple(slice(step - 1, None, step) for _ in range(v.ndim))]


def rate(vc, vm, vf, p):
    """R_p of eq. (rich) from the three values on the coarse grid."""
    def norm(x):
        x = np.asarray(x).ravel()
        return float(np.max(np.abs(x))) if p == np.inf else float(np.linalg.norm(x, p))
    return (math.log(norm(vf - vm)) - math.log(norm(vm - vc))) / math.log(0.5)


def nested(n_coarse):
    """The coarse, medium and fine grid sizes."""
    return n_coarse, 2 * n_coarse + 1, 4 * n_coarse + 3


def elliptic_rates(d, alpha, n_coarse, tol=1e-12, stream=None, mixed=0):
    """R_2 and R_inf of the application (g_1) and the solution (g_2 = 1)."""
    fs, us, info = [], [], []
    for level, n in enumerate(nested(n_coarse)):
        op = Op(d, alpha, 1.0 / (n + 1), (n,) * d, stream=stream)
        g1 = torch.from_numpy(bump(n, d)).cuda()
        fs.append(coarse_view(op.apply(g1).cpu().numpy(), level))
        one = torch.ones((n,) * d, dtype=torch.float64, device="cuda")
        u, inf = op.solve(one, tol=tol, opts=solve_opts(pc=FL_PC_FD, mixed=mixed))
        us.append(coarse_view(u.cpu().numpy(), level))
        info.append({"n": n, "iters": inf["iters"], "rel_res_true": inf["rel_res_true"]})
        op.close()
    out = {f"{q}_R{p}": rate(*vals, np.inf if p == "inf" else 2)
           for q, vals in (("u", us), ("f", fs)) for p in ("2", "inf")}
    out["solves"] = info
    return out


def parabolic_final(d, alpha, n, nu=(3, 11, 2), T=0.25, tol=1e-12, stream=None):
    """u at time T of the Crank-Nicolson schedule on the n^d grid (dt = 1/(n+1))."""
    op = Op(d, alpha, 1.0 / (n + 1), (n,) * d, stream=stream)
    dt = 1.0 / (n + 1)
    steps = int(round(T / dt))
    u = torch.from_numpy(bump(n, d, nu[:d])).cuda()
    iters = 0
    for _ in range(steps):
        u, inf = op.step(u, dt, 0.5, tol=tol, opts=solve_opts(pc=FL_PC_FD))
        iters += inf["iters"]
    out = u.cpu().numpy()
    op.close()
    return out, steps, iters


def parabolic_rates(d, alpha, n_coarse, tol=1e-12, stream=None):
    """R_2 and R_inf of the solution at T = 0.25 under simultaneous refinement in space and time."""
    vals, info = [], []
    for level, n in enumerate(nested(n_coarse)):
        u, steps, iters = parabolic_final(d, alpha, n, tol=tol, stream=stream)
        vals.append(coarse_view(u, level))
        info.append({"n": n, "steps": steps, "iters": iters})
    return {"R2": rate(*vals, 2), "Rinf": rate(*vals, np.inf), "runs": info}


def single_step_iterations(d, alpha, n, seed=0, tol=1e-9, stream=None):
    """CG iterations of one Crank-Nicolson system (I + dt/2 M) x = b, dt = 1/(n+1),
    b ~ N(0, 1) (seeded), x_0 = 0, with the preconditioner I + dt/2 C h^d L and without."""
    op = Op(d, alpha, 1.0 / (n + 1), (n,) * d, stream=stream)
    dt = 1.0 / (n + 1)
    b = np.random.Generator(np.random.PCG64(seed)).standard_normal((n,) * d)
    # from u^k = 0 the step's right-hand side is dt theta f^{k+1}: f^{k+1} = b / (dt / 2)
    fk1 = torch.from_numpy(b / (0.5 * dt)).cuda()
    out = {}
    for name, pc in (("pcg", FL_PC_FD), ("cg", FL_PC_NONE)):
        u = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
        _, inf = op.step(u, dt, 0.5, f_k1=fk1, tol=tol, opts=solve_opts(pc=pc, maxit=1000))
        out[name] = inf["iters"]
    op.close()
    return out


def subsample(v, n_fine, n):
    """Values of a fine-grid function (n_fine points per axis) at the points of
    the n-point grid; (n + 1) must divide (n_fine + 1)."""
    step, rem = divmod(n_fine + 1, n + 1)
    if rem:
        raise ValueError("n + 1 must divide n_fine + 1")
    sl = slice(step - 1, None, step)
    return np.ascontiguousarray(v[tuple(sl for _ in range(v.ndim))])


def smooth_errors(alpha, ns=(127, 255, 511, 1023), n_fine=4095, tol=1e-13, stream=None):
    """Sec. 4.2, the smooth 2D example: u_true = g_1 on the n_fine^2 grid of
    [0, 1]^2, f = M^(n_fine) u_true (one FP64 application); for each n, the
    subsampled f is solved on the n^2 grid (FP64 PCG, the preconditioner chosen
    by alpha) and e = ||u_true - u|| / ||u_true|| on that grid.  Also the growth
    rate gamma of e ~ n^gamma, the least-squares slope of log e against log n."""
    opf = Op(2, alpha, 1.0 / (n_fine + 1), (n_fine, n_fine), stream=stream)
    uf = bump(n_fine, 2)
    ff = opf.apply(torch.from_numpy(uf.copy()).cuda()).cpu().numpy()
    opf.close()
    errs, solves = [], []
    for n in ns:
        f = subsample(ff, n_fine, n)
        ut = subsample(uf, n_fine, n)
        op = Op(2, alpha, 1.0 / (n + 1), (n, n), stream=stream)
        u, inf = op.solve(torch.from_numpy(f).cuda(), tol=tol, opts=solve_opts(pc=FL_PC_AUTO, maxit=20000))
        op.close()
        errs.append(float(np.linalg.norm(u.cpu().numpy() - ut) / np.linalg.norm(ut)))
        solves.append({"n": n, "iters": inf["iters"], "rel_res_true": inf["rel_res_true"]})
    gamma = float(np.polyfit(np.log(np.asarray(ns, dtype=float)), np.log(errs), 1)[0])
    return {"errors": errs, "rate": gamma, "solves": solves}
