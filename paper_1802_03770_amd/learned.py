"""Training of the learned preconditioner on solver-generated pairs (host
orchestration of the C entry points; every arithmetic step runs in the HIP
library).

Pairs: for each problem of the plan (alpha, right-hand side f):
  * the errors x* - x_k of the first `iters` iterates x_k of the spectral PCG
    solve (x* the same solve to 1e-12),
  * `fields` random errors e (power-law Gaussian fields),
each turned by fl_learned_pairs into R = r/s, T = (D e - r)/s with r = M e.
"""
import numpy as np
import torch

from . import (FL_PC_SPECTRAL, Net, Op, learned_pairs, solve_opts)


def init_params(seed=0, d=2):
    """He-uniform weights, zero biases, output layer scaled by 0.1 (seeded host draw);
    3^d taps per kernel."""
    rng = np.random.Generator(np.random.PCG64(seed))
    layers = [("cin", 2, 32)] + [(k, 32, 32) for k in ("d1", "d2", "d3", "b3", "u2", "u1", "u0")] + [("out", 32, 1)]
    K = 3 ** d
    parts = []
    for name, ci, co in layers:
        lim = np.sqrt(6.0 / (K * ci))
        w = rng.uniform(-lim, lim, size=(K, ci, co))
        if name == "out":
            w *= 0.1
        parts += [w.ravel(), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


def make_pairs(plan, iters=10, fields=10, stream=None, log=None):
    """Training set (R, T, A) on the device from a list of problems
    ({"n", "alpha", "rhs_seed", "field_seed"}, "d" 2 or 3), all on one n^d grid."""
    from workloads import bump_field, power_law_field
    stream = stream or torch.cuda.Stream()
    Rs, Ts, As = [], [], []
    for i, pr in enumerate(plan):
        n, alpha, d = pr["n"], pr["alpha"], pr.get("d", 2)
        f_np, h = bump_field(n, d, 32 if d == 2 else 16, pr["rhs_seed"], width=(0.05, 0.2))
        op = Op(d, alpha, h, (n,) * d, stream=stream)
        f = torch.from_numpy(f_np).cuda()
        xs, info = op.solve(f, tol=1e-12, opts=solve_opts(pc=FL_PC_SPECTRAL))
        # iterates strictly before the converged one (x_k of the same solve with
        # maxit = k equals x* bitwise once k reaches its iteration count)
        nit = min(iters, max(1, info["iters"] - 1))
        xk = []
        for k in range(nit):
            u, _ = op.solve(f, tol=1e-30, opts=solve_opts(pc=FL_PC_SPECTRAL, maxit=k + 1), check=False)
            xk.append(u)
        xk = torch.stack([torch.zeros_like(xs)] + xk[:-1]) if iters > 0 else None
        if xk is not None:
            R, T = learned_pairs(op, xs, e_sub=xk)
            Rs.append(R)
            Ts.append(T)
            As += [alpha] * nit
        if fields > 0:
            e = np.stack([power_law_field((n,) * d, pr["field_seed"] + j) for j in range(fields)])
            R, T = learned_pairs(op, torch.from_numpy(e).cuda())
            Rs.append(R)
            Ts.append(T)
        As += [alpha] * fields
        op.close()
        if log and (i + 1) % 10 == 0:
            log(f"[learned] pairs from {i + 1}/{len(plan)} problems")
    torch.cuda.synchronize()
    return torch.cat(Rs), torch.cat(Ts), torch.tensor(As, dtype=torch.float32, device="cuda")


def train(R, T, A, steps=2000, batch=16, lr=1e-3, seed=0, params=None, stream=None, lr_decay_at=0.7):
    """Train a Net on the pairs (minibatch indices drawn on the host from a
    seeded generator); lr drops 10x after `lr_decay_at` of the steps.  The
    network's dimension follows the pairs: R [npairs, H, W] or [npairs, D, H, W]."""
    d = R.dim() - 1
    net = Net(stream=stream, params=init_params(seed, d) if params is None else params, d=d)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    idx = rng.integers(0, R.shape[0], size=(steps, batch))
    k1 = int(steps * lr_decay_at)
    losses = net.train(R, T, A, idx[:k1], batch, lr)
    if steps > k1:
        losses += net.train(R, T, A, idx[k1:], batch, lr * 0.1)
    return net, losses
