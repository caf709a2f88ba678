"""True residuals of full-size solutions recomputed by the FP64 oracle.

The library reports ||f - M u|| / ||f|| of its own solution from its own FP64
application.  These tests recompute that residual with the oracle (explicit
DFT matrices, or direct sums organised along grid lines) for the solver
configurations and workloads the benchmark times:

* 1024^2, alpha = 1 (the metric's workload): FP64 PCG with the FD
  preconditioner and learned + FP32 refinement, full residual by the
  oracle's naive-DFT application;
* 128^3, alpha = 1.5: learned + FP32 refinement, full residual;
* 16 right-hand sides at 256^3: two of them, residual estimated from 4096
  points on 16 random grid lines (exact direct sums at those points), scaled
  by sqrt(N) to an l2 norm;
* the uneven backward-Euler batch: four of its problems (the largest grid
  among them) for every one of 200 steps, each step's residual
  (I + dt M) u^{k+1} - u^k in full by the oracle (numpy's FFT as its
  transform), and the smallest problem's
  whole trajectory against the oracle's own theta steps.

The learned solves use a network trained here on fewer pairs and steps than
the benchmark's (the solution's accuracy comes from the FP64 refinement
loop, whatever the network).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import krylov as KR  # noqa: E402
from oracle import operator as O  # noqa: E402
from oracle import precond as PC  # noqa: E402
from workloads import (bump_field, learned_training_plan, workload_elliptic_1024,  # noqa: E402
                       workload_rhs_256cubed, workload_uneven_steps)


def _fl():
    import paper_1802_03770_amd as fl
    return fl


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def _full_residual(ref, f, u):
    return float(np.linalg.norm(f - ref.apply(u, method="dft")) / np.linalg.norm(f))


@pytest.fixture(scope="module")
def net2d():
    from paper_1802_03770_amd import learned as L
    s = torch.cuda.Stream()
    plan = learned_training_plan(nalpha=16, n=128, seed=5000)
    R, T, A = L.make_pairs(plan, iters=6, fields=6, stream=s)
    net, _ = L.train(R, T, A, steps=400, batch=8, lr=2e-3, seed=1, stream=s)
    return net


def test_1024_fp64_pcg_and_learned_full_residual(net2d):
    _say("1024^2 full residuals")
    fl = _fl()
    w = workload_elliptic_1024(1.0)
    n, alpha, h, f = w["n"], w["alpha"], w["h"], w["f"]
    op = fl.Op(2, alpha, h, (n, n), stream=net2d.stream)
    ref = O.Operator(2, alpha, h, (n, n))
    for name, opts in (("fp64_pcg", fl.solve_opts(pc=fl.FL_PC_FD, mixed=0)),
                       ("learned_f32", fl.solve_opts(pc=fl.FL_PC_LEARNED, mixed=1, net=net2d))):
        u, info = op.solve(_dev(f), tol=1e-8, opts=opts)
        res = _full_residual(ref, f, u.cpu().numpy())
        _say(name, info["iters"], info["rel_res_true"], res)
        assert res <= 1e-8, (name, res)
        # the library's own FP64 residual agrees with the oracle's
        assert abs(info["rel_res_true"] - res) <= 1e-3 * res + 1e-14, (name, info["rel_res_true"], res)


def test_128cubed_learned_full_residual():
    _say("128^3 learned full residual")
    fl = _fl()
    from paper_1802_03770_amd import learned as L
    s = torch.cuda.Stream()
    plan = learned_training_plan(nalpha=8, n=16, seed=5600, d=3)
    R, T, A = L.make_pairs(plan, iters=3, fields=3, stream=s)
    net, _ = L.train(R, T, A, steps=100, batch=4, lr=2e-3, seed=2, stream=s)
    n, alpha = 128, 1.5
    f, h = bump_field(n, 3, 16, 5500, width=(0.05, 0.2))
    op = fl.Op(3, alpha, h, (n,) * 3, stream=s)
    ref = O.Operator(3, alpha, h, (n,) * 3)
    u, info = op.solve(_dev(f), tol=1e-8, opts=fl.solve_opts(pc=fl.FL_PC_LEARNED, mixed=1, net=net))
    res = _full_residual(ref, f, u.cpu().numpy())
    _say("128^3", info["iters"], info["rel_res_true"], res)
    assert res <= 1e-8
    assert abs(info["rel_res_true"] - res) <= 1e-3 * res + 1e-14


@pytest.mark.parametrize("pc", [1, 3])
def test_256cubed_batched_sampled_lines(pc):
    _say("256^3 batched, sampled lines, pc", pc)
    fl = _fl()
    w0 = workload_rhs_256cubed(0)
    n, alpha, h = w0["n"], w0["alpha"], w0["h"]
    s = torch.cuda.Stream()
    op = fl.Op(3, alpha, h, (n,) * 3, stream=s)
    wts = O.weights_folded(3, alpha, h, (n,) * 3)
    fs = [workload_rhs_256cubed(k)["f"] for k in (0, 9)]
    us, infos = fl.solve_batched([op, op], [_dev(f) for f in fs], tol=1e-8, opts=fl.solve_opts(pc=pc, mixed=1))
    rng = np.random.default_rng(256 + pc)
    leads = [tuple(int(v) for v in rng.integers(0, n, 2)) for _ in range(16)]
    N = n ** 3
    for f, u, inf in zip(fs, us, infos):
        assert inf["status"] == 0 and inf["rel_res_true"] <= 1e-8, inf
        un = u.cpu().numpy()
        r2 = []
        for lead in leads:
            r = f[lead] - O.apply_line(wts, un, lead)
            r2.append(r * r)
        est = float(np.sqrt(N * np.mean(np.concatenate(r2))) / np.linalg.norm(f))
        _say("sampled residual estimate", est, "library", inf["rel_res_true"])
        # 4096 points: the estimate of the l2 residual is within a small
        # factor of the whole-grid value, which the tolerance bounds by 1e-8
        assert est <= 3e-8, est


UNEVEN = workload_uneven_steps(32)
# four of the 32 problems: the first of each grid size (the largest included)
PICK = [next(i for i, p in enumerate(UNEVEN) if p["n"] == v) for v in (128, 256, 384, 512)]


@pytest.fixture(scope="module")
def uneven_trajectories():
    fl = _fl()
    s = torch.cuda.Stream()
    ops = [fl.Op(2, p["alpha"], p["h"], (p["n"], p["n"]), stream=s) for p in UNEVEN]
    opts = fl.solve_opts(pc=fl.FL_PC_SPECTRAL)
    us = [_dev(p["u0"]) for p in UNEVEN]
    states = {i: [UNEVEN[i]["u0"].copy()] for i in PICK}
    for k in range(200):
        fl.step_batched(ops, us, [1e-3] * 32, theta=1.0, nsteps=1, tol=1e-10, opts=opts)
        for i in PICK:
            states[i].append(us[i].cpu().numpy())
    # the benchmark advances all 200 steps in one call
    us200 = [_dev(p["u0"]) for p in UNEVEN]
    fl.step_batched(ops, us200, [1e-3] * 32, theta=1.0, nsteps=200, tol=1e-10, opts=opts)
    final200 = {i: us200[i].cpu().numpy() for i in PICK}
    return states, final200


@pytest.mark.parametrize("which", range(4))
def test_uneven_batch_every_step_against_oracle(uneven_trajectories, which):
    states, final200 = uneven_trajectories
    i = PICK[which]
    p = UNEVEN[i]
    n, alpha, h = p["n"], p["alpha"], p["h"]
    _say("uneven problem", i, "n", n, "alpha", alpha)
    ref = O.Operator(2, alpha, h, (n, n))
    traj = states[i]
    worst = 0.0
    for k in range(200):
        b, u1 = traj[k], traj[k + 1]
        r = b - (u1 + 1e-3 * ref.apply(u1, method="fft"))
        worst = max(worst, float(np.linalg.norm(r) / np.linalg.norm(b)))
    _say("worst step residual", worst)
    assert worst <= 2e-10, worst
    # single-step calls and the one 200-step call take the same path
    assert float(np.abs(final200[i] - traj[-1]).max()) <= 1e-12 * float(np.abs(traj[-1]).max())
    if n == 128:
        # the whole trajectory against the oracle's own backward-Euler steps
        sc = PC.pc_scale(2, alpha, h)
        u = p["u0"].copy()
        for k in range(200):
            u, _ = KR.theta_step(lambda v: ref.apply(v, method="fft"),
                                 lambda r: PC.apply_inverse(r, sc, 1.0, 1e-3), u, 1e-3, 1.0, tol=1e-12)
        err = float(np.linalg.norm(traj[-1] - u) / np.linalg.norm(u))
        _say("trajectory error vs oracle", err)
        assert err <= 1e-7, err
