"""GPU parity of the batched driver (fl_solve_batched / fl_step_batched).

Every member of a batch is checked against the oracle on its own: dense
Cholesky-class solves and the exact eigen-propagator on small grids, and
sampled residuals (direct sums at chosen points) on the uneven C4-size grids.
A batch shares one stream, so every test creates its ops on one stream.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import krylov as KR  # noqa: E402
from oracle import operator as O  # noqa: E402
from oracle import precond as PC  # noqa: E402
from workloads import bump_field, random_mask, white_noise  # noqa: E402


def _fl():
    import paper_1802_03770_amd as fl
    return fl


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def _rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


# (n, alpha): uneven 2D grids; the last two share one op (two right-hand sides)
PROBS_2D = [((24, 30), 0.6), ((31, 31), 1.0), ((40, 36), 1.5), ((17, 45), 1.9)]


def _make(fl, probs, stream):
    ops, refs = [], []
    for n, alpha in probs:
        h = 2.0 / (max(n) + 1)
        ops.append(fl.Op(len(n), alpha, h, n, stream=stream))
        refs.append(O.Operator(len(n), alpha, h, n))
    return ops, refs


@pytest.mark.parametrize("pc,mixed", [(1, 0), (0, 0), (1, 1)])
def test_solve_batched_uneven_against_dense(pc, mixed):
    _say("batched solve 2D uneven pc", pc, "mixed", mixed)
    fl = _fl()
    s = torch.cuda.Stream()
    ops, refs = _make(fl, PROBS_2D, s)
    ops.append(ops[1])  # second right-hand side of the 31^2 operator
    refs.append(refs[1])
    fs = [white_noise(r.n, 50 + i) for i, r in enumerate(refs)]
    fs[1] = bump_field(31, 2, 6, 51)[0]  # a smooth right-hand side for the shared operator
    us, infos = fl.solve_batched(ops, [_dev(f) for f in fs], tol=1e-12,
                                 opts=fl.solve_opts(pc=pc, mixed=mixed))
    for i, (u, r, f, inf) in enumerate(zip(us, refs, fs, infos)):
        M = r.dense()
        xs = np.linalg.solve(M, f.ravel())
        got = u.cpu().numpy().ravel()
        res = np.linalg.norm(f.ravel() - M @ got) / np.linalg.norm(f)
        assert inf["status"] == 0
        assert res <= 2e-12, (i, res)
        assert _rel(got, xs) <= 1e-9, i


def test_solve_batched_matches_standalone_iterations():
    _say("batched vs standalone iteration counts")
    fl = _fl()
    s = torch.cuda.Stream()
    ops, refs = _make(fl, PROBS_2D, s)
    fs = [white_noise(r.n, 70 + i) for i, r in enumerate(refs)]
    _, infos = fl.solve_batched(ops, [_dev(f) for f in fs], tol=1e-10, opts=fl.solve_opts(pc=1))
    for i, (op, r, f) in enumerate(zip(ops, refs, fs)):
        _, one = op.solve(_dev(f), tol=1e-10, opts=fl.solve_opts(pc=1))
        assert abs(one["iters"] - infos[i]["iters"]) <= 1, (i, one["iters"], infos[i]["iters"])
        # and the oracle's PCG on the same system
        M = r.dense()
        sc = PC.pc_scale(2, r.alpha, r.h)
        _, it, _, _ = KR.pcg(lambda v: (M @ v.ravel()).reshape(v.shape), f, lambda q: PC.apply_inverse(q, sc),
                             tol=1e-10)
        assert abs(it - infos[i]["iters"]) <= 1, (i, it, infos[i]["iters"])


@pytest.mark.parametrize("probs", [
    [((37,), 0.7), ((46,), 1.3), ((64,), 1.8), ((37,), 0.7)],
    [((12, 10, 9), 1.2), ((8, 9, 10), 0.5), ((12, 10, 9), 1.2)],
])
def test_solve_batched_1d_3d(probs):
    _say("batched solve", probs)
    fl = _fl()
    s = torch.cuda.Stream()
    ops, refs = _make(fl, probs, s)
    fs = [white_noise(r.n, 90 + i) for i, r in enumerate(refs)]
    us, infos = fl.solve_batched(ops, [_dev(f) for f in fs], tol=1e-12, opts=fl.solve_opts(pc=1))
    for i, (u, r, f) in enumerate(zip(us, refs, fs)):
        M = r.dense()
        xs = np.linalg.solve(M, f.ravel())
        assert _rel(u.cpu().numpy().ravel(), xs) <= 1e-9, i
        assert infos[i]["rel_res_true"] <= 2e-12


def test_solve_batched_masked_and_zero_rhs():
    _say("batched masked + zero rhs")
    fl = _fl()
    s = torch.cuda.Stream()
    probs = [((30, 26), 1.1), ((33, 33), 0.8), ((20, 22), 1.4)]
    ops, refs = _make(fl, probs, s)
    masks = [random_mask(refs[0].n, 5), None, random_mask(refs[2].n, 6)]
    fs = [white_noise(refs[0].n, 1) * masks[0], np.zeros(refs[1].n), white_noise(refs[2].n, 3) * masks[2]]
    us, infos = fl.solve_batched(ops, [_dev(f) for f in fs], tol=1e-12, opts=fl.solve_opts(pc=1),
                                 masks=[None if m is None else _dev(m, torch.uint8) for m in masks])
    assert infos[1]["iters"] == 0 and np.all(us[1].cpu().numpy() == 0.0)
    for i in (0, 2):
        m = masks[i].ravel().astype(bool)
        M = refs[i].dense()[np.ix_(m, m)]
        xs = np.linalg.solve(M, fs[i].ravel()[m])
        got = us[i].cpu().numpy().ravel()
        assert np.all(got[~m] == 0.0)
        assert _rel(got[m], xs) <= 1e-9, i


def test_batched_graph_and_eager_agree():
    _say("batched graph vs eager")
    fl = _fl()
    s = torch.cuda.Stream()
    ops, refs = _make(fl, PROBS_2D, s)
    fs = [_dev(white_noise(r.n, 11 + i)) for i, r in enumerate(refs)]
    ug, ig = fl.solve_batched(ops, fs, tol=1e-11, opts=fl.solve_opts(pc=1, graph=1))
    ue, ie = fl.solve_batched(ops, fs, tol=1e-11, opts=fl.solve_opts(pc=1, graph=0))
    for a, b, x, y in zip(ug, ue, ig, ie):
        assert torch.equal(a, b)
        assert x["iters"] == y["iters"]


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_step_batched_against_exact_propagator(theta):
    _say("batched steps theta", theta)
    fl = _fl()
    s = torch.cuda.Stream()
    probs = [((12, 12), 1.2), ((10, 14), 0.7), ((9, 11), 1.7)]
    dts = [0.01, 0.02, 0.005]
    ops, refs = _make(fl, probs, s)
    u0 = [white_noise(r.n, 21 + i) for i, r in enumerate(refs)]
    us = [_dev(u) for u in u0]
    fl.step_batched(ops, us, dts, theta=theta, nsteps=4, tol=1e-14)
    for i, r in enumerate(refs):
        want = KR.exact_propagator(r.dense(), dts[i], theta, 4, u0[i]).reshape(r.n)
        assert _rel(us[i].cpu().numpy(), want) <= 1e-11, i


def test_step_batched_c4_sizes_sampled():
    # one backward-Euler step of uneven problems at the sizes of the uneven
    # batch workload, dt = 1e-3; the residual of (I + dt M) u1 = u0 is checked
    # at sampled points with the oracle's direct sums
    _say("batched step at 128..512 sampled")
    fl = _fl()
    from workloads import workload_uneven_steps
    probs = workload_uneven_steps(nprob=6)
    sizes = sorted({p["n"] for p in probs})
    probs = [next(p for p in probs if p["n"] == n) for n in sizes] + probs[:2]
    s = torch.cuda.Stream()
    ops = [fl.Op(2, p["alpha"], p["h"], (p["n"], p["n"]), stream=s) for p in probs]
    us = [_dev(p["u0"]) for p in probs]
    _, infos = fl.step_batched(ops, us, [1e-3] * len(ops), theta=1.0, nsteps=1, tol=1e-10)
    rng = np.random.default_rng(3)
    for i, p in enumerate(probs):
        n = p["n"]
        u1 = us[i].cpu().numpy()
        w = O.weights_folded(2, p["alpha"], p["h"], (n, n))
        pts = [(0, 0), (n - 1, n - 1), (n // 2, n // 2)] + [tuple(rng.integers(0, n, 2)) for _ in range(5)]
        Mu = O.apply_at(w, u1, pts)
        scale = np.linalg.norm(p["u0"]) / np.sqrt(n * n)
        for q, mv in zip(pts, Mu):
            r = p["u0"][q] - (u1[q] + 1e-3 * mv)
            # pointwise residual: well inside the 1e-10 relative l2 tolerance
            assert abs(r) <= 1e-8 * max(scale, np.abs(p["u0"]).max()), (i, q, r)
        assert infos[i]["rel_res_true"] <= 1e-10
        # the same step through the single-problem entry point
        one = _dev(p["u0"])
        ops[i].step(one, 1e-3, 1.0, tol=1e-10)
        assert _rel(u1, one.cpu().numpy()) <= 1e-8, i


def test_batched_rejects_mixed_dimensions():
    fl = _fl()
    s = torch.cuda.Stream()
    a = fl.Op(2, 1.0, 0.1, (8, 8), stream=s)
    b = fl.Op(1, 1.0, 0.1, (8,), stream=s)
    with pytest.raises(ValueError):
        fl.solve_batched([a, b], [_dev(np.ones((8, 8))), _dev(np.ones(8))])
    c = fl.Op(2, 1.0, 0.1, (8, 8))  # its own stream
    with pytest.raises(ValueError):
        fl.solve_batched([a, c], [_dev(np.ones((8, 8))), _dev(np.ones((8, 8)))])


@pytest.mark.parametrize("mixed", [0, 1])
def test_repeat_batched_calls_allocate_nothing_and_take_per_problem_tol(mixed):
    # A repeat of a batched call with the same problems reuses every buffer,
    # descriptor table and captured graph (the library's device allocation
    # count does not move), and each problem stops at its own tolerance.
    _say("batched reuse, mixed", mixed)
    fl = _fl()
    s = torch.cuda.Stream()
    ops, refs = _make(fl, PROBS_2D, s)
    fs = [_dev(white_noise(r.n, 51 + i)) for i, r in enumerate(refs)]
    tols = [1e-6, 1e-12, 1e-9, 1e-11]
    opts = fl.solve_opts(pc=fl.FL_PC_FD, mixed=mixed)
    fl.solve_batched(ops, fs, tol=tols, opts=opts)
    a0 = fl.device_allocations()
    us, infos = fl.solve_batched(ops, fs, tol=tols, opts=opts)
    torch.cuda.synchronize()
    assert fl.device_allocations() == a0
    for i, r in enumerate(refs):
        M = r.dense()
        f = fs[i].cpu().numpy().ravel()
        res = np.linalg.norm(f - M @ us[i].cpu().numpy().ravel()) / np.linalg.norm(f)
        assert res <= tols[i] * 1.5, (i, res, tols[i])
        assert abs(infos[i]["rel_res_true"] - res) <= 1e-3 * res + 1e-14
    # the loosest problem needs fewer iterations than the same one at the tightest tolerance
    _, tight = fl.solve_batched(ops, fs, tol=1e-12, opts=opts)
    assert infos[0]["iters"] < tight[0]["iters"]
    # repeated time-step calls with one dt set reuse their batch as well
    u0 = [_dev(white_noise(r.n, 61 + i)) for i, r in enumerate(refs)]
    dts = [1e-3, 2e-3, 1e-3, 5e-4]
    fl.step_batched(ops, u0, dts, theta=0.5, nsteps=1, tol=1e-11)
    a1 = fl.device_allocations()
    fl.step_batched(ops, u0, dts, theta=0.5, nsteps=3, tol=1e-11)
    torch.cuda.synchronize()
    assert fl.device_allocations() == a1
    # and single-problem solves of a built op allocate nothing after the first
    ops[0].solve(fs[0], tol=1e-10, opts=opts)
    a2 = fl.device_allocations()
    ops[0].solve(fs[0], tol=1e-10, opts=opts)
    assert fl.device_allocations() == a2
