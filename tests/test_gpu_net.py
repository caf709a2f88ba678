"""GPU parity of the learned preconditioner's network (BF16 activations, FP32
accumulation) against the FP64 numpy oracle (oracle/net.py), of its training
pairs against the oracle's operator and sine-basis diagonal, and the ablation:
what the trained network gains inside flexible CG over the same solver
without it.

Tolerances: the network keeps activations in BF16 (8-bit significand, unit
roundoff 2^-9 ~ 2e-3) through nine layers, so outputs and gradients are
compared in relative l2 norm against the FP64 oracle.

* ReLU-active regime (weights scaled by 0.1, hidden biases 1: every
  pre-activation stays positive, checked on the oracle): the network is
  linear in its input and BF16 rounding is the only difference, about 20
  roundings deep.  Measured per-layer gradient errors stay below 1e-2 in 2D
  and 3D; bound 2e-2 per layer, 1e-2 for the whole gradient and 2e-2 for the
  output.  These are the tight pins of the reverse pass: an indexing error
  shows as an O(1) error in the layer it touches.
* Random biases (ReLUs switch inside the test grids): a pre-activation near
  zero can take the other side of the ReLU in BF16 than in FP64, which
  changes that pixel's gradient entirely.  The coarse levels of small test
  grids sum few pixels, so single flips show: measured per-layer errors run
  3e-2 .. 2e-1 across seeds and shapes in 2D and 3D alike, whole-gradient
  errors up to 6.6e-2 with cosine similarity at least 0.9978.  Bounds: 3e-2
  for outputs, 2.5e-1 per layer, 1e-1 whole, cosine 0.997.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import net as NN  # noqa: E402
from oracle import operator as O  # noqa: E402
from oracle import precond as PC  # noqa: E402
from oracle import spectral as SP  # noqa: E402
from workloads import bump_field, power_law_field, white_noise  # noqa: E402


def _fl():
    import paper_1802_03770_amd as fl
    return fl


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rl2(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _check_grad(g, want, d, per_layer, whole, cos_min):
    o = 0
    for name, ci, co in NN.LAYERS:
        nw = 3 ** d * ci * co
        for part, m in (("W", nw), ("b", co)):
            if np.linalg.norm(want[o:o + m]) > 0:
                err = _rl2(g[o:o + m], want[o:o + m])
                assert err <= per_layer, (name, part, err)
            o += m
    cos = float(g @ want / (np.linalg.norm(g) * np.linalg.norm(want)))
    assert cos >= cos_min, cos
    assert _rl2(g, want) <= whole, _rl2(g, want)


def _params_relu_active(seed, d):
    """Weights scaled by 0.1 and hidden biases 1 (output layer as drawn): every
    pre-activation of the test inputs stays positive."""
    th = NN.init_params(seed, d)
    for name, (w, b) in NN.unpack(th, d).items():
        if name != "out":
            w *= 0.1
            b[:] = 1.0
    return th


@pytest.mark.parametrize("d,shape", [(2, (2, 16, 24)), (2, (3, 8, 16)), (3, (2, 8, 16, 8)), (3, (1, 16, 16, 16))])
def test_net_grad_relu_active_against_oracle(d, shape):
    _say("net grad relu-active", d, shape)
    fl = _fl()
    th = _params_relu_active(4 + d, d)
    rng = np.random.Generator(np.random.PCG64(31 + sum(shape)))
    x = rng.standard_normal(shape).astype(np.float32)
    gy = rng.standard_normal(shape).astype(np.float32)
    al = rng.uniform(0.2, 1.9, size=shape[0])
    th64 = th.astype(np.float32).astype(np.float64)
    want_y, act = NN.forward(th64, x.astype(np.float64), al, keep=True)
    assert min(float(act[k].min()) for k in ("a0", "a1", "a2", "a3", "c3", "c2", "c1", "c0")) > 0.05
    net = fl.Net(params=th, d=d)
    y = net.forward(torch.from_numpy(x).cuda(), list(al)).cpu().numpy()
    assert _rl2(y, want_y) <= 2e-2
    g = net.grad(torch.from_numpy(x).cuda(), list(al), torch.from_numpy(gy).cuda()).cpu().numpy()
    want = NN.grad(th64, x.astype(np.float64), al, gy.astype(np.float64))
    _check_grad(g, want, d, per_layer=2e-2, whole=1e-2, cos_min=0.9999)


@pytest.mark.parametrize("B,H,W", [(1, 24, 136), (2, 16, 64), (1, 40, 128)])
def test_net_forward_tiles_pixelwise_against_oracle(B, H, W):
    # Every layer runs on 4 x 64 tiles with a one-pixel halo staged in LDS
    # (the coarse levels on the same tiles of smaller grids): these shapes
    # cross tile rows and columns at every level and end in ragged tiles.
    # With parameters that keep every ReLU active the BF16 error is smooth,
    # so a wrong halo or boundary padding shows as a pixel far above the rest.
    _say("net forward tiles", B, H, W)
    fl = _fl()
    th = _params_relu_active(9, 2)
    rng = np.random.Generator(np.random.PCG64(77 + H + W))
    x = rng.standard_normal((B, H, W)).astype(np.float32)
    al = rng.uniform(0.2, 1.9, size=B)
    th64 = th.astype(np.float32).astype(np.float64)
    want, act = NN.forward(th64, x.astype(np.float64), al, keep=True)
    assert min(float(act[k].min()) for k in ("a0", "a1", "a2", "a3", "c3", "c2", "c1", "c0")) > 0.05
    net = fl.Net(params=th, d=2)
    y = net.forward(torch.from_numpy(x).cuda(), list(al)).cpu().numpy()
    err = np.abs(y - want)
    scale = float(np.abs(want).max())
    assert _rl2(y, want) <= 2e-2, _rl2(y, want)
    assert float(err.max()) <= 3e-2 * scale, (float(err.max()) / scale, np.unravel_index(err.argmax(), err.shape))
    # tile-edge columns and rows are no worse than the interior
    cols = [c for c in (0, 63, 64, 127, 128, W - 1) if c < W]
    rows = [r for r in range(0, H, 4)] + [r for r in range(3, H, 4)] + [H - 1]
    interior = float(np.sqrt(np.mean(err ** 2)))
    assert float(err[:, :, cols].max()) <= 10 * interior + 1e-3 * scale
    assert float(err[:, rows, :].max()) <= 10 * interior + 1e-3 * scale


def _params(seed):
    th = NN.init_params(seed)
    rng = np.random.Generator(np.random.PCG64(seed + 50))
    P = NN.unpack(th)
    for name, (w, b) in P.items():  # nonzero biases, output layer at full scale
        b[:] = 0.1 * rng.standard_normal(b.shape)
    P["out"][0][:] *= 10.0
    return th


@pytest.mark.parametrize("B,H,W", [(2, 16, 24), (1, 8, 8), (3, 64, 72), (1, 128, 64)])
def test_net_forward_against_oracle(B, H, W):
    _say("net forward", B, H, W)
    fl = _fl()
    th = _params(3)
    rng = np.random.Generator(np.random.PCG64(B * 1000 + H + W))
    x = rng.standard_normal((B, H, W))
    al = rng.uniform(0.2, 1.9, size=B)
    net = fl.Net(params=th)
    y = net.forward(torch.from_numpy(x.astype(np.float32)).cuda(), list(al)).cpu().numpy()
    want = NN.forward(th.astype(np.float32).astype(np.float64), x.astype(np.float32).astype(np.float64), al)
    assert _rl2(y, want) <= 3e-2, _rl2(y, want)


@pytest.mark.parametrize("B,H,W", [(2, 16, 24), (1, 32, 32)])
def test_net_grad_against_oracle(B, H, W):
    _say("net grad", B, H, W)
    fl = _fl()
    th = _params(4)
    rng = np.random.Generator(np.random.PCG64(7 + H))
    x = rng.standard_normal((B, H, W)).astype(np.float32)
    gy = rng.standard_normal((B, H, W)).astype(np.float32)
    al = rng.uniform(0.2, 1.9, size=B)
    net = fl.Net(params=th)
    g = net.grad(torch.from_numpy(x).cuda(), list(al), torch.from_numpy(gy).cuda()).cpu().numpy()
    want = NN.grad(th.astype(np.float32).astype(np.float64), x.astype(np.float64), al, gy.astype(np.float64))
    _check_grad(g, want, 2, per_layer=2.5e-1, whole=1e-1, cos_min=0.997)


def test_net_params_roundtrip_and_zero_output():
    fl = _fl()
    th = NN.init_params(1).astype(np.float32)
    net = fl.Net(params=th)
    assert np.array_equal(net.get_params().cpu().numpy(), th)
    z = th.copy()
    z[-(9 * 32 + 1):] = 0.0  # output layer zero: N = 0
    net.set_params(z)
    y = net.forward(torch.ones((1, 16, 16), dtype=torch.float32, device="cuda"), 1.0)
    assert torch.count_nonzero(y).item() == 0


def test_learned_pairs_against_oracle():
    _say("learned pairs")
    fl = _fl()
    n, alpha = (24, 30), 1.3
    h = 2.0 / 31
    op = fl.Op(2, alpha, h, n)
    ref = O.Operator(2, alpha, h, n)
    e = np.stack([power_law_field(n, 11), power_law_field(n, 12)])
    sub = np.stack([np.zeros(n), 0.5 * power_law_field(n, 13)])
    R, T = fl.learned_pairs(op, torch.from_numpy(e).cuda(), e_sub=torch.from_numpy(sub).cuda())
    assert R.shape == (2, 24, 32)
    m = SP.tau_eigenvalues(2, alpha, n) * ref.C * h ** -alpha
    Q0 = PC.sine_matrix(n[0]) * math.sqrt(2 / (n[0] + 1))
    Q1 = PC.sine_matrix(n[1]) * math.sqrt(2 / (n[1] + 1))
    for k in range(2):
        ek = e[k] - sub[k]
        r = ref.apply(ek)
        De = Q0 @ ((Q0.T @ ek @ Q1) * m) @ Q1.T
        s = np.sqrt((r * r).mean())
        got_R, got_T = R[k].cpu().numpy(), T[k].cpu().numpy()
        assert np.all(got_R[:, 30:] == 0) and np.all(got_T[:, 30:] == 0)
        assert _rl2(got_R[:, :30], r / s) <= 1e-6
        assert _rl2(got_T[:, :30], (De - r) / s) <= 1e-5


def test_learned_fcg_falls_back_to_fd():
    # a network whose output is a large negative constant makes r.z < 0 on a
    # positive residual: the solver must switch to the FD preconditioner
    _say("learned fallback")
    fl = _fl()
    n, alpha = 32, 1.0
    h = 2.0 / (n + 1)
    s = torch.cuda.Stream()
    op = fl.Op(2, alpha, h, (n, n), stream=s)
    th = np.zeros(NN.nparams(), dtype=np.float32)
    th[-1] = -1000.0
    net = fl.Net(stream=s, params=th)
    f = torch.ones((n, n), dtype=torch.float64, device="cuda")
    u, info = op.solve(f, tol=1e-10, opts=fl.solve_opts(pc=fl.FL_PC_LEARNED, net=net))
    assert info["fell_back"] == 1
    M = O.Operator(2, alpha, h, (n, n)).dense()
    res = np.linalg.norm(1.0 - M @ u.cpu().numpy().ravel()) / n
    assert res <= 1e-9


@pytest.mark.parametrize("mixed", [0, 1])
def test_learned_fcg_graph_matches_eager(mixed):
    # Iterations replayed from captured graphs must give the eager launches'
    # result bit for bit: on the first solve (graphs captured), on a second
    # with another right-hand side (graphs reused; the stopping threshold
    # differs and is read from device memory), after the network's weights
    # change in place (graphs reused, new weights read), and after a larger
    # forward pass has reallocated the network's activations (graphs captured
    # again: the old ones hold the old buffers).
    _say("learned graph vs eager", mixed)
    fl = _fl()
    n, alpha = 96, 1.2
    rhs = [bump_field(n, 2, 16, seed, width=(0.05, 0.2)) for seed in (5, 6)]
    h = rhs[0][1]
    rhs = [f for f, _ in rhs]
    s = torch.cuda.Stream()
    op = fl.Op(2, alpha, h, (n, n), stream=s)
    th = (0.05 * NN.init_params(41, 2)).astype(np.float32)
    net = fl.Net(stream=s, params=th)
    M = O.Operator(2, alpha, h, (n, n)).dense()

    def run(f_np, graph):
        f = torch.from_numpy(f_np).cuda()
        u, info = op.solve(f, tol=1e-9, opts=fl.solve_opts(pc=fl.FL_PC_LEARNED, net=net, mixed=mixed,
                                                            graph=graph))
        s.synchronize()
        return u.cpu().numpy(), info

    for step, f_np in enumerate(rhs + [rhs[0], rhs[1]]):
        if step == 2:
            net.set_params((0.04 * NN.init_params(42, 2)).astype(np.float32))
        if step == 3:
            with torch.cuda.stream(s):
                net.forward(torch.zeros((4, 256, 256), dtype=torch.float32, device="cuda"), alpha)
            s.synchronize()
        ug, ig = run(f_np, 1)
        ue, ie = run(f_np, 0)
        _say("step", step, "iters", ig["iters"], ie["iters"], "fell back", ig["fell_back"])
        assert ig["iters"] == ie["iters"] >= 3
        assert ig["fell_back"] == ie["fell_back"] == 0
        assert np.array_equal(ug, ue)
        res = np.linalg.norm(f_np.ravel() - M @ ug.ravel()) / np.linalg.norm(f_np)
        assert res <= 2e-9, res


def test_learned_rejects_masks_steps_and_3d():
    fl = _fl()
    s = torch.cuda.Stream()
    op = fl.Op(2, 1.0, 0.1, (16, 16), stream=s)
    net = fl.Net(stream=s, params=np.zeros(NN.nparams(), dtype=np.float32))
    f = torch.ones((16, 16), dtype=torch.float64, device="cuda")
    mk = torch.ones((16, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(fl.FlError):
        op.solve(f, mask=mk, opts=fl.solve_opts(pc=fl.FL_PC_LEARNED, net=net))
    with pytest.raises(fl.FlError):
        op.step(f.clone(), 1e-3, opts=fl.solve_opts(pc=fl.FL_PC_LEARNED, net=net))
    with pytest.raises(fl.FlError):
        op.solve(f, opts=fl.solve_opts(pc=fl.FL_PC_LEARNED))  # no network
    op3 = fl.Op(3, 1.0, 0.1, (8, 8, 8), stream=s)
    with pytest.raises(fl.FlError):
        op3.solve(torch.ones((8, 8, 8), dtype=torch.float64, device="cuda"),
                  opts=fl.solve_opts(pc=fl.FL_PC_LEARNED, net=net))


def test_training_and_ablation():
    # Train on solver-generated pairs at 64^2 (a few hundred Adam steps) and
    # compare, on a right-hand side outside the training set, flexible CG with
    # the trained network against the same solver with N = 0 (the spectral
    # preconditioner alone) and against the FD preconditioner.
    _say("training + ablation")
    fl = _fl()
    from paper_1802_03770_amd import learned as L
    from workloads import learned_training_plan
    s = torch.cuda.Stream()
    plan = learned_training_plan(nalpha=24, n=64, seed=777)
    R, T, A = L.make_pairs(plan, iters=6, fields=6, stream=s)
    assert R.shape[0] == A.shape[0] >= 24 * 10 and R.shape[1:] == (64, 64)
    net, losses = L.train(R, T, A, steps=400, batch=8, lr=2e-3, seed=3, stream=s)
    first, last = np.mean(losses[:20]), np.mean(losses[-20:])
    _say("loss", first, "->", last)
    assert last < 0.5 * first
    zero = fl.Net(stream=s, params=np.zeros(NN.nparams(), dtype=np.float32))
    out = {}
    for alpha in (0.6, 1.0, 1.5):
        n = 64
        f_np, h = bump_field(n, 2, 32, 99, width=(0.05, 0.2))
        op = fl.Op(2, alpha, h, (n, n), stream=s)
        f = torch.from_numpy(f_np).cuda()
        M = O.Operator(2, alpha, h, (n, n)).dense()
        its = {}
        for name, opts in (("learned", fl.solve_opts(pc=fl.FL_PC_LEARNED, net=net)),
                           ("spectral_fcg", fl.solve_opts(pc=fl.FL_PC_LEARNED, net=zero)),
                           ("fd", fl.solve_opts(pc=fl.FL_PC_FD))):
            u, info = op.solve(f, tol=1e-10, opts=opts)
            res = np.linalg.norm(f_np.ravel() - M @ u.cpu().numpy().ravel()) / np.linalg.norm(f_np)
            assert res <= 1e-9, (name, res)
            its[name] = info["iters"]
        out[alpha] = its
    _say("iterations", out)
    assert sum(v["learned"] for v in out.values()) < sum(v["spectral_fcg"] for v in out.values())
    for v in out.values():
        assert v["learned"] <= v["spectral_fcg"]
        assert v["spectral_fcg"] < v["fd"]


# ---------------------------------------------------------------------------
# 3D network (3 x 3 x 3 kernels)
# ---------------------------------------------------------------------------
def _params3(seed):
    th = NN.init_params(seed, 3)
    rng = np.random.Generator(np.random.PCG64(seed + 50))
    P = NN.unpack(th, 3)
    for name, (w, b) in P.items():
        b[:] = 0.1 * rng.standard_normal(b.shape)
    P["out"][0][:] *= 10.0
    return th


@pytest.mark.parametrize("B,D,H,W", [(1, 8, 8, 8), (2, 16, 8, 24), (1, 8, 16, 72)])
def test_net3d_forward_against_oracle(B, D, H, W):
    _say("net3d forward", B, D, H, W)
    fl = _fl()
    th = _params3(5)
    rng = np.random.Generator(np.random.PCG64(B * 100 + D + H + W))
    x = rng.standard_normal((B, D, H, W))
    al = rng.uniform(0.2, 1.9, size=B)
    net = fl.Net(params=th, d=3)
    assert net.nparams == NN.nparams(3)
    y = net.forward(torch.from_numpy(x.astype(np.float32)).cuda(), list(al)).cpu().numpy()
    want = NN.forward(th.astype(np.float32).astype(np.float64), x.astype(np.float32).astype(np.float64), al)
    assert _rl2(y, want) <= 3e-2, _rl2(y, want)


@pytest.mark.parametrize("B,D,H,W", [(1, 8, 8, 16), (2, 8, 16, 8)])
def test_net3d_grad_against_oracle(B, D, H, W):
    _say("net3d grad", B, D, H, W)
    fl = _fl()
    th = _params3(6)
    rng = np.random.Generator(np.random.PCG64(9 + D + H))
    x = rng.standard_normal((B, D, H, W)).astype(np.float32)
    gy = rng.standard_normal((B, D, H, W)).astype(np.float32)
    al = rng.uniform(0.2, 1.9, size=B)
    net = fl.Net(params=th, d=3)
    g = net.grad(torch.from_numpy(x).cuda(), list(al), torch.from_numpy(gy).cuda()).cpu().numpy()
    want = NN.grad(th.astype(np.float32).astype(np.float64), x.astype(np.float64), al, gy.astype(np.float64))
    _check_grad(g, want, 3, per_layer=2.5e-1, whole=1e-1, cos_min=0.997)


def test_net3d_dimension_checks():
    fl = _fl()
    net = fl.Net(params=np.zeros(NN.nparams(3), dtype=np.float32), d=3)
    with pytest.raises(fl.FlError):  # depth not a multiple of 8
        net.forward(torch.zeros((1, 12, 8, 8), dtype=torch.float32, device="cuda"), 1.0)
    with pytest.raises(ValueError):  # a 2D grid for a 3D network
        net.forward(torch.zeros((2, 3, 8, 8, 8), dtype=torch.float32, device="cuda"), 1.0)
    net2 = fl.Net(params=np.zeros(NN.nparams(), dtype=np.float32))
    with pytest.raises((fl.FlError, ValueError)):  # parameter count of the other dimension
        net2.set_params(np.zeros(NN.nparams(3), dtype=np.float32))


def test_learned_pairs_3d_against_oracle():
    _say("learned pairs 3d")
    fl = _fl()
    n, alpha = (10, 12, 9), 1.3
    h = 2.0 / 13
    op = fl.Op(3, alpha, h, n)
    ref = O.Operator(3, alpha, h, n)
    e = np.stack([power_law_field(n, 21), power_law_field(n, 22)])
    sub = np.stack([np.zeros(n), 0.5 * power_law_field(n, 23)])
    R, T = fl.learned_pairs(op, torch.from_numpy(e).cuda(), e_sub=torch.from_numpy(sub).cuda())
    assert R.shape == (2, 16, 16, 16)
    m = SP.tau_eigenvalues(3, alpha, n) * ref.C * h ** -alpha
    Q = [PC.sine_matrix(k) * math.sqrt(2 / (k + 1)) for k in n]
    for k in range(2):
        ek = e[k] - sub[k]
        r = ref.apply(ek)
        c = np.einsum("ia,jb,kc,ijk->abc", Q[0], Q[1], Q[2], ek)
        De = np.einsum("ia,jb,kc,abc->ijk", Q[0], Q[1], Q[2], c * m)
        s = np.sqrt((r * r).mean())
        got_R, got_T = R[k].cpu().numpy(), T[k].cpu().numpy()
        assert np.all(got_R[10:] == 0) and np.all(got_R[:, 12:] == 0) and np.all(got_R[:, :, 9:] == 0)
        assert np.all(got_T[10:] == 0) and np.all(got_T[:, 12:] == 0) and np.all(got_T[:, :, 9:] == 0)
        assert _rl2(got_R[:10, :12, :9], r / s) <= 1e-6
        assert _rl2(got_T[:10, :12, :9], (De - r) / s) <= 1e-5


@pytest.mark.parametrize("mixed", [0, 1])
def test_learned_fcg_3d_against_dense(mixed):
    # flexible CG with a 3D network (random weights, then N = 0, the spectral
    # preconditioner alone) on an uneven 3D grid padded to multiples of 8
    _say("learned fcg 3d mixed", mixed)
    fl = _fl()
    n, alpha = (11, 12, 10), 1.5
    h = 2.0 / 13
    s = torch.cuda.Stream()
    op = fl.Op(3, alpha, h, n, stream=s)
    M = O.Operator(3, alpha, h, n).dense()
    f = white_noise(n, 40)
    for th in (_params3(7) * 0.1, np.zeros(NN.nparams(3), dtype=np.float32)):
        net = fl.Net(stream=s, params=th, d=3)
        u, info = op.solve(torch.from_numpy(f).cuda(), tol=1e-10,
                           opts=fl.solve_opts(pc=fl.FL_PC_LEARNED, net=net, mixed=mixed))
        res = np.linalg.norm(f.ravel() - M @ u.cpu().numpy().ravel()) / np.linalg.norm(f)
        assert info["status"] == 0 and res <= 2e-10, (info, res)
    with pytest.raises(fl.FlError):  # a 2D network on a 3D op
        op.solve(torch.from_numpy(f).cuda(), opts=fl.solve_opts(
            pc=fl.FL_PC_LEARNED, net=fl.Net(stream=s, params=np.zeros(NN.nparams(), dtype=np.float32))))


def test_training_and_ablation_3d():
    # Train a 3D network on solver-generated pairs at 16^3 and compare on a
    # right-hand side outside the training set: flexible CG with the trained
    # network, with N = 0 (spectral preconditioner alone), and FD PCG.
    _say("training + ablation 3d")
    fl = _fl()
    from paper_1802_03770_amd import learned as L
    from workloads import learned_training_plan
    s = torch.cuda.Stream()
    plan = learned_training_plan(nalpha=16, n=16, seed=880, d=3)
    R, T, A = L.make_pairs(plan, iters=5, fields=5, stream=s)
    assert R.shape[1:] == (16, 16, 16) and R.shape[0] == A.shape[0] >= 16 * 6
    net, losses = L.train(R, T, A, steps=300, batch=4, lr=2e-3, seed=4, stream=s)
    first, last = np.mean(losses[:20]), np.mean(losses[-20:])
    _say("loss 3d", first, "->", last)
    assert last < 0.6 * first
    zero = fl.Net(stream=s, params=np.zeros(NN.nparams(3), dtype=np.float32), d=3)
    out = {}
    for alpha in (0.7, 1.5):
        n = 16
        f_np, h = bump_field(n, 3, 16, 98, width=(0.05, 0.2))
        op = fl.Op(3, alpha, h, (n,) * 3, stream=s)
        M = O.Operator(3, alpha, h, (n,) * 3).dense()
        its = {}
        for name, opts in (("learned", fl.solve_opts(pc=fl.FL_PC_LEARNED, net=net)),
                           ("spectral_fcg", fl.solve_opts(pc=fl.FL_PC_LEARNED, net=zero)),
                           ("fd", fl.solve_opts(pc=fl.FL_PC_FD))):
            u, info = op.solve(torch.from_numpy(f_np).cuda(), tol=1e-10, opts=opts)
            res = np.linalg.norm(f_np.ravel() - M @ u.cpu().numpy().ravel()) / np.linalg.norm(f_np)
            assert res <= 1e-9, (name, res)
            its[name] = info["iters"]
        out[alpha] = its
    _say("iterations 3d", out)
    for v in out.values():
        assert v["spectral_fcg"] < v["fd"]
        assert v["learned"] <= v["spectral_fcg"] + 1


def _adam_problem(d, shape, seed):
    th = _params_relu_active(seed, d)
    rng = np.random.Generator(np.random.PCG64(seed + 900))
    R = rng.standard_normal(shape).astype(np.float32)
    T = (0.3 * rng.standard_normal(shape)).astype(np.float32)
    A = rng.uniform(0.2, 1.9, size=shape[0]).astype(np.float32)
    return th, R, T, A


@pytest.mark.parametrize("d,shape", [(2, (2, 16, 24)), (3, (2, 8, 8, 16))])
def test_adam_steps_against_oracle_with_device_gradients(d, shape):
    # Three Adam steps of fl_net_train on one fixed minibatch.  Before each
    # step the same gradient is taken through fl_net_grad (same kernels, same
    # fixed-order reductions, the loss gradient 2 (y - t) / n formed in FP32
    # as the training step forms it), and the oracle's adam_step is fed that
    # gradient: the parameters after every step must agree to FP32 rounding.
    # This pins the update, both moments and the bias corrections by step
    # number, independently of the BF16 gradient error.
    _say("adam vs oracle (device gradients)", d, shape)
    fl = _fl()
    th0, R, T, A = _adam_problem(d, shape, 21 + d)
    B = shape[0]
    lr = 1e-3
    net = fl.Net(params=th0, d=d)
    Rd, Td, Ad = (torch.from_numpy(v).cuda() for v in (R, T, A))
    n = R.size
    th = th0.astype(np.float32).astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for k in range(1, 4):
        y = net.forward(Rd, [float(a) for a in A]).cpu().numpy()
        gy = np.float32(2.0 / n) * (y - T)
        g = net.grad(Rd, [float(a) for a in A], torch.from_numpy(gy).cuda()).cpu().numpy().astype(np.float64)
        net.train(Rd, Td, Ad, np.arange(B).reshape(1, B), batch=B, lr=lr)
        got = net.get_params().cpu().numpy().astype(np.float64)
        th, m, v = NN.adam_step(th, g, m, v, k, lr)
        step = np.abs(got - th)
        assert float(step.max()) <= 2e-3 * lr + 1e-6 * float(np.abs(th).max()), (k, float(step.max()))


@pytest.mark.parametrize("d,shape", [(2, (2, 16, 24)), (3, (2, 8, 8, 16))])
def test_adam_trajectory_against_oracle(d, shape):
    # Three training steps from fixed parameters on a fixed minibatch, against
    # the oracle run end to end (its own FP64 forward, loss gradient, reverse
    # pass and adam_step).  Adam divides each coordinate's step by its own
    # gradient scale, so a coordinate whose gradient is below the BF16
    # gradient error can step the other way; the comparison is therefore on
    # the whole step theta_3 - theta_0 per layer (relative l2) and on the
    # fraction of coordinates that moved in the oracle's direction.
    _say("adam trajectory vs oracle", d, shape)
    fl = _fl()
    th0, R, T, A = _adam_problem(d, shape, 41 + d)
    B = shape[0]
    lr = 1e-3
    net = fl.Net(params=th0, d=d)
    Rd, Td, Ad = (torch.from_numpy(v).cuda() for v in (R, T, A))
    net.train(Rd, Td, Ad, np.tile(np.arange(B), (3, 1)), batch=B, lr=lr)
    got = net.get_params().cpu().numpy().astype(np.float64)
    th = th0.astype(np.float32).astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    x64, t64, a64 = R.astype(np.float64), T.astype(np.float64), A.astype(np.float64)
    for k in range(1, 4):
        g = NN.loss_grad(th, x64, a64, t64)
        th, m, v = NN.adam_step(th, g, m, v, k, lr)
    th0_64 = th0.astype(np.float32).astype(np.float64)
    dg, dw = got - th0_64, th - th0_64
    assert _rl2(dg, dw) <= 0.3, _rl2(dg, dw)
    # coordinates whose gradient stands clear of the BF16 gradient error
    # (above 5% of the RMS gradient of its layer) move the oracle's way
    g0 = NN.loss_grad(th0_64, x64, a64, t64)
    o, strong = 0, np.zeros(g0.size, dtype=bool)
    for name, ci, co in NN.LAYERS:
        for m_ in (3 ** d * ci * co, co):
            seg = g0[o:o + m_]
            strong[o:o + m_] = np.abs(seg) > 0.05 * np.sqrt(np.mean(seg ** 2))
            o += m_
    agree = float(np.mean(np.sign(dg[strong]) == np.sign(dw[strong])))
    assert agree >= 0.99, agree
