"""GPU parity of the length-specialised kernels against the FP64 oracle.

The row and column FFT kernels of the application have compile-time versions
for padded lengths 256, 512, 1024 and 2048 (grids of 128, 256, 512, 1024
points on an axis); the sine kernels have compile-time versions for the
chirp-z form with FFT length 256, 512 or 1024 (n = 126, 256, 508 here: 2(n+1)
has a prime factor above 43, so the odd extension is not used) and for the
prime form of n = 256 (n + 1 = 257 prime: Rader's identity, FFT length 256).  Each shape
below puts such an axis last (row passes), first (symbol / scaled sine column
pass) or in the middle of a 3D grid (forward / inverse column passes and the
unscaled sine column pass).  The batched cases give every member the same
shape, which lets the batched launches use the same specialisations.

Tolerances as in the other parity tests: FP64 1e-12, FP32 2e-5 relative
(max-norm against the oracle's max).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import operator as O  # noqa: E402
from oracle import precond as PC  # noqa: E402
from oracle import spectral as SP  # noqa: E402
from workloads import bump_field, white_noise  # noqa: E402


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


APPLY_SHAPES = [(3, 4, 256), (256, 3, 5), (4, 256, 3), (128, 6), (6, 128), (5, 512), (3, 1024), (130, 4, 3)]


@pytest.mark.parametrize("n", APPLY_SHAPES)
def test_apply_specialised_lengths(n):
    _say("apply specialised", n)
    fl = _fl()
    d, alpha, h = len(n), 1.2, 2.0 / (max(n) + 1)
    op = fl.Op(d, alpha, h, n)
    ref = O.Operator(d, alpha, h, n)
    u = white_noise(n, 21)
    want = ref.apply(u, method="dft")
    assert _rel(op.apply(_dev(u)).cpu().numpy(), want) <= 1e-12
    want32 = ref.apply(u.astype(np.float32).astype(np.float64), method="dft")
    got32 = op.apply(_dev(u, torch.float32)).double().cpu().numpy()
    assert _rel(got32, want32) <= 2e-5


PRECOND_SHAPES = [(3, 4, 256), (256, 3, 4), (4, 256, 3), (126, 5), (5, 126), (3, 508), (508, 3), (256, 6)]


@pytest.mark.parametrize("n", PRECOND_SHAPES)
@pytest.mark.parametrize("mode", [2, 1])
def test_precond_specialised_chirp_lengths(n, mode):
    # mode 2: every axis in the chirp-z form; mode 1: n = 256 in the prime form
    # (n + 1 = 257, Rader's identity with an FFT of length 256), 126 and 508
    # still chirp-z (2(n+1) = 2 * 127, 2 * 509)
    _say("precond specialised", n, mode)
    fl = _fl()
    d, alpha, h = len(n), 0.9, 2.0 / (max(n) + 1)
    op = fl.Op(d, alpha, h, n, dst_mode=mode)
    forms = op.plan()
    for a, k in enumerate(n):
        if k in (126, 256, 508):
            want = (3, 256) if (mode == 1 and k == 256) else (2, {126: 256, 256: 512, 508: 1024}[k])
            assert tuple(forms["f64"][a]) == want and tuple(forms["f32"][a]) == want, forms
    r = white_noise(n, 22)
    for shift in ((0.0, 1.0), (1.0, 0.01)):
        want = PC.apply_inverse(r, PC.pc_scale(d, alpha, h), *shift)
        assert _rel(op.precond(_dev(r), p0=shift[0], p1=shift[1]).cpu().numpy(), want) <= 1e-12
        got32 = op.precond(_dev(r, torch.float32), p0=shift[0], p1=shift[1]).double().cpu().numpy()
        assert _rel(got32, want) <= 2e-5
    m = SP.tau_eigenvalues(d, alpha, n)
    want_s = SP.apply_tau_inverse(r, m, O.Operator(d, alpha, h, n).C * h ** -alpha)
    assert _rel(op.precond(_dev(r), kind=fl.FL_PC_SPECTRAL).cpu().numpy(), want_s) <= 1e-12
    got_s32 = op.precond(_dev(r, torch.float32), kind=fl.FL_PC_SPECTRAL).double().cpu().numpy()
    assert _rel(got_s32, want_s) <= 2e-5


@pytest.mark.parametrize("shape,pc,mixed,mode", [((256, 4, 256), 1, 1, 2), ((256, 256), 3, 0, 2), ((6, 126, 5), 1, 0, 0),
                                                 ((256, 4, 256), 1, 1, 1), ((256, 256), 3, 0, 1), ((256,), 1, 0, 1)])
def test_batched_uniform_specialised(shape, pc, mixed, mode):
    # two right-hand sides of one operator and a third problem of the same
    # shape and another alpha: every launch takes the shared specialisation
    _say("batched uniform", shape, pc, mixed, mode)
    fl = _fl()
    s = torch.cuda.Stream()
    d, h = len(shape), 2.0 / (max(shape) + 1)
    op_a = fl.Op(d, 1.2, h, shape, stream=s, dst_mode=mode)
    op_b = fl.Op(d, 0.7, h, shape, stream=s, dst_mode=mode)
    refs = [O.Operator(d, 1.2, h, shape), O.Operator(d, 0.7, h, shape)]
    fs = [white_noise(shape, 30), bump_field(shape[0], d, 8, 31)[0] if len(set(shape)) == 1 else
          white_noise(shape, 31), white_noise(shape, 32)]
    us, infos = fl.solve_batched([op_a, op_a, op_b], [_dev(f) for f in fs], tol=1e-10,
                                 opts=fl.solve_opts(pc=pc, mixed=mixed))
    for i, (u, f, inf) in enumerate(zip(us, fs, infos)):
        ref = refs[0] if i < 2 else refs[1]
        res = np.linalg.norm(f - ref.apply(u.cpu().numpy(), method="dft")) / np.linalg.norm(f)
        assert inf["status"] == 0, (i, inf)
        assert res <= 1e-9, (i, res)
    # same iteration counts as the standalone solves (same kernels, same order)
    for i, (op, f) in enumerate(((op_a, fs[0]), (op_a, fs[1]), (op_b, fs[2]))):
        _, inf = op.solve(_dev(f), tol=1e-10, opts=fl.solve_opts(pc=pc, mixed=mixed))
        assert abs(inf["iters"] - infos[i]["iters"]) <= 1, (i, inf["iters"], infos[i]["iters"])
