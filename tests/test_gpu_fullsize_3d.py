"""GPU parity at the 3D benchmark size (256^3, alpha = 1.2), in the launch
configuration the batched 16 x 256^3 workload and the single-op solves use:
the length-512 row and column FFT kernels and the chirp-z sine kernels of
length 512 (2(n+1) = 514 = 2 * 257).

* Application: sampled outputs against the oracle's direct sums over all
  16.7M points (FP64 1e-12 and FP32 2e-5 relative to the largest output).
* Preconditioners (FD and sine-basis diagonal): the whole result against the
  oracle's dense sine-matrix products (1e-12 / 2e-5).
* Batched solves of two of the workload's right-hand sides: the residual at
  sampled points, from the oracle's direct sums, is bounded by the 2-norm
  tolerance (|r_i| <= ||r||_2 <= tol ||f||_2; factor 2 for the evaluation).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import constants as K  # noqa: E402
from oracle import operator as O  # noqa: E402
from oracle import precond as PC  # noqa: E402
from oracle import spectral as SP  # noqa: E402
from workloads import white_noise, workload_rhs_256cubed  # noqa: E402

N3, ALPHA = 256, 1.2
POINTS = [(0, 0, 0), (255, 255, 255), (128, 3, 250), (17, 200, 64), (255, 0, 129)]


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


@pytest.fixture(scope="module")
def setup():
    fl = _fl()
    h = 2.0 / (N3 + 1)
    op = fl.Op(3, ALPHA, h, (N3,) * 3)
    plan = op.plan()
    # prime form (FFT length 256) or chirp-z (length 512), as the autotuner timed them
    assert all((form, L) in ((3, 256), (2, 512)) for form, L in plan["f64"] + plan["f32"]), plan
    ref = O.Operator(3, ALPHA, h, (N3,) * 3)
    return fl, op, ref, h


def test_apply_256cubed_sampled(setup):
    fl, op, ref, h = setup
    _say("apply 256^3 sampled")
    u = white_noise((N3,) * 3, 41)
    got = op.apply(_dev(u)).cpu().numpy()
    want = O.apply_at(ref.w, u, POINTS)
    scale = np.abs(got).max()
    for p, wv in zip(POINTS, want):
        assert abs(got[p] - wv) <= 1e-12 * scale, (p, got[p], wv)
    u32 = u.astype(np.float32)
    got32 = op.apply(_dev(u32, torch.float32)).double().cpu().numpy()
    want32 = O.apply_at(ref.w, u32.astype(np.float64), POINTS)
    for p, wv in zip(POINTS, want32):
        assert abs(got32[p] - wv) <= 2e-5 * scale, (p, got32[p], wv)


def test_precond_256cubed(setup):
    fl, op, ref, h = setup
    _say("precond 256^3")
    r = white_noise((N3,) * 3, 42)
    want = PC.apply_inverse(r, PC.pc_scale(3, ALPHA, h))
    assert _rel(op.precond(_dev(r)).cpu().numpy(), want) <= 1e-12
    assert _rel(op.precond(_dev(r, torch.float32)).double().cpu().numpy(), want) <= 2e-5
    m = SP.tau_eigenvalues(3, ALPHA, (N3,) * 3)
    want_s = SP.apply_tau_inverse(r, m, K.c_alpha(ALPHA, 3) * h ** -ALPHA)
    assert _rel(op.precond(_dev(r), kind=fl.FL_PC_SPECTRAL).cpu().numpy(), want_s) <= 1e-12
    got_s32 = op.precond(_dev(r, torch.float32), kind=fl.FL_PC_SPECTRAL).double().cpu().numpy()
    assert _rel(got_s32, want_s) <= 2e-5


@pytest.mark.parametrize("pc", [1, 3])
def test_batched_256cubed_sampled_residual(setup, pc):
    fl, op, ref, h = setup
    _say("batched 256^3 pc", pc)
    fs = [workload_rhs_256cubed(k)["f"] for k in range(2)]
    assert fs[0].shape == (N3,) * 3
    us, infos = fl.solve_batched([op, op], [_dev(f) for f in fs], tol=1e-8, opts=fl.solve_opts(pc=pc, mixed=1))
    for f, u, inf in zip(fs, us, infos):
        assert inf["status"] == 0 and inf["rel_res_true"] <= 1e-8, inf
        un = u.cpu().numpy()
        Mu = O.apply_at(ref.w, un, POINTS[:3])
        bound = 2e-8 * np.linalg.norm(f)
        for p, mv in zip(POINTS[:3], Mu):
            assert abs(f[p] - mv) <= bound, (p, f[p] - mv, bound)
