"""GPU parity of the application on grids padded to 8192 points along an axis
(n = 4081 .. 4096), the fine grid of the smooth 2D example (Sec. 4.2): the
row, symbol-column and symbol (DCT-I) kernels specialised for FFT lines of
8192 points, 256 lanes per line.

* FP64 application at 4095^2 and on a mixed 1000 x 4095 grid: sampled outputs
  against the oracle's direct sums over all points (1e-12 relative to the
  largest output); FP32 at 2e-5.
* Such grids are application-only: the solver, preconditioner, step, batched
  and profiling entry points refuse them with FL_E_UNSUPPORTED.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import operator as O  # noqa: E402
from workloads import white_noise  # noqa: E402


def _fl():
    import paper_1802_03770_amd as fl
    return fl


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("shape,alpha", [((4095, 4095), 1.25), ((1000, 4095), 0.75), ((4090, 600), 1.6)])
def test_apply_8192_lines_sampled(shape, alpha):
    _say("apply, lines of 8192", shape, alpha)
    fl = _fl()
    h = 1.0 / (max(shape) + 1)
    op = fl.Op(2, alpha, h, shape)
    assert max(op.padded()) == 8192
    # a smooth separable field plus seeded noise (any input serves: the
    # application is linear)
    x0 = np.linspace(0.0, 1.0, shape[0])[:, None]
    x1 = np.linspace(0.0, 1.0, shape[1])[None, :]
    u = np.sin(3.0 * x0 + 0.5) * np.cos(5.0 * x1) + 0.05 * white_noise(shape, 12)
    g64 = op.apply(_dev(u)).cpu().numpy()
    g32 = op.apply(_dev(u, torch.float32)).cpu().numpy()
    w = O.weights_folded(2, alpha, h, shape)
    rng = np.random.default_rng(sum(shape))
    pts = [(0, 0), (shape[0] - 1, shape[1] - 1), (shape[0] // 2, 5),
           (int(rng.integers(0, shape[0])), int(rng.integers(0, shape[1])))]
    want = O.apply_at(w, u, pts)
    scale = np.abs(g64).max()
    for p, wv in zip(pts, want):
        assert abs(g64[p] - wv) <= 1e-12 * scale, (p, g64[p], wv)
        assert abs(g32[p] - wv) <= 2e-5 * scale, (p, g32[p], wv)
    op.close()


def test_8192_lines_are_application_only():
    fl = _fl()
    n = 4095
    op = fl.Op(2, 1.0, 1.0 / (n + 1), (n, n))
    f = torch.ones((n, n), dtype=torch.float64, device="cuda")
    with pytest.raises(fl.FlError):
        op.solve(f, tol=1e-8)
    with pytest.raises(fl.FlError):
        op.precond(f)
    with pytest.raises(fl.FlError):
        op.step(f.clone(), 1e-3, 1.0)
    with pytest.raises(fl.FlError):
        op.profile_pass(torch.float64, 4)
    with pytest.raises(fl.FlError):
        fl.solve_batched([op], [f], tol=1e-8)
    op.close()
    with pytest.raises(fl.FlError):  # 1D and 3D grids of 8192-point lines are not built
        fl.Op(1, 1.0, 1.0 / (n + 1), (n,))
