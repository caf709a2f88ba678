"""The allocation-free application (fl_apply_noalloc) against fl_apply: same
kernels on the same inputs, so the outputs are bitwise equal.  Two calls in a
row, the second with a smaller input (the shared scratch keeps the first
call's contents), in 2D and 3D, FP64 and FP32, with a mask and a shift; a
request beyond the scratch is rejected before any work."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from workloads import random_mask, white_noise  # noqa: E402


def _fl():
    import paper_1802_03770_amd as fl
    return fl


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("first,second", [((2, 1024, 1024), (1, 300, 257)), ((2, 96, 80, 72), (1, 40, 33, 30))])
def test_noalloc_matches_apply(dtype, first, second):
    _say("noalloc", dtype, first, second)
    fl = _fl()
    s = torch.cuda.Stream()
    for k, shape in enumerate((first, second)):
        batch, n = shape[0], shape[1:]
        d = len(n)
        op = fl.Op(d, 1.3, 2.0 / (n[0] + 1), n, stream=s)
        u = _dev(white_noise(shape, 40 + k), dtype)
        m = _dev(random_mask(n, 41 + k), torch.uint8)
        for mask, sh in ((None, (0.0, 1.0)), (m, (1.0, 0.3))):
            want = op.apply(u, mask=mask, shift0=sh[0], shift1=sh[1])
            got = torch.full_like(u, float("nan"))
            op.apply_noalloc(u, got, mask=mask, shift0=sh[0], shift1=sh[1])
            torch.cuda.synchronize()
            assert torch.equal(got, want), (shape, mask is not None)
        op.close()


def test_noalloc_rejects_beyond_scratch():
    fl = _fl()
    op = fl.Op(2, 1.0, 2.0 / 1025, (1024, 1024))
    u = torch.zeros((4, 1024, 1024), dtype=torch.float64, device="cuda")  # 4 x 16.8 MB > 64 MiB
    out = torch.empty_like(u)
    with pytest.raises(fl.FlError) as e:
        op.apply_noalloc(u, out)
    assert e.value.status == fl.FL_E_INVALID and "scratch" in str(e.value)
