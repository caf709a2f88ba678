"""GPU parity of the sine-basis diagonal preconditioner (fl_precond_spectral,
pc = FL_PC_SPECTRAL) against the FP64 oracle (oracle/spectral.py)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import constants as K  # noqa: E402
from oracle import krylov as KR  # noqa: E402
from oracle import operator as O  # noqa: E402
from oracle import spectral as SP  # noqa: E402
from workloads import random_mask, white_noise  # noqa: E402


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


CASES = [(37,), (46,), (48, 40), (46, 40), (40, 52), (64, 64), (9, 10, 12), (6, 7, 46)]


@pytest.mark.parametrize("n", CASES)
def test_tau_table(n):
    _say("tau table", n)
    fl = _fl()
    d, alpha = len(n), 1.3
    h = 2.0 / (max(n) + 1)
    op = fl.Op(d, alpha, h, n)
    want = SP.tau_eigenvalues(d, alpha, n) * O.Operator(d, alpha, h, n).C * h ** -alpha
    got = op.tau().cpu().numpy()
    assert _rel(got, want) <= 1e-12
    g32 = op.tau(torch.float32).cpu().numpy()
    assert _rel(g32, want) <= 1e-6


@pytest.mark.parametrize("n", CASES)
@pytest.mark.parametrize("shift", [(0.0, 1.0), (1.0, 0.01)])
def test_precond_spectral(n, shift):
    _say("precond spectral", n, shift)
    fl = _fl()
    d, alpha = len(n), 0.8
    h = 2.0 / (max(n) + 1)
    op = fl.Op(d, alpha, h, n)
    m = SP.tau_eigenvalues(d, alpha, n)
    sc = O.Operator(d, alpha, h, n).C * h ** -alpha
    r = white_noise(n, 4)
    want = SP.apply_tau_inverse(r, m, sc, *shift)
    got = op.precond(_dev(r), p0=shift[0], p1=shift[1], kind=fl.FL_PC_SPECTRAL).cpu().numpy()
    assert _rel(got, want) <= 1e-12
    g32 = op.precond(_dev(r, torch.float32), p0=shift[0], p1=shift[1], kind=fl.FL_PC_SPECTRAL).cpu().numpy()
    assert _rel(g32, want) <= 2e-5
    # masked form: P_Omega B P_Omega
    if d == 2:
        mk = random_mask(n, 1).astype(np.float64)
        gm = op.precond(_dev(r), mask=_dev(mk, torch.uint8), p0=shift[0], p1=shift[1],
                        kind=fl.FL_PC_SPECTRAL).cpu().numpy()
        assert _rel(gm, mk * SP.apply_tau_inverse(r * mk, m, sc, *shift)) <= 1e-12


@pytest.mark.parametrize("mixed", [0, 1])
def test_solve_spectral_against_dense(mixed):
    _say("solve spectral mixed", mixed)
    fl = _fl()
    from workloads import workload_elliptic_64
    w = workload_elliptic_64()
    n, alpha, h, f = w["n"], w["alpha"], w["h"], w["f"]
    op = fl.Op(2, alpha, h, (n, n))
    ref = O.Operator(2, alpha, h, (n, n))
    M = ref.dense()
    xs = np.linalg.solve(M, f.ravel()).reshape(n, n)
    u, info = op.solve(_dev(f), tol=1e-12, opts=fl.solve_opts(pc=fl.FL_PC_SPECTRAL, mixed=mixed))
    u = u.cpu().numpy()
    res = np.linalg.norm(f.ravel() - M @ u.ravel()) / np.linalg.norm(f)
    assert res <= 2e-12
    assert _rel(u, xs) <= 1e-9
    if not mixed:
        # iteration count of the oracle's PCG with the same preconditioner, within 1
        m = SP.tau_eigenvalues(2, alpha, (n, n))
        _, it, _, _ = KR.pcg(lambda v: (M @ v.ravel()).reshape(v.shape), f,
                             lambda r: SP.apply_tau_inverse(r, m, ref.C * h ** -alpha), tol=1e-10)
        _, i10 = op.solve(_dev(f), tol=1e-10, opts=fl.solve_opts(pc=fl.FL_PC_SPECTRAL))
        assert abs(i10["iters"] - it) <= 1
        assert it <= 15


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_step_spectral_against_exact_propagator(theta):
    _say("step spectral", theta)
    fl = _fl()
    n = (12, 12)
    d, alpha, h, dt, steps = 2, 1.2, 0.08, 0.01, 5
    op = fl.Op(d, alpha, h, n)
    M = O.Operator(d, alpha, h, n).dense()
    u0 = white_noise(n, 17)
    u = _dev(u0)
    for _ in range(steps):
        u, _ = op.step(u, dt, theta, tol=1e-14, opts=fl.solve_opts(pc=fl.FL_PC_SPECTRAL))
    want = KR.exact_propagator(M, dt, theta, steps, u0).reshape(n)
    assert _rel(u.cpu().numpy(), want) <= 1e-11


def test_batched_spectral_uneven():
    _say("batched spectral")
    fl = _fl()
    s = torch.cuda.Stream()
    probs = [((24, 30), 0.6), ((31, 31), 1.0), ((40, 36), 1.5)]
    ops, refs, fs = [], [], []
    for i, (n, a) in enumerate(probs):
        h = 2.0 / (max(n) + 1)
        ops.append(fl.Op(2, a, h, n, stream=s))
        refs.append(O.Operator(2, a, h, n))
        fs.append(white_noise(n, 30 + i))
    us, infos = fl.solve_batched(ops, [_dev(f) for f in fs], tol=1e-12,
                                 opts=fl.solve_opts(pc=fl.FL_PC_SPECTRAL))
    for u, r, f, inf in zip(us, refs, fs, infos):
        xs = np.linalg.solve(r.dense(), f.ravel())
        assert _rel(u.cpu().numpy().ravel(), xs) <= 1e-9
        assert inf["iters"] <= 20


def test_full_size_tau_sampled():
    # 1024^2 table in the configuration the solver uses: sampled entries
    # against the oracle's separable sum, one mode at a time
    _say("tau 1024^2 sampled")
    fl = _fl()
    n, alpha = 1024, 1.0
    h = 2.0 / (n + 1)
    op = fl.Op(2, alpha, h, (n, n))
    got = op.tau().cpu().numpy()
    om = O.omega_folded(2, alpha, (n, n))
    G = SP.sine_correlation(n)
    C = K.c_alpha(alpha, 2)
    for k0, k1 in [(0, 0), (0, 1), (5, 700), (1023, 1023), (511, 3)]:
        want = C * h ** -alpha * float(G[k0] @ om @ G[k1])
        assert abs(got[k0, k1] - want) <= 1e-11 * abs(got).max(), (k0, k1)


@pytest.mark.parametrize("n", [(37,), (64, 64), (48, 40), (9, 10, 12), (1024,), (256,), (256, 37), (5, 256, 7)])
@pytest.mark.parametrize("mode", [1, 2])
def test_precond_both_sine_plans(n, mode):
    # the sine-transform plans the autotuner chooses between: direct odd
    # extension (mode 1, where 2(n+1) factors over radices <= 43), the prime
    # form (mode 1, n + 1 = 257) and chirp-z
    _say("sine plan", mode, n)
    fl = _fl()
    from oracle import precond as PCO
    d, alpha = len(n), 1.1
    h = 2.0 / (max(n) + 1)
    op = fl.Op(d, alpha, h, n, dst_mode=mode)
    plan = op.plan()
    if mode == 2:
        assert all(f == 2 for f, _ in plan["f64"] + plan["f32"])
    else:
        for a, k in enumerate(n):
            if k == 256:
                assert tuple(plan["f64"][a]) == (3, 256) and tuple(plan["f32"][a]) == (3, 256), plan
    r = white_noise(n, 8)
    want = PCO.apply_inverse(r, PCO.pc_scale(d, alpha, h))
    assert _rel(op.precond(_dev(r)).cpu().numpy(), want) <= 1e-12
    assert _rel(op.precond(_dev(r, torch.float32)).cpu().numpy(), want) <= 2e-5
    m = SP.tau_eigenvalues(d, alpha, n)
    want_s = SP.apply_tau_inverse(r, m, O.Operator(d, alpha, h, n).C * h ** -alpha)
    assert _rel(op.precond(_dev(r), kind=fl.FL_PC_SPECTRAL).cpu().numpy(), want_s) <= 1e-12


def test_autotuned_plan_is_recorded():
    fl = _fl()
    op = fl.Op(2, 1.0, 2.0 / 1025, (1024, 1024))
    plan = op.plan()
    for p in ("f64", "f32"):
        for form, L in plan[p]:
            assert (form, L) in ((1, 2050), (2, 2048)), plan


@pytest.mark.parametrize("lanes", [-1, 128])
def test_precond_full_size_sine_column_forms(lanes):
    # 1024^2 (direct length 2050) with the plan's lanes and with 128 lanes per
    # FFT line in the sine column pass; whole result against the oracle's dense
    # sine matrices (FD) and its sine-basis diagonal (spectral)
    _say("1024^2 sine column lanes", lanes)
    fl = _fl()
    from oracle import precond as PCO
    n, alpha = 1024, 1.0
    h = 2.0 / (n + 1)
    op = fl.Op(2, alpha, h, (n, n), sine_col_lanes=lanes, dst_mode=1)
    assert op.plan()["sine_col_lanes"]["f32"] == (128 if lanes > 0 else 0)
    r = white_noise((n, n), 21)
    want = PCO.apply_inverse(r, PCO.pc_scale(2, alpha, h))
    assert _rel(op.precond(_dev(r)).cpu().numpy(), want) <= 1e-12
    assert _rel(op.precond(_dev(r, torch.float32)).cpu().numpy(), want) <= 2e-5
    m = SP.tau_eigenvalues(2, alpha, (n, n))
    want_s = SP.apply_tau_inverse(r, m, K.c_alpha(alpha, 2) * h ** -alpha)
    assert _rel(op.precond(_dev(r), kind=fl.FL_PC_SPECTRAL).cpu().numpy(), want_s) <= 1e-12
