"""The paper's grid-refinement studies run through the library at the
paper's grid sizes (paper_1802_03770_amd.convergence, every application,
solve and time step on the GPU), against the printed tables:

* Table 2drich (2D, 255^2 / 511^2 / 1023^2): solution rates within the
  printed digits; application rates at 4 - alpha (the quadrature's order for
  the smooth g_1), 0.09-0.13 above the printed ones (see the reading in
  tests/test_oracle_convergence.py);
* Table 3Drich (3D, 63^3 / 127^3 / 255^3);
* Table richpara (Crank-Nicolson to T = 0.25 with dt = 1/(n+1), 2D and 3D);
* Table td_its (one Crank-Nicolson system with a random right-hand side):
  PCG counts within one of the printed ones.
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
    assert all(s["rel_res_true"] <= 1e-11 for s in r["solves"])


@pytest.mark.parametrize("alpha", [1.25, 1.5, 1.75])
def test_3d_richardson_rates(alpha):
    from paper_1802_03770_amd import convergence as CV
    row = _row("tab_3drich.txt", alpha)
    r = CV.elliptic_rates(3, alpha, 63)
    _say("3D", alpha, {k: v for k, v in r.items() if k != "solves"}, "printed", row[1:])
    assert abs(r["u_R2"] - row[1]) <= 0.05 and abs(r["u_Rinf"] - row[2]) <= 0.05
    assert abs(r["f_R2"] - row[3]) <= 0.3 and abs(r["f_Rinf"] - row[4]) <= 0.3
    assert all(s["rel_res_true"] <= 1e-11 for s in r["solves"])


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("alpha", [1.25, 1.5, 1.75])
def test_parabolic_rates(d, alpha):
    from paper_1802_03770_amd import convergence as CV
    row = _row("tab_richpara.txt", alpha)
    r = CV.parabolic_rates(d, alpha, 255 if d == 2 else 31)
    want = row[1:3] if d == 2 else row[3:5]
    _say("richpara", d, alpha, r, "printed", want)
    assert [v["steps"] for v in r["runs"]] == ([64, 128, 256] if d == 2 else [8, 16, 32])
    assert abs(r["R2"] - want[0]) <= 0.05 and abs(r["Rinf"] - want[1]) <= 0.05


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
