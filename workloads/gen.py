"""Seeded input generators (numpy PCG64).

Draw order for a bump sum: centres (G x d), then widths (G), then amplitudes
(G).  "Width" is the standard deviation of the bump.  Every field is float64
C-contiguous with shape (n,)*d, last axis fastest, evaluated at the interior
grid points x_j = lo + j h, j = 1..n, h = (hi - lo)/(n + 1).
"""
import numpy as np


def grid_axis(n, lo=-1.0, hi=1.0):
    h = (hi - lo) / (n + 1)
    return lo + h * np.arange(1, n + 1), h


def bump_field(n, d, nbumps, seed, width=(0.1, 0.3), centre=(-0.6, 0.6), lo=-1.0, hi=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(centre[0], centre[1], size=(nbumps, d))
    w = rng.uniform(width[0], width[1], size=nbumps)
    a = rng.standard_normal(nbumps)
    x, h = grid_axis(n, lo, hi)
    # separable evaluation: bump g is a_g prod_ax exp(-(x - c_{g,ax})^2 / (2 w_g^2));
    # the sum over bumps is a product of per-axis factor matrices E[ax][g, i]
    E = [np.exp(-((x[None, :] - c[:, ax:ax + 1]) ** 2) / (2.0 * w[:, None] ** 2)) for ax in range(d)]
    acc = a[:, None] * E[0]  # [G, n]
    for ax in range(1, d):
        acc = (acc[:, :, None] * E[ax][:, None, :]).reshape(nbumps, -1) if ax < d - 1 else acc
    if d == 1:
        out = acc.sum(axis=0)
    else:
        out = acc.T @ E[d - 1]  # [prod n_{<d-1}, n]
    return np.ascontiguousarray(out.reshape((n,) * d)), h


def white_noise(shape, seed):
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(shape)


def random_mask(shape, seed, frac_out=0.2):
    """uint8 mask: an L-shaped occlusion plus a few random holes (1 = inside the domain)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = np.ones(shape, dtype=np.uint8)
    sl = tuple(slice(s // 2, s) for s in shape[:2]) + tuple(slice(None) for _ in shape[2:])
    m[sl] = 0
    holes = rng.random(shape) < frac_out * 0.1
    m[holes] = 0
    return m


def workload_elliptic_64(seed=1000):
    """2D, alpha = 1, 64 x 64 on (-1,1)^2, 8 bumps, widths U[0.1,0.3], amplitudes N(0,1)."""
    f, h = bump_field(64, 2, 8, seed, width=(0.1, 0.3))
    return {"d": 2, "n": 64, "alpha": 1.0, "h": h, "f": f}


def workload_elliptic_1024(alpha=1.0, seed=2000):
    """2D, 1024 x 1024 on (-1,1)^2, 32 bumps, widths U[0.05,0.2], amplitudes N(0,1)."""
    f, h = bump_field(1024, 2, 32, seed, width=(0.05, 0.2))
    return {"d": 2, "n": 1024, "alpha": alpha, "h": h, "f": f}


def workload_rhs_256cubed(k, n=256, seed0=3000):
    """3D, 256^3 on (-1,1)^3, alpha = 1.2, right-hand side k (16 bumps, widths U[0.05,0.2], amplitudes N(0,1))."""
    f, h = bump_field(n, 3, 16, seed0 + k, width=(0.05, 0.2))
    return {"d": 3, "n": n, "alpha": 1.2, "h": h, "f": f}


def workload_uneven_steps(nprob=32, seed=4000, sizes=(128, 256, 384, 512)):
    """Batch of uneven 2D backward-Euler problems: n from sizes, alpha ~ U[0.3, 1.8]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.choice(np.array(sizes), size=nprob)
    alphas = rng.uniform(0.3, 1.8, size=nprob)
    probs = []
    for i in range(nprob):
        u0, h = bump_field(int(ns[i]), 2, 8, seed + 1 + i, width=(0.1, 0.3))
        probs.append({"d": 2, "n": int(ns[i]), "alpha": float(alphas[i]), "h": h, "u0": u0})
    return probs


def power_law_field(shape, seed, slope=(0.0, 3.0)):
    """Gaussian random field with a random spectral slope: white noise on the
    doubled periodic box, amplitudes scaled by (1 + |k|)^-beta with beta drawn
    from U[slope], cropped to `shape` and normalised to unit l2 norm.  Draw
    order: beta, then the noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    beta = rng.uniform(slope[0], slope[1])
    big = tuple(2 * v for v in shape)
    w = rng.standard_normal(big)
    kk = 0.0
    for a, v in enumerate(big):
        k = np.fft.fftfreq(v) * v
        sh = [1] * len(big)
        sh[a] = v
        kk = kk + (k.reshape(sh)) ** 2
    amp = (1.0 + np.sqrt(kk)) ** (-beta)
    f = np.fft.ifftn(np.fft.fftn(w) * amp).real[tuple(slice(0, v) for v in shape)]
    return np.ascontiguousarray(f / np.linalg.norm(f))


def learned_training_plan(nalpha=100, n=256, seed=5000, lo=0.2, hi=1.9, d=2):
    """Problems of the learned-preconditioner training set: alpha ~ U[lo, hi]
    on an n^d grid of (-1,1)^d, each with a bump right-hand side (32 bumps in
    2D, 16 in 3D; widths U[0.05,0.2], amplitudes N(0,1)) and random-field seeds."""
    rng = np.random.Generator(np.random.PCG64(seed))
    alphas = rng.uniform(lo, hi, size=nalpha)
    return [{"n": n, "d": d, "alpha": float(a), "rhs_seed": seed + 1 + i, "field_seed": seed + 100000 + 1000 * i}
            for i, a in enumerate(alphas)]


def l_shape_mask(n):
    """uint8 mask of the L-shaped domain on an n x n grid of [0,1]^2 (n odd,
    h = 1/(n+1)): the (n+1)/2 x (n+1)/2 block of points in one corner,
    x_i, y_j <= 1/2 (1-based i, j <= (n+1)/2), is removed.  n = 127 leaves
    127^2 - 64^2 = 12033 points."""
    m = np.ones((n, n), dtype=np.uint8)
    q = (n + 1) // 2
    m[:q, :q] = 0
    return m


def octagon_mask(n):
    """uint8 mask of the octagon with vertices on the grid: the square [0,1]^2
    with its four corners cut along the lines x + y = 1/4 (and mirror images),
    points on a cut line removed.  1-based i, j: a point is outside when
    i + j <= (n+1)/4 or one of its three mirror images is.  n = 127 leaves
    127^2 - 4 * 496 = 14145 points."""
    i = np.arange(1, n + 1)
    I, J = np.meshgrid(i, i, indexing="ij")
    c = (n + 1) / 4.0
    out = (I + J <= c) | ((n + 1 - I) + J <= c) | (I + (n + 1 - J) <= c) | ((n + 1 - I) + (n + 1 - J) <= c)
    return (~out).astype(np.uint8)
