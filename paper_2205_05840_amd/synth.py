"""Seeded synthetic inputs shared by the tests, the smoke run and the benchmark.

Only random numbers and sampled input fields live here: no step of the solver's
arithmetic.  Every right-hand side is a field f sampled at the 2x2x2 Gauss points of
each element, an array [n^3][8][3] (element (c0, c1, c2) at row (c2 n + c1) n + c0,
point q = q0 + 2 q1 + 4 q2 at local coordinates (x_{q0}, x_{q1}, x_{q2}) with
x = (1 -+ 1/sqrt 3)/2, components x, y, z).
"""
import numpy as np

GAUSS_1D = np.array([(1.0 - 1.0 / np.sqrt(3.0)) / 2.0, (1.0 + 1.0 / np.sqrt(3.0)) / 2.0])


def gauss_points(n, L=1.0):
    """Physical coordinates (n^3, 8, 3) of the 2x2x2 Gauss points of every element."""
    h = L / n
    c2, c1, c0 = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    corner = np.stack([c0.ravel(), c1.ravel(), c2.ravel()], 1) * h
    q2, q1, q0 = np.meshgrid(GAUSS_1D, GAUSS_1D, GAUSS_1D, indexing="ij")
    loc = np.stack([q0.ravel(), q1.ravel(), q2.ravel()], 1) * h
    return corner[:, None, :] + loc[None, :, :]


def normal_samples(n, seed, nrhs=None):
    """f ~ N(0, 1) i.i.d. per Gauss point and component; shape [n^3, 8, 3] or [nrhs, ...]."""
    rng = np.random.default_rng(seed)
    shape = (n ** 3, 8, 3) if nrhs is None else (nrhs, n ** 3, 8, 3)
    return rng.standard_normal(shape)


def manufactured_field(x, y, z):
    """u* = (sin pi y sin pi z, sin pi z sin pi x, sin pi x sin pi y) on the unit cube."""
    s = np.sin
    p = np.pi
    return s(p * y) * s(p * z), s(p * z) * s(p * x), s(p * x) * s(p * y)


def manufactured_samples(n, alpha, seed, noise=1e-3):
    """f = (2 pi^2 alpha + 1) u* at the Gauss points plus N(0, noise^2) per component.

    curl curl u* = 2 pi^2 u* and n x u* = 0 on the unit cube, so u* solves the model
    problem with this f when noise = 0.
    """
    X = gauss_points(n)
    u = np.stack(manufactured_field(X[..., 0], X[..., 1], X[..., 2]), -1)
    rng = np.random.default_rng(seed)
    return (2.0 * np.pi ** 2 * alpha + 1.0) * u + noise * rng.standard_normal(u.shape)


def batched_problems(nprob=512, seed=3, sizes=(8, 12, 16, 24, 32)):
    """Sizes drawn uniformly from ``sizes`` and alpha log-uniform in [1e-2, 1e2]."""
    rng = np.random.default_rng(seed)
    n = rng.choice(np.asarray(sizes), size=nprob)
    alpha = 10.0 ** rng.uniform(-2.0, 2.0, size=nprob)
    return n.astype(np.int64), alpha


def unit_directions(ndim, count, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((count, ndim))
    return v / np.linalg.norm(v, axis=1, keepdims=True)
