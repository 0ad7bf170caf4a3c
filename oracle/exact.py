"""Exact discrete solutions u_h = A^{-1} b of eq. (fem).

Two routes:
  * ``solve_direct``: sparse LU of the assembled matrix (small n).
  * ``solve_fft``: for constant alpha on a box the orthonormal DST-I (node axes,
    modes 1..n-1) and DCT-II (cell axes, modes 0..n-1) diagonalise the 1-D blocks:
    T -> (2 + cos(pi a / n)) / 3 and D maps sine mode a to cosine mode a with factor
    g_a = 2 sin(pi a / (2 n)).  A then splits into one 3x3 block per wave vector
    (a, b, c):  h [alpha C^T diag(tau_a, tau_b, tau_c) C + h^2 diag(tau_b tau_c,
    tau_a tau_c, tau_a tau_b)] with C = [[0, -g_c, g_b], [g_c, 0, -g_a],
    [-g_b, g_a, 0]], keeping only the components whose modes exist.
"""
import numpy as np
import scipy.fft as sfft
import scipy.sparse.linalg as spla

from . import assemble, mesh


def solve_direct(n, h, alpha, b):
    A = assemble.matrix_kron(n, h, alpha).tocsc()
    return spla.splu(A, permc_spec="MMD_AT_PLUS_A").solve(np.asarray(b, dtype=np.float64))


def _split(n, v):
    out = []
    for d in range(3):
        o = mesh.block_offset(n, d)
        s = mesh.block_shape(n, d)
        out.append(v[..., o:o + int(np.prod(s))].reshape(v.shape[:-1] + s))
    return out


def _fwd(X, d):
    lead = X.ndim - 3
    for ax in range(3):
        geo = 2 - ax
        if geo == d:
            X = sfft.dct(X, type=2, norm="ortho", axis=lead + ax)
        else:
            X = sfft.dst(X, type=1, norm="ortho", axis=lead + ax)
    return X


def _inv(X, d):
    lead = X.ndim - 3
    for ax in range(3):
        geo = 2 - ax
        if geo == d:
            X = sfft.idct(X, type=2, norm="ortho", axis=lead + ax)
        else:
            X = sfft.idst(X, type=1, norm="ortho", axis=lead + ax)
    return X


def _embed(n, Xd, d):
    """Place the transformed block of direction d on the full (n,n,n) mode grid [c][b][a]."""
    full = np.zeros(Xd.shape[:-3] + (n, n, n), dtype=Xd.dtype)
    sl = [slice(None)] * (Xd.ndim - 3)
    for ax in range(3):
        geo = 2 - ax
        sl.append(slice(0, n) if geo == d else slice(1, n))
    full[tuple(sl)] = Xd
    return full, tuple(sl)


def blocks(n, h, alpha, alpha_curl=None, dtype=np.float64, mass=1):
    """3x3 symbol of A (or of alpha_curl*K + mass*M) on the (n,n,n) mode grid, and the
    mask of existing components.  Returns (Ablk[..., 3, 3], mask[..., 3])."""
    if alpha_curl is None:
        alpha_curl = alpha
    k = np.arange(n)
    kf = k.astype(dtype)
    pi = np.asarray(np.pi, dtype=dtype) if dtype == np.float64 else np.arccos(np.asarray(-1, dtype=dtype))
    h, alpha_curl = np.asarray(h, dtype=dtype), np.asarray(alpha_curl, dtype=dtype)
    g = 2 * np.sin(pi * kf / (2 * n))
    tau = (2 + np.cos(pi * kf / n)) / 3
    c, b, a = np.meshgrid(k, k, k, indexing="ij")
    ga, gb, gc = g[a], g[b], g[c]
    ta, tb, tc = tau[a], tau[b], tau[c]
    Z = np.zeros_like(ga)
    C = np.stack([np.stack([Z, -gc, gb], -1),
                  np.stack([gc, Z, -ga], -1),
                  np.stack([-gb, ga, Z], -1)], -2)
    Tf = np.stack([ta, tb, tc], -1)
    K = np.einsum("...fi,...f,...fj->...ij", C, Tf, C)
    Mdiag = np.stack([tb * tc, ta * tc, ta * tb], -1)
    A = h * (alpha_curl * K + mass * h * h * (np.eye(3, dtype=dtype) * Mdiag[..., None, :]))
    mask = np.stack([(b >= 1) & (c >= 1), (a >= 1) & (c >= 1), (a >= 1) & (b >= 1)], -1)
    return A, mask


def transform(n, v, dtype=np.float64):
    """Orthonormal transform of compact vector(s) v onto the (..., n, n, n, 3) mode grid."""
    parts = _split(n, np.asarray(v, dtype=dtype))
    return np.stack([_embed(n, _fwd(parts[d], d), d)[0] for d in range(3)], -1)


def inverse_transform(n, U):
    out = []
    for d in range(3):
        full = U[..., d]
        sl = [slice(None)] * (full.ndim - 3)
        for ax in range(3):
            geo = 2 - ax
            sl.append(slice(0, n) if geo == d else slice(1, n))
        out.append(_inv(full[tuple(sl)], d).reshape(full.shape[:-3] + (-1,)))
    return np.concatenate(out, -1)


def _solve3(A, b):
    """Solutions of the 3x3 systems A x = b by the adjugate (any float dtype, including
    the x86 extended long double, which LAPACK does not take)."""
    a = [[A[..., i, j] for j in range(3)] for i in range(3)]
    adj = np.empty_like(A)
    for i in range(3):
        for j in range(3):
            r0, r1 = [x for x in range(3) if x != j]
            c0, c1 = [x for x in range(3) if x != i]
            adj[..., i, j] = (-1) ** (i + j) * (a[r0][c0] * a[r1][c1] - a[r0][c1] * a[r1][c0])
    det = a[0][0] * adj[..., 0, 0] + a[0][1] * adj[..., 1, 0] + a[0][2] * adj[..., 2, 0]
    return np.einsum("...ij,...j->...i", adj, b) / det[..., None]


def solve_fft(n, h, alpha, b, dtype=np.float64):
    """u = A^{-1} b for one or several right-hand sides (last axis = compact dofs).

    dtype=np.longdouble runs the transforms and the 3x3 solves in x86 extended precision
    (unit roundoff 2^-64) and returns the result in that precision: for references that
    difference nearly equal solutions (the adjoint of a tracking loss)."""
    A, mask = blocks(n, h, alpha, dtype=dtype)
    B = transform(n, b, dtype)
    Afix = np.where(mask[..., :, None] & mask[..., None, :], A, 0)
    Afix = Afix + np.eye(3, dtype=dtype) * (~mask)[..., None, :]
    if np.dtype(dtype) == np.float64:
        U = np.linalg.solve(Afix, (B * mask)[..., None])[..., 0]
    else:
        U = _solve3(Afix, B * mask)
    return inverse_transform(n, U * mask)


def apply_fft(n, h, alpha, x, dtype=np.float64, mass=1):
    """y = A x (mass=0: y = alpha K x) for one or several vectors (last axis = compact
    dofs) through the 3x3 symbols: transform, multiply each wave vector's block,
    transform back."""
    A, mask = blocks(n, h, alpha, dtype=dtype, mass=mass)
    X = transform(n, x, dtype) * mask
    Afix = np.where(mask[..., :, None] & mask[..., None, :], A, 0.0)
    Y = np.einsum("...ij,...j->...i", Afix, X)
    return inverse_transform(n, Y * mask)


def eigenvalues(n, h, alpha):
    """All eigenvalues of A, ascending (from the 3x3 symbols)."""
    A, mask = blocks(n, h, alpha)
    both = mask[..., :, None] & mask[..., None, :]
    Afix = np.where(both, A, 0.0) - np.eye(3) * (~mask)[..., None, :]
    ev = np.linalg.eigvalsh(Afix).ravel()
    return np.sort(ev[ev > 0])
