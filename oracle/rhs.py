"""Load vector f_h: <f_h, phi_e> = (f, phi_e) (Sec. 2, eq. fem).

The integral over each element uses tensor Gauss-Legendre quadrature.  The sampled
form takes f at the 2x2x2 Gauss points of every element, an array [n^3][8][3]
(element (c0, c1, c2) at row (c2 n + c1) n + c0, point q = q0 + 2 q1 + 4 q2 at
local coordinates (x_{q0}, x_{q1}, x_{q2}), x = (1 -+ 1/sqrt 3)/2, components
x, y, z), with weight h^3/8 per point.  This rule is exact for the ND(T) mass.
"""
import numpy as np

from . import assemble, element, mesh


def _psi(a, t):
    return t if a == 1 else 1.0 - t


def _local_basis_values(pts):
    """(npts, 12, 3) values of the 12 local basis functions at local points."""
    out = np.zeros((pts.shape[0], 12, 3))
    for d in range(3):
        ea, eb = [ax for ax in range(3) if ax != d]
        for b in range(2):
            for a in range(2):
                out[:, element.local_edge(d, a, b), d] = _psi(a, pts[:, ea]) * _psi(b, pts[:, eb])
    return out


def gauss_rule(q):
    x, w = np.polynomial.legendre.leggauss(q)
    x = (x + 1.0) / 2.0
    w = w / 2.0
    g2, g1, g0 = np.meshgrid(x, x, x, indexing="ij")
    w2, w1, w0 = np.meshgrid(w, w, w, indexing="ij")
    pts = np.stack([g0.ravel(), g1.ravel(), g2.ravel()], 1)
    return pts, (w0 * w1 * w2).ravel()


def load_from_samples(n, h, f):
    """b from f sampled at the 2x2x2 Gauss points, f of shape [n^3, 8, 3] (or [..., n^3, 8, 3])."""
    f = np.asarray(f, dtype=np.float64)
    pts, w = gauss_rule(2)
    phi = _local_basis_values(pts)                       # (8, 12, 3)
    elem = np.einsum("...eqc,qlc,q->...el", f, phi, w) * h ** 3
    dofs = assemble.element_dofs(n)                      # (n^3, 12)
    N = mesh.ndof(n)
    lead = f.shape[:-3]
    elem = elem.reshape((-1,) + elem.shape[-2:])
    out = np.zeros((elem.shape[0], N))
    keep = dofs.ravel() >= 0
    for r in range(elem.shape[0]):
        out[r] = np.bincount(dofs.ravel()[keep], weights=elem[r].ravel()[keep], minlength=N)
    return out.reshape(lead + (N,))


def load_from_function(n, L, fun, q=5):
    """b for a smooth field fun(x, y, z) -> (fx, fy, fz) with q^3-point Gauss per element."""
    h = L / n
    pts, w = gauss_rule(q)
    phi = _local_basis_values(pts)
    c2, c1, c0 = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    corner = np.stack([c0.ravel(), c1.ravel(), c2.ravel()], 1) * h   # (n^3, 3)
    X = corner[:, None, :] + h * pts[None, :, :]
    F = np.stack(fun(X[..., 0], X[..., 1], X[..., 2]), -1)           # (n^3, npts, 3)
    elem = np.einsum("eqc,qlc,q->el", F, phi, w) * h ** 3
    dofs = assemble.element_dofs(n)
    keep = dofs.ravel() >= 0
    return np.bincount(dofs.ravel()[keep], weights=elem.ravel()[keep], minlength=mesh.ndof(n))


def interpolate(n, L, fun, q=8):
    """Edge averages lambda_e(u) (eq. NDdof) of a smooth field, by q-point Gauss on each edge."""
    h = L / n
    x, w = np.polynomial.legendre.leggauss(q)
    x = (x + 1.0) / 2.0
    w = w / 2.0
    d_all, p = mesh.edge_coords(n)
    out = np.zeros(d_all.shape[0])
    for d in range(3):
        sel = d_all == d
        base = p[sel].astype(np.float64) * h
        acc = np.zeros(sel.sum())
        for xi, wi in zip(x, w):
            pt = base.copy()
            pt[:, d] += xi * h
            acc += wi * np.stack(fun(pt[:, 0], pt[:, 1], pt[:, 2]), -1)[:, d]
        out[sel] = acc
    return out
