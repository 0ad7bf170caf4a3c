"""Global matrices A_h = alpha K + M of eq. (fem), assembled two independent ways.

(i) Kronecker form.  With D the (n x (n-1)) node-to-cell difference (Dirichlet
nodes removed), T = tridiag(1/6, 2/3, 1/6) the 1-D hat mass / h on interior nodes
and I the identity on cells, the discrete curl of an edge vector is the face
circulation C u (right-hand rule, divided by h):
    F_x = D_y u_z - D_z u_y,  F_y = D_z u_x - D_x u_z,  F_z = D_x u_y - D_y u_x,
the face (Raviart-Thomas) mass is T along each face normal, the edge mass is T (x) T
across each edge direction, and
    K = h C^T M_F C,   M = h^3 M_E,   A = alpha K + M.
(ii) Element by element from the 12x12 matrices of ``oracle.element``.

Vectors use the compact numbering of ``oracle.mesh``.
"""
import numpy as np
import scipy.sparse as sp

from . import element, mesh


def _D(n):
    """(n x (n-1)) map from interior node values to cell differences phi_{c+1} - phi_c."""
    D = sp.lil_matrix((n, n - 1))
    for c in range(n):
        if c + 1 <= n - 1:
            D[c, c] = 1.0          # node c+1 -> column c
        if c >= 1:
            D[c, c - 1] = -1.0     # node c   -> column c-1
    return D.tocsr()


def _T(n):
    """Tridiagonal 1-D hat-function mass (divided by h) on the n-1 interior nodes."""
    m = n - 1
    return sp.diags([np.full(m - 1, 1 / 6), np.full(m, 2 / 3), np.full(m - 1, 1 / 6)],
                    [-1, 0, 1], format="csr")


def _kron3(az, ay, ax):
    return sp.kron(az, sp.kron(ay, ax, format="csr"), format="csr")


def curl_operator(n):
    """Integer face-circulation matrix C (faces x edges) and face mass M_F."""
    D, Ic, In = _D(n), sp.identity(n, format="csr"), sp.identity(n - 1, format="csr")
    T = _T(n)
    Z = None
    # face blocks: x-faces (z cell, y cell, x node), y-faces (z cell, y node, x cell),
    #              z-faces (z node, y cell, x cell)
    Cx = [Z, -_kron3(D, Ic, In), _kron3(Ic, D, In)]            # -D_z u_y + D_y u_z
    Cy = [_kron3(D, In, Ic), Z, -_kron3(Ic, In, D)]            #  D_z u_x - D_x u_z
    Cz = [-_kron3(In, D, Ic), _kron3(In, Ic, D), Z]            # -D_y u_x + D_x u_y
    C = sp.bmat([Cx, Cy, Cz], format="csr")
    MF = sp.block_diag([_kron3(Ic, Ic, T), _kron3(Ic, T, Ic), _kron3(T, Ic, Ic)], format="csr")
    return C, MF


def edge_mass_kron(n):
    """M_E with M = h^3 M_E: T (x) T across each edge direction."""
    Ic, T = sp.identity(n, format="csr"), _T(n)
    return sp.block_diag([_kron3(T, T, Ic), _kron3(T, Ic, T), _kron3(Ic, T, T)], format="csr")


def stiffness_kron(n, h):
    """K = h C^T M_F C (curl-curl part, the derivative of A with respect to alpha)."""
    C, MF = curl_operator(n)
    return (h * (C.T @ MF @ C)).tocsr()


def mass_kron(n, h):
    return (h ** 3 * edge_mass_kron(n)).tocsr()


def matrix_kron(n, h, alpha):
    """A = alpha K + M in Kronecker form."""
    return (alpha * stiffness_kron(n, h) + mass_kron(n, h)).tocsr()


def element_dofs(n):
    """(n^3, 12) compact indices of the 12 edges of every element (-1 on the boundary)."""
    c2, c1, c0 = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    c = [c0.ravel(), c1.ravel(), c2.ravel()]
    out = np.empty((c0.size, 12), dtype=np.int64)
    for d in range(3):
        ea, eb = [ax for ax in range(3) if ax != d]
        for b in range(2):
            for a in range(2):
                p = [c[0].copy(), c[1].copy(), c[2].copy()]
                p[ea] = p[ea] + a
                p[eb] = p[eb] + b
                out[:, element.local_edge(d, a, b)] = mesh.compact_index(n, d, *p)
    return out


def matrix_elementwise(n, h, alpha):
    """A assembled element by element from the 12x12 element matrix."""
    Ae = element.element_matrix(h, alpha)
    dofs = element_dofs(n)
    rows = np.repeat(dofs, 12, axis=1).ravel()
    cols = np.tile(dofs, (1, 12)).ravel()
    vals = np.tile(Ae.ravel(), dofs.shape[0])
    keep = (rows >= 0) & (cols >= 0)
    N = mesh.ndof(n)
    return sp.csr_matrix((vals[keep], (rows[keep], cols[keep])), shape=(N, N))


def gradient(n, h):
    """Discrete gradient G of interior nodal values (Lagrange space W_h, Sec. 4).

    Edge average of the tangential derivative of a Q1 function: (phi_b - phi_a) / h.
    Interior nodes are ordered [z][y][x] over 1..n-1.
    """
    D, In, Ic = _D(n), sp.identity(n - 1, format="csr"), sp.identity(n, format="csr")
    del Ic
    Gx = _kron3(In, In, D)
    Gy = _kron3(In, D, In)
    Gz = _kron3(D, In, In)
    return (sp.vstack([Gx, Gy, Gz], format="csr") / h).tocsr()


def apply_rows(n, h, alpha, x, rows):
    """Selected entries of A x by the element definition: (A x)_e is the sum, over the
    (at most four) cubes T that contain edge e, of the row of the element matrix for e's
    local edge times T's edge values (boundary edges contribute zero).  For sizes where
    assembling A is too costly; ``rows`` are compact indices."""
    Ae = element.element_matrix(h, alpha)
    rows = np.asarray(rows, dtype=np.int64)
    d_all, p_all = mesh.edge_coords(n)
    d = d_all[rows]
    p = p_all[rows]
    x = np.asarray(x)
    out = np.zeros(rows.size)
    for b in range(2):
        for a in range(2):
            # the cube in which e is the local edge (d, a, b): its lower node is e's node
            # minus a along the first and b along the second transverse axis
            c = p.copy()
            for dd in range(3):
                ea, eb = [ax for ax in range(3) if ax != dd]
                m = d == dd
                c[m, ea] -= a
                c[m, eb] -= b
            inside = np.all((c >= 0) & (c < n), axis=1)
            vals = np.zeros((rows.size, 12))
            for dd in range(3):
                ea, eb = [ax for ax in range(3) if ax != dd]
                for bb in range(2):
                    for aa in range(2):
                        q = c.copy()
                        q[:, ea] += aa
                        q[:, eb] += bb
                        q = np.where(inside[:, None], q, 0)
                        idx = np.asarray(mesh.compact_index(n, dd, q[:, 0], q[:, 1], q[:, 2]))
                        ok = inside & (idx >= 0)
                        vals[ok, element.local_edge(dd, aa, bb)] = x[idx[ok]]
            loc = 4 * d + a + 2 * b
            out += np.where(inside, np.einsum("ij,ij->i", Ae[loc], vals), 0.0)
    return out
