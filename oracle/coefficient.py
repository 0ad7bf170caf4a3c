"""Coefficients with jumps (Sec. 6: the analysis assumes a constant alpha; jumps are
named there as the first extension).

alpha(x) = alpha * c(x) with c constant on each box of an r x r x r grid of boxes that
tile the cube, given as an array ``boxes[z][y][x]`` of positive values.  When r divides
the element count of the coarsest level, every element of every level, and so every
subdomain (an element of the next coarser level, Sec. 3.2), lies inside one box.  The
bilinear form of eq. (def bilinear form) becomes a(u, v) = sum_T (alpha_T (curl u,
curl v)_T + (u, v)_T), so the element-by-element assembly of eq. (fem) takes each
cube's own alpha_T, and with nested spaces the coarse form is the restriction of the
fine one (P^T A_k P = A_{k-1}, the property tests pin).

Vectors use the compact numbering of ``oracle.mesh``; cells are ordered (z, y, x) with x
fastest, as in ``assemble.element_dofs``.
"""
import numpy as np
import scipy.sparse as sp

from . import assemble, element, mesh


def cell_field(n, boxes):
    """[n, n, n] array ([z][y][x]) of the box values on the cells of an n^3 mesh."""
    boxes = np.asarray(boxes, dtype=np.float64)
    r = boxes.shape[0]
    if boxes.shape != (r, r, r) or n % r:
        raise ValueError("boxes must be r x r x r with r dividing n")
    w = n // r
    return np.repeat(np.repeat(np.repeat(boxes, w, axis=0), w, axis=1), w, axis=2)


def _assemble(n, Ke_scale, Me_scale, h):
    """sum_T (Ke_scale_T K_T + Me_scale M_T) over the n^3 cells."""
    K = element.curl_matrix(h)
    M = element.mass_matrix(h)
    dofs = assemble.element_dofs(n)
    a = np.asarray(Ke_scale, dtype=np.float64).reshape(-1)
    vals = (a[:, None] * K.ravel()[None, :] + Me_scale * M.ravel()[None, :]).ravel()
    rows = np.repeat(dofs, 12, axis=1).ravel()
    cols = np.tile(dofs, (1, 12)).ravel()
    keep = (rows >= 0) & (cols >= 0)
    N = mesh.ndof(n)
    return sp.csr_matrix((vals[keep], (rows[keep], cols[keep])), shape=(N, N))


def matrix_cells(n, h, alpha_cells):
    """A = sum_T (alpha_T K_T + M_T) with one alpha per cell ([n, n, n], [z][y][x])."""
    return _assemble(n, alpha_cells, 1.0, h)


def stiffness_cells(n, h, alpha_cells):
    """sum_T alpha_T K_T: the derivative of A with respect to a common factor of alpha."""
    return _assemble(n, alpha_cells, 0.0, h)


def level_matrices(sizes, L, alpha, boxes):
    """A_k of every level size in ``sizes`` for alpha(x) = alpha * boxes (r divides each)."""
    return [matrix_cells(nk, L / nk, alpha * cell_field(nk, boxes)) for nk in sizes]


def apply_rows(n, h, alpha_cells, x, rows, absolute=False):
    """Selected entries of A x, row by row from the element definition, for sizes where
    assembling A is too costly: (A x)_e sums, over the (at most four) cubes T holding edge
    e, alpha_T K_T + M_T's row of e's local edge times T's edge values.  absolute: the same
    sum of |alpha_T K_T + M_T| |x| instead, an upper bound of (|A| |x|)_e (the rounding
    scale of the row)."""
    K = element.curl_matrix(h)
    M = element.mass_matrix(h)
    if absolute:
        x = np.abs(x)
    ac = np.asarray(alpha_cells, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    d_all, p_all = mesh.edge_coords(n)
    d = d_all[rows]
    p = p_all[rows]
    x = np.asarray(x)
    out = np.zeros(rows.size)
    for b in range(2):
        for a in range(2):
            c = p.copy()
            for dd in range(3):
                ea, eb = [ax for ax in range(3) if ax != dd]
                m = d == dd
                c[m, ea] -= a
                c[m, eb] -= b
            inside = np.all((c >= 0) & (c < n), axis=1)
            cc = np.where(inside[:, None], c, 0)
            aT = ac[cc[:, 2], cc[:, 1], cc[:, 0]]
            vals = np.zeros((rows.size, 12))
            for dd in range(3):
                ea, eb = [ax for ax in range(3) if ax != dd]
                for bb in range(2):
                    for aa in range(2):
                        q = cc.copy()
                        q[:, ea] += aa
                        q[:, eb] += bb
                        idx = np.asarray(mesh.compact_index(n, dd, q[:, 0], q[:, 1], q[:, 2]))
                        ok = inside & (idx >= 0)
                        vals[ok, element.local_edge(dd, aa, bb)] = x[idx[ok]]
            loc = 4 * d + a + 2 * b
            row = aT[:, None] * K[loc] + M[loc]
            if absolute:
                row = np.abs(row)
            out += np.where(inside, np.einsum("ij,ij->i", row, vals), 0.0)
    return out
