"""Non-box domains (Sec. 6: the analysis assumes a convex domain; the paper names
nonconvex domains as an extension): Omega a union of boxes of an r x r x r grid of boxes
tiling the cube, given as a boolean array ``active[z][y][x]`` (for instance the cube with
one octant removed, a Fichera corner).

With r dividing the coarsest level, every element of every level lies in Omega or outside
it.  The Nedelec space on Omega with zero tangential trace on its boundary has one
unknown per edge of the mesh whose open segment lies in the interior of Omega: an edge
whose (up to four) surrounding cells are all in Omega.  Its matrix is the cube's matrix
restricted to those edges (the rows and columns of an interior edge only involve the
cells around it), the transfers are the cube's restricted the same way (a coarse field
with zero trace on the boundary of Omega is one on the fine mesh), and the smoother's
sets are the cube's sets intersected with the unknowns of Omega.

Vectors of Omega are numbered by the cube's compact numbering (``oracle.mesh``) with the
edges outside Omega left out, in order.
"""
import numpy as np
import scipy.sparse as sp

from . import coefficient, mesh


def cell_active(n, active):
    """[n, n, n] booleans ([z][y][x]) of the cells of an n^3 mesh inside Omega."""
    a = np.asarray(active, dtype=bool)
    return coefficient.cell_field(n, a.astype(np.float64)) > 0.5


def unknown_mask(n, active):
    """Boolean over the cube's unknowns (compact order): the edge's surrounding cells are
    all in Omega."""
    cells = cell_active(n, active)
    d, p = mesh.edge_coords(n)
    keep = np.ones(d.size, dtype=bool)
    for b in range(2):
        for a in range(2):
            c = p.copy()
            for dd in range(3):
                ea, eb = [ax for ax in range(3) if ax != dd]
                m = d == dd
                c[m, ea] -= a
                c[m, eb] -= b
            keep &= cells[c[:, 2], c[:, 1], c[:, 0]]
    return keep


def restriction(n, active):
    """R (unknowns of Omega x unknowns of the cube) selecting Omega's unknowns."""
    keep = np.flatnonzero(unknown_mask(n, active))
    return sp.csr_matrix((np.ones(keep.size), (np.arange(keep.size), keep)), shape=(keep.size, mesh.ndof(n)))


def matrix(n, h, alpha_cells, active):
    """A on Omega: the cube's cell-by-cell matrix restricted to Omega's unknowns."""
    R = restriction(n, active)
    return (R @ coefficient.matrix_cells(n, h, alpha_cells) @ R.T).tocsr()
