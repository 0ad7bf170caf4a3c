"""Grid transfers (Sec. 3.1, eq. F2C).

The Nedelec spaces are nested, so the coarse-to-fine operator I_{k-1}^k is the
natural injection: a coarse basis function written in fine basis functions.  Along
the edge direction a coarse cell indicator is the sum of the two fine cell
indicators (weights 1, 1); across it a coarse hat function is the fine hat at the
same node plus half of each neighbouring fine hat (weights 1/2, 1, 1/2).  The
fine-to-coarse operator I_k^{k-1} is the transpose (eq. F2C).
"""
import scipy.sparse as sp


def _P0(nc):
    """Cells: coarse cell c -> fine cells 2c, 2c+1 with weight 1."""
    P = sp.lil_matrix((2 * nc, nc))
    for c in range(nc):
        P[2 * c, c] = 1.0
        P[2 * c + 1, c] = 1.0
    return P.tocsr()


def _P1(nc):
    """Interior nodes: coarse node C (1..nc-1) -> fine node 2C (1) and 2C +- 1 (1/2)."""
    P = sp.lil_matrix((2 * nc - 1, nc - 1))
    for C in range(1, nc):
        P[2 * C - 1, C - 1] = 1.0
        P[2 * C - 2, C - 1] = 0.5
        P[2 * C, C - 1] = 0.5
    return P.tocsr()


def prolongation(nc):
    """I_{k-1}^k from the level with nc elements per axis to the level with 2 nc."""
    P0, P1 = _P0(nc), _P1(nc)

    def k3(az, ay, ax):
        return sp.kron(az, sp.kron(ay, ax))

    return sp.block_diag([k3(P1, P1, P0), k3(P1, P0, P1), k3(P0, P1, P1)], format="csr")


def restriction(nc):
    """I_k^{k-1} = (I_{k-1}^k)^T (eq. F2C)."""
    return prolongation(nc).T.tocsr()
