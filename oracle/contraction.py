"""Contraction number of the V-cycle (Sec. 5, Tables 1-2).

The error propagation operator is E_k = I - B_k A_k with B_k g = MG(k, g, 0, m)
(Sec. 4.2, eq. VCycleRecursion).  E_k is a-symmetric positive semidefinite (Remark
after eq. RkDef), so ||E_k||_a is its largest eigenvalue, i.e. one minus the
smallest eigenvalue of the generalized problem (A B A) x = lambda A x.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import exact


def dense_preconditioner(H):
    """B = MG(J, ., 0, m) as a dense matrix (columns are V-cycles of unit vectors)."""
    N = H.A[-1].shape[0]
    return H.mg(H.J, np.eye(N))


def contraction_dense(H):
    A = H.A[-1].toarray()
    B = dense_preconditioner(H)
    B = 0.5 * (B + B.T)
    lam = sla.eigh(A @ B @ A, A, eigvals_only=True)
    return 1.0 - lam.min(), lam


def contraction_lanczos(H, tol=1e-8):
    """||E_J||_a by Lanczos on the a-self-adjoint E = I - B A (large levels)."""
    A = H.A[-1]
    n = H.sizes[-1]
    h = H.L / n
    N = A.shape[0]
    AE = spla.LinearOperator((N, N), matvec=lambda x: A @ x - A @ H.precondition(A @ x),
                             dtype=np.float64)
    Minv = spla.LinearOperator((N, N), matvec=lambda x: exact.solve_fft(n, h, H.alpha, x),
                               dtype=np.float64)
    vals = spla.eigsh(AE, k=1, M=A, Minv=Minv, which="LA", tol=tol,
                      return_eigenvectors=False)
    return float(vals.max())
