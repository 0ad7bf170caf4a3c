"""Preconditioned conjugate gradients with the V-cycle as preconditioner.

Not in the paper, which iterates the V-cycle itself; the V-cycle operator
B = MG(J, ., 0, m) is symmetric positive definite because R_k is a-symmetric and
E_k = I - B A is a-symmetric positive semidefinite (Sec. 4.2, Remark after eq.
RkDef) with norm below one (Theorem), so textbook PCG applies.

Start u_0 = 0, stop when ||b - A u_k||_2 <= rtol ||b||_2 using the recursively
updated residual.  ``flexible`` selects the Polak-Ribiere form
beta = z_{k+1}^T (r_{k+1} - r_k) / z_k^T r_k.
"""
import numpy as np


def pcg(A, b, precond, rtol=1e-10, maxit=500, flexible=False):
    """Returns (u, iterations, relres_recursive, history)."""
    b = np.asarray(b, dtype=np.float64)
    u = np.zeros_like(b)
    r = b.copy()
    bnorm = np.linalg.norm(b)
    hist = [1.0]
    if bnorm == 0.0:
        return u, 0, 0.0, hist
    z = precond(r)
    p = z.copy()
    rz = r @ z
    for it in range(1, maxit + 1):
        q = A @ p
        pq = p @ q
        if not (pq > 0.0) or not np.isfinite(pq):
            raise FloatingPointError("PCG breakdown: p^T A p <= 0")
        a = rz / pq
        u += a * p
        r_old = r.copy() if flexible else None
        r -= a * q
        rel = np.linalg.norm(r) / bnorm
        hist.append(rel)
        if rel <= rtol:
            return u, it, rel, hist
        z = precond(r)
        rz_new = r @ z
        beta = (z @ (r - r_old)) / rz if flexible else rz_new / rz
        rz = rz_new
        p = z + beta * p
    return u, maxit, hist[-1], hist
