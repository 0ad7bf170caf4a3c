"""Gradients of L = sum_k ||u_k - t_k||_2^2 with A(alpha) u_k = b_k.

A(alpha) = alpha K + M (eq. def bilinear form) is symmetric, so the adjoint system
uses the same operator: A lambda_k = 2 (u_k - t_k).  Then dL/db_k = lambda_k and
dL/dalpha = -sum_k lambda_k^T K u_k since dA/dalpha = K.
"""
import numpy as np

from . import assemble, exact


def loss_and_grads(n, L, alpha, B, T, solve=None, dtype=np.float64):
    """B, T: (nrhs, N) right-hand sides and targets.  Returns (L, dL/dB, dL/dalpha).

    dtype=np.longdouble takes the exact solves, the residual U - T and the curl-curl
    form in extended precision (results rounded to FP64).  A tracking loss against
    targets near U differences nearly equal vectors, and lambda = A^{-1} 2 (U - T)
    then amplifies the rounding of U in the smallest eigenmodes of A: at 96^3 with
    targets from alpha = 2, |U - T| is 6e-5 |U| and two FP64 routes to lambda differ by
    3e-5, so a 1e-6 reference for dL/dB needs the extra precision."""
    h = L / n
    if dtype != np.float64:
        U = exact.solve_fft(n, h, alpha, B, dtype)
        R = U - np.asarray(T, dtype=dtype)
        loss = np.sum(R * R)
        Lam = exact.solve_fft(n, h, alpha, 2 * R, dtype)
        KU = exact.apply_fft(n, h, 1.0, U, dtype, mass=0)
        return float(loss), Lam.astype(np.float64), -float(np.sum(Lam * KU))
    if solve is None:
        def solve(rhs):
            return exact.solve_fft(n, h, alpha, rhs)
    U = solve(B)
    R = U - T
    loss = float(np.sum(R * R))
    Lam = solve(2.0 * R)
    K = assemble.stiffness_kron(n, h)
    KU = (K @ U.T).T
    dalpha = -float(np.sum(Lam * KU))
    return loss, Lam, dalpha
