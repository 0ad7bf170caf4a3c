"""Gradients of L = sum_k ||u_k - t_k||_2^2 with A(alpha) u_k = b_k.

A(alpha) = alpha K + M (eq. def bilinear form) is symmetric, so the adjoint system
uses the same operator: A lambda_k = 2 (u_k - t_k).  Then dL/db_k = lambda_k and
dL/dalpha = -sum_k lambda_k^T K u_k since dA/dalpha = K.
"""
import numpy as np

from . import assemble, exact


def loss_and_grads(n, L, alpha, B, T, solve=None):
    """B, T: (nrhs, N) right-hand sides and targets.  Returns (L, dL/dB, dL/dalpha)."""
    h = L / n
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
