"""Symmetric V-cycle multigrid MG(k, g, z0, m) (Sec. 3.3, Fig. 1).

Level k = 0 is solved exactly.  For k >= 1: m smoothing steps
z_l = z_{l-1} + M_k^{-1}(g - A_k z_{l-1}), restriction of the residual with
I_k^{k-1}, a coarse correction with MG(k-1, gbar, 0, m) prolongated by I_{k-1}^k,
and m more smoothing steps.  Every level is the same problem rediscretised on the
refined mesh (Sec. 3.1, eq. kthEq).
"""
import numpy as np
import scipy.linalg as sla

from . import assemble, coefficient, domain, mesh, smoother as sm, transfer


class Hierarchy:
    """All levels of the V-cycle for n elements per axis on a cube of side L."""

    def __init__(self, n, alpha, L=1.0, s=2, m=1, kind="vertex", eta=None,
                 factored=None, damp_interior=True, boundary=True, inverse="lu", levels=None,
                 boxes=None, active=None):
        """levels: keep only that many levels from the finest down (the coarsest kept
        level is then solved exactly, k = 0 of Fig. 1); None keeps all of them.
        boxes: alpha(x) = alpha * boxes[z][y][x] on an r x r x r grid of boxes (r divides
        the coarsest kept level), every level assembled cell by cell
        (``oracle.coefficient``) and smoothed by the literal smoother; None: constant.
        active: Omega as the boxes of an r x r x r grid that it keeps (``oracle.domain``):
        every level restricted to Omega's unknowns, the literal smoother on its sets."""
        self.sizes = mesh.level_sizes(n)          # coarsest first
        if levels is not None:
            if not 1 <= levels <= len(self.sizes):
                raise ValueError("levels out of range")
            self.sizes = self.sizes[len(self.sizes) - levels:]
        self.alpha, self.L, self.m, self.boxes, self.active = alpha, L, m, boxes, active
        if (boxes is not None or active is not None) and factored:
            raise ValueError("the factored smoother assumes one alpha for every subdomain of the cube")
        self.A, self.M, self.P, self.R = [], [], [None], []
        for k, nk in enumerate(self.sizes):
            h = L / nk
            if boxes is None and active is None:
                A = assemble.matrix_kron(nk, h, alpha)
            else:
                cf = np.ones((1, 1, 1)) if boxes is None else boxes
                A = coefficient.matrix_cells(nk, h, alpha * coefficient.cell_field(nk, cf))
            keep = None
            if active is not None:
                keep = domain.unknown_mask(nk, active)
                Rk = domain.restriction(nk, active)
                A = (Rk @ A @ Rk.T).tocsr()
                self.R.append(Rk)
            self.A.append(A)
            if k == 0:
                self.M.append(None)
                self.coarse_chol = sla.cho_factor(A.toarray())
                continue
            sk = min(s, nk // 2)
            if nk % sk:
                raise ValueError(f"level with {nk} elements is not divisible by {sk}")
            use_f = (factored if factored is not None else (nk >= 24)) and boxes is None and active is None
            if kind == "vertex" and use_f and damp_interior:
                e = 1.0 / 9.0 if eta is None else eta
                self.M.append(sm.FactoredVertexSmoother(A, nk, sk, e, boundary, inverse))
            else:
                self.M.append(sm.LiteralSmoother(A, nk, sk, kind, eta, damp_interior, boundary, inverse, keep))
            P = transfer.prolongation(self.sizes[k - 1])
            if active is not None:
                P = (self.R[k] @ P @ self.R[k - 1].T).tocsr()
            self.P.append(P)

    @property
    def J(self):
        return len(self.sizes) - 1

    def mg(self, k, g, z0=None, m=None):
        """MG(k, g, z0, m) of Fig. 1."""
        m = self.m if m is None else m
        if k == 0:
            return sla.cho_solve(self.coarse_chol, g)
        A, Minv, P = self.A[k], self.M[k], self.P[k]
        z = np.zeros_like(g) if z0 is None else np.array(z0, dtype=np.float64)
        for _ in range(m):
            z = z + Minv(g - A @ z)
        gbar = P.T @ (g - A @ z)
        z = z + P @ self.mg(k - 1, gbar, None, m)
        for _ in range(m):
            z = z + Minv(g - A @ z)
        return z

    def precondition(self, g):
        """B g = MG(J, g, 0, m): the V-cycle used as a preconditioner."""
        return self.mg(self.J, np.asarray(g, dtype=np.float64))
