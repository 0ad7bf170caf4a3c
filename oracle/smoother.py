"""Nonoverlapping substructuring smoothers (Sec. 3.2).

Vertex-based smoother, eq. (Preconditioner P):
    M_V^{-1} = eta_V ( sum_T J_T A_T^{-1} J_T^t + sum_V J_V A_V^{-1} J_V^t ),
edge-based smoother, eq. (Preconditioner E): the same with the edge spaces N_h^E.

* N_h^T (eq. SubdomainSpace): fine fields supported in coarse element T, i.e. spanned
  by the basis functions of the edges strictly inside T.  A_T (eq. ATDef) is the
  principal submatrix of A on those edges.
* N_h^V (eq. vertex space): fields that are free on the interface edges Gamma_V
  (interiors of the 12 coarse faces and the 6 coarse edges through V), zero on every
  other edge outside the 8 elements around V, and a-orthogonal to the interior
  spaces of those 8 elements.  A basis is Phi_V = [I ; -A_pp^{-1} A_p,Gamma] (the
  discrete-harmonic extension into the patch interior p), and in that basis
  J_V A_V^{-1} J_V^t = Phi_V (Phi_V^T A Phi_V)^{-1} Phi_V^T (eq. AVDef).
* N_h^E (eq. edge space): the same with the 4 faces and 4 elements around coarse
  edge E.

``LiteralSmoother`` builds every patch separately from the assembled A and assumes
nothing about translation invariance.  ``FactoredVertexSmoother`` evaluates the same
operator through a global condensation: z_I = A_II^{-1} r_I, g = r - A z_I,
y_V = S_V^{-1} g|Gamma_V with one Schur complement S_V per level, w = sum_V R_V^T y_V,
w_I = -A_II^{-1} (A w)_I, M^{-1} r = eta (z_I + w_I + w).  The two agree because
A_II is block diagonal over coarse elements and every coupling of a Gamma_V edge to
interior edges stays inside the patch of V.
"""
import numpy as np
import scipy.linalg as sla

from . import mesh


def _sub(A, rows, cols):
    return A[rows][:, cols].toarray()


class LiteralSmoother:
    """M^{-1} for kind='vertex' (eta defaults to 1/9) or kind='edge' (eta 1/13)."""

    def __init__(self, A, n, s=2, kind="vertex", eta=None, damp_interior=True, boundary=True,
                 inverse="lu", keep=None):
        """inverse: 'lu' (LAPACK solves and inverses) or 'cholesky' (Cholesky solves and
        inverses); two FP64 routes to the same local matrices whose difference measures how
        far rounding in the setup moves the result.  keep: for a domain inside the cube
        (``oracle.domain``), the cube's unknowns that are Omega's; A is then Omega's matrix
        and every set is the cube's set intersected with them (empty sets are dropped)."""
        if n % s or n // s < 2:
            raise ValueError("need n divisible by s with at least 2 subdomains per axis")
        self.A, self.n, self.s, self.kind = A.tocsr(), n, s, kind
        if inverse == "cholesky":
            self._inv = lambda M: sla.cho_solve(sla.cho_factor(M), np.eye(M.shape[0]))
            self._solve = lambda M, B: sla.cho_solve(sla.cho_factor(M), B)
        else:
            self._inv = np.linalg.inv
            self._solve = np.linalg.solve
        self.eta = eta if eta is not None else (1.0 / 9.0 if kind == "vertex" else 1.0 / 13.0)
        self.damp_interior = damp_interior
        if keep is None:
            to_local = lambda ix: np.asarray(ix)
        else:
            pos = np.full(len(keep), -1)
            pos[np.asarray(keep)] = np.arange(int(np.count_nonzero(keep)))

            def to_local(ix):
                q = pos[np.asarray(ix, dtype=np.int64)]
                return q[q >= 0]
        self.T = []
        self.Iof = {}
        for t in mesh.coarse_elements(n, s):
            I = to_local(mesh.interior_set(n, s, t))
            self.Iof[t] = I
            if len(I):
                self.T.append((I, self._inv(_sub(self.A, I, I))))
        self.P = []
        if kind == "vertex":
            for v in mesh.coarse_vertices(n, s, boundary):
                G = to_local(mesh.vertex_interface_set(n, s, v))
                if len(G):
                    self.P.append(self._patch(G, mesh.patch_elements(n, s, v)))
        elif kind == "edge":
            for axis, c in mesh.coarse_edges(n, s, boundary):
                G = to_local(mesh.edge_interface_set(n, s, axis, c))
                if len(G):
                    self.P.append(self._patch(G, mesh.edge_patch_elements(n, s, axis, c)))
        else:
            raise ValueError(kind)

    def _patch(self, G, elems):
        Ip = np.sort(np.concatenate([self.Iof[t] for t in elems]))
        ext = -self._solve(_sub(self.A, Ip, Ip), _sub(self.A, Ip, G))
        idx = np.concatenate([G, Ip])
        Phi = np.vstack([np.eye(len(G)), ext])           # rows follow idx
        # A_V = Phi^T A Phi with A restricted to idx (Phi vanishes elsewhere)
        Aloc = _sub(self.A, idx, idx)
        AV = Phi.T @ Aloc @ Phi
        AV = 0.5 * (AV + AV.T)
        return idx, Phi, self._inv(AV), AV

    def patch_matrices(self):
        """A_V (or A_E) of every patch, in the order of the sorted interface indices."""
        return [p[3] for p in self.P]

    def interior_matrices(self):
        return [np.linalg.inv(Ainv) for _, Ainv in self.T]

    def apply(self, r):
        r = np.asarray(r, dtype=np.float64)
        zi = np.zeros_like(r)
        for I, Ainv in self.T:
            zi[I] += Ainv @ r[I]
        zp = np.zeros_like(r)
        for idx, Phi, AVinv, _ in self.P:
            zp[idx] += Phi @ (AVinv @ (Phi.T @ r[idx]))
        if self.damp_interior:
            return self.eta * (zi + zp)
        return zi + self.eta * zp

    __call__ = apply


class FactoredVertexSmoother:
    """The vertex smoother through global condensation.

    One Schur complement S_V per vertex type (interior, or which faces of the box the
    vertex lies on), taken from the first patch of that type.
    """

    def __init__(self, A, n, s=2, eta=1.0 / 9.0, boundary=True, inverse="lu"):
        """inverse: 'lu' (numpy inverse, LAPACK solve for the Schur complement) or
        'cholesky' (explicit Cholesky inverses); two FP64 routes to the same factors whose
        difference measures how far rounding in the setup moves the result."""
        if n % s or n // s < 2:
            raise ValueError("need n divisible by s with at least 2 subdomains per axis")
        self.A, self.n, self.s, self.eta = A.tocsr(), n, s, eta
        self.Iidx = mesh.interior_sets(n, s)
        I0 = self.Iidx[0]
        self.AT = _sub(self.A, I0, I0)

        def inv(M):
            if inverse == "cholesky":
                return sla.cho_solve(sla.cho_factor(M), np.eye(M.shape[0]))
            return np.linalg.inv(M)

        self.ATinv = inv(self.AT)
        groups = {}
        for v in mesh.coarse_vertices(n, s, boundary):
            groups.setdefault(mesh.vertex_type(n, s, v), []).append(v)
        self.groups = []
        for typ in sorted(groups):
            verts = groups[typ]
            Gidx = mesh.vertex_interface_sets(n, s, verts)
            v0 = verts[0]
            G0 = Gidx[0]
            Ip = np.sort(np.concatenate([mesh.interior_set(n, s, t)
                                         for t in mesh.patch_elements(n, s, v0)]))
            App = _sub(self.A, Ip, Ip)
            ApG = _sub(self.A, Ip, G0)
            if inverse == "cholesky":
                X = inv(App) @ ApG
            else:
                X = np.linalg.solve(App, ApG)
            S = _sub(self.A, G0, G0) - ApG.T @ X
            self.groups.append((typ, Gidx, S, inv(S)))

    def schur(self, typ=13):
        for t, _, S, _ in self.groups:
            if t == typ:
                return S
        raise KeyError(typ)

    def apply(self, r):
        r = np.asarray(r, dtype=np.float64)
        N = r.shape[0]
        # interior solves z_I = A_II^{-1} r_I
        zi = np.zeros_like(r)
        zi[self.Iidx] = np.einsum("ij,tj...->ti...", self.ATinv, r[self.Iidx])
        # condensed interface residual g = r - A z_I  (zero on interior rows)
        g = r - self.A @ zi
        # vertex patch solves and the scatter-sum w = sum_V R_V^T S_V^{-1} R_V g
        w = np.zeros_like(r)
        for _, Gidx, _, Sinv in self.groups:
            y = np.einsum("ij,vj...->vi...", Sinv, g[Gidx])
            flat = Gidx.ravel()
            if r.ndim == 1:
                w += np.bincount(flat, weights=y.reshape(-1), minlength=N)
            else:
                yy = y.reshape(-1, r.shape[1])
                for c in range(r.shape[1]):
                    w[:, c] += np.bincount(flat, weights=yy[:, c], minlength=N)
        # discrete-harmonic extension into the subdomain interiors
        q = self.A @ w
        wi = np.zeros_like(r)
        wi[self.Iidx] = -np.einsum("ij,tj...->ti...", self.ATinv, q[self.Iidx])
        return self.eta * (zi + wi + w)

    __call__ = apply
