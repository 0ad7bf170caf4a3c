"""Pins of the oracle's non-box domains (``oracle.domain``; Sec. 6 names nonconvex
domains as an extension): Omega a union of boxes of an r x r x r grid.

* with every box kept, the hierarchy is the cube's, preconditioner for preconditioner;
* the unknowns are exactly the edges whose open segment lies inside Omega, found here by
  testing four points just off the edge's midpoint against the boxes (an independent
  geometric test of the cell rule);
* Galerkin identity P^T A P = A_coarse on Omega (nested spaces with zero trace on the
  boundary of Omega);
* the V-cycle is symmetric with contraction in [(8/9)^2, 1), and PCG reaches the sparse
  direct solution.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import contraction, domain, mesh, pcg, vcycle


def fichera():
    a = np.ones((2, 2, 2), dtype=bool)
    a[1, 1, 1] = False          # the octant x, y, z > 1/2 removed
    return a


def l_prism():
    a = np.ones((2, 2, 2), dtype=bool)
    a[:, 1, 1] = False          # an L-shaped cross-section extruded along z
    return a


def random_union(r, seed):
    rng = np.random.default_rng(seed)
    a = rng.random((r, r, r)) < 0.7
    a[0, 0, 0] = True
    return a


def test_all_boxes_is_the_cube():
    n = 8
    g = np.random.default_rng(0).standard_normal(mesh.ndof(n))
    H1 = vcycle.Hierarchy(n, 1.3, factored=False)
    H2 = vcycle.Hierarchy(n, 1.3, active=np.ones((2, 2, 2), dtype=bool))
    assert H2.A[-1].shape == H1.A[-1].shape
    assert abs(H2.A[-1] - H1.A[-1]).max() <= 1e-14 * abs(H1.A[-1]).max()
    z1, z2 = H1.precondition(g), H2.precondition(g)
    assert np.linalg.norm(z1 - z2) <= 1e-12 * np.linalg.norm(z1)


@pytest.mark.parametrize("n,active", [(8, fichera()), (8, l_prism()), (12, random_union(3, 1))])
def test_unknowns_are_edges_inside_omega(n, active):
    r = active.shape[0]
    w = n // r
    eps = 1e-3

    def inside(x):   # x in cell units; strictly inside an active box, and inside the cube
        if np.any(x <= 0) or np.any(x >= n):
            return False
        bx, by, bz = (np.floor(x / w)).astype(int)
        return bool(active[bz, by, bx])

    d_all, p_all = mesh.edge_coords(n)
    want = np.zeros(d_all.size, dtype=bool)
    for e in range(d_all.size):
        d, p = d_all[e], p_all[e].astype(float)
        mid = p.copy()
        mid[d] += 0.5
        ta, tb = [ax for ax in range(3) if ax != d]
        ok = True
        for sa in (-eps, eps):
            for sb in (-eps, eps):
                q = mid.copy()
                q[ta] += sa
                q[tb] += sb
                ok = ok and inside(q)
        want[e] = ok
    got = domain.unknown_mask(n, active)
    assert np.array_equal(got, want)
    assert 0 < got.sum() < d_all.size


@pytest.mark.parametrize("n,active", [(8, fichera()), (8, l_prism()), (16, fichera()), (12, random_union(3, 2))])
def test_galerkin_on_omega(n, active):
    H = vcycle.Hierarchy(n, 0.7, active=active)
    for k in range(1, len(H.sizes)):
        G = (H.P[k].T @ H.A[k] @ H.P[k]).tocsr()
        assert abs(G - H.A[k - 1]).max() <= 1e-13 * abs(H.A[k - 1]).max()


@pytest.mark.parametrize("active", [fichera(), l_prism()])
def test_vcycle_on_omega(active):
    n = 8
    H = vcycle.Hierarchy(n, 1.0, active=active)
    N = H.A[-1].shape[0]
    B = np.column_stack([H.precondition(e) for e in np.eye(N)])
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    c, _ = contraction.contraction_dense(H)
    assert (8.0 / 9.0) ** 2 - 1e-10 <= c < 1.0


@pytest.mark.parametrize("n,active", [(8, fichera()), (16, fichera()), (16, l_prism())])
def test_pcg_on_omega_reaches_direct_solution(n, active):
    H = vcycle.Hierarchy(n, 1.0, active=active)
    A = H.A[-1]
    b = np.random.default_rng(4).standard_normal(A.shape[0])
    u, it, _, _ = pcg.pcg(A, b, H.precondition, rtol=1e-12)
    ue = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(u - ue) <= 1e-9 * np.linalg.norm(ue)
    assert it <= 40
