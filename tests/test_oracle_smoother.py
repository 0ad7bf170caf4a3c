"""Pins of the substructuring smoothers (Sec. 3.2) and their index sets."""
import numpy as np
import pytest

from oracle import assemble, element, mesh, smoother


def _dense(S, N):
    return S(np.eye(N))


@pytest.mark.parametrize("s,nI,nGV,nGE", [(2, 6, 60, 18), (4, 108, 312, 100)])
def test_set_sizes(s, nI, nGV, nGE):
    n = 3 * s
    assert len(mesh.interior_set(n, s, (1, 1, 1))) == nI == 3 * s * (s - 1) ** 2
    assert len(mesh.vertex_interface_set(n, s, (1, 1, 1))) == nGV == 6 * s + 24 * s * (s - 1)
    assert len(mesh.edge_interface_set(n, s, 0, (0, s, s))) == nGE == s + 8 * s * (s - 1)


@pytest.mark.parametrize("s", [2, 4])
def test_partition_and_coverage(s):
    """Interiors are disjoint; with boundary patches every face-interior unknown lies in
    exactly 4 vertex sets and every unknown on a coarse edge in exactly 2."""
    n = 3 * s
    N = mesh.ndof(n)
    cover_I = np.zeros(N, int)
    for t in mesh.coarse_elements(n, s):
        cover_I[mesh.interior_set(n, s, t)] += 1
    cover_V = np.zeros(N, int)
    for v in mesh.coarse_vertices(n, s, boundary=True):
        cover_V[mesh.vertex_interface_set(n, s, v)] += 1
    d, p = mesh.edge_coords(n)
    trans = np.stack([p[np.arange(N), (d + 1) % 3], p[np.arange(N), (d + 2) % 3]], 1)
    on = (trans % s == 0).sum(1)          # 0: interior, 1: face interior, 2: coarse edge
    assert np.all(cover_I[on == 0] == 1) and np.all(cover_I[on > 0] == 0)
    assert np.all(cover_V[on == 0] == 0)
    assert np.all(cover_V[on == 1] == 4)
    assert np.all(cover_V[on == 2] == 2)


@pytest.mark.parametrize("n,boundary", [(4, True), (8, True), (8, False), (12, True)])
def test_literal_equals_factored(n, boundary):
    A = assemble.matrix_kron(n, 1.0 / n, 0.3)
    r = np.random.default_rng(n).standard_normal((A.shape[0], 2))
    a = smoother.LiteralSmoother(A, n, boundary=boundary)(r)
    b = smoother.FactoredVertexSmoother(A, n, boundary=boundary)(r)
    assert abs(a - b).max() <= 1e-13 * abs(a).max()


def test_factored_s4_equals_literal():
    n = 8
    A = assemble.matrix_kron(n, 1.0 / n, 2.0)
    r = np.random.default_rng(0).standard_normal(A.shape[0])
    a = smoother.LiteralSmoother(A, n, s=4)(r)
    b = smoother.FactoredVertexSmoother(A, n, s=4)(r)
    assert abs(a - b).max() <= 1e-12 * abs(a).max()


@pytest.mark.parametrize("kind,eta,bound", [("vertex", 1 / 9, 1 / 8), ("edge", 1 / 13, 1 / 12)])
@pytest.mark.parametrize("boundary", [True, False])
def test_symmetry_and_spectral_condition(kind, eta, bound, boundary):
    """M^{-1} is symmetric and the spectrum of M^{-1} A lies in (0, 1] for eta at the
    bound of Sec. 3.2 (eta_V <= 1/8, eta_E <= 1/12)."""
    n = 6
    A = assemble.matrix_kron(n, 1.0 / n, 1.0)
    N = A.shape[0]
    for e in (eta, bound):
        Mi = _dense(smoother.LiteralSmoother(A, n, kind=kind, eta=e, boundary=boundary), N)
        assert abs(Mi - Mi.T).max() <= 1e-13 * abs(Mi).max()
        lam = np.linalg.eigvals(Mi @ A.toarray()).real
        assert lam.min() > 0 and lam.max() <= 1 + 1e-10


@pytest.mark.parametrize("kind", ["vertex", "edge"])
def test_bubbles_scaled_by_eta(kind):
    n = 6
    A = assemble.matrix_kron(n, 1.0 / n, 5.0)
    S = smoother.LiteralSmoother(A, n, kind=kind)
    w = np.zeros(A.shape[0])
    I = mesh.interior_set(n, 2, (1, 0, 2))
    w[I] = np.random.default_rng(1).standard_normal(len(I))
    np.testing.assert_allclose(S(A @ w), S.eta * w, atol=1e-13 * abs(w).max())


def _coarse_element_energy(n, h, alpha, t, s):
    """a_T restricted to the fine elements of coarse element t (assembled locally)."""
    Ae = element.element_matrix(h, alpha)
    dofs = assemble.element_dofs(n)
    N = mesh.ndof(n)
    out = np.zeros((N, N))
    for c2 in range(s * t[2], s * t[2] + s):
        for c1 in range(s * t[1], s * t[1] + s):
            for c0 in range(s * t[0], s * t[0] + s):
                e = dofs[(c2 * n + c1) * n + c0]
                for i in range(12):
                    for j in range(12):
                        if e[i] >= 0 and e[j] >= 0:
                            out[e[i], e[j]] += Ae[i, j]
    return out


def test_minimum_energy_vertex():
    """eq. MinimumEnergyV: the discrete-harmonic field has the least energy on each
    element of the patch among fields with the same interface values."""
    n, s, alpha = 4, 2, 0.8
    h = 1.0 / n
    A = assemble.matrix_kron(n, h, alpha)
    S = smoother.LiteralSmoother(A, n)
    idx, Phi, _, _ = S.P[0]
    nG = Phi.shape[1]
    rng = np.random.default_rng(3)
    v = np.zeros(A.shape[0])
    v[idx] = Phi @ rng.standard_normal(nG)
    # a-orthogonal to every bubble of the patch (harmonic)
    for t in mesh.patch_elements(n, s, (1, 1, 1)):
        I = mesh.interior_set(n, s, t)
        assert abs((A @ v)[I]).max() <= 1e-13 * abs(A @ v).max()
    for t in mesh.patch_elements(n, s, (1, 1, 1)):
        aT = _coarse_element_energy(n, h, alpha, t, s)
        for _ in range(3):
            w = v.copy()
            I = mesh.interior_set(n, s, t)
            w[I] += rng.standard_normal(len(I))
            assert v @ aT @ v <= w @ aT @ w + 1e-14


def test_patch_matrices_translation_invariant():
    """All patches of one vertex type have the same A_V (the GPU stores one per type)."""
    n = 10
    A = assemble.matrix_kron(n, 1.0 / n, 0.5)
    S = smoother.LiteralSmoother(A, n)
    by_type = {}
    for v, AV in zip(mesh.coarse_vertices(n, 2), S.patch_matrices()):
        by_type.setdefault(mesh.vertex_type(n, 2, v), []).append(AV)
    assert len(by_type) == 19
    for mats in by_type.values():
        for M in mats[1:]:
            assert abs(M - mats[0]).max() <= 1e-14 * abs(mats[0]).max()


@pytest.mark.parametrize("n,s", [(8, 2), (12, 2), (8, 4)])
def test_vectorized_sets_equal_per_item_sets(n, s):
    I = mesh.interior_sets(n, s)
    I2 = np.stack([mesh.interior_set(n, s, t) for t in mesh.coarse_elements(n, s)])
    assert np.array_equal(I, I2)
    groups = {}
    for v in mesh.coarse_vertices(n, s):
        groups.setdefault(mesh.vertex_type(n, s, v), []).append(v)
    for verts in groups.values():
        G = mesh.vertex_interface_sets(n, s, verts)
        G2 = np.stack([mesh.vertex_interface_set(n, s, v) for v in verts])
        assert np.array_equal(G, G2)


def _edge_geometry(n):
    """Compact indices with the doubled coordinates of each unknown's midpoint (2 p, with
    the cell axis at 2 p + 1), so that every geometric test below is on integers."""
    d, p = mesh.edge_coords(n)
    mid = 2 * p.astype(np.int64)
    mid[np.arange(d.size), d] += 1
    return d, mid


def _in_open_face(mid, d, normal, plane, box):
    """Edges (doubled midpoints) lying in the open interior of the axis-parallel square
    {x_normal = plane} x box[a] x box[b] (box in doubled coordinates, closed intervals):
    the edge is parallel to the face, its midpoint in the open square, and it does not
    lie on the square's boundary lines."""
    ok = (d != normal) & (mid[:, normal] == plane)
    for ax in range(3):
        if ax == normal:
            continue
        lo, hi = box[ax]
        ok &= (mid[:, ax] > lo) & (mid[:, ax] < hi)
    return ok


@pytest.mark.parametrize("s,n", [(2, 6), (2, 8), (4, 12)])
@pytest.mark.parametrize("boundary", [True, False])
def test_edge_sets_brute_force(s, n, boundary):
    """Each edge interface set (eq. edge space) equals, by brute force over all unknowns,
    the fine edges lying on the closed coarse edge E or in the open interior of one of
    the (up to) 4 coarse faces containing E; and every face-interior unknown lies in as
    many sets as its face has coarse edges carrying a space (4 with boundary edges, the
    interior coarse edges of its face otherwise), every coarse-edge unknown in exactly 1."""
    d, mid = _edge_geometry(n)
    m = n // s
    cover = np.zeros(mesh.ndof(n), int)
    for axis, c in mesh.coarse_edges(n, s, boundary):
        got = np.asarray(mesh.edge_interface_set(n, s, axis, c))
        cover[got] += 1
        C = 2 * np.asarray(c)
        ea, eb = [ax for ax in range(3) if ax != axis]
        on_e = (d == axis) & (mid[:, ea] == C[ea]) & (mid[:, eb] == C[eb]) & \
            (mid[:, axis] > C[axis]) & (mid[:, axis] < C[axis] + 2 * s)
        sel = on_e.copy()
        for t, other in ((ea, eb), (eb, ea)):
            for sign in (-1, 1):
                box = {axis: (C[axis], C[axis] + 2 * s),
                       t: tuple(sorted((C[t], C[t] + sign * 2 * s)))}
                sel |= _in_open_face(mid, d, other, C[other], box)
        np.testing.assert_array_equal(got, np.flatnonzero(sel))
    trans = np.stack([mid[np.arange(d.size), (d + 1) % 3], mid[np.arange(d.size), (d + 2) % 3]], 1)
    on = (trans % (2 * s) == 0).sum(1)
    assert np.all(cover[on == 0] == 0) and np.all(cover[on == 2] == 1)
    face = np.flatnonzero(on == 1)
    if boundary:
        assert np.all(cover[face] == 4)
    else:
        # the face of a face-interior unknown: normal axis = the transverse axis at a
        # coarse node; its 4 coarse edges are interior unless they lie on the box boundary
        for e in face:
            dd = d[e]
            a1, a2 = (dd + 1) % 3, (dd + 2) % 3
            normal, t = (a1, a2) if trans[e, 0] % (2 * s) == 0 else (a2, a1)
            f0 = mid[e, dd] // (2 * s) * (2 * s)
            g0 = mid[e, t] // (2 * s) * (2 * s)
            interior = lambda x: 0 < x < 2 * n
            pl = mid[e, normal]
            want = 0
            for along, fixed, pos in ((dd, t, g0), (dd, t, g0 + 2 * s), (t, dd, f0), (t, dd, f0 + 2 * s)):
                want += interior(pl) and interior(pos)
            assert cover[e] == want, (e, cover[e], want)


@pytest.mark.parametrize("s,n", [(2, 6), (4, 12)])
@pytest.mark.parametrize("boundary", [True, False])
def test_vertex_sets_brute_force(s, n, boundary):
    """Each vertex interface set (eq. vertex space) equals, by brute force, the fine edges
    on the 6 closed coarse edges through V or in the open interiors of the 12 coarse faces
    containing V (cut to the unknowns)."""
    d, mid = _edge_geometry(n)
    for v in mesh.coarse_vertices(n, s, boundary):
        V = 2 * s * np.asarray(v)
        sel = np.zeros(d.size, bool)
        for axis in range(3):
            ea, eb = [ax for ax in range(3) if ax != axis]
            sel |= (d == axis) & (mid[:, ea] == V[ea]) & (mid[:, eb] == V[eb]) & \
                (np.abs(mid[:, axis] - V[axis]) < 2 * s)
            for normal in range(3):
                if normal == axis:
                    continue
                t = 3 - axis - normal
                for sa in (-1, 1):
                    for sb in (-1, 1):
                        box = {axis: tuple(sorted((V[axis], V[axis] + sa * 2 * s))),
                               t: tuple(sorted((V[t], V[t] + sb * 2 * s)))}
                        sel |= _in_open_face(mid, d, normal, V[normal], box)
        np.testing.assert_array_equal(np.asarray(mesh.vertex_interface_set(n, s, v)),
                                      np.flatnonzero(sel))
