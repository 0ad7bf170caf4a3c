"""Pins of the V-cycle (Sec. 3.3, Fig. 1), its contraction numbers (Table 2), PCG
and the adjoint gradient."""
import os

import numpy as np
import pytest

from oracle import adjoint, assemble, contraction, exact, mesh, pcg, rhs, vcycle

HERE = os.path.dirname(os.path.abspath(__file__))


def _table(name):
    rows = {}
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = line.split()
            rows[(float(v[0]), int(v[1]))] = [float(x) for x in v[2:]]
    return rows


TABLE2 = _table("table2_vertex.txt")


@pytest.mark.parametrize("alpha", [0.01, 0.1, 1.0, 10.0, 100.0])
@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_table2_k1_exact(alpha, m):
    """At k = 1 the one vertex patch and the 8 interiors split N_1 a-orthogonally, so
    M^{-1} = eta A^{-1} and ||E_1||_a = (8/9)^(2m): every printed digit of Table 2."""
    H = vcycle.Hierarchy(4, alpha, L=2.0, m=m)
    c, _ = contraction.contraction_dense(H)
    assert abs(c - (8.0 / 9.0) ** (2 * m)) < 1e-8
    assert round(c, 3) == TABLE2[(alpha, 1)][m - 1]


@pytest.mark.parametrize("alpha,m", [(0.01, 1), (1.0, 1), (1.0, 5), (100.0, 5)])
def test_table2_k2(alpha, m):
    """k = 2 (8^3 elements on (-1,1)^3): within 1.5% of Table 2, never below the
    bubble bound (8/9)^(2m)."""
    H = vcycle.Hierarchy(8, alpha, L=2.0, m=m)
    c, lam = contraction.contraction_dense(H)
    ref = TABLE2[(alpha, 2)][m - 1]
    assert c >= (8.0 / 9.0) ** (2 * m) - 1e-10
    assert abs(c - ref) <= 0.015 * ref, (c, ref)
    assert lam.max() <= 1 + 1e-9


@pytest.mark.slow
def test_table2_k3_lanczos():
    H = vcycle.Hierarchy(16, 0.01, L=2.0, m=1)
    c = contraction.contraction_lanczos(H)
    assert round(c, 3) == TABLE2[(0.01, 3)][0]


def test_interior_only_reading_misses_table2():
    """With vertex spaces only at interior coarse vertices the k = 2 contraction is
    clearly above Table 2 (the reason the boundary patches are the default)."""
    H = vcycle.Hierarchy(8, 1.0, L=2.0, m=5, boundary=False)
    c, _ = contraction.contraction_dense(H)
    assert c > 1.04 * TABLE2[(1.0, 2)][4]


def test_coarsest_exact():
    H = vcycle.Hierarchy(2, 1.0)
    A0 = H.A[0].toarray()
    g = np.random.default_rng(0).standard_normal(A0.shape[0])
    np.testing.assert_allclose(A0 @ H.mg(0, g), g, rtol=1e-13)


def test_preconditioner_symmetric_positive():
    """B = MG(J, ., 0, 1) on the 8^3 unit-cube problem: symmetric, lambda(BA) in
    [1 - ||E||, 1] (Sec. 4.2, Remark on R_k and E_k)."""
    H = vcycle.Hierarchy(8, 1.0)
    B = contraction.dense_preconditioner(H)
    assert abs(B - B.T).max() <= 1e-13 * abs(B).max()
    c, lam = contraction.contraction_dense(H)
    assert lam.min() >= 1 - c - 1e-12 and lam.max() <= 1 + 1e-9
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


def test_contraction_decreases_with_m():
    cs = [contraction.contraction_dense(vcycle.Hierarchy(8, 0.1, m=m))[0] for m in (1, 2, 3)]
    assert cs[0] > cs[1] > cs[2]


def test_vcycle_steps_follow_figure1():
    """With m = 1 and z0 = 0: z1 = M^{-1} g, z2 = z1 + P MG(k-1, P^T (g - A z1)),
    z3 = z2 + M^{-1}(g - A z2), written out by hand for a two-level hierarchy."""
    H = vcycle.Hierarchy(4, 2.0)
    A, M, P = H.A[1], H.M[1], H.P[1]
    g = np.random.default_rng(5).standard_normal(A.shape[0])
    z1 = M(g)
    e = np.linalg.solve(H.A[0].toarray(), P.T @ (g - A @ z1))
    z2 = z1 + P @ e
    z3 = z2 + M(g - A @ z2)
    np.testing.assert_allclose(H.precondition(g), z3, rtol=0, atol=1e-12 * abs(z3).max())


@pytest.mark.parametrize("alpha", [0.01, 1.0, 100.0])
def test_pcg_solves_to_tolerance(alpha):
    from paper_2205_05840_amd import synth
    n = 8
    h = 1.0 / n
    b = rhs.load_from_samples(n, h, synth.normal_samples(n, 0))
    H = vcycle.Hierarchy(n, alpha)
    A = H.A[-1]
    u, it, rel, _ = pcg.pcg(A, b, H.precondition, rtol=1e-10)
    assert rel <= 1e-10 and np.linalg.norm(b - A @ u) <= 1.01e-10 * np.linalg.norm(b) * 10
    ue = exact.solve_fft(n, h, alpha, b)
    assert np.linalg.norm(u - ue) <= 1e-8 * np.linalg.norm(ue)
    assert it <= 30


@pytest.mark.slow
def test_pcg_mesh_independent():
    from paper_2205_05840_amd import synth
    its = []
    for n in (8, 16, 32):
        h = 1.0 / n
        b = rhs.load_from_samples(n, h, synth.normal_samples(n, 0))
        H = vcycle.Hierarchy(n, 1.0)
        _, it, rel, _ = pcg.pcg(H.A[-1], b, H.precondition, rtol=1e-10)
        assert rel <= 1e-10
        its.append(it)
    assert max(its) - min(its) <= 2 and max(its) <= 30, its


def test_adjoint_gradient_matches_central_differences():
    """dL/dalpha = -sum_k lambda_k^T K u_k and dL/db_k = lambda_k against central
    differences of L computed with exact solves."""
    n, L, alpha = 6, 1.0, 1.0
    h = L / n
    N = mesh.ndof(n)
    rng = np.random.default_rng(4)
    B = rng.standard_normal((3, N))
    T = exact.solve_fft(n, h, 2.0, B)
    loss, dB, da = adjoint.loss_and_grads(n, L, alpha, B, T)

    def Lof(a, Bm):
        U = exact.solve_fft(n, h, a, Bm)
        return float(np.sum((U - T) ** 2))

    d = 1e-4
    fd = (Lof(alpha + d, B) - Lof(alpha - d, B)) / (2 * d)
    assert abs(fd - da) <= 1e-6 * abs(da)
    for k in range(2):
        Dir = rng.standard_normal(B.shape)
        eps = 1e-3 * np.linalg.norm(B) / np.linalg.norm(Dir)
        fdb = (Lof(alpha, B + eps * Dir) - Lof(alpha, B - eps * Dir)) / (2 * eps)
        assert abs(fdb - np.sum(dB * Dir)) <= 1e-6 * abs(fdb)
    del loss


def test_stiffness_is_alpha_derivative():
    n, h = 4, 0.25
    K = assemble.stiffness_kron(n, h)
    A1 = assemble.matrix_kron(n, h, 1.0)
    A2 = assemble.matrix_kron(n, h, 3.0)
    assert abs((A2 - A1) / 2.0 - K).max() <= 1e-14 * abs(K).max()


def test_fewer_levels_two_grid_is_exact_coarse_correction():
    """With two levels kept, MG(1, g, 0, 1) of Fig. 1 is the two-grid cycle whose coarse
    step is the exact solve with A_{J-1}: pre-smoothing, exact coarse correction of the
    restricted residual, post-smoothing, written out here by hand."""
    import numpy as np
    import scipy.linalg as sla
    n, alpha = 8, 0.7
    H = vcycle.Hierarchy(n, alpha, levels=2)
    assert H.sizes == [4, 8]
    g = np.random.default_rng(1).standard_normal(mesh.ndof(n))
    A, M, P = H.A[1], H.M[1], H.P[1]
    z = M(g)
    z = z + P @ sla.solve(H.A[0].toarray(), P.T @ (g - A @ z), assume_a="pos")
    z = z + M(g - A @ z)
    assert np.abs(H.precondition(g) - z).max() <= 1e-12 * np.abs(z).max()


def test_cg_lanczos_matrix_gives_contraction():
    """The contraction estimate the library takes: preconditioned CG on A u = b records
    alpha_j = r_j.z_j / p_j.A p_j and beta_j = r_{j+1}.z_{j+1} / r_j.z_j; the tridiagonal
    matrix with diagonal 1/alpha_j + beta_{j-1}/alpha_{j-1} and off-diagonal
    sqrt(beta_j)/alpha_j is the Lanczos matrix of B A, whose smallest eigenvalue converges to
    lambda_min(B A) = 1 - ||E||_a.  CG is continued past the convergence of u (the process
    is scale-free, and the Lanczos recurrence goes on in the directions the rounding
    leaves): the extreme eigenvalue sits just below a large cluster (the bubbles at
    1 - (8/9)^2) and is resolved only after about 60 steps.  Checked here against the
    dense eigensolve at k = 2."""
    import numpy as np
    H = vcycle.Hierarchy(8, 1.0, L=2.0, m=1)
    A = H.A[-1]
    b = np.random.default_rng(0).standard_normal(A.shape[0])
    r = b.copy()
    z = H.precondition(r)
    p = z.copy()
    rz = r @ z
    al, be = [], []
    for _ in range(120):
        q = A @ p
        a = rz / (p @ q)
        al.append(a)
        r = r - a * q
        z = H.precondition(r)
        rz_new = r @ z
        be.append(rz_new / rz)
        p = z + be[-1] * p
        rz = rz_new
    m = len(al)
    d = [1 / al[0]] + [1 / al[j] + be[j - 1] / al[j - 1] for j in range(1, m)]
    e = [np.sqrt(be[j]) / al[j] for j in range(m - 1)]
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    c_lanczos = 1 - np.linalg.eigvalsh(T).min()
    c_dense, _ = contraction.contraction_dense(H)
    assert abs(c_lanczos - c_dense) <= 1e-9, (c_lanczos, c_dense)
