"""Pins of the global operator, the grid transfers and the exact solvers."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import assemble, exact, mesh, rhs, transfer


@pytest.mark.parametrize("n", [2, 3, 4, 5, 8])
def test_kron_equals_elementwise(n):
    h, alpha = 1.0 / n, 0.37
    A1 = assemble.matrix_kron(n, h, alpha)
    A2 = assemble.matrix_elementwise(n, h, alpha)
    assert abs(A1 - A2).max() <= 1e-15 * abs(A1).max()
    assert abs(A1 - A1.T).max() == 0.0


@pytest.mark.parametrize("n", [3, 4, 8])
def test_de_rham(n):
    """curl grad = 0 exactly for integer nodal data; hence A G phi = M G phi."""
    C, _ = assemble.curl_operator(n)
    G = assemble.gradient(n, 1.0)                      # integer differences
    phi = np.random.default_rng(n).integers(-50, 50, size=(n - 1) ** 3).astype(float)
    assert np.all(C @ (G @ phi) == 0.0)
    h = 1.0 / n
    Gh = assemble.gradient(n, h)
    A = assemble.matrix_kron(n, h, 3.0)
    M = assemble.mass_kron(n, h)
    v = Gh @ phi
    bound = 1e-14 * (abs(A) @ np.abs(v)).max()       # rounding of the cancelling sum
    np.testing.assert_allclose(A @ v, M @ v, rtol=0, atol=bound)


def test_ndof_counts():
    for n, N in [(4, 108), (8, 1176), (16, 10800), (32, 92256), (64, 762048), (128, 6193536)]:
        assert mesh.ndof(n) == N


@pytest.mark.parametrize("n", [3, 4, 6])
def test_spd_and_spectrum(n):
    h = 1.0 / n
    A = assemble.matrix_kron(n, h, 2.0).toarray()
    ev = np.linalg.eigvalsh(A)
    assert ev.min() > 0 and ev.min() >= h ** 3 / 9.0 * (1 - 1e-12)
    np.testing.assert_allclose(np.sort(exact.eigenvalues(n, h, 2.0)), ev, rtol=1e-12,
                               atol=1e-14 * ev.max())


@pytest.mark.parametrize("nc", [2, 3, 4])
def test_galerkin(nc):
    """I_k^{k-1} A_k I_{k-1}^k = A_{k-1}: nested spaces and one bilinear form."""
    L, alpha = 1.0, 0.7
    P = transfer.prolongation(nc)
    Af = assemble.matrix_kron(2 * nc, L / (2 * nc), alpha)
    Ac = assemble.matrix_kron(nc, L / nc, alpha)
    D = (P.T @ Af @ P - Ac)
    assert abs(D).max() <= 1e-14 * abs(Ac).max()


@pytest.mark.parametrize("nc", [2, 3, 5])
def test_commuting_gradient(nc):
    """Prolongation of a coarse gradient is the fine gradient of the Q1-prolongated field."""
    P = transfer.prolongation(nc)
    P1 = transfer._P1(nc)
    Q1 = sp.kron(P1, sp.kron(P1, P1))
    Gc = assemble.gradient(nc, 1.0)
    Gf = assemble.gradient(2 * nc, 0.5)
    phi = np.random.default_rng(1).integers(-9, 9, size=(nc - 1) ** 3).astype(float)
    assert np.all(P @ (Gc @ phi) == Gf @ (Q1 @ phi))


def test_prolongation_weights():
    """A fine x-edge on a coarse x-edge takes the coarse value (weight 1); one halfway
    between two coarse node lines takes their mean (hat weights 1/2)."""
    nc = 3
    P = transfer.prolongation(nc)
    c = np.random.default_rng(2).standard_normal(mesh.ndof(nc))
    fine = P @ c
    d, p = mesh.edge_coords(2 * nc)
    sel = (d == 0) & (p[:, 1] % 2 == 0) & (p[:, 2] % 2 == 0)
    ci = mesh.compact_index(nc, 0, p[sel, 0] // 2, p[sel, 1] // 2, p[sel, 2] // 2)
    np.testing.assert_array_equal(fine[sel], c[ci])
    sel = (d == 0) & (p[:, 1] % 2 == 1) & (p[:, 2] % 2 == 0)
    lo = mesh.compact_index(nc, 0, p[sel, 0] // 2, p[sel, 1] // 2, p[sel, 2] // 2)
    hi = mesh.compact_index(nc, 0, p[sel, 0] // 2, p[sel, 1] // 2 + 1, p[sel, 2] // 2)
    ref = 0.5 * (np.where(lo >= 0, c[lo], 0.0) + np.where(hi >= 0, c[hi], 0.0))
    np.testing.assert_array_equal(fine[sel], ref)


@pytest.mark.parametrize("n", [4, 8, 12, 16, 24])
def test_fft_matches_sparse_direct(n):
    h, alpha = 1.0 / n, 1.7
    b = np.random.default_rng(n).standard_normal(mesh.ndof(n))
    u1 = exact.solve_direct(n, h, alpha, b)
    u2 = exact.solve_fft(n, h, alpha, b)
    A = assemble.matrix_kron(n, h, alpha)
    # both are backward stable: small residuals, forward difference within kappa * eps
    ev = exact.eigenvalues(n, h, alpha)
    for u in (u1, u2):
        assert np.linalg.norm(b - A @ u) <= 1e-14 * ev.max() * np.linalg.norm(u)
    kappa = ev.max() / ev.min()
    assert np.linalg.norm(u1 - u2) <= 10 * kappa * 2.2e-16 * np.linalg.norm(u1)


def test_fft_multiple_rhs():
    n, h = 6, 1.0 / 6
    B = np.random.default_rng(0).standard_normal((3, mesh.ndof(n)))
    U = exact.solve_fft(n, h, 0.5, B)
    for r in range(3):
        np.testing.assert_allclose(U[r], exact.solve_fft(n, h, 0.5, B[r]), rtol=1e-13, atol=1e-14)


def test_load_vector_quadrature():
    """The 2x2x2 Gauss rule is exact for f in Q1 per element; compare with 5^3 Gauss."""
    n, L = 4, 1.0
    f = lambda x, y, z: (1 + x + 2 * y - z + 3 * y * z, x * y - 2 * z + 1, 2 + x * z + y)
    from paper_2205_05840_amd import synth
    X = synth.gauss_points(n, L)
    F = np.stack(f(X[..., 0], X[..., 1], X[..., 2]), -1)
    b1 = rhs.load_from_samples(n, L / n, F)
    b2 = rhs.load_from_function(n, L, f, q=5)
    np.testing.assert_allclose(b1, b2, rtol=1e-13, atol=1e-16)


@pytest.mark.slow
def test_manufactured_first_order():
    """Energy error ||u* - u_h||_a^2 = a(u*,u*) - b^T u_h decreases like h (Sec. 2)."""
    alpha = 1.0
    from paper_2205_05840_amd import synth
    aa = (2 * np.pi ** 2 * alpha + 1) * 0.75
    errs = []
    for n in (8, 16, 32):
        f = lambda x, y, z: tuple((2 * np.pi ** 2 * alpha + 1) * c
                                  for c in synth.manufactured_field(x, y, z))
        b = rhs.load_from_function(n, 1.0, f, q=5)
        u = exact.solve_fft(n, 1.0 / n, alpha, b)
        errs.append(np.sqrt(aa - b @ u))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(0.95 < r < 1.1 for r in rates), (errs, rates)


@pytest.mark.parametrize("n,alpha", [(4, 1.0), (7, 0.3), (10, 25.0)])
def test_apply_rows_equals_assembled(n, alpha):
    """The sampled-row product (element definition, used at sizes too large to assemble)
    equals the Kronecker-assembled matrix on every row."""
    from oracle import assemble, mesh
    h = 1.0 / n
    x = np.random.default_rng(n).standard_normal(mesh.ndof(n))
    rows = np.random.default_rng(1).permutation(mesh.ndof(n))
    y = assemble.apply_rows(n, h, alpha, x, rows)
    ref = (assemble.matrix_kron(n, h, alpha) @ x)[rows]
    assert np.abs(y - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("n", [3, 5, 8])
def test_interpolate_gradient_commutes(n):
    """Canonical interpolation (edge averages, eq. NDdof) of a gradient equals the
    discrete gradient of the nodal values: the average of d phi / dx_d along an edge is
    (phi(end) - phi(start)) / h, the commuting property of the de Rham sequence."""
    L = 1.3
    h = L / n
    p = np.pi / L
    phi = lambda x, y, z: np.sin(p * x) * np.sin(2 * p * y) * np.sin(p * z) * (1 + x * y)
    grad = lambda x, y, z: (
        np.sin(2 * p * y) * np.sin(p * z) * (p * np.cos(p * x) * (1 + x * y) + np.sin(p * x) * y),
        np.sin(p * x) * np.sin(p * z) * (2 * p * np.cos(2 * p * y) * (1 + x * y) + np.sin(2 * p * y) * x),
        np.sin(p * x) * np.sin(2 * p * y) * p * np.cos(p * z) * (1 + x * y))
    ii = np.arange(1, n) * h
    z2, y2, x2 = np.meshgrid(ii, ii, ii, indexing="ij")
    nodal = phi(x2, y2, z2).ravel()                     # [z][y][x] over interior nodes
    got = rhs.interpolate(n, L, grad, q=10)
    ref = assemble.gradient(n, h) @ nodal
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_interpolate_polynomial_edge_average():
    """Edge averages of a field polynomial along each edge, against the closed form
    (1/h) int_{ih}^{(i+1)h} t^3 dt = h^3 ((i+1)^4 - i^4) / 4 times the transverse factors."""
    n, L = 4, 2.0
    h = L / n
    f = lambda x, y, z: (x ** 3 * y, z * y ** 3, 2.0 + 0 * x)
    got = rhs.interpolate(n, L, f, q=4)
    d, pp = mesh.edge_coords(n)
    c = pp.astype(float)
    avg3 = lambda i: h ** 3 * ((i + 1) ** 4 - i ** 4) / 4.0
    ref = np.where(d == 0, avg3(c[:, 0]) * c[:, 1] * h,
                   np.where(d == 1, c[:, 2] * h * avg3(c[:, 1]), 2.0))
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("n,alpha", [(3, 1.0), (6, 0.05), (9, 40.0)])
def test_apply_fft_equals_assembled(n, alpha):
    """A x through the 3x3 symbols of the orthonormal DST/DCT transforms equals the
    assembled matrix (the matrix-free reference for sizes too large to assemble)."""
    h = 1.0 / n
    X = np.random.default_rng(n).standard_normal((2, mesh.ndof(n)))
    ref = (assemble.matrix_kron(n, h, alpha) @ X.T).T
    got = exact.apply_fft(n, h, alpha, X)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("n,alpha", [(4, 1.0), (6, 30.0)])
def test_fft_extended_precision(n, alpha):
    """The extended-precision transform solve: its residual with the extended symbol
    product is at the level of the extended unit roundoff (2^-64, far below FP64's),
    the FP64-assembled matrix sees an FP64-level residual (its entries are rounded to
    FP64), and it agrees with the FP64 solve within kappa * eps."""
    h = 1.0 / n
    b = np.random.default_rng(n).standard_normal(mesh.ndof(n))
    ul = exact.solve_fft(n, h, alpha, b, dtype=np.longdouble)
    assert ul.dtype == np.longdouble
    A = assemble.matrix_kron(n, h, alpha).toarray()
    scale = (np.abs(A) @ np.abs(ul.astype(np.float64))).max()
    rl = exact.apply_fft(n, h, alpha, ul, dtype=np.longdouble) - b
    assert np.abs(rl).max() <= 1e-17 * scale
    res = np.abs(A.astype(np.longdouble) @ ul - b).max()
    assert res <= 1e-15 * scale
    ev = exact.eigenvalues(n, h, alpha)
    u64 = exact.solve_fft(n, h, alpha, b)
    assert np.linalg.norm(u64 - ul.astype(np.float64)) <= 10 * ev.max() / ev.min() * 2.2e-16 * np.linalg.norm(u64)


def test_adjoint_extended_matches_fp64_small():
    """At 8^3 (no strong cancellation) the extended-precision adjoint reference equals
    the FP64 one to 1e-9 in dL/db and 1e-12 in the loss and dL/dalpha."""
    from oracle import adjoint
    n, h = 8, 1.0 / 8
    B = np.random.default_rng(3).standard_normal((2, mesh.ndof(n)))
    T = exact.solve_fft(n, h, 2.0, B)
    l1, d1, a1 = adjoint.loss_and_grads(n, 1.0, 1.0, B, T)
    l2, d2, a2 = adjoint.loss_and_grads(n, 1.0, 1.0, B, T, dtype=np.longdouble)
    assert abs(l1 - l2) <= 1e-12 * l2 and abs(a1 - a2) <= 1e-12 * abs(a2)
    assert np.linalg.norm(d1 - d2) <= 1e-9 * np.linalg.norm(d2)
