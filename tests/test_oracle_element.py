"""Pins of the element matrices (Sec. 2, eq. nedlec form and eq. NDdof).

The reference values are derived here symbolically, straight from the definition of
ND(T) and its edge-average degrees of freedom, not from the oracle's closed form.
"""
import numpy as np
import pytest
import sympy as sp

from oracle import element

x1, x2, x3 = sp.symbols("x1 x2 x3")
X = (x1, x2, x3)


def _nd_monomials():
    """The 12 monomial fields spanning ND(T) of eq. (nedlec form)."""
    z = sp.Integer(0)
    mons = []
    one = sp.Integer(1)
    for f in (one, x2, x3, x2 * x3):
        mons.append((f, z, z))
    for f in (one, x3, x1, x3 * x1):
        mons.append((z, f, z))
    for f in (one, x1, x2, x1 * x2):
        mons.append((z, z, f))
    return mons


def _edge_average(u, d, a, b):
    """(1/|e|) int_e u . t_e on the unit cube, edge of direction d at offsets (a, b)."""
    ea, eb = [ax for ax in range(3) if ax != d]
    sub = {X[ea]: a, X[eb]: b}
    return sp.integrate(u[d].subs(sub), (X[d], 0, 1))


@pytest.fixture(scope="module")
def symbolic_matrices():
    mons = _nd_monomials()
    # dof matrix: rows = the 12 functionals in the oracle's local order, cols = monomials
    Dm = sp.zeros(12, 12)
    for d in range(3):
        for b in range(2):
            for a in range(2):
                r = element.local_edge(d, a, b)
                for c, m in enumerate(mons):
                    Dm[r, c] = _edge_average(m, d, a, b)
    coef = Dm.inv()                     # column e: coefficients of the dual basis phi_e
    basis = []
    for e in range(12):
        u = [sum(coef[c, e] * mons[c][k] for c in range(12)) for k in range(3)]
        basis.append(u)

    def curl(u):
        return (sp.diff(u[2], x2) - sp.diff(u[1], x3),
                sp.diff(u[0], x3) - sp.diff(u[2], x1),
                sp.diff(u[1], x1) - sp.diff(u[0], x2))

    def integ(f):
        return sp.integrate(sp.expand(f), (x1, 0, 1), (x2, 0, 1), (x3, 0, 1))

    M = np.zeros((12, 12))
    K = np.zeros((12, 12))
    curls = [curl(u) for u in basis]
    for i in range(12):
        for j in range(i, 12):
            M[i, j] = M[j, i] = float(integ(sum(basis[i][k] * basis[j][k] for k in range(3))))
            K[i, j] = K[j, i] = float(integ(sum(curls[i][k] * curls[j][k] for k in range(3))))
    return M, K, basis


def test_dual_basis_is_edge_hat(symbolic_matrices):
    _, _, basis = symbolic_matrices
    # x-edge at (eta, zeta) = (1, 0): (x2 (1 - x3), 0, 0)
    u = basis[element.local_edge(0, 1, 0)]
    assert sp.simplify(u[0] - x2 * (1 - x3)) == 0 and u[1] == 0 and u[2] == 0


@pytest.mark.parametrize("h", [1.0, 0.25, 1.0 / 128])
def test_mass_matrix_matches_definition(symbolic_matrices, h):
    M, _, _ = symbolic_matrices
    np.testing.assert_allclose(element.mass_matrix(h), h ** 3 * M, rtol=1e-14, atol=1e-17)


@pytest.mark.parametrize("h", [1.0, 0.25, 1.0 / 128])
def test_curl_matrix_matches_definition(symbolic_matrices, h):
    _, K, _ = symbolic_matrices
    np.testing.assert_allclose(element.curl_matrix(h), h * K, rtol=1e-14, atol=1e-15 * h)


def test_closed_form_blocks():
    M4 = np.array([[4, 2, 2, 1], [2, 4, 1, 2], [2, 1, 4, 2], [1, 2, 2, 4]]) / 36.0
    M = element.mass_matrix(1.0)
    for d in range(3):
        np.testing.assert_allclose(M[4 * d:4 * d + 4, 4 * d:4 * d + 4], M4, rtol=1e-15)
    # the constant field (1,0,0) has edge values 1 on the 4 x-edges and energy |T| = 1
    u = np.zeros(12)
    u[:4] = 1.0
    assert abs(u @ M @ u - 1.0) < 1e-15


def test_curl_kernel_is_gradients():
    K = element.curl_matrix(1.0)
    assert np.linalg.matrix_rank(K, tol=1e-12) == 5
    # gradients of the 8 trilinear nodal functions: edge value = phi(end) - phi(start)
    G = np.zeros((12, 8))
    for d in range(3):
        ea, eb = [ax for ax in range(3) if ax != d]
        for b in range(2):
            for a in range(2):
                start = [0, 0, 0]
                start[ea], start[eb] = a, b
                end = list(start)
                end[d] = 1
                e = element.local_edge(d, a, b)
                G[e, start[0] + 2 * start[1] + 4 * start[2]] -= 1
                G[e, end[0] + 2 * end[1] + 4 * end[2]] += 1
    assert np.linalg.matrix_rank(G) == 7
    np.testing.assert_allclose(K @ G, 0.0, atol=1e-14)
