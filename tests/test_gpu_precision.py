"""GPU parity of the single-precision V-cycle (the mixed-precision form) step by step:
operator apply, restriction, prolongation (with level sizes that are not multiples of
four, so the clamped last planes of the prolongation run), the smoother (boundary
patches on and off, including the permuted last row block of S^{-1} in the patch
products and the in-place X_T / A_T^{-1} reads of the interface sum and extension) and
the whole V-cycle, each against the FP64 oracle.

Tolerances.
* Operator and transfers are short sums: every output entry is a sum of k <= 33 terms
  (operator) or <= 18 terms (restriction) whose inputs and coefficients are rounded to
  single precision, so |fl(y) - y| <= (k + 2) u |A| |x| entrywise (u = 2^-24), the
  standard bound for recursive summation plus one rounding of each factor.
* Smoother and V-cycle: the library builds every local factor (A_T^{-1}, X_T =
  A_T^{-1} A_{I,dT}, S^{-1}, the coarsest inverse) in FP64 and rounds it once, and it
  evaluates the condensed form through X_T, so the cancellation of the large curl part
  on discrete gradients (A grad phi = M grad phi) happens in the FP64 setup, not in
  single precision.  What remains is a handful of roundings of relative size u per
  entry along each chain of products and sums.  Measured over the cases below the
  relative l2 error against the FP64 oracle is 0.8e-7 .. 1.5e-7 (1.3 .. 2.5 u) for
  every alpha, size and boundary choice; the tolerance is 12 u = 7.2e-7, 4.7 to 9 times
  every observed value, and any defect that changes a factor entry, a slot or a
  coefficient (errors of 1e-3 .. 1) exceeds it by orders of magnitude.
"""
import numpy as np
import pytest

from layout import boundary_mask, from_padded, to_padded
from oracle import assemble, mesh, smoother, transfer, vcycle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
TOL32 = 12 * U32


def _solver(n, alpha=1.0, **kw):
    from paper_2205_05840_amd import Solver
    print(f"[case] fp32 n={n} alpha={alpha} {kw}", flush=True)
    return Solver(n, alpha, precision="fp32", **kw)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _lvl(S, level):
    info = S.layout(level)
    return info[0], info[1], info[2]


@pytest.mark.parametrize("n,alpha", [(4, 1.0), (10, 3.0), (14, 0.2), (40, 1.0), (80, 7.0)])
def test_apply_fp32(n, alpha):
    S = _solver(n, alpha)
    h = 1.0 / n
    A = assemble.matrix_kron(n, h, alpha)
    x = np.random.default_rng(n).standard_normal(mesh.ndof(n))
    y = _host(S.level_op(S.levels - 1, "apply", _dev(to_padded(n, S.P, S.B, x))))
    got = from_padded(n, S.P, S.B, y)
    bound = 35 * U32 * (abs(A) @ np.abs(x))
    err = np.abs(got - A @ x)
    print(f"apply fp32: max err / bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound)
    assert np.all(y[boundary_mask(n, S.P, S.B)] == 0.0)


@pytest.mark.parametrize("n", [8, 10, 12, 14, 20, 32])
def test_transfers_fp32(n):
    S = _solver(n, 1.0)
    J = S.levels - 1
    nf, Pf, Bf = _lvl(S, J)
    nc, Pc, Bc = _lvl(S, J - 1)
    Pm = transfer.prolongation(nc)
    rng = np.random.default_rng(n)
    rf = rng.standard_normal(mesh.ndof(nf))
    gc = from_padded(nc, Pc, Bc, _host(S.level_op(J, "restrict", _dev(to_padded(nf, Pf, Bf, rf)))))
    err = np.abs(gc - Pm.T @ rf)
    bound = 20 * U32 * (abs(Pm.T) @ np.abs(rf))
    print(f"restrict fp32: max err / bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound)
    ec = rng.standard_normal(mesh.ndof(nc))
    zf0 = rng.standard_normal(mesh.ndof(nf))
    zf = _dev(to_padded(nf, Pf, Bf, zf0))
    S.level_op(J, "prolong", _dev(to_padded(nc, Pc, Bc, ec)), out=zf)
    zh = _host(zf)
    err = np.abs(from_padded(nf, Pf, Bf, zh) - (zf0 + Pm @ ec))
    bound = 6 * U32 * (np.abs(zf0) + abs(Pm) @ np.abs(ec))
    print(f"prolong fp32: max err / bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound)
    assert not zh[boundary_mask(nf, Pf, Bf)].any()


@pytest.mark.parametrize("n,alpha,boundary", [(4, 1.0, True), (8, 0.3, True), (8, 3.0, False),
                                              (10, 1.0, True), (10, 1.0, False), (12, 10.0, True),
                                              (14, 0.5, True), (14, 2.0, False), (16, 0.01, True),
                                              (32, 1.0, True)])
def test_smoother_fp32(n, alpha, boundary):
    S = _solver(n, alpha, boundary_patches=boundary)
    A = assemble.matrix_kron(n, 1.0 / n, alpha)
    r = np.random.default_rng(2).standard_normal(mesh.ndof(n))
    z = from_padded(n, S.P, S.B, _host(S.level_op(S.levels - 1, "smooth", _dev(to_padded(n, S.P, S.B, r)))))
    ref = smoother.FactoredVertexSmoother(A, n, 2, boundary=boundary)(r)
    err = _rel(z, ref)
    print(f"smoother fp32: err {err:.2e} = {err / U32:.2f} u")
    assert err <= TOL32


@pytest.mark.parametrize("n,alpha,m,boundary", [(4, 1.0, 1, True), (8, 1.0, 1, True),
                                                (8, 0.01, 2, True), (10, 1.0, 1, True),
                                                (12, 100.0, 1, False), (14, 3.0, 1, True),
                                                (14, 0.3, 1, False), (16, 1.0, 1, True),
                                                (32, 1.0, 1, True), (40, 0.1, 1, True)])
def test_vcycle_fp32(n, alpha, m, boundary):
    S = _solver(n, alpha, m=m, boundary_patches=boundary)
    g = np.random.default_rng(3).standard_normal(mesh.ndof(n))
    z = from_padded(n, S.P, S.B, _host(S.vcycle(_dev(to_padded(n, S.P, S.B, g)))))
    ref = vcycle.Hierarchy(n, alpha, m=m, boundary=boundary, factored=True).precondition(g)
    err = _rel(z, ref)
    print(f"V-cycle fp32: err {err:.2e} = {err / U32:.2f} u")
    assert err <= TOL32
