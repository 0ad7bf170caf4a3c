"""GPU parity on non-box domains (Sec. 6): Omega a union of boxes of an r x r x r grid
(ndmg_opts.domain), against the oracle's restriction of the cube (``oracle.domain``,
``vcycle.Hierarchy(active=...)``): the cube less one octant (a Fichera corner), an
L-shaped prism, and a random union of 3^3 boxes.

Vectors live in the cube's padded layout with zeros at every edge outside Omega's
unknowns; every test checks that those entries stay exactly zero.

Tolerances (the derivations of the cube and jump tests):
* operator apply: 1e-14 of max |A||x| entrywise;
* smoother and V-cycle in FP64: 0.03 (0.02) of u kappa(A_T) kappa(S) over the oracle's
  local matrices (the library forms X_T and S^{-1} explicitly); FP32 V-cycle 12 u;
* PCG: residual recomputed with the oracle's matrix <= 1.5e-10, iterations within one
  of the oracle's PCG, the solution against a sparse direct solve.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from layout import from_padded, to_padded
from oracle import coefficient, domain, mesh, pcg, rhs, smoother, vcycle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def fichera():
    a = np.ones((2, 2, 2), dtype=bool)
    a[1, 1, 1] = False
    return a


def l_prism():
    a = np.ones((2, 2, 2), dtype=bool)
    a[:, 1, 1] = False
    return a


def union3(seed=7):
    rng = np.random.default_rng(seed)
    a = rng.random((3, 3, 3)) < 0.7
    a[0, 0, 0] = a[1, 1, 1] = True
    return a


DOMAINS = {"fichera": fichera, "l_prism": l_prism, "union3": union3}


def _solver(n, active, **kw):
    from paper_2205_05840_amd import Solver
    print(f"[case] domain n={n} r={active.shape[0]} kept {int(active.sum())} {kw}", flush=True)
    return Solver(n, kw.pop("alpha", 1.0), domain=active, **kw)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


class Omega:
    """Maps between Omega's unknowns and the cube's padded layout."""

    def __init__(self, S, n, active):
        self.S, self.n = S, n
        self.keep = domain.unknown_mask(n, active)

    def dev(self, x_omega):
        full = np.zeros(mesh.ndof(self.n))
        full[self.keep] = x_omega
        return torch.from_numpy(to_padded(self.n, self.S.P, self.S.B, full)).cuda()

    def host(self, t):
        """Omega's entries of a device vector; asserts zeros everywhere else."""
        v = _host(t)
        full = from_padded(self.n, self.S.P, self.S.B, v)
        assert not full[~self.keep].any(), "nonzero outside Omega"
        outside = np.ones(v.size, dtype=bool)
        outside[np.flatnonzero(to_padded(self.n, self.S.P, self.S.B, np.ones(mesh.ndof(self.n))))] = False
        assert not v[outside].any(), "nonzero off the unknowns"
        return full[self.keep]


def _scale(lit):
    return U64 * max(np.linalg.cond(Ai) for _, Ai in lit.T) * max(np.linalg.cond(p[3]) for p in lit.P)


@pytest.mark.parametrize("name,n", [("fichera", 8), ("fichera", 16), ("l_prism", 16), ("union3", 12),
                                    ("fichera", 64)])
def test_apply_and_rhs(name, n):
    from paper_2205_05840_amd import synth
    active = DOMAINS[name]()
    S = _solver(n, active, alpha=0.8)
    W = Omega(S, n, active)
    A = domain.matrix(n, 1.0 / n, 0.8 * np.ones((n, n, n)), active)
    assert S.ndof == A.shape[0]
    assert np.array_equal(_host(S.unknown_mask()), to_padded(n, S.P, S.B, W.keep.astype(np.float64)))
    x = np.random.default_rng(n).standard_normal(A.shape[0])
    y = W.host(S.apply(W.dev(x)))
    err = np.abs(y - A @ x).max() / (abs(A) @ np.abs(x)).max()
    print(f"{name} n={n}: apply {err:.2e} of max |A||x|")
    assert err <= 1e-14
    f = synth.normal_samples(n, 1)
    b = W.host(S.assemble_rhs(torch.from_numpy(f)))
    b_o = rhs.load_from_samples(n, 1.0 / n, f)[W.keep]
    assert _rel(b, b_o) <= 1e-14


@pytest.mark.parametrize("name,n,kind,s", [("fichera", 8, "vertex", 2), ("fichera", 16, "vertex", 2),
                                           ("l_prism", 16, "vertex", 2), ("union3", 12, "vertex", 2),
                                           ("fichera", 16, "vertex", 4), ("fichera", 8, "edge", 2)])
def test_smoother(name, n, kind, s):
    active = DOMAINS[name]()
    S = _solver(n, active, smoother=kind, subdomain=s)
    W = Omega(S, n, active)
    A = domain.matrix(n, 1.0 / n, np.ones((n, n, n)), active)
    g = np.random.default_rng(3).standard_normal(A.shape[0])
    z = W.host(S.level_op(S.levels - 1, "smooth", W.dev(g)))
    lit = smoother.LiteralSmoother(A, n, s, kind=kind, keep=W.keep)
    ref = lit(g)
    err, scale = _rel(z, ref), _scale(lit)
    print(f"{name} n={n} {kind} s={s}: smoother err {err:.2e}, scale {scale:.2e}, ratio {err / scale:.4f}")
    assert err <= max(1e-13, 0.03 * scale)


@pytest.mark.parametrize("name,n,kind", [("fichera", 8, "vertex"), ("fichera", 16, "vertex"),
                                         ("l_prism", 16, "vertex"), ("union3", 12, "vertex"),
                                         ("fichera", 8, "edge")])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_vcycle(name, n, kind, precision):
    active = DOMAINS[name]()
    S = _solver(n, active, smoother=kind, precision=precision)
    W = Omega(S, n, active)
    H = vcycle.Hierarchy(n, 1.0, kind=kind, active=active)
    g = np.random.default_rng(5).standard_normal(H.A[-1].shape[0])
    z = W.host(S.vcycle(W.dev(g)))
    ref = H.precondition(g)
    err = _rel(z, ref)
    if precision == "fp32":
        print(f"{name} n={n} {kind} V-cycle fp32: err {err:.2e} = {err / U32:.2f} u")
        assert err <= 12 * U32
    else:
        scale = _scale(H.M[-1])
        print(f"{name} n={n} {kind} V-cycle fp64: err {err:.2e}, scale {scale:.2e}, ratio {err / scale:.4f}")
        assert err <= max(1e-12, 0.02 * scale)


@pytest.mark.parametrize("name,n,precision", [("fichera", 16, "fp64"), ("fichera", 16, "fp32"),
                                              ("l_prism", 16, "fp64"), ("union3", 24, "fp64")])
def test_pcg_against_oracle(name, n, precision):
    from paper_2205_05840_amd import synth
    active = DOMAINS[name]()
    S = _solver(n, active, precision=precision)
    W = Omega(S, n, active)
    f = synth.normal_samples(n, 0)
    b_o = rhs.load_from_samples(n, 1.0 / n, f)[W.keep]
    u, it, rel = S.solve(S.assemble_rhs(torch.from_numpy(f)), rtol=1e-10)
    u_c = W.host(u)
    H = vcycle.Hierarchy(n, 1.0, active=active)
    A = H.A[-1]
    true_rel = _rel(A @ u_c, b_o)
    _, it_o, _, _ = pcg.pcg(A, b_o, H.precondition, rtol=1e-10, flexible=(precision == "fp32"))
    ue = spla.spsolve(A.tocsc(), b_o)
    print(f"{name} n={n} {precision}: {it} iterations (oracle {it_o}), relres {rel:.2e}, true {true_rel:.2e}, "
          f"error {_rel(u_c, ue):.2e}")
    assert rel <= 1e-10 and true_rel <= 1.5e-10
    assert abs(it - it_o) <= 1
    lam_min = spla.eigsh(A, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
    assert np.linalg.norm(u_c - ue) <= 1.5e-10 * np.linalg.norm(b_o) / lam_min


@pytest.mark.parametrize("n", [64, 128])
def test_pcg_fichera_large(n):
    """The Fichera domain at full size, mixed precision: the residual recomputed in FP64 on
    the GPU, rows of it against the oracle's row-by-row apply of the cube (Omega's rows
    only involve cells inside Omega), and zeros outside Omega."""
    from paper_2205_05840_amd import synth
    active = fichera()
    S = _solver(n, active, precision="fp32")
    W = Omega(S, n, active)
    f = synth.normal_samples(n, 0)
    b = S.assemble_rhs(torch.from_numpy(f))
    u, it, rel = S.solve(b, rtol=1e-10)
    res = b - S.apply(u)
    true_rel = float(torch.linalg.norm(res) / torch.linalg.norm(b))
    print(f"fichera n={n}: {it} iterations, relres {rel:.2e}, true {true_rel:.2e}")
    assert rel <= 1e-10 and true_rel <= 1.5e-10
    u_c = W.host(u)
    full = np.zeros(mesh.ndof(n))
    full[W.keep] = u_c
    rows = np.flatnonzero(W.keep)[np.random.default_rng(2).choice(int(W.keep.sum()), 3000, replace=False)]
    b_c = from_padded(n, S.P, S.B, _host(b))
    cells = np.ones((n, n, n))
    r_o = b_c[rows] - coefficient.apply_rows(n, 1.0 / n, cells, full, rows)
    absAu = coefficient.apply_rows(n, 1.0 / n, cells, full, rows, absolute=True)
    r_g = from_padded(n, S.P, S.B, _host(res))[rows]
    assert np.all(np.abs(r_o - r_g) <= 1e-14 * absAu + 1e-300)


@pytest.mark.parametrize("dims,box", [((16, 8, 8), (2.0, 1.0, 1.0)), ((8, 16, 8), (1.0, 2.0, 1.0)),
                                      ((12, 12, 8), (3.0, 3.0, 2.0))])
def test_box_not_a_cube(dims, box):
    """A box that is not a cube (Sec. 1), served inside the cube of max(n_d) elements: the
    unknown count against its closed form nx (ny-1)(nz-1) + (nx-1) ny (nz-1) + (nx-1)(ny-1) nz,
    zeros outside the box, and PCG against the oracle on the same union of boxes."""
    from paper_2205_05840_amd import Solver, synth
    nx, ny, nz = dims
    n = max(dims)
    L = box[dims.index(n)]
    g = int(np.gcd.reduce(dims))
    r = n // g
    active = np.zeros((r, r, r), dtype=bool)
    active[: nz // g, : ny // g, : nx // g] = True
    print(f"[case] box {dims} {box}", flush=True)
    S = Solver(dims, 1.0, length=box)
    assert (S.n, S.ndof) == (n, nx * (ny - 1) * (nz - 1) + (nx - 1) * ny * (nz - 1) + (nx - 1) * (ny - 1) * nz)
    W = Omega(S, n, active)
    want = to_padded(n, S.P, S.B, W.keep.astype(np.float64))
    assert np.array_equal(_host(S.unknown_mask()), want)
    h = L / n
    f = synth.normal_samples(n, 3)
    b_o = rhs.load_from_samples(n, h, f)[W.keep]
    u, it, rel = S.solve(S.assemble_rhs(torch.from_numpy(f)), rtol=1e-10)
    u_c = W.host(u)
    H = vcycle.Hierarchy(n, 1.0, L=L, active=active)
    A = H.A[-1]
    _, it_o, _, _ = pcg.pcg(A, b_o, H.precondition, rtol=1e-10)
    print(f"box {dims}: {it} iterations (oracle {it_o}), relres {rel:.2e}, true {_rel(A @ u_c, b_o):.2e}")
    assert rel <= 1e-10 and _rel(A @ u_c, b_o) <= 1.5e-10 and abs(it - it_o) <= 1
