"""GPU tests of the batched form: problems of uneven sizes and alphas with several
right-hand sides each, solved by one batched call.  Every (problem, right-hand side)
pair is checked against the FP64 oracle (its matrix, its PCG iteration count and the
exact discrete solution from the FFT solver), and the batched kernels against the
single-problem path (same arithmetic per pair, so apply and V-cycle agree bitwise)."""
import numpy as np
import pytest

from layout import from_padded, to_padded
from oracle import assemble, exact, mesh, pcg, rhs, vcycle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _batch(ns, alphas, nrhs, precision="fp64", **kw):
    from paper_2205_05840_amd import BatchedSolver
    print(f"[case] batch ns={list(ns)} nrhs={nrhs} {precision} {kw}", flush=True)
    return BatchedSolver(ns, alphas, nrhs=nrhs, precision=precision, **kw)


def _true_residual_ok(A, b, u, rtol):
    """||b - A u|| against the stopping tolerance plus the residual gap of CG in FP64:
    the updated residual drifts from b - A u by rounding of order eps || |A| |u| ||
    (the FP64 oracle's own PCG shows a gap of 0.3 times that at alpha ~ 100)."""
    gap = 2.0 * np.finfo(float).eps * np.linalg.norm(abs(A) @ np.abs(u))
    return np.linalg.norm(b - A @ u) <= 1.5 * rtol * np.linalg.norm(b) + gap


def _loads(ns, nrhs, seed):
    """Oracle load vectors (compact numbering) per problem: [nrhs, ndof(n)]."""
    from paper_2205_05840_amd import synth
    out = []
    for p, n in enumerate(ns):
        f = synth.normal_samples(int(n), seed + p, nrhs=nrhs)
        out.append(rhs.load_from_samples(int(n), 1.0 / n, f))
    return out


def _pack(BS, blocks):
    X = np.zeros(BS.total_len)
    for p, blk in enumerate(blocks):
        off, vl, n, P, B, _ = BS.offset(p)
        X[off:off + BS.nrhs * vl] = to_padded(n, P, B, blk).reshape(-1)
    return torch.from_numpy(X).cuda()


def _unpack(BS, X):
    X = _host(X)
    out = []
    for p in range(BS.nprob):
        off, vl, n, P, B, _ = BS.offset(p)
        out.append(from_padded(n, P, B, X[off:off + BS.nrhs * vl].reshape(BS.nrhs, vl)))
    return out


def test_layout_groups_sizes():
    ns = [12, 8, 16, 8, 6]
    BS = _batch(ns, [1.0] * 5, 2)
    offs = [BS.offset(p) for p in range(5)]
    # classes in ascending n, problems of a class in input order, nrhs vectors each
    order = sorted(range(5), key=lambda p: (ns[p], p))
    pos = 0
    for p in order:
        off, vl, n, P, B, _ = offs[p]
        assert off == pos and n == ns[p] and vl == 3 * B and B == (n + 1) ** 2 * P
        pos += 2 * vl
    assert pos == BS.total_len


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_apply_and_vcycle_equal_single(precision):
    from paper_2205_05840_amd import Solver
    ns, alphas, nrhs = [8, 16, 12, 8], [0.05, 3.0, 40.0, 1.0], 2
    BS = _batch(ns, alphas, nrhs, precision)
    rng = np.random.default_rng(4)
    blocks = [rng.standard_normal((nrhs, mesh.ndof(n))) for n in ns]
    X = _pack(BS, blocks)
    Y = _host(BS.apply(X))
    Z = _host(BS.vcycle(X))
    for p, n in enumerate(ns):
        S = Solver(n, alphas[p], precision=precision)
        off, vl = BS.offset(p)[:2]
        for r in range(nrhs):
            x = torch.from_numpy(to_padded(n, S.P, S.B, blocks[p][r])).cuda()
            sl = slice(off + r * vl, off + (r + 1) * vl)
            assert np.array_equal(Y[sl], _host(S.apply(x))), (p, r)
            assert np.array_equal(Z[sl], _host(S.vcycle(x))), (p, r)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_operator_kernel_classes(precision):
    """Classes of 24^3 and 32^3 with four pairs each run the plane-marching operator
    kernel with one position per lane (a single problem of these sizes takes the
    per-thread kernel): the batched apply against the assembled matrix for every pair,
    and the batched PCG (whose V-cycle residuals use the same kernel, in FP32 for the
    mixed form) against the exact discrete solution."""
    ns, alphas, nrhs = [24, 32, 24, 32], [0.3, 2.0, 45.0, 0.01], 2
    BS = _batch(ns, alphas, nrhs, precision)
    rng = np.random.default_rng(24)
    blocks = [rng.standard_normal((nrhs, mesh.ndof(n))) for n in ns]
    Y = _unpack(BS, BS.apply(_pack(BS, blocks)))
    for p, n in enumerate(ns):
        A = assemble.matrix_kron(n, 1.0 / n, alphas[p])
        for r in range(nrhs):
            assert _rel(Y[p][r], A @ blocks[p][r]) <= 1e-14, (p, r)
    b = _loads(ns, nrhs, 240)
    U, it, rel = BS.solve(_pack(BS, b), rtol=1e-10)
    u = _unpack(BS, U)
    assert (rel <= 1e-10).all()
    for p, n in enumerate(ns):
        h = 1.0 / n
        A = assemble.matrix_kron(n, h, alphas[p])
        ev = exact.eigenvalues(n, h, alphas[p])
        ue = exact.solve_fft(n, h, alphas[p], b[p])
        for r in range(nrhs):
            bn = np.linalg.norm(b[p][r])
            assert _true_residual_ok(A, b[p][r], u[p][r], 1e-10), (p, r)
            assert np.linalg.norm(u[p][r] - ue[r]) <= 2e-10 * bn / ev.min(), (p, r)


def test_batched_pcg_fp64_matches_oracle():
    ns = [8, 12, 16, 6, 8, 12]
    alphas = [0.01, 2.5, 0.3, 100.0, 17.0, 1.0]
    nrhs = 3
    BS = _batch(ns, alphas, nrhs)
    b = _loads(ns, nrhs, 20)
    b[3][1] = 0.0                                   # a zero right-hand side: done at once
    U, it, rel = BS.solve(_pack(BS, b), rtol=1e-10)
    u = _unpack(BS, U)
    for p, n in enumerate(ns):
        h = 1.0 / n
        A = assemble.matrix_kron(n, h, alphas[p])
        H = vcycle.Hierarchy(n, alphas[p])
        ev = exact.eigenvalues(n, h, alphas[p])
        ue = exact.solve_fft(n, h, alphas[p], b[p])
        for r in range(nrhs):
            if p == 3 and r == 1:
                assert it[p, r] == 0 and rel[p, r] == 0.0 and not u[p][r].any()
                continue
            assert rel[p, r] <= 1e-10
            bn = np.linalg.norm(b[p][r])
            assert _true_residual_ok(A, b[p][r], u[p][r], 1e-10), (p, r)
            _, it_o, _, _ = pcg.pcg(A, b[p][r], H.precondition, rtol=1e-10)
            assert abs(it[p, r] - it_o) <= 1, (p, r, it[p, r], it_o)
            assert np.linalg.norm(u[p][r] - ue[r]) <= 2e-10 * bn / ev.min()


def test_batched_pcg_solution_to_tight_tolerance():
    ns, alphas, nrhs = [16, 8, 24], [1.0, 30.0, 0.02], 2
    BS = _batch(ns, alphas, nrhs)
    b = _loads(ns, nrhs, 40)
    U, it, rel = BS.solve(_pack(BS, b), rtol=1e-13)
    u = _unpack(BS, U)
    for p, n in enumerate(ns):
        ue = exact.solve_fft(n, 1.0 / n, alphas[p], b[p])
        for r in range(nrhs):
            assert _rel(u[p][r], ue[r]) <= 1e-9, (p, r)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_six_rhs_with_idle_pairs(precision):
    """Six right-hand sides per problem: the patch products of one-group segments run
    four right-hand sides of a problem per workgroup, so the second workgroup of each
    problem holds two.  Zero right-hand sides are done at once and idle from the first
    iteration: one that leads a workgroup (r = 0) and one in the second (r = 5)."""
    ns, alphas, nrhs = [16, 12, 16], [0.5, 20.0, 0.02], 6
    BS = _batch(ns, alphas, nrhs, precision)
    b = _loads(ns, nrhs, 70)
    b[1][0] = 0.0
    b[2][5] = 0.0
    U, it, rel = BS.solve(_pack(BS, b), rtol=1e-10)
    u = _unpack(BS, U)
    for p, n in enumerate(ns):
        h = 1.0 / n
        A = assemble.matrix_kron(n, h, alphas[p])
        ev = exact.eigenvalues(n, h, alphas[p])
        ue = exact.solve_fft(n, h, alphas[p], b[p])
        for r in range(nrhs):
            if (p, r) in ((1, 0), (2, 5)):
                assert it[p, r] == 0 and not u[p][r].any(), (p, r)
                continue
            bn = np.linalg.norm(b[p][r])
            assert rel[p, r] <= 1e-10, (p, r)
            assert _true_residual_ok(A, b[p][r], u[p][r], 1e-10), (p, r)
            assert np.linalg.norm(u[p][r] - ue[r]) <= 2e-10 * bn / ev.min(), (p, r)


def test_batched_mixed_precision_uneven():
    """Sizes from {8, 12, 16, 24, 32}, alpha log-uniform in [1e-2, 1e2], four N(0, 1)
    right-hand sides each, FP32 V-cycle in FP64 CG."""
    from paper_2205_05840_amd import synth
    ns, alphas = synth.batched_problems(12, seed=5)
    nrhs = 4
    BS = _batch(ns, alphas, nrhs, "fp32")
    b = _loads(ns, nrhs, 60)
    U, it, rel = BS.solve(_pack(BS, b), rtol=1e-10)
    u = _unpack(BS, U)
    print("iterations per pair:", it.tolist())
    assert (rel <= 1e-10).all()
    for p, n in enumerate(ns):
        n = int(n)
        h = 1.0 / n
        A = assemble.matrix_kron(n, h, alphas[p])
        ev = exact.eigenvalues(n, h, alphas[p])
        ue = exact.solve_fft(n, h, alphas[p], b[p])
        for r in range(nrhs):
            bn = np.linalg.norm(b[p][r])
            assert _true_residual_ok(A, b[p][r], u[p][r], 1e-10), (p, r)
            assert np.linalg.norm(u[p][r] - ue[r]) <= 2e-10 * bn / ev.min()


def test_batched_graph_replays_match_eager():
    ns, alphas, nrhs = [8, 16, 12, 16], [1.0, 0.1, 10.0, 2.0], 2
    Bg = _batch(ns, alphas, nrhs, "fp32", use_graphs=True)
    Be = _batch(ns, alphas, nrhs, "fp32", use_graphs=False)
    X = _pack(Bg, _loads(ns, nrhs, 80))
    Ue, ite, rele = Be.solve(X)
    Ue = _host(Ue)
    U = Bg.zeros()
    for rep in range(3):
        U.fill_(3.0)                     # eager work between replays
        _, it, rel = Bg.solve(X, U=U)
        assert np.array_equal(it, ite) and np.array_equal(rel, rele)
        assert np.array_equal(_host(U), Ue), rep


def test_batched_pairs_stop_independently():
    from paper_2205_05840_amd import _lib
    ns, alphas, nrhs = [8, 12], [1.0, 1.0], 2
    BS = _batch(ns, alphas, nrhs)
    b = _loads(ns, nrhs, 90)
    b[0][1] = 0.0
    X = _pack(BS, b)
    U, it, rel = BS.solve(X, maxit=2, raise_on_noconv=False)
    assert it[0, 1] == 0 and (it[0, 0] == 2) and (it[1] == 2).all()
    with pytest.raises(_lib.NdmgError) as e:
        BS.solve(X, maxit=2)
    assert e.value.code == _lib.NDMG_ENOCONV
    # a non-finite right-hand side breaks its own pair only
    Xn = X.clone()
    off = BS.offset(1)[0]
    Xn[off + BS.offset(1)[3] + 1] = float("nan")
    code, itn, reln = _lib.ndmg_pcg_solve_batched(BS.ctx, Xn.data_ptr(), BS.zeros().data_ptr(), 1e-10,
                                                  500, BS.npairs, raise_on_noconv=False,
                                                  raise_on_breakdown=False)
    torch.cuda.synchronize()
    assert code == _lib.NDMG_EBREAKDOWN
    itn = np.array(itn).reshape(2, 2)
    reln = np.array(reln).reshape(2, 2)
    assert itn[1, 0] == 0
    assert (reln[0, 0] <= 1e-10) and (reln[1, 1] <= 1e-10) and itn[0, 1] == 0


def test_multi_rhs_solver_and_autograd():
    """A single-problem solver holding k right-hand sides solves them in one call and
    gives the same iterations and (to rounding) the same solutions as k single solves;
    the differentiable solve uses it."""
    from paper_2205_05840_amd import Solver, solve
    n, k = 16, 3
    b = _loads([n], k, 100)[0]
    S1 = Solver(n, 1.0)
    Sk = Solver(n, 1.0, nrhs=k)
    Bk = torch.from_numpy(to_padded(n, Sk.P, Sk.B, b)).cuda()
    Uk, itk, relk = Sk.solve(Bk, rtol=1e-12)
    for r in range(k):
        u1, it1, rel1 = S1.solve(Bk[r].contiguous(), rtol=1e-12)
        assert abs(itk[r] - it1) <= 1
        assert _rel(_host(Uk[r]), _host(u1)) <= 1e-10
    Bg = Bk.clone().requires_grad_(True)
    a = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    L = (solve(Bg, a, Sk, rtol=1e-13) ** 2).sum()
    Lv = float(L.detach())
    L.backward()
    Bh = Bk.clone().requires_grad_(True)
    a1 = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    L1 = (solve(Bh, a1, S1, rtol=1e-13) ** 2).sum()
    L1v = float(L1.detach())
    L1.backward()
    assert abs(Lv - L1v) <= 1e-10 * abs(L1v)
    assert abs(float(a.grad) - float(a1.grad)) <= 1e-8 * abs(float(a1.grad))
    assert _rel(_host(Bg.grad), _host(Bh.grad)) <= 1e-9


def test_batched_bottom_levels_one_launch():
    """The one-launch bottom of the V-cycle (levels n_k <= 16 in one workgroup per pair)
    gives the same solves as the per-level launches, to rounding."""
    ns, alphas, nrhs = [8, 12, 16, 24], [1.0, 0.2, 30.0, 3.0], 2
    b = _loads(ns, nrhs, 120)
    Bs = [_batch(ns, alphas, nrhs, "fp64", bottom_n=bn) for bn in (0, 16)]
    out = []
    for BS in Bs:
        U, it, rel = BS.solve(_pack(BS, b), rtol=1e-12)
        assert (rel <= 1e-12).all()
        out.append((_unpack(BS, U), it))
    for p, n in enumerate(ns):
        ue = exact.solve_fft(n, 1.0 / n, alphas[p], b[p])
        for r in range(nrhs):
            assert abs(int(out[0][1][p, r]) - int(out[1][1][p, r])) <= 1
            assert _rel(out[1][0][p][r], ue[r]) <= 1e-9, (p, r)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_dense_bottom_matches_recursion(precision):
    """The bottom of the V-cycle as one dense matrix per problem (levels n_k <= 8, the
    default) against the recursion all the way down: V-cycle outputs agree to rounding
    and both solve every pair to the exact discrete solution."""
    ns, alphas, nrhs = [8, 12, 16, 6, 24, 8], [1.0, 0.2, 30.0, 3.0, 0.05, 7.0], 3
    b = _loads(ns, nrhs, 140)
    Bd = _batch(ns, alphas, nrhs, precision)
    Br = _batch(ns, alphas, nrhs, precision, dense_n=0)
    rng = np.random.default_rng(6)
    blocks = [rng.standard_normal((nrhs, mesh.ndof(n))) for n in ns]
    Zd = _unpack(Bd, Bd.vcycle(_pack(Bd, blocks)))
    Zr = _unpack(Br, Br.vcycle(_pack(Br, blocks)))
    if precision == "fp64":
        for p in range(len(ns)):
            for r in range(nrhs):
                assert _rel(Zd[p][r], Zr[p][r]) <= 1e-11, (p, r, _rel(Zd[p][r], Zr[p][r]))
    else:
        # FP32 rounding is amplified by the conditioning of the local solves (up to
        # 1e-3 relative at alpha h^-2 ~ 1e4): the dense form must be as close to the FP64
        # V-cycle as the recursion is
        B64 = _batch(ns, alphas, nrhs, "fp64", dense_n=0)
        Z64 = _unpack(B64, B64.vcycle(_pack(B64, blocks)))
        for p in range(len(ns)):
            for r in range(nrhs):
                ed, er = _rel(Zd[p][r], Z64[p][r]), _rel(Zr[p][r], Z64[p][r])
                assert ed <= 3.0 * max(er, 1e-6), (p, r, ed, er)
    rtol = 1e-12 if precision == "fp64" else 1e-11
    sols = []
    for BS in (Bd, Br):
        U, it, rel = BS.solve(_pack(BS, b), rtol=rtol)
        assert (rel <= rtol).all()
        sols.append((_unpack(BS, U), it))
    for p, n in enumerate(ns):
        ue = exact.solve_fft(n, 1.0 / n, alphas[p], b[p])
        for r in range(nrhs):
            assert abs(int(sols[0][1][p, r]) - int(sols[1][1][p, r])) <= 1
            for k in range(2):
                assert _rel(sols[k][0][p][r], ue[r]) <= 1e-7, (k, p, r)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_dense_bottom_many_problems(precision):
    """Classes of eight or more problems keep the dense bottom transposed (one thread per
    row); the V-cycle agrees with the recursion and solves reach the exact solution."""
    ns = [8] * 9 + [16] * 8 + [12] * 8
    alphas = [10.0 ** (-1.5 + 3.0 * p / (len(ns) - 1)) for p in range(len(ns))]
    nrhs = 2
    Bd = _batch(ns, alphas, nrhs, precision)
    Br = _batch(ns, alphas, nrhs, precision, dense_n=0)
    rng = np.random.default_rng(8)
    blocks = [rng.standard_normal((nrhs, mesh.ndof(n))) for n in ns]
    Zd = _unpack(Bd, Bd.vcycle(_pack(Bd, blocks)))
    Zr = _unpack(Br, Br.vcycle(_pack(Br, blocks)))
    if precision == "fp64":
        for p in range(len(ns)):
            for r in range(nrhs):
                assert _rel(Zd[p][r], Zr[p][r]) <= 1e-11, (p, r, _rel(Zd[p][r], Zr[p][r]))
    else:
        B64 = _batch(ns, alphas, nrhs, "fp64", dense_n=0)
        Z64 = _unpack(B64, B64.vcycle(_pack(B64, blocks)))
        for p in range(len(ns)):
            for r in range(nrhs):
                ed, er = _rel(Zd[p][r], Z64[p][r]), _rel(Zr[p][r], Z64[p][r])
                assert ed <= 3.0 * max(er, 1e-6), (p, r, ed, er)
    b = _loads(ns, nrhs, 160)
    rtol = 1e-12 if precision == "fp64" else 1e-11
    U, it, rel = Bd.solve(_pack(Bd, b), rtol=rtol)
    assert (rel <= rtol).all()
    sol = _unpack(Bd, U)
    for p, n in enumerate(ns):
        ue = exact.solve_fft(n, 1.0 / n, alphas[p], b[p])
        for r in range(nrhs):
            assert _rel(sol[p][r], ue[r]) <= 1e-7, (p, r)
