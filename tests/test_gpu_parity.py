"""GPU parity: the HIP library (through the C ABI) against the FP64 CPU oracle.

Tolerances (FP64, relative l2): apply 1e-14, transfers 1e-15.  The smoother and the
V-cycle go through inverted local matrices (A_T, and Schur complements S_V whose
condition grows like alpha h^-2), so any two correct FP64 evaluations already differ by
the rounding of those inverses, of relative size u kappa.  The scale of that rounding
is measured per case as the spread between the oracle evaluated with its factors from
two FP64 routes (LU and Cholesky).  The library's factors come from a third route (host
Cholesky with its own Schur complement sums), so its error is a third sample of the
same rounding: over the 29 smoother and V-cycle cases here it lies between 0.47 and
3.5 times the spread (deterministic: no atomics on either side).  The tolerance is
max(1e-13 resp. 1e-12, 5 * spread): 1.4 to 10.6 times every observed error.  PCG:
relative residual <= 1e-10 with the oracle's iteration count +-1; solution error
within the residual bound ||e|| <= ||r|| / lambda_min(A).
"""
import numpy as np
import pytest

from layout import boundary_mask, from_padded, to_padded
from oracle import assemble, exact, mesh, pcg, rhs, smoother, transfer, vcycle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

C64 = 5.0   # tolerance / spread of the oracle's two FP64 routes (see above)


def _solver(n, alpha=1.0, **kw):
    from paper_2205_05840_amd import Solver
    print(f"[case] n={n} alpha={alpha} {kw}", flush=True)
    return Solver(n, alpha, **kw)


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


@pytest.mark.parametrize("n,alpha", [(4, 1.0), (7, 2.0), (8, 0.37), (14, 5.0), (16, 100.0),
                                     (40, 1.0)])
def test_apply(n, alpha):
    S = _solver(n, alpha)
    h = 1.0 / n
    x = np.random.default_rng(n).standard_normal(mesh.ndof(n))
    y = _host(S.apply(_dev(to_padded(n, S.P, S.B, x))))
    ref = assemble.matrix_kron(n, h, alpha) @ x
    assert _rel(from_padded(n, S.P, S.B, y), ref) <= 1e-14
    assert np.all(y[boundary_mask(n, S.P, S.B)] == 0.0)


@pytest.mark.parametrize("n", [8, 10, 12, 14, 32])
def test_transfers(n):
    S = _solver(n, 1.0)
    J = S.levels - 1
    nf, Pf, Bf = _lvl(S, J)
    nc, Pc, Bc = _lvl(S, J - 1)
    rng = np.random.default_rng(1)
    rf = rng.standard_normal(mesh.ndof(nf))
    gc = _host(S.level_op(J, "restrict", _dev(to_padded(nf, Pf, Bf, rf))))
    Pm = transfer.prolongation(nc)
    assert _rel(from_padded(nc, Pc, Bc, gc), Pm.T @ rf) <= 1e-15
    ec = rng.standard_normal(mesh.ndof(nc))
    zf0 = rng.standard_normal(mesh.ndof(nf))
    zf = _dev(to_padded(nf, Pf, Bf, zf0))
    S.level_op(J, "prolong", _dev(to_padded(nc, Pc, Bc, ec)), out=zf)
    zh = _host(zf)
    assert _rel(from_padded(nf, Pf, Bf, zh), zf0 + Pm @ ec) <= 1e-15
    assert not zh[boundary_mask(nf, Pf, Bf)].any()   # non-unknown entries untouched (zero)


@pytest.mark.parametrize("n,alpha,boundary", [(4, 1.0, True), (8, 0.3, True), (8, 3.0, False),
                                              (10, 1.0, True), (10, 2.0, False), (12, 10.0, True),
                                              (14, 0.5, True), (14, 5.0, False), (16, 0.01, True)])
def test_smoother(n, alpha, boundary):
    S = _solver(n, alpha, boundary_patches=boundary)
    h = 1.0 / n
    A = assemble.matrix_kron(n, h, alpha)
    r = np.random.default_rng(2).standard_normal(mesh.ndof(n))
    z = _host(S.level_op(S.levels - 1, "smooth", _dev(to_padded(n, S.P, S.B, r))))
    ref = smoother.FactoredVertexSmoother(A, n, 2, boundary=boundary)(r)
    alt = smoother.FactoredVertexSmoother(A, n, 2, boundary=boundary, inverse="cholesky")(r)
    tol = max(1e-13, C64 * _rel(alt, ref))
    err = _rel(from_padded(n, S.P, S.B, z), ref)
    print(f"smoother fp64: err {err:.2e}, spread {_rel(alt, ref):.2e}, ratio {err / max(_rel(alt, ref), 1e-300):.2f}")
    assert err <= tol
    if n <= 8:
        ref2 = smoother.LiteralSmoother(A, n, 2, boundary=boundary)(r)
        assert _rel(from_padded(n, S.P, S.B, z), ref2) <= tol


@pytest.mark.parametrize("boundary", [True, False])
def test_smoother_after_small_level_kernel(boundary):
    """The one-launch small-level kernel and the per-level smoother share a level's buffer
    of patch results in different layouts; vertices without a patch must still read
    zeros in the per-level smoother after the small-level kernel has filled the buffer."""
    n, alpha = 16, 0.5
    S = _solver(n, alpha, boundary_patches=boundary, bottom_n=n)
    rng = np.random.default_rng(11)
    g = rng.standard_normal(mesh.ndof(n))
    S.vcycle(_dev(to_padded(n, S.P, S.B, g)))   # fills the buffers in the small-level layout
    A = assemble.matrix_kron(n, 1.0 / n, alpha)
    r = rng.standard_normal(mesh.ndof(n))
    z = _host(S.level_op(S.levels - 1, "smooth", _dev(to_padded(n, S.P, S.B, r))))
    ref = smoother.FactoredVertexSmoother(A, n, 2, boundary=boundary)(r)
    alt = smoother.FactoredVertexSmoother(A, n, 2, boundary=boundary, inverse="cholesky")(r)
    assert _rel(from_padded(n, S.P, S.B, z), ref) <= max(1e-13, C64 * _rel(alt, ref))


@pytest.mark.parametrize("precision,n,nrhs", [("fp32", 64, 1), ("fp64", 64, 1), ("fp32", 32, 4),
                                               ("fp64", 24, 4)])
def test_patch_addressing_forms_agree(precision, n, nrhs):
    """The smoother's condensation and vertex patch products address their loads and
    stores either through buffer descriptors with 32-bit byte offsets (in the patch
    products an absent slot's offset lies past the range and reads zero) or with 64-bit
    addresses (the form for vectors of 2 GB or more, selected here by table entries
    "patchaddr" for every level).  The V-cycle must come out the same bit for bit; several
    right-hand sides take the waves that serve one pair each."""
    import os
    from paper_2205_05840_amd import _lib
    L = _lib.lib()
    cls = 0 if nrhs == 1 else 2
    S = _solver(n, 0.8, precision=precision, nrhs=nrhs)
    rng = np.random.default_rng(n)
    g = (torch.from_numpy(rng.standard_normal((nrhs, S.vec_len))).cuda() * S.unknown_mask()).contiguous()
    if nrhs == 1:
        g = g[0].contiguous()
    z32 = _host(S.vcycle(g))
    try:
        k = n
        while k >= 4:
            _lib.check(L.ndmg_tuning_set(f"patchaddr {k} {precision} 0 {cls} 64 1".encode()))
            k //= 2
        S64 = _solver(n, 0.8, precision=precision, nrhs=nrhs)
        z64 = _host(S64.vcycle(g))
    finally:
        L.ndmg_tuning_clear()
        if os.path.exists(_lib.TUNING_PATH):
            L.ndmg_tuning_load(_lib.TUNING_PATH.encode())
    print(f"{precision} n={n} nrhs={nrhs}: max |z| {np.abs(z32).max():.3e}, "
          f"differing entries {int((z32 != z64).sum())}")
    assert np.array_equal(z32, z64)


def test_exported_factors_match_patch_matrices():
    n, alpha = 8, 0.7
    S = _solver(n, alpha)
    A = assemble.matrix_kron(n, 1.0 / n, alpha)
    F = smoother.FactoredVertexSmoother(A, n, 2)
    Sinv = S.export_factor(S.levels - 1, 1, 13)[:60, :60]
    np.testing.assert_allclose(Sinv, np.linalg.inv(F.schur(13)), rtol=1e-11,
                               atol=1e-12 * abs(Sinv).max())
    ATinv = S.export_factor(S.levels - 1, 0)
    np.testing.assert_allclose(ATinv, F.ATinv, rtol=1e-12, atol=1e-13 * abs(ATinv).max())


@pytest.mark.parametrize("n", [2, 3, 5, 7])
def test_coarse_only(n):
    S = _solver(n, 2.0)
    assert S.levels == 1
    b = np.random.default_rng(n).standard_normal(mesh.ndof(n))
    z = _host(S.vcycle(_dev(to_padded(n, S.P, S.B, b))))
    ref = exact.solve_direct(n, 1.0 / n, 2.0, b)
    assert _rel(from_padded(n, S.P, S.B, z), ref) <= 1e-12


@pytest.mark.parametrize("n,alpha,m,boundary", [(4, 1.0, 1, True), (8, 1.0, 1, True),
                                                (8, 0.01, 2, True), (10, 1.0, 1, True),
                                                (12, 100.0, 1, False), (16, 1.0, 1, True)])
def test_vcycle(n, alpha, m, boundary):
    _check_vcycle(n, alpha, m, boundary, None)


@pytest.mark.parametrize("n,alpha,m,bottom", [(8, 1.0, 1, 0), (12, 3.0, 2, 0), (16, 0.5, 1, 16),
                                              (24, 1.0, 1, 12), (32, 20.0, 1, 16)])
def test_vcycle_bottom_levels(n, alpha, m, bottom):
    """The bottom of the V-cycle as one launch (bottom levels n_k <= bottom) and as one
    launch per step (bottom = 0) both match the oracle."""
    _check_vcycle(n, alpha, m, True, bottom)


@pytest.mark.parametrize("n,alpha,m,dense", [(4, 1.0, 1, 8), (8, 0.01, 2, 8), (12, 100.0, 1, 8),
                                             (16, 1.0, 1, 8), (16, 1.0, 1, 4), (32, 3.0, 1, 8),
                                             (8, 1.0, 1, 0), (16, 1.0, 1, 0), (12, 100.0, 1, 0)])
def test_vcycle_dense_bottom(n, alpha, m, dense):
    """The V-cycle with its bottom (from the finest level with n_k <= dense down) applied
    as one dense matrix per problem, and with the recursion all the way (dense = 0),
    against the oracle."""
    _check_vcycle(n, alpha, m, True, None, dense)


def test_vcycle_dense_top_clears_output():
    """At n = 8 the whole V-cycle is the dense matrix; entries of the output that are not
    unknowns come out zero whatever the buffer held."""
    n = 8
    S = _solver(n, 1.0)
    g = np.random.default_rng(5).standard_normal(mesh.ndof(n))
    z = torch.full((S.vec_len,), 7.0, dtype=torch.float64, device="cuda")
    z = _host(S.vcycle(_dev(to_padded(n, S.P, S.B, g)), z))
    assert not z[boundary_mask(n, S.P, S.B)].any()
    ref = vcycle.Hierarchy(n, 1.0, m=1, boundary=True, factored=True).precondition(g)
    assert _rel(from_padded(n, S.P, S.B, z), ref) <= 1e-12


@pytest.mark.parametrize("n,levels,alpha", [(12, 2, 1.0), (16, 3, 0.2), (32, 4, 5.0)])
def test_vcycle_fewer_levels(n, levels, alpha):
    """levels = L keeps the L finest levels; the coarsest kept level is solved exactly."""
    _check_vcycle(n, alpha, 1, True, None, levels=levels)
    S = _solver(n, alpha, levels=levels)
    assert S.levels == levels and S.layout(0)[0] == n >> (levels - 1)


def _check_vcycle(n, alpha, m, boundary, bottom, dense=None, levels=None):
    S = _solver(n, alpha, m=m, boundary_patches=boundary, bottom_n=bottom, dense_n=dense,
                **({"levels": levels} if levels else {}))
    H = vcycle.Hierarchy(n, alpha, m=m, boundary=boundary, factored=True, levels=levels)
    H2 = vcycle.Hierarchy(n, alpha, m=m, boundary=boundary, factored=True, inverse="cholesky",
                          levels=levels)
    g = np.random.default_rng(3).standard_normal(mesh.ndof(n))
    z = _host(S.vcycle(_dev(to_padded(n, S.P, S.B, g))))
    ref = H.precondition(g)
    spread = _rel(H2.precondition(g), ref)
    tol = max(1e-12, C64 * spread)
    err = _rel(from_padded(n, S.P, S.B, z), ref)
    print(f"V-cycle fp64: err {err:.2e}, spread {spread:.2e}, ratio {err / max(spread, 1e-300):.2f}")
    assert err <= tol


@pytest.mark.parametrize("n,alpha", [(8, 1.0), (16, 0.01), (16, 100.0), (24, 1.0), (32, 1.0)])
def test_pcg(n, alpha):
    from paper_2205_05840_amd import synth
    S = _solver(n, alpha)
    h = 1.0 / n
    f = synth.normal_samples(n, 0)
    b_o = rhs.load_from_samples(n, h, f)
    b = S.assemble_rhs(torch.from_numpy(f))
    assert _rel(from_padded(n, S.P, S.B, _host(b)), b_o) <= 1e-14
    u, it, rel = S.solve(b, rtol=1e-10)
    u_c = from_padded(n, S.P, S.B, _host(u))
    A = assemble.matrix_kron(n, h, alpha)
    assert rel <= 1e-10
    assert np.linalg.norm(b_o - A @ u_c) <= 1.5e-10 * np.linalg.norm(b_o)
    H = vcycle.Hierarchy(n, alpha)
    _, it_o, _, _ = pcg.pcg(A, b_o, H.precondition, rtol=1e-10)
    assert abs(it - it_o) <= 1, (it, it_o)
    ue = exact.solve_fft(n, h, alpha, b_o)
    ev = exact.eigenvalues(n, h, alpha)
    # error bound from the residual: ||e|| <= ||r|| / lambda_min
    assert np.linalg.norm(u_c - ue) <= 2e-10 * np.linalg.norm(b_o) / ev.min()


def test_pcg_solution_to_tight_tolerance():
    """Solution protocol: run to 1e-13 and compare with the exact discrete solution."""
    n, alpha = 32, 1.0
    S = _solver(n, alpha)
    b_o = np.random.default_rng(7).standard_normal(mesh.ndof(n))
    u, it, rel = S.solve(_dev(to_padded(n, S.P, S.B, b_o)), rtol=1e-13)
    ue = exact.solve_fft(n, 1.0 / n, alpha, b_o)
    assert _rel(from_padded(n, S.P, S.B, _host(u)), ue) <= 1e-9


def test_pcg_edge_cases():
    from paper_2205_05840_amd import _lib
    n = 8
    S = _solver(n, 1.0)
    zero = S.zeros()
    u, it, rel = S.solve(zero)
    assert it == 0 and rel == 0.0 and float(_host(u).max()) == 0.0
    b = _dev(to_padded(n, S.P, S.B, np.random.default_rng(0).standard_normal(mesh.ndof(n))))
    u, it, rel = S.solve(b, rtol=1e-10, maxit=1, raise_on_noconv=False)
    assert it == 1 and rel > 1e-10 and np.isfinite(_host(u)).all()
    with pytest.raises(_lib.NdmgError) as e:
        S.solve(b, rtol=1e-10, maxit=1)
    assert e.value.code == _lib.NDMG_ENOCONV
    bn = b.clone()
    bn[S.P + 1] = float("nan")
    with pytest.raises(_lib.NdmgError) as e:
        S.solve(bn)
    assert e.value.code == _lib.NDMG_EBREAKDOWN
    # vectors one double off 16-byte alignment are refused before any work
    buf = torch.zeros(S.vec_len + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.NdmgError) as e:
        S.solve(b, u=buf[1:])
    assert e.value.code == _lib.NDMG_EINVAL


def test_curlcurl_form():
    n = 8
    S = _solver(n, 1.0)
    rng = np.random.default_rng(5)
    lam = rng.standard_normal((3, mesh.ndof(n)))
    uu = rng.standard_normal((3, mesh.ndof(n)))
    K = assemble.stiffness_kron(n, 1.0 / n)
    ref = sum(lam[r] @ (K @ uu[r]) for r in range(3))
    got = S.curlcurl_form(_dev(to_padded(n, S.P, S.B, lam)), _dev(to_padded(n, S.P, S.B, uu)))
    assert abs(got - ref) <= 1e-13 * np.sum(np.abs(lam) * np.abs((abs(K) @ np.abs(uu).T).T))


@pytest.mark.parametrize("n", [4, 7, 10])
def test_assemble_rhs(n):
    from paper_2205_05840_amd import synth
    S = _solver(n, 1.0)
    f = synth.normal_samples(n, 11)
    b = _host(S.assemble_rhs(torch.from_numpy(f)))
    assert _rel(from_padded(n, S.P, S.B, b), rhs.load_from_samples(n, 1.0 / n, f)) <= 1e-14


def test_mixed_precision_pcg():
    """FP32 V-cycle inside FP64 flexible CG still reaches 1e-10; error vs FP64 reported."""
    from paper_2205_05840_amd import synth
    n, alpha = 32, 1.0
    h = 1.0 / n
    S64 = _solver(n, alpha)
    S32 = _solver(n, alpha, precision="fp32")
    f = synth.normal_samples(n, 2)
    b = S64.assemble_rhs(torch.from_numpy(f))
    u64, it64, rel64 = S64.solve(b)
    u32, it32, rel32 = S32.solve(b)
    assert rel32 <= 1e-10 and abs(it32 - it64) <= 1
    b_o = rhs.load_from_samples(n, h, f)
    A = assemble.matrix_kron(n, h, alpha)
    u_c = from_padded(n, S32.P, S32.B, _host(u32))
    assert np.linalg.norm(b_o - A @ u_c) <= 1.5e-10 * np.linalg.norm(b_o)
    err = _rel(u_c, from_padded(n, S64.P, S64.B, _host(u64)))
    print(f"mixed vs fp64: iters {it32} vs {it64}, rel diff {err:.2e}")
    # the V-cycle itself agrees with the FP64 oracle to single precision
    g = np.random.default_rng(3).standard_normal(mesh.ndof(n))
    z = _host(S32.vcycle(_dev(to_padded(n, S32.P, S32.B, g))))
    ref = vcycle.Hierarchy(n, alpha).precondition(g)
    # a few roundings of relative size 2^-24 per entry (see test_gpu_precision.py)
    err32 = _rel(from_padded(n, S32.P, S32.B, z), ref)
    print(f"FP32 V-cycle vs FP64 oracle: {err32:.2e}")
    assert err32 <= 12 * 2.0 ** -24


def test_graph_replays_match_eager():
    """The CG iterations replayed from captured graphs give bitwise the same iterates as
    the eager launches; several solves in a row (replays with eager work and host
    synchronisation in between), then a solve into a different output (re-capture)."""
    from paper_2205_05840_amd import synth
    n = 16
    Sg = _solver(n, 1.0, use_graphs=True)
    Se = _solver(n, 1.0, use_graphs=False)
    b = Sg.assemble_rhs(torch.from_numpy(synth.normal_samples(n, 5)))
    ue, ite, rele = Se.solve(b)
    ue = _host(ue)
    u = Sg.zeros()
    for rep in range(3):
        u.fill_(7.0)                     # eager work between replays
        _, it, rel = Sg.solve(b, u=u)
        assert it == ite and rel == rele
        assert np.array_equal(_host(u), ue), rep
    u2, it, rel = Sg.solve(b)
    assert np.array_equal(_host(u2), ue)
    S32 = _solver(n, 1.0, precision="fp32")
    S32e = _solver(n, 1.0, precision="fp32", use_graphs=False)
    assert np.array_equal(_host(S32.solve(b)[0]), _host(S32e.solve(b)[0]))
