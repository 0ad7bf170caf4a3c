"""GPU parity of the plane-marching operator kernel (one position per lane up to n = 64,
two up to 128) against the FP64 oracle: the apply on sampled rows (element definition, up to the 128^3 bench
size), the FP64 V-cycle (its residuals use the kernel's residual mode), and PCG (its
p^T A p uses the dot mode) in FP64 and mixed precision against the exact discrete
solution.  n = 80 and 112 give tile counts that leave padding workgroups."""
import numpy as np
import pytest

from layout import boundary_mask, from_padded, to_padded
from oracle import assemble, exact, mesh, pcg, rhs, vcycle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _solver(n, alpha=1.0, **kw):
    from paper_2205_05840_amd import Solver
    print(f"[case] n={n} alpha={alpha} {kw}", flush=True)
    return Solver(n, alpha, **kw)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("n,alpha", [(80, 1.0), (96, 0.01), (112, 37.0), (128, 1.0)])
def test_apply_sampled_rows(n, alpha):
    S = _solver(n, alpha)
    h = 1.0 / n
    x = np.random.default_rng(n).standard_normal(mesh.ndof(n))
    y = _host(S.apply(torch.from_numpy(to_padded(n, S.P, S.B, x)).cuda()))
    # random rows plus every row next to a tile edge in y and z (rows 0, 1, 7, 8, ...)
    rng = np.random.default_rng(1)
    d, p = mesh.edge_coords(n)
    edge = np.nonzero((p[:, 1] % 8 <= 1) | (p[:, 1] % 8 == 7) | (p[:, 2] % 8 <= 1) |
                      (p[:, 2] % 8 == 7))[0]
    rows = np.unique(np.concatenate([rng.choice(mesh.ndof(n), 20000, replace=False),
                                     rng.choice(edge, 20000, replace=False)]))
    ref = assemble.apply_rows(n, h, alpha, x, rows)
    got = from_padded(n, S.P, S.B, y)[rows]
    assert _rel(got, ref) <= 1e-14
    assert np.all(y[boundary_mask(n, S.P, S.B)] == 0.0)


@pytest.mark.parametrize("n,alpha", [(80, 1.0), (96, 40.0)])
def test_vcycle_fp64(n, alpha):
    S = _solver(n, alpha)
    H = vcycle.Hierarchy(n, alpha, factored=True)
    H2 = vcycle.Hierarchy(n, alpha, factored=True, inverse="cholesky")
    g = np.random.default_rng(3).standard_normal(mesh.ndof(n))
    z = _host(S.vcycle(torch.from_numpy(to_padded(n, S.P, S.B, g)).cuda()))
    ref = H.precondition(g)
    spread = _rel(H2.precondition(g), ref)
    tol = max(1e-12, 5 * spread)   # as in test_gpu_parity.py
    err = _rel(from_padded(n, S.P, S.B, z), ref)
    print(f"V-cycle fp64: err {err:.2e}, spread {spread:.2e}, ratio {err / spread:.2f}")
    assert err <= tol


@pytest.mark.parametrize("n,alpha,precision", [(80, 1.0, "fp64"), (80, 1.0, "fp32"),
                                               (112, 0.05, "fp32")])
def test_pcg(n, alpha, precision):
    from paper_2205_05840_amd import synth
    S = _solver(n, alpha, precision=precision)
    h = 1.0 / n
    f = synth.normal_samples(n, 0)
    b_o = rhs.load_from_samples(n, h, f)
    b = S.assemble_rhs(torch.from_numpy(f))
    u, it, rel = S.solve(b, rtol=1e-10)
    assert rel <= 1e-10
    u_c = from_padded(n, S.P, S.B, _host(u))
    ue = exact.solve_fft(n, h, alpha, b_o)
    ev = exact.eigenvalues(n, h, alpha)
    # error bound from the residual (plus the recursive/true residual gap)
    assert np.linalg.norm(u_c - ue) <= 3e-10 * np.linalg.norm(b_o) / ev.min()
    if precision == "fp64" and n == 80:
        A = assemble.matrix_kron(n, h, alpha)
        H = vcycle.Hierarchy(n, alpha)
        _, it_o, _, _ = pcg.pcg(A, b_o, H.precondition, rtol=1e-10)
        assert abs(it - it_o) <= 1, (it, it_o)
    if precision == "fp32":
        # the mixed form needs no more iterations than the FP64 V-cycle (+-1)
        S64 = _solver(n, alpha)
        _, it64, _ = S64.solve(b, rtol=1e-10)
        print(f"fp32 {it} vs fp64 {it64} iterations")
        assert abs(it - it64) <= 1, (it, it64)
    print(f"{precision} n={n}: {it} iterations, relres {rel:.2e}")


def test_pcg_bench_size_mixed():
    """The 128^3 bench configuration (alpha = 1, f ~ N(0, 1) at the Gauss points, seed 2,
    FP32 V-cycle in FP64 CG): relative residual and solution against the exact discrete
    solution (FFT)."""
    from paper_2205_05840_amd import synth
    n = 128
    h = 1.0 / n
    S = _solver(n, 1.0, precision="fp32")
    f = synth.normal_samples(n, 2)
    b = S.assemble_rhs(torch.from_numpy(f))
    u, it, rel = S.solve(b, rtol=1e-10)
    assert rel <= 1e-10 and it <= 30
    S64 = _solver(n, 1.0)
    _, it64, _ = S64.solve(b, rtol=1e-10)
    assert abs(it - it64) <= 1, (it, it64)
    del S64
    b_o = rhs.load_from_samples(n, h, f)
    ue = exact.solve_fft(n, h, 1.0, b_o)
    ev_min = h ** 3 / 9.0   # lower bound of the spectrum (symbol of A)
    err = np.linalg.norm(from_padded(n, S.P, S.B, _host(u)) - ue)
    print(f"128^3 mixed: {it} iterations, relres {rel:.2e}, |u - u_exact| / |u_exact| "
          f"{err / np.linalg.norm(ue):.2e}")
    assert err <= 3e-10 * np.linalg.norm(b_o) / ev_min


# (precision, mode, n, planes per workgroup, [(two-barrier variant, one-barrier variant)])
SYNC_CASES = [("fp64", 0, 64, 4, [(2, 3)]), ("fp64", 0, 128, 16, [(2, 3)]),
              ("fp64", 1, 64, 4, [(2, 3)]),
              ("fp32", 1, 64, 3, [(0, 2), (1, 3)]), ("fp32", 1, 128, 12, [(0, 2), (1, 3)])]


@pytest.mark.parametrize("prec,mode,n,kz,pairs", SYNC_CASES)
def test_one_barrier_form_agrees(prec, mode, n, kz, pairs):
    """The operator kernel's form with one barrier per step (two copies of the y-exchange
    area, used by step parity) against the form with two, at the same tiling: the FP64
    apply (mode 0) and the FP32 V-cycle whose level-n residuals use mode 1 must agree bit
    for bit, on every one of repeated launches (an ordering fault would show as a change
    between launches)."""
    import os
    from paper_2205_05840_amd import _lib
    L = _lib.lib()
    S = _solver(n, 0.9, precision=prec)
    g = torch.Generator(device="cuda")
    g.manual_seed(n + mode)
    x = (torch.randn(S.vec_len, generator=g, dtype=torch.float64, device="cuda") * S.unknown_mask()).contiguous()
    run = (lambda: S.apply(x)) if mode == 0 else (lambda: S.vcycle(x))
    try:
        for two, one in pairs:
            outs = {}
            for v in (two, one):
                L.ndmg_tuning_clear()
                _lib.check(L.ndmg_tuning_set(f"stencil {n} {prec} {mode} 0 {v} {kz}".encode()))
                ref = _host(run())
                same = all(np.array_equal(_host(run()), ref) for _ in range(10))
                outs[v] = ref
                print(f"{prec} mode {mode} n={n} variant {v} kz {kz}: repeats identical {same}")
                assert same
            assert np.array_equal(outs[two], outs[one])
    finally:
        L.ndmg_tuning_clear()
        if os.path.exists(_lib.TUNING_PATH):
            L.ndmg_tuning_load(_lib.TUNING_PATH.encode())


@pytest.mark.parametrize("n", [40, 64])
def test_one_position_per_lane_shapes(n):
    """Up to n = 64 the operator kernel gives each lane one position of a row (n = 64: the
    position i = n is written apart).  Every launch variant and several plane counts per
    workgroup must give the same apply bit for bit, and it must match the element
    definition on sampled rows (random, and next to tile edges in y and z)."""
    import os
    from paper_2205_05840_amd import _lib
    L = _lib.lib()
    S = _solver(n, 2.5)
    h = 1.0 / n
    x = np.random.default_rng(n + 7).standard_normal(mesh.ndof(n))
    xd = torch.from_numpy(to_padded(n, S.P, S.B, x)).cuda()
    outs = []
    try:
        for v in range(4):
            for kz in (2, 5, n):
                L.ndmg_tuning_clear()
                _lib.check(L.ndmg_tuning_set(f"stencil {n} fp64 0 0 {v} {kz}".encode()))
                outs.append(((v, kz), _host(S.apply(xd))))
    finally:
        L.ndmg_tuning_clear()
        if os.path.exists(_lib.TUNING_PATH):
            L.ndmg_tuning_load(_lib.TUNING_PATH.encode())
    ref_shape, y = outs[0]
    for shape, o in outs[1:]:
        assert np.array_equal(o, y), (shape, ref_shape)
    rng = np.random.default_rng(2)
    d, p = mesh.edge_coords(n)
    edge = np.nonzero((p[:, 1] % 8 <= 1) | (p[:, 1] % 8 == 7) | (p[:, 2] % 5 <= 1))[0]
    rows = np.unique(np.concatenate([rng.choice(mesh.ndof(n), 8000, replace=False),
                                     rng.choice(edge, 8000, replace=False)]))
    ref = assemble.apply_rows(n, h, 2.5, x, rows)
    assert _rel(from_padded(n, S.P, S.B, y)[rows], ref) <= 1e-14
    assert np.all(y[boundary_mask(n, S.P, S.B)] == 0.0)
