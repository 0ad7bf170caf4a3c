"""Benchmark: V-cycle-preconditioned CG at 128^3 on one MI355X, mixed precision vs FP64.

A step is one complete ndmg_pcg_solve (u0 = 0 to ||b - A u|| <= 1e-10 ||b||) of the
128^3 unit-cube problem (6,193,536 interior-edge unknowns, alpha = 1, f ~ N(0, 1) at
the 2x2x2 Gauss points, seed 2), with the right-hand side already resident in HBM and
the setup done before the timed region.  The headline leg runs the V-cycle in FP32
inside FP64 flexible CG; the FP64 leg (V-cycle in FP64) is reported next to it, and
both are repeated at alpha = 1e-3.

More forms are measured next to the plain FP64 path and reported under "forms":
batched (512 problems with n drawn from {8, 12, 16, 24, 32} and alpha log-uniform in
[1e-2, 1e2], 4 right-hand sides each, FP32 V-cycle in FP64 CG, one batched solve per
step; against single FP64 solves of a sample of the same problems), differentiated
(96^3, 16 right-hand sides, loss sum_k ||u_k - t_k||^2 with t_k the alpha = 2
solutions, forward and adjoint solves plus dL/dalpha per step; against the same
gradient through single-right-hand-side solves), the 64^3 manufactured-field
configuration (alpha 0.01, 1, 100; subdomains of 2 and 4 elements; the edge smoother at
alpha = 1), implicit Maxwell time stepping at 128^3 (steps per second) and a coefficient with
jumps at 128^3 (alpha constant on each of 4^3 boxes, contrast up to 1e4) and a non-box
domain at 128^3 (the cube less one octant).

Prints one JSON line.  Options: --gpus N (only 1 is supported), --steps K, --warmup W,
--no-cpu-baseline, --no-forms.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_ELEM = 128
SEED = 2
RTOL = 1e-10
BATCH_NPROB, BATCH_NRHS, BATCH_SEED = 512, 4, 3
BATCH_SAMPLE = 16          # problems of the sequential FP64 comparison
DIFF_N, DIFF_NRHS, DIFF_SEED = 96, 16, 4


def log(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(files):
    """Hash of library sources (a counter reading is valid for the sources it was taken on)."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2205_05840_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, prec):
    """HBM bytes per launch (per solve for kernel "solve") from the committed rocprofv3
    counter summary, if its entry was taken on the current sources it lists; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get("kernels", {}).get(f"{kernel}:{prec}")
    if ent is None or ent.get("source_hash") != source_hash(ent.get("sources", [])):
        return None
    return ent.get("bytes")


def run_leg(torch, Solver, f, alpha, precision, steps, warmup):
    S = Solver(N_ELEM, alpha, precision=precision)
    b = S.assemble_rhs(f)
    u = S.zeros()
    for _ in range(warmup):
        S.solve(b, rtol=RTOL, u=u)
    torch.cuda.synchronize()
    times, iters, rels = [], [], []
    t_all0 = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        _, it, rel = S.solve(b, rtol=RTOL, u=u)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        iters.append(it)
        rels.append(rel)
    t_all = time.perf_counter() - t_all0
    # true residual in FP64
    r = b - S.apply(u)
    true_rel = float(torch.linalg.norm(r) / torch.linalg.norm(b))
    return S, b, u, {"s_per_solve_total": t_all / steps, "s_per_solve_median": sorted(times)[len(times) // 2],
                     "iters": iters[-1], "relres": rels[-1], "true_relres": true_rel}


def time_apply(torch, S, reps=40, nbuf=8):
    """Average duration of the operator-apply kernel (one launch per ndmg_apply), timed
    with HIP events on the library's stream, rotating over nbuf input/output pairs so that
    the 256 MB last-level cache cannot hold them.  The loop calls the C ABI directly (a
    few microseconds per call) so that the launches queue up ahead of the GPU and the
    events measure the kernels, not the host."""
    from paper_2205_05840_amd import _lib
    xs = [torch.randn(S.vec_len, dtype=torch.float64, device=S.device) for _ in range(nbuf)]
    mask = S.unknown_mask()
    xs = [(x * mask).contiguous() for x in xs]
    ys = [S.zeros() for _ in range(nbuf)]
    for i in range(nbuf):
        S.apply(xs[i], ys[i])
    ptrs = [(xs[i].data_ptr(), ys[i].data_ptr()) for i in range(nbuf)]
    L = _lib.lib()
    torch.cuda.synchronize()
    st = S.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # a first batch of launches keeps the GPU busy while the timed ones are queued
    for i in range(nbuf):
        _lib.check(L.ndmg_apply(S.ctx, *ptrs[i]))
    e0.record(st)
    for i in range(reps):
        _lib.check(L.ndmg_apply(S.ctx, *ptrs[i % nbuf]))
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def patch_flops(n):
    """Useful flops of one launch of the fine-level vertex patch products at n^3 (2 x 2 x 2
    subdomains, vertex spaces at boundary coarse vertices too): 2 |Gamma_V|^2 per
    non-empty patch.  With nH = n / 2 coarse cells per axis there are (nH - 1)^3 interior
    vertices with 60 interface unknowns, 6 (nH - 1)^2 on the faces of the box with 18
    (the 2 fine edges of the inward coarse edge and 4 in each of the 4 inward faces) and
    12 (nH - 1) on its edges with 4 (the one face between the two boundary planes); the 8
    corners have none.  The padding of the MFMA tiles is not counted."""
    m = n // 2 - 1
    return 2 * (m ** 3 * 60 ** 2 + 6 * m ** 2 * 18 ** 2 + 12 * m * 4 ** 2)


def time_patch(torch, S, reps=40):
    """Average duration of the fine-level patch products (k_sm_patch alone, one launch per
    call), timed with HIP events on the library's stream over `reps` launches queued
    behind a first batch, on the condensed residual left by one smoother application."""
    from paper_2205_05840_amd import _lib
    r = (torch.randn(S.vec_len, dtype=torch.float64, device=S.device) * S.unknown_mask()).contiguous()
    S.level_op(-1, "smooth", r)
    L = _lib.lib()
    ptr = r.data_ptr()
    torch.cuda.synchronize()
    st = S.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(8):
        _lib.check(L.ndmg_level_op(S.ctx, -1, _lib.NDMG_OP_PATCH, ptr, ptr))
    e0.record(st)
    for _ in range(reps):
        _lib.check(L.ndmg_level_op(S.ctx, -1, _lib.NDMG_OP_PATCH, ptr, ptr))
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def batched_leg(torch, steps, warmup):
    """512 uneven problems x 4 right-hand sides in one batched solve per step (FP32
    V-cycle in FP64 CG); the same batch with the FP64 V-cycle; and single FP64 solves of
    the first BATCH_SAMPLE problems one after another."""
    from paper_2205_05840_amd import BatchedSolver, Solver, synth
    ns, alphas = synth.batched_problems(BATCH_NPROB, seed=BATCH_SEED)
    dof = [3 * int(n) * (int(n) - 1) ** 2 for n in ns]
    out = {"nprob": BATCH_NPROB, "nrhs": BATCH_NRHS, "sizes": sorted(set(int(n) for n in ns)),
           "dof_rhs_total": sum(dof) * BATCH_NRHS}
    B = None
    for prec in ("fp32", "fp64"):
        t0 = time.perf_counter()
        BS = BatchedSolver(ns, alphas, nrhs=BATCH_NRHS, precision=prec)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        if B is None:
            g = torch.Generator(device=BS.device)
            g.manual_seed(BATCH_SEED)
            f = torch.randn(BS.sample_len(), generator=g, dtype=torch.float64, device=BS.device)
            B = BS.assemble_rhs(f)
            del f
        U = BS.zeros()
        for _ in range(warmup):
            BS.solve(B, rtol=RTOL, U=U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, it, rel = BS.solve(B, rtol=RTOL, U=U)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        npairs = BATCH_NPROB * BATCH_NRHS
        log(f"batched {prec}: setup {setup:.1f} s, {t * 1e3:.1f} ms per batch of {npairs} solves")
        out[prec] = {"s_per_batch": t, "solves_per_s": npairs / t,
                     "dof_rhs_per_s": out["dof_rhs_total"] / t, "setup_s": setup,
                     "iters_max": int(it.max()), "iters_mean": float(it.mean()),
                     "relres_max": float(rel.max())}
        if prec == "fp32":
            U32 = U.clone()
        else:
            out["fp32"]["rel_diff_vs_fp64_max"] = max(
                float(torch.linalg.norm(BS.view(U32, p) - BS.view(U, p)) /
                      torch.linalg.norm(BS.view(U, p))) for p in range(BATCH_NPROB))
            # single FP64 solves of a sample, one after another (setup untimed)
            sample = []
            for p in range(BATCH_SAMPLE):
                S = Solver(int(ns[p]), float(alphas[p]))
                Bp = BS.view(B, p).clone()
                Up = S.zeros()
                S.solve(Bp[0].contiguous(), rtol=RTOL, u=Up)     # warm-up (graph capture)
                sample.append((S, Bp, Up))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for S, Bp, Up in sample:
                for r in range(BATCH_NRHS):
                    S.solve(Bp[r].contiguous(), rtol=RTOL, u=Up)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            nsol = BATCH_SAMPLE * BATCH_NRHS
            sdof = sum(dof[:BATCH_SAMPLE]) * BATCH_NRHS
            out["sequential_fp64_sample"] = {"problems": BATCH_SAMPLE, "solves": nsol,
                                             "solves_per_s": nsol / t, "dof_rhs_per_s": sdof / t}
            del sample
        del BS, U
        torch.cuda.empty_cache()
    out["speedup_batched_fp32_vs_sequential_fp64_dof_rate"] = (
        out["fp32"]["dof_rhs_per_s"] / out["sequential_fp64_sample"]["dof_rhs_per_s"])
    return out


def diff_leg(torch, steps, warmup):
    """dL/dB and dL/dalpha for L = sum_k ||u_k - t_k||^2 at 96^3 with 16 right-hand sides:
    all right-hand sides in one batched solve (forward and adjoint), against the same
    gradient through one solve per right-hand side.  FP64 V-cycle."""
    from paper_2205_05840_amd import Solver, solve
    n, k = DIFF_N, DIFF_NRHS
    Sk = Solver(n, 1.0, nrhs=k)
    S2 = Solver(n, 2.0, nrhs=k)
    S1 = Solver(n, 1.0)
    g = torch.Generator(device=Sk.device)
    g.manual_seed(DIFF_SEED)
    f = torch.randn(k * n ** 3 * 24, generator=g, dtype=torch.float64, device=Sk.device)
    B = Sk.assemble_rhs(f)
    del f
    T, _, _ = S2.solve(B, rtol=1e-12)
    del S2
    res = {"n": n, "nrhs": k, "ndof": 3 * n * (n - 1) ** 2}

    def grad(S):
        Bg = B.clone().requires_grad_(True)
        a = torch.tensor(1.0, dtype=torch.float64, device=B.device, requires_grad=True)
        L = ((solve(Bg, a, S, rtol=RTOL) - T) ** 2).sum()
        L.backward()
        return float(L.detach()), Bg.grad, float(a.grad)

    for name, S in (("batched_rhs", Sk), ("single_rhs", S1)):
        for _ in range(warmup):
            grad(S)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            L, gB, ga = grad(S)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        res[name] = {"s_per_gradient": t, "loss": L, "dL_dalpha": ga}
        log(f"differentiation {name}: {t:.3f} s per gradient")
        if name == "batched_rhs":
            gB0 = gB
        else:
            res["batched_vs_single_grad_rel_diff"] = {
                "dL_dB": float(torch.linalg.norm(gB - gB0) / torch.linalg.norm(gB)),
                "dL_dalpha": abs(res["batched_rhs"]["dL_dalpha"] - ga) / abs(ga)}
    res["speedup_batched_vs_single_rhs"] = (res["single_rhs"]["s_per_gradient"] /
                                            res["batched_rhs"]["s_per_gradient"])
    return res


def manufactured_leg(torch, steps):
    """The 64^3 configuration: plain FP64 V-cycle PCG to 1e-10 for f = (2 pi^2 alpha + 1) u*
    at the Gauss points plus N(0, 1e-6) noise (seed 1), alpha in {0.01, 1, 100}, subdomains
    of 2 and of 4 elements; and the edge-based smoother (eta 1/13) on the same problem at
    alpha = 1."""
    from paper_2205_05840_amd import Solver, synth
    n = 64
    ndof = 3 * n * (n - 1) ** 2
    out = {"n": n, "ndof": ndof, "precision": "fp64"}
    cases = [(a, "vertex", s) for s in (2, 4) for a in (0.01, 1.0, 100.0)] + [(1.0, "edge", 2)]
    for alpha, kind, sd in cases:
        S = Solver(n, alpha, subdomain=sd, smoother=kind)
        b = S.assemble_rhs(torch.from_numpy(synth.manufactured_samples(n, alpha, 1)))
        u = S.zeros()
        S.solve(b, rtol=RTOL, u=u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, it, rel = S.solve(b, rtol=RTOL, u=u)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        name = f"{kind}_s{sd}@alpha={alpha:g}"
        out[name] = {"s_per_solve": t, "dof_per_s": ndof / t, "iters": it, "relres": rel}
        log(f"64^3 {name}: {t * 1e3:.2f} ms/solve, {it} iterations")
        del S, b, u
    return out


def jumps_leg(torch, steps):
    """Coefficient with jumps at 128^3: alpha = 10^U(-2, 2) on a 4 x 4 x 4 grid of boxes
    (seed 3; contrast up to 1e4), six levels (coarsest 4^3, so that the boxes hold whole
    coarse elements), FP32 V-cycle in FP64 CG to 1e-10; the per-cell operator kernel and the
    gathered-product smoother on every level."""
    import numpy as np
    from paper_2205_05840_amd import Solver, synth
    n = N_ELEM
    boxes = 10.0 ** np.random.default_rng(3).uniform(-2.0, 2.0, size=(4, 4, 4))
    t0 = time.perf_counter()
    S = Solver(n, 1.0, precision="fp32", levels=6, coef=boxes)
    t_setup = time.perf_counter() - t0
    b = S.assemble_rhs(torch.from_numpy(synth.normal_samples(n, SEED)))
    u = S.zeros()
    S.solve(b, rtol=RTOL, u=u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, it, rel = S.solve(b, rtol=RTOL, u=u)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    true_rel = float(torch.linalg.norm(b - S.apply(u)) / torch.linalg.norm(b))
    ndof = 3 * n * (n - 1) ** 2
    log(f"128^3 jumps (4^3 boxes): setup {t_setup:.2f} s, {t * 1e3:.2f} ms/solve, {it} iterations")
    return {"n": n, "boxes": 4, "contrast": float(boxes.max() / boxes.min()), "setup_s": t_setup,
            "s_per_solve": t, "dof_per_s": ndof / t, "iters": it, "relres": rel, "true_relres": true_rel}


def fichera_leg(torch, steps):
    """A non-box domain at 128^3: the unit cube less the octant x, y, z > 1/2 (a Fichera
    corner), FP32 V-cycle in FP64 CG to 1e-10; every level on the per-cell operator kernel
    and the gathered-product smoother."""
    import numpy as np
    from paper_2205_05840_amd import Solver, synth
    n = N_ELEM
    active = np.ones((2, 2, 2), dtype=bool)
    active[1, 1, 1] = False
    t0 = time.perf_counter()
    S = Solver(n, 1.0, precision="fp32", domain=active)
    t_setup = time.perf_counter() - t0
    b = S.assemble_rhs(torch.from_numpy(synth.normal_samples(n, SEED)))
    u = S.zeros()
    S.solve(b, rtol=RTOL, u=u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, it, rel = S.solve(b, rtol=RTOL, u=u)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    true_rel = float(torch.linalg.norm(b - S.apply(u)) / torch.linalg.norm(b))
    log(f"128^3 Fichera domain: setup {t_setup:.2f} s, {t * 1e3:.2f} ms/solve, {it} iterations")
    return {"n": n, "domain": "unit cube less the octant x, y, z > 1/2", "ndof": S.ndof, "setup_s": t_setup,
            "s_per_solve": t, "dof_per_s": S.ndof / t, "iters": it, "relres": rel, "true_relres": true_rel}


def timestep_leg(torch, nsteps=20):
    """Implicit Maxwell time stepping at 128^3 (average-acceleration Newmark, eps = 1,
    sigma = 1, mu = 1, dt = 0.01: each step the model problem with alpha = dt^2 / (4 (1 +
    dt / 2))), FP32 V-cycle, solves to 1e-10 started from the predictor."""
    from paper_2205_05840_amd import Solver, synth
    n, dt, eps, sigma, mu = N_ELEM, 0.01, 1.0, 1.0, 1.0
    alpha = dt * dt / (4 * mu * (eps + 0.5 * sigma * dt))
    S = Solver(n, alpha, precision="fp32")
    f = S.assemble_rhs(torch.from_numpy(synth.normal_samples(n, SEED)))
    u, v, a = S.zeros(), S.zeros(), S.zeros()
    S.maxwell_step(f, u, v, a, dt, eps, sigma, mu, rtol=RTOL)   # warm-up (graph capture)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for _ in range(nsteps):
        it, _ = S.maxwell_step(f, u, v, a, dt, eps, sigma, mu, rtol=RTOL)
        iters.append(it[0])
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / nsteps
    log(f"time stepping 128^3: {t * 1e3:.2f} ms per step, iterations {iters[0]} .. {iters[-1]}")
    return {"n": n, "alpha": alpha, "dt": dt, "s_per_step": t, "steps_per_s": 1.0 / t,
            "iters_first": iters[0], "iters_last": iters[-1], "iters_mean": sum(iters) / len(iters)}


def cpu_baseline(f, iters_expected, gpu_solutions=None, sample_iters=3):
    """The FP64 CPU oracle (assembled sparse matrices, factored vertex smoother) on a
    bounded sample of the same 128^3 solve: setup untimed, then `sample_iters` PCG
    iterations timed and scaled to a full solve of `iters_expected` iterations.

    Also the second CPU reference: the oracle's exact solve of the same discrete system
    (sine/cosine transforms diagonalise A on the box into 3 x 3 blocks), timed, and the
    relative error of the GPU solutions (padded layout, host copies) against it."""
    import numpy as np
    from oracle import exact, mesh, pcg, rhs, vcycle
    h = 1.0 / N_ELEM
    b = rhs.load_from_samples(N_ELEM, h, f)
    t0 = time.perf_counter()
    ue = exact.solve_fft(N_ELEM, h, 1.0, b)
    t_fft = time.perf_counter() - t0
    exact_ref = {"s_per_solve": t_fft, "method": "oracle exact solve (DST/DCT, 3x3 blocks)"}
    if gpu_solutions:
        P = (N_ELEM + 1 + 7) // 8 * 8
        B = (N_ELEM + 1) ** 2 * P
        d, pc = mesh.edge_coords(N_ELEM)
        idx = d * B + (pc[:, 2] * (N_ELEM + 1) + pc[:, 1]) * P + pc[:, 0]
        nrm = float(np.linalg.norm(ue))
        for name, u in gpu_solutions.items():
            exact_ref[f"rel_error_{name}"] = float(np.linalg.norm(u[idx] - ue)) / nrm
    del ue
    # one thread: SciPy's sparse products are single-threaded, and the BLAS pools (which
    # the dense local products would use) are held to one thread, so that `cores` is exact
    try:
        from threadpoolctl import threadpool_limits
        limit = threadpool_limits(limits=1)
    except Exception:
        limit = None
    t0 = time.perf_counter()
    H = vcycle.Hierarchy(N_ELEM, 1.0)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    pcg.pcg(H.A[-1], b, H.precondition, rtol=RTOL, maxit=sample_iters)
    t = time.perf_counter() - t0
    threads_timed = blas_threads()
    if limit is not None:
        limit.restore_original_limits()
    per_iter = t / sample_iters
    s_solve = per_iter * iters_expected
    ndof = 3 * N_ELEM * (N_ELEM - 1) ** 2
    return {"value": ndof / s_solve, "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "sample": (f"{sample_iters} V-cycle-PCG iterations of the 128^3 alpha=1 solve "
                       f"({t:.1f} s, setup {t_setup:.1f} s untimed), scaled to "
                       f"{iters_expected} iterations; one thread (SciPy SpMV, BLAS pools held to 1)"),
            "s_per_solve_est": s_solve,
            "affinity_cpus": len(os.sched_getaffinity(0)),
            "cpu_model": cpu_model(),
            "blas_threads": threads_timed,
            "exact": exact_ref}


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def blas_threads():
    """Threads of the BLAS / OpenMP pools loaded in this process (threadpoolctl), per library."""
    try:
        import threadpoolctl
        return {f"{p.get('internal_api')}:{os.path.basename(p.get('filepath', ''))}": p.get("num_threads")
                for p in threadpoolctl.threadpool_info()}
    except Exception:
        return None


def kernel_probe(torch, Solver, reps):
    """For hardware-counter runs: a device copy of 256 MiB (calibration of the byte
    counters against a kernel of known traffic), then `reps` FP64 operator applies at
    128^3, and 4 fine-level smoother applications (condensation, patch products,
    pull/extend) in FP64 and in FP32."""
    src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    out = {"probe": "apply+smooth", "n": N_ELEM, "reps": reps, "copy_bytes_each_way": src.numel() * 8}
    for prec in ("fp64", "fp32"):
        S = Solver(N_ELEM, 1.0, precision=prec)
        if prec == "fp64":
            out["apply_avg_launch_us"] = time_apply(torch, S, reps=reps) * 1e6
        r = (torch.randn(S.vec_len, dtype=torch.float64, device=S.device) * S.unknown_mask()).contiguous()
        for _ in range(4):
            S.level_op(-1, "smooth", r)
        torch.cuda.synchronize()
        del S
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched and differentiated forms")
    ap.add_argument("--kernel-probe", action="store_true",
                    help="only run the calibration copy and the apply kernel (counter runs)")
    ap.add_argument("--solve-probe", choices=["fp32", "fp64"],
                    help="only run one warm-up and --probe-solves timed 128^3 solves in this "
                         "precision (counter runs; the difference of runs with 2 and 1 timed "
                         "solves is the traffic of one solve)")
    ap.add_argument("--probe-solves", type=int, default=1)
    ap.add_argument("--batched-probe", choices=["fp32", "fp64"],
                    help="only run one warm-up and one timed solve of the batched form in this "
                         "precision (counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2205_05840_amd import Solver, synth
    from paper_2205_05840_amd import _lib
    _lib.lib()   # fail loudly if the HIP library is missing

    if args.kernel_probe:
        kernel_probe(torch, Solver, 10)
        return
    if args.solve_probe:
        f = torch.from_numpy(synth.normal_samples(N_ELEM, SEED))
        _, _, _, res = run_leg(torch, Solver, f, 1.0, args.solve_probe, args.probe_solves, 1)
        print(json.dumps({"probe": "solve", "precision": args.solve_probe, "n": N_ELEM,
                          "s_per_solve": res["s_per_solve_total"], "iters": res["iters"]}), flush=True)
        return
    if args.batched_probe:
        from paper_2205_05840_amd import BatchedSolver
        ns, alphas = synth.batched_problems(BATCH_NPROB, seed=BATCH_SEED)
        BS = BatchedSolver(ns, alphas, nrhs=BATCH_NRHS, precision=args.batched_probe)
        g = torch.Generator(device=BS.device)
        g.manual_seed(BATCH_SEED)
        B = BS.assemble_rhs(torch.randn(BS.sample_len(), generator=g, dtype=torch.float64, device=BS.device))
        U = BS.zeros()
        BS.solve(B, rtol=RTOL, U=U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, it, _ = BS.solve(B, rtol=RTOL, U=U)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "batched", "precision": args.batched_probe, "nprob": BATCH_NPROB,
                          "nrhs": BATCH_NRHS, "s_per_batch": time.perf_counter() - t0,
                          "iters_max": int(it.max())}), flush=True)
        return
    f = torch.from_numpy(synth.normal_samples(N_ELEM, SEED))
    ndof = 3 * N_ELEM * (N_ELEM - 1) ** 2
    legs = {}
    sols = {}
    for alpha in (1.0, 1e-3):
        for prec in ("fp32", "fp64"):
            S, b, u, res = run_leg(torch, Solver, f, alpha, prec, args.steps, args.warmup)
            res["dof_per_s"] = ndof / res["s_per_solve_total"]
            legs[f"{prec}@alpha={alpha:g}"] = res
            log(f"128^3 {prec} alpha={alpha:g}: {res['s_per_solve_total'] * 1e3:.1f} ms/solve, "
                f"{res['iters']} iterations")
            sols[(alpha, prec)] = u.clone()
            if alpha == 1.0 and prec == "fp64":
                t_apply = time_apply(torch, S)
                t_patch64 = time_patch(torch, S)
            if alpha == 1.0 and prec == "fp32":
                t_patch = time_patch(torch, S)
            del S, b, u
            torch.cuda.empty_cache()
    for alpha in (1.0, 1e-3):
        u32, u64 = sols[(alpha, "fp32")], sols[(alpha, "fp64")]
        legs[f"fp32@alpha={alpha:g}"]["rel_diff_vs_fp64"] = float(
            torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64))

    head = legs["fp32@alpha=1"]
    fp64 = legs["fp64@alpha=1"]
    bytes_apply = 2 * ndof * 8
    achieved = bytes_apply / t_apply / 1e9
    roofline_apply = {"kernel": "k_stencil (operator apply y = A x, 128^3, FP64)",
                      "bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                      "frac": achieved / 8000.0, "traffic": load_traffic("apply", "fp64"),
                      "avg_launch_us": t_apply * 1e6, "algorithmic_bytes_per_launch": bytes_apply}
    # the dominant kernel of the headline (FP32 V-cycle) solve: the fine-level patch
    # products, two launches per CG iteration, priced against the FP32 MFMA peak
    flops = patch_flops(N_ELEM)
    roofline = {"kernel": "k_sm_patch (vertex patch products y_V = S_V^-1 g|Gamma_V, 128^3, FP32)",
                "bound": "mfma", "achieved": flops / t_patch / 1e12, "peak": 157.3, "unit": "TFLOP/s",
                "frac": flops / t_patch / 1e12 / 157.3, "traffic": load_traffic("patch", "fp32"),
                "avg_launch_us": t_patch * 1e6, "algorithmic_flops_per_launch": flops}
    roofline_patch64 = {"kernel": "k_sm_patch (128^3, FP64)", "bound": "mfma",
                        "achieved": flops / t_patch64 / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                        "frac": flops / t_patch64 / 1e12 / 78.6, "traffic": load_traffic("patch", "fp64"),
                        "avg_launch_us": t_patch64 * 1e6, "algorithmic_flops_per_launch": flops}
    solve_bytes = {p: load_traffic("solve", p) for p in ("fp32", "fp64")}
    solve_traffic = {p: (None if solve_bytes[p] is None else
                         {"bytes_per_solve": solve_bytes[p],
                          "achieved_GBps": solve_bytes[p] / legs[f"{p}@alpha=1"]["s_per_solve_total"] / 1e9,
                          "frac_of_hbm_peak": solve_bytes[p] / legs[f"{p}@alpha=1"]["s_per_solve_total"] / 8e12})
                     for p in ("fp32", "fp64")}
    out = {
        "metric": "DOF/s and s/solve to 1e-10 rel. residual at 128^3, mixed vs FP64 V-cycle-PCG",
        "value": head["dof_per_s"], "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["s_per_solve_total"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 CG + f32 V-cycle", "data": "synthetic",
        "config": {"workload": ("128^3 unit-cube hex mesh, lowest-order Nedelec, alpha=1, f~N(0,1) "
                                "at 2x2x2 Gauss points (seed 2), vertex-smoother V(1,1)-PCG to "
                                "1e-10, FP32 V-cycle in FP64 flexible CG"),
                   "n": N_ELEM, "ndof": ndof, "levels": 7, "parallelism": "single GPU"},
        "s_per_solve": head["s_per_solve_total"], "s_per_solve_median": head["s_per_solve_median"],
        "iters": head["iters"],
        "relres": head["relres"], "true_relres": head["true_relres"],
        "fp64": {"value": fp64["dof_per_s"], "s_per_solve": fp64["s_per_solve_total"],
                 "iters": fp64["iters"], "true_relres": fp64["true_relres"]},
        "speedup_mixed_vs_fp64": fp64["s_per_solve_total"] / head["s_per_solve_total"],
        "legs": legs, "roofline": roofline,
        "roofline_other": {"apply_fp64": roofline_apply, "patch_fp64": roofline_patch64},
        "solve_traffic": solve_traffic,
    }
    if not args.no_forms:
        out["forms"] = {"batched": batched_leg(torch, max(1, args.steps // 2), 1),
                        "differentiation": diff_leg(torch, 1, 1),
                        "manufactured_64": manufactured_leg(torch, max(1, args.steps // 2)),
                        "time_stepping": timestep_leg(torch),
                        "jumps_128": jumps_leg(torch, max(1, args.steps // 2)),
                        "fichera_128": fichera_leg(torch, max(1, args.steps // 2))}
    if not args.no_cpu_baseline:
        host = {"fp32": sols[(1.0, "fp32")].cpu().numpy(), "fp64": sols[(1.0, "fp64")].cpu().numpy()}
        out["cpu_baseline"] = cpu_baseline(f.numpy(), fp64["iters"], host)
    print(json.dumps(out), flush=True)
    del np


if __name__ == "__main__":
    main()
