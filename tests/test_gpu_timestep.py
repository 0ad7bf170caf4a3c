"""Implicit Maxwell time stepping on the GPU (Sec. 1, eq. Maxwell timestep): the
average-acceleration Newmark step (ndmg_maxwell_step, each step the model problem solved
by V-cycle PCG started from the predictor) against the oracle's stepping with exact
solves, its energy conservation without damping, and the warm-started PCG.

Tolerances: every GPU solve runs to 1e-13, so each step's u carries a relative error of
about 1e-13 times the conditioning of A on the error's components; a = 4/dt^2 (u - w)
divides a small difference by dt^2/4.  Observed after 8 steps: u within 1.1e-12 .. 1.4e-12
of the oracle, v and a within 4e-13 .. 5e-13; the tolerance is 1e-11.
"""
import numpy as np
import pytest

from layout import from_padded, to_padded
from oracle import exact, mesh, rhs, timestep

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("n,dt,eps,sigma,mu", [(16, 0.05, 1.0, 2.0, 1.0), (32, 0.02, 2.0, 0.0, 0.5)])
def test_steps_match_oracle(n, dt, eps, sigma, mu):
    from paper_2205_05840_amd import Solver, synth
    print(f"[case] maxwell n={n} dt={dt} eps={eps} sigma={sigma} mu={mu}", flush=True)
    O = timestep.Newmark(n, 1.0, dt, eps, sigma, mu)
    S = Solver(n, O.alpha)
    rng = np.random.default_rng(n)
    u, v = rng.standard_normal(mesh.ndof(n)), rng.standard_normal(mesh.ndof(n))
    f = rhs.load_from_samples(n, 1.0 / n, synth.normal_samples(n, 9))
    a = O.initial_acceleration(u, v, f)
    dev = lambda x: torch.from_numpy(to_padded(n, S.P, S.B, x)).cuda()
    gu, gv, ga, gf = dev(u), dev(v), dev(a), dev(f)
    iters = []
    for _ in range(8):
        it, rel = S.maxwell_step(gf, gu, gv, ga, dt, eps, sigma, mu, rtol=1e-13)
        iters.append(it[0])
        assert rel[0] <= 1e-13
        u, v, a = O.step(u, v, a, f)
    print(f"iterations per step (warm start): {iters}")
    for name, g, o in (("u", gu, u), ("v", gv, v), ("a", ga, a)):
        e = _rel(from_padded(n, S.P, S.B, _host(g)), o)
        print(f"{name}: relative error {e:.2e}")
        assert e <= 1e-11


def test_energy_conserved_on_gpu():
    """sigma = 0 and no source: the discrete energy eps/2 v^T M v + 1/(2 mu) u^T K u of the
    GPU's states stays at its initial value (to the accuracy of the solves)."""
    from paper_2205_05840_amd import Solver
    n, dt = 16, 0.1
    O = timestep.Newmark(n, 1.0, dt, eps=1.0, sigma=0.0, mu=1.0)
    S = Solver(n, O.alpha)
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal(mesh.ndof(n)), rng.standard_normal(mesh.ndof(n))
    a = O.initial_acceleration(u, v, np.zeros_like(u))
    e0 = O.energy(u, v)
    dev = lambda x: torch.from_numpy(to_padded(n, S.P, S.B, x)).cuda()
    gu, gv, ga, gf = dev(u), dev(v), dev(a), dev(np.zeros_like(u))
    for k in range(20):
        S.maxwell_step(gf, gu, gv, ga, dt, 1.0, 0.0, 1.0, rtol=1e-13)
        e = O.energy(from_padded(n, S.P, S.B, _host(gu)), from_padded(n, S.P, S.B, _host(gv)))
        assert abs(e - e0) <= 1e-9 * e0, (k, e, e0)


def test_warm_start():
    """From the exact solution the warm-started PCG stops after its first iteration; from
    the solution of a nearby right-hand side it needs fewer iterations than from zero, and
    it reaches the same residual bound."""
    from paper_2205_05840_amd import Solver, synth
    n, alpha = 32, 1.0
    S = Solver(n, alpha)
    h = 1.0 / n
    b_o = rhs.load_from_samples(n, h, synth.normal_samples(n, 2))
    b = torch.from_numpy(to_padded(n, S.P, S.B, b_o)).cuda()
    u0, it_cold, _ = S.solve(b, rtol=1e-10)
    ue = exact.solve_fft(n, h, alpha, b_o)
    u = torch.from_numpy(to_padded(n, S.P, S.B, ue)).cuda()
    _, it_exact, rel = S.solve(b, rtol=1e-10, u=u, warm=True)
    assert it_exact == 1 and rel <= 1e-10
    b2_o = b_o + 1e-4 * np.linalg.norm(b_o) / np.sqrt(b_o.size) * np.random.default_rng(1).standard_normal(b_o.size)
    b2 = torch.from_numpy(to_padded(n, S.P, S.B, b2_o)).cuda()
    _, it_cold2, _ = S.solve(b2, rtol=1e-10)
    u2, it_warm2, rel2 = S.solve(b2, rtol=1e-10, u=u0.clone(), warm=True)
    print(f"cold {it_cold}, from the exact solution {it_exact}, nearby rhs: cold {it_cold2}, warm {it_warm2}")
    assert it_warm2 < it_cold2 and rel2 <= 1e-10
    res = exact.apply_fft(n, h, alpha, from_padded(n, S.P, S.B, _host(u2))) - b2_o
    assert np.linalg.norm(res) <= 1.5e-10 * np.linalg.norm(b2_o)
