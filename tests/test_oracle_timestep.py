"""Pins of the oracle's implicit Maxwell time stepping (Sec. 1, eq. Maxwell timestep)."""
import numpy as np
import pytest

from oracle import assemble, exact, mesh, timestep


def _field(n, seed):
    return np.random.default_rng(seed).standard_normal(mesh.ndof(n))


def test_step_operator_is_the_model_problem():
    """The per-step operator (dt^2/4) mu^{-1} K + (eps + sigma dt/2) M, divided by
    eps + sigma dt/2, is A(alpha) with alpha = dt^2 / (4 mu (eps + sigma dt/2))."""
    n, dt, eps, sigma, mu = 6, 0.03, 2.0, 5.0, 0.7
    S = timestep.Newmark(n, 1.0, dt, eps, sigma, mu)
    op = (0.25 * dt * dt / mu * S.K + (eps + 0.5 * sigma * dt) * S.M) / (eps + 0.5 * sigma * dt)
    A = assemble.matrix_kron(n, 1.0 / n, S.alpha)
    assert abs(op - A).max() <= 1e-14 * abs(A).max()


@pytest.mark.parametrize("n,dt", [(4, 0.05), (6, 0.2)])
def test_energy_conserved_without_damping(n, dt):
    """sigma = 0, no source: the average-acceleration scheme (the trapezoidal rule) keeps
    eps/2 v^T M v + 1/(2 mu) u^T K u exactly, step after step."""
    S = timestep.Newmark(n, 1.0, dt, eps=1.5, sigma=0.0, mu=0.8)
    u, v = _field(n, 1), _field(n, 2)
    a = S.initial_acceleration(u, v, np.zeros_like(u))
    e0 = S.energy(u, v)
    for _ in range(20):
        u, v, a = S.step(u, v, a, np.zeros_like(u))
        assert abs(S.energy(u, v) - e0) <= 1e-11 * e0


def test_energy_decays_with_damping():
    n = 5
    S = timestep.Newmark(n, 1.0, 0.1, eps=1.0, sigma=3.0, mu=1.0)
    u, v = _field(n, 3), _field(n, 4)
    a = S.initial_acceleration(u, v, np.zeros_like(u))
    e = S.energy(u, v)
    for _ in range(10):
        u, v, a = S.step(u, v, a, np.zeros_like(u))
        e1 = S.energy(u, v)
        assert e1 < e
        e = e1


def test_second_order_in_time():
    """Errors at t = 0.4 against a run with dt / 16 fall by about 4 per halving of dt."""
    n = 4
    u0, v0 = _field(n, 5), _field(n, 6)
    f = 0.3 * _field(n, 7)

    def run(dt):
        S = timestep.Newmark(n, 1.0, dt, eps=1.0, sigma=0.5, mu=1.0)
        u, v = u0.copy(), v0.copy()
        a = S.initial_acceleration(u, v, f)
        for _ in range(int(round(0.4 / dt))):
            u, v, a = S.step(u, v, a, f)
        return u

    ref = run(0.4 / 256)
    errs = [np.linalg.norm(run(0.4 / k) - ref) for k in (16, 32, 64)]
    rates = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.5 < r < 4.5 for r in rates), (errs, rates)
