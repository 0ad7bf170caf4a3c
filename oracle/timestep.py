"""Implicit time stepping of Maxwell's equations (Sec. 1, eq. Maxwell timestep).

With the magnetic field eliminated, the electric field of the system in Sec. 1 solves
    eps E'' + sigma E' + curl(mu^{-1} curl E) = J'
(constant eps, sigma, mu; zero tangential trace).  In the Nedelec space this is
    eps M u'' + sigma M u' + mu^{-1} K u = f,     f = (J', phi_e),
with M the mass matrix and K the curl-curl matrix (A = alpha K + M, eq. def bilinear
form).  The average-acceleration Newmark scheme (beta = 1/4, gamma = 1/2) reads
    u_{n+1} = u_n + dt v_n + dt^2/4 (a_n + a_{n+1}),   v_{n+1} = v_n + dt/2 (a_n + a_{n+1}),
    eps M a_{n+1} + sigma M v_{n+1} + mu^{-1} K u_{n+1} = f_{n+1}.
Eliminating a_{n+1} and v_{n+1} and multiplying by dt^2/4 leaves, per step,
    (dt^2/4) mu^{-1} K u_{n+1} + (eps + sigma dt/2) M u_{n+1} = R.H.S.,
the operator of eq. (Maxwell timestep); divided by eps + sigma dt/2 it is the model
problem with alpha = dt^2 / (4 mu (eps + sigma dt/2)).  Each step here solves it exactly
(transform solve).

TEST INFRASTRUCTURE: part of the oracle package (see oracle/__init__.py).
"""
import numpy as np
import scipy.sparse.linalg as spla

from . import assemble, exact


class Newmark:
    """The scheme above on the cube (0, L)^3 with n^3 elements."""

    def __init__(self, n, L, dt, eps=1.0, sigma=0.0, mu=1.0):
        self.n, self.h, self.dt = n, L / n, dt
        self.eps, self.sigma, self.mu = eps, sigma, mu
        self.d = eps + 0.5 * sigma * dt
        self.alpha = dt * dt / (4.0 * mu * self.d)
        self.M = assemble.mass_kron(n, self.h)
        self.K = assemble.stiffness_kron(n, self.h)

    def initial_acceleration(self, u0, v0, f0):
        """a_0 from the equation at t = 0: eps M a_0 = f_0 - sigma M v_0 - mu^{-1} K u_0."""
        rhs = f0 - self.sigma * (self.M @ v0) - (self.K @ u0) / self.mu
        return spla.spsolve(self.M.tocsc(), rhs) / self.eps

    def step(self, u, v, a, f_next):
        dt, h2 = self.dt, 0.25 * self.dt ** 2
        w = u + dt * v + h2 * a
        rhs = (h2 * f_next + self.M @ (self.eps * w + self.sigma * (0.5 * dt * u + h2 * v))) / self.d
        u1 = exact.solve_fft(self.n, self.h, self.alpha, rhs)
        a1 = (u1 - w) / h2
        v1 = v + 0.5 * dt * (a + a1)
        return u1, v1, a1

    def energy(self, u, v):
        """eps/2 v^T M v + 1/(2 mu) u^T K u: conserved by the scheme when sigma = 0 and f = 0."""
        return 0.5 * self.eps * v @ (self.M @ v) + 0.5 / self.mu * u @ (self.K @ u)
