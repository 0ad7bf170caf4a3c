"""The benchmarked configurations asserted against the FP64 oracle at their full sizes.

* 128^3, FP64 V-cycle PCG (alpha = 1 and 1e-3, f ~ N(0, 1) at the Gauss points, seed
  2): relative residual <= 1e-10 recomputed with the oracle's operator (the exact
  transform-domain product), the iteration count against the oracle's at 64^3 (mesh
  independence, Sec. 4), and the solution protocol: run to 1e-13 and compare with the
  exact discrete solution (transform solve) to 1e-9 in l2 and in the energy norm.
* 64^3, FP64, manufactured field plus N(0, 1e-6) noise at alpha = 0.01, 1, 100: residual,
  iteration count within +-1 of the oracle's own V-cycle PCG, and the solution protocol.
* 96^3 differentiated form: loss and gradients (dL/db_k and dL/dalpha) against the
  oracle's adjoint with exact solves in extended precision, and directional central
  differences along random
  unit directions of b (the loss is quadratic in b, so the difference quotient is exact
  up to the accuracy of the solves).
"""
import numpy as np
import pytest

from layout import from_padded, to_padded
from oracle import exact, mesh, pcg, rhs, vcycle, adjoint

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


def _energy_rel(n, h, alpha, u, ue):
    e = u - ue
    return np.sqrt(e @ exact.apply_fft(n, h, alpha, e)) / np.sqrt(ue @ exact.apply_fft(n, h, alpha, ue))


def _check_solve(S, n, alpha, b_o, b, it_ref=None):
    h = 1.0 / n
    u, it, rel = S.solve(b, rtol=1e-10)
    u_c = from_padded(n, S.P, S.B, _host(u))
    true_rel = _rel(exact.apply_fft(n, h, alpha, u_c), b_o)
    print(f"n={n} alpha={alpha}: {it} iterations, relres {rel:.2e}, true {true_rel:.2e}")
    assert rel <= 1e-10 and true_rel <= 1.5e-10
    if it_ref is not None:
        assert abs(it - it_ref) <= 1, (it, it_ref)
    ut, it2, rel2 = S.solve(b, rtol=1e-13, raise_on_noconv=False)
    ut = from_padded(n, S.P, S.B, _host(ut))
    ue = exact.solve_fft(n, h, alpha, b_o)
    e2, ea = _rel(ut, ue), _energy_rel(n, h, alpha, ut, ue)
    print(f"  at 1e-13: {it2} iterations, relres {rel2:.2e}; error l2 {e2:.2e}, energy {ea:.2e}; "
          f"at 1e-10: l2 {_rel(u_c, ue):.2e}")
    assert e2 <= 1e-9 and ea <= 1e-9
    return it


@pytest.mark.parametrize("alpha", [1.0, 1e-3])
def test_pcg_fp64_128(alpha):
    from paper_2205_05840_amd import synth
    n = 128
    S = _solver(n, alpha)
    f = synth.normal_samples(n, 2)
    b_o = rhs.load_from_samples(n, 1.0 / n, f)
    b = S.assemble_rhs(torch.from_numpy(f))
    assert _rel(from_padded(n, S.P, S.B, _host(b)), b_o) <= 1e-14
    it = _check_solve(S, n, alpha, b_o, b)
    # mesh independence: the oracle's iteration count at 64^3 (same alpha and seed)
    n2 = 64
    H = vcycle.Hierarchy(n2, alpha)
    b2 = rhs.load_from_samples(n2, 1.0 / n2, synth.normal_samples(n2, 2))
    _, it_o, _, _ = pcg.pcg(H.A[-1], b2, H.precondition, rtol=1e-10)
    print(f"  oracle at 64^3: {it_o} iterations")
    assert abs(it - it_o) <= 2


@pytest.mark.parametrize("alpha", [0.01, 1.0, 100.0])
def test_manufactured_64(alpha):
    from paper_2205_05840_amd import synth
    n = 64
    S = _solver(n, alpha)
    f = synth.manufactured_samples(n, alpha, 1)
    b_o = rhs.load_from_samples(n, 1.0 / n, f)
    b = S.assemble_rhs(torch.from_numpy(f))
    H = vcycle.Hierarchy(n, alpha)
    _, it_o, _, _ = pcg.pcg(H.A[-1], b_o, H.precondition, rtol=1e-10)
    _check_solve(S, n, alpha, b_o, b, it_ref=it_o)


def _loss_grads_gpu(S, B_o, T_o, n, rtol):
    from paper_2205_05840_amd import solve
    B = torch.from_numpy(to_padded(n, S.P, S.B, B_o)).cuda().requires_grad_(True)
    T = torch.from_numpy(to_padded(n, S.P, S.B, T_o)).cuda()
    a = torch.tensor(S.alpha, dtype=torch.float64, device="cuda", requires_grad=True)
    U = solve(B, a, S, rtol=rtol)
    L = ((U - T) ** 2).sum()
    L.backward()
    return float(L.detach()), from_padded(n, S.P, S.B, B.grad.cpu().numpy()), float(a.grad)


def test_gradients_96():
    from paper_2205_05840_amd import synth
    n, nrhs = 96, 3
    h = 1.0 / n
    B_o = rhs.load_from_samples(n, h, synth.normal_samples(n, 4, nrhs=nrhs))
    T_o = exact.solve_fft(n, h, 2.0, B_o)
    S = _solver(n, 1.0, nrhs=nrhs)
    L, dB, da = _loss_grads_gpu(S, B_o, T_o, n, 1e-13)
    # extended-precision reference: |U - T| is 6e-5 |U| here, and an FP64 reference
    # gradient dL/db carries 1.3e-5 of rounding (two FP64 routes disagree by that much)
    L_o, dB_o, da_o = adjoint.loss_and_grads(n, 1.0, 1.0, B_o, T_o, dtype=np.longdouble)
    print(f"96^3: L {L:.6e} ({abs(L - L_o) / L_o:.1e}), dL/dalpha {da:.6e} "
          f"({abs(da - da_o) / abs(da_o):.1e}), dL/db {_rel(dB, dB_o):.1e}")
    assert abs(L - L_o) <= 1e-9 * L_o
    assert abs(da - da_o) <= 1e-6 * abs(da_o)
    assert _rel(dB, dB_o) <= 1e-6


def test_gradient_directions_96():
    """dL/db . d against (L(b + eps d) - L(b - eps d)) / (2 eps) for 4 random unit
    directions d of the stacked right-hand sides.  L is quadratic in b, so the central
    difference equals the directional derivative for any eps; eps = 1e-3 |b| keeps the
    change of L well above the rounding of the solves."""
    from paper_2205_05840_amd import synth
    n, nrhs = 96, 2
    h = 1.0 / n
    B_o = rhs.load_from_samples(n, h, synth.normal_samples(n, 4, nrhs=nrhs))
    T_o = exact.solve_fft(n, h, 2.0, B_o)
    S = _solver(n, 1.0, nrhs=nrhs)
    _, dB, _ = _loss_grads_gpu(S, B_o, T_o, n, 1e-13)
    D = synth.unit_directions(B_o.size, 4, 21).reshape((4,) + B_o.shape)
    eps = 1e-3 * np.linalg.norm(B_o)
    for k in range(4):
        Lp = _loss_grads_gpu(S, B_o + eps * D[k], T_o, n, 1e-13)[0]
        Lm = _loss_grads_gpu(S, B_o - eps * D[k], T_o, n, 1e-13)[0]
        fd = (Lp - Lm) / (2 * eps)
        an = float(np.sum(dB * D[k]))
        print(f"direction {k}: adjoint {an:.10e}, central difference {fd:.10e}")
        assert abs(fd - an) <= 1e-6 * abs(an)


def test_alpha_central_difference_96():
    """dL/dalpha from the adjoint solves against (L(1 + d) - L(1 - d)) / (2 d), d = 1e-6,
    with every solve run to 1e-13."""
    from paper_2205_05840_amd import synth
    n, nrhs, d = 96, 2, 1e-6
    h = 1.0 / n
    B_o = rhs.load_from_samples(n, h, synth.normal_samples(n, 4, nrhs=nrhs))
    T_o = exact.solve_fft(n, h, 2.0, B_o)
    _, _, da = _loss_grads_gpu(_solver(n, 1.0, nrhs=nrhs), B_o, T_o, n, 1e-13)
    Lp = _loss_grads_gpu(_solver(n, 1.0 + d, nrhs=nrhs), B_o, T_o, n, 1e-13)[0]
    Lm = _loss_grads_gpu(_solver(n, 1.0 - d, nrhs=nrhs), B_o, T_o, n, 1e-13)[0]
    fd = (Lp - Lm) / (2 * d)
    print(f"dL/dalpha: adjoint {da:.10e}, central difference {fd:.10e}")
    assert abs(fd - da) <= 1e-6 * abs(da)
