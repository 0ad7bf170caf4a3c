"""Solver: a torch-facing wrapper of one ndmg context.

PyTorch supplies device memory (the workspace and the vectors) and the stream; every
computation runs in libndmg.so.
"""
import numpy as np
import torch

from . import _lib

PRECISIONS = {"fp64": 0, "fp32": 1}
SMOOTHERS = {"vertex": 0, "edge": 1}


def _opts(m, eta, precision, boundary_patches, flexible, use_graphs, bottom_n=None, dense_n=None,
          smoother="vertex", subdomain=2, coef=None, domain=None):
    """ndmg_opts; with coef (an r x r x r array of box factors, [z][y][x]) or domain (an
    r x r x r array of flags, the boxes a non-box domain keeps) also the copies the struct
    points to, which must live through the plan and setup calls."""
    o = _lib.ndmg_default_opts()
    o.smoother = SMOOTHERS[smoother]
    o.subdomain = int(subdomain)
    o.m = int(m)
    if eta is not None:
        o.eta = float(eta)
    o.precision = PRECISIONS[precision]
    o.boundary_patches = 1 if boundary_patches else 0
    o.flexible = -1 if flexible is None else int(bool(flexible))
    if use_graphs is not None:   # None: the library's choice by problem size
        o.use_graphs = 1 if use_graphs else 0
    if bottom_n is not None:
        o.bottom_n = int(bottom_n)
    if dense_n is not None:
        o.dense_n = int(dense_n)
    keep = []
    if coef is not None:
        c = np.ascontiguousarray(coef, dtype=np.float64)
        r = c.shape[0]
        if c.shape != (r, r, r):
            raise ValueError("coef must be an r x r x r array of box factors")
        o.coef_r = r
        o.coef = c.ctypes.data_as(_lib.ctypes.POINTER(_lib.ctypes.c_double))
        keep.append(c)
    if domain is not None:
        d = np.ascontiguousarray(np.asarray(domain, dtype=bool), dtype=np.uint8)
        r = d.shape[0]
        if d.shape != (r, r, r) or (coef is not None and o.coef_r != r):
            raise ValueError("domain must be an r x r x r array of flags on the grid of coef")
        o.coef_r = r
        o.domain = d.ctypes.data_as(_lib.ctypes.POINTER(_lib.ctypes.c_ubyte))
        keep.append(d)
    o._keep = keep
    return o


class _Context:
    """Workspace, private stream and context handle shared by both solver kinds."""

    def _alloc(self, ws_bytes, device):
        self.device = torch.device(device)
        self.ws_bytes = ws_bytes
        self.ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=self.device)
        self._ws_ptr = (self.ws.data_ptr() + 255) // 256 * 256
        # the library works on a stream of its own (default priority; graph capture needs a
        # non-null stream); calls are ordered after the caller's current stream and the
        # caller's stream waits for them
        self.stream = torch.cuda.Stream(device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _run(self, fn, *args):
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        try:
            return fn(self.ctx, *args)
        finally:
            cur.wait_stream(self.stream)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            self.stream.synchronize()
            _lib.ndmg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver(_Context):
    """V-cycle-preconditioned CG for curl(alpha curl u) + u = f on (0, length)^3 with
    n^3 cubes, lowest-order Nedelec edge elements and zero tangential trace.  On a box that
    is not a cube, n = (nx, ny, nz) and length = its three side lengths (cubic elements):
    vectors and load samples then refer to the cube of max(n_d) elements, with zeros
    outside the box (the library serves the box as a domain inside that cube).  Smoother
    "vertex" (eq. Preconditioner P) or "edge" (eq. Preconditioner E) on subdomains of
    subdomain^3 elements (2 or 4).  coef: an r x r x r array of box factors, alpha(x) =
    alpha * coef[z][y][x] of x's box (jumps, Sec. 6; r divides the coarsest level).
    domain: an r x r x r array of flags, the boxes a non-box domain keeps (Sec. 6).  With
    nrhs > 1 every call works on nrhs vectors at once ([nrhs, vec_len] tensors), each
    right-hand side with its own CG scalars."""

    def __init__(self, n, alpha, length=1.0, m=1, eta=None, precision="fp64",
                 boundary_patches=True, flexible=None, use_graphs=None, device="cuda:0", nrhs=1,
                 bottom_n=None, dense_n=None, levels=0, smoother="vertex", subdomain=2, coef=None,
                 domain=None):
        dims = (int(n),) * 3 if np.ndim(n) == 0 else tuple(int(v) for v in n)
        box = (float(length),) * 3 if np.ndim(length) == 0 else tuple(float(v) for v in length)
        if len(dims) != 3 or len(box) != 3:
            raise ValueError("n and length: a number (cube) or three per axis (box)")
        cube = dims[0] == dims[1] == dims[2]
        # a box that is not a cube runs inside the cube of max(n_d) elements (zeros outside)
        self.dims, self.box = dims, box
        self.n = max(dims)
        self.length = box[dims.index(self.n)]
        self.alpha, self.nrhs = float(alpha), int(nrhs)
        self._domain = domain
        if self.nrhs > 1 and levels:
            raise ValueError("levels applies to single right-hand-side solvers")
        if self.nrhs > 1 and not cube:
            raise ValueError("several right-hand sides at once need a cube")
        o = _opts(m, eta, precision, boundary_patches, flexible, use_graphs, bottom_n, dense_n,
                  smoother, subdomain, coef, domain)
        self.opts = o
        self.precision = precision
        if self.nrhs == 1:
            ws_bytes, self.vec_len = _lib.ndmg_plan(dims, box, self.alpha, o, levels)
        else:
            ws_bytes, tl = _lib.ndmg_plan_batched([self.n], self.length, self.nrhs, o)
            self.vec_len = tl // self.nrhs
        self._alloc(ws_bytes, device)
        if self.nrhs == 1:
            self.ctx = _lib.ndmg_setup(dims, box, self.alpha, o, self._ws_ptr, ws_bytes,
                                       self.stream.cuda_stream, levels)
        else:
            self.ctx = _lib.ndmg_setup_batched([self.n], self.length, [self.alpha], self.nrhs, o,
                                               self._ws_ptr, ws_bytes, self.stream.cuda_stream)
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        info = _lib.ndmg_layout(self.ctx, -1)
        self.P, self.B, self.levels, self.ndof = info[1], info[2], info[4], info[5]

    # ---- helpers -------------------------------------------------------------------
    def zeros(self, *lead):
        if not lead and self.nrhs > 1:
            lead = (self.nrhs,)
        return torch.zeros(*lead, self.vec_len, dtype=torch.float64, device=self.device)

    def _check(self, t):
        if t.dtype != torch.float64 or t.device != self.device or not t.is_contiguous():
            raise ValueError("vectors must be contiguous float64 tensors on the solver's device")
        if t.shape[-1] != self.vec_len:
            raise ValueError(f"vector length {t.shape[-1]} != {self.vec_len}")
        if t.numel() != self.nrhs * self.vec_len:
            raise ValueError(f"expected {self.nrhs} vector(s) of length {self.vec_len}")
        return t.data_ptr()

    def layout(self, level=-1):
        return _lib.ndmg_layout(self.ctx, level)

    def unknown_mask(self):
        """1.0 at the entries of the padded layout that are unknowns, else 0: the edges
        whose four cells lie inside the domain (the interior edges of the cube, or of the
        box or union of boxes solved on)."""
        if getattr(self, "_mask", None) is None:
            n = self.n
            # cell flags, [z][y][x], with a layer of outside cells around the cube
            c = torch.zeros(n + 2, n + 2, n + 2, dtype=torch.bool, device=self.device)
            c[1:n + 1, 1:n + 1, 1:n + 1] = self._cells_inside()
            m = torch.zeros(3, n + 1, n + 1, self.P, dtype=torch.float64, device=self.device)
            # an x edge (cell i, nodes j, k) touches cells (i, j-1..j, k-1..k); likewise y, z
            m[0, :, :, :n] = (c[:-1, :-1, 1:-1] & c[:-1, 1:, 1:-1] & c[1:, :-1, 1:-1] & c[1:, 1:, 1:-1]).double()
            m[1, :, :n, :n + 1] = (c[:-1, 1:-1, :-1] & c[:-1, 1:-1, 1:] & c[1:, 1:-1, :-1] & c[1:, 1:-1, 1:]).double()
            m[2, :n, :, :n + 1] = (c[1:-1, :-1, :-1] & c[1:-1, :-1, 1:] & c[1:-1, 1:, :-1] & c[1:-1, 1:, 1:]).double()
            self._mask = m.reshape(-1)
        return self._mask

    def _cells_inside(self):
        """[n, n, n] flags ([z][y][x]) of the cells of the cube that belong to the domain."""
        n = self.n
        if self._domain is not None:
            flags = torch.as_tensor(np.asarray(self._domain, dtype=bool), device=self.device)
            w = n // flags.shape[0]
            return flags.repeat_interleave(w, 0).repeat_interleave(w, 1).repeat_interleave(w, 2)
        inside = torch.zeros(n, n, n, dtype=torch.bool, device=self.device)
        nx, ny, nz = self.dims
        inside[:nz, :ny, :nx] = True
        return inside

    # ---- operations -----------------------------------------------------------------

    def apply(self, x, y=None):
        y = self.zeros() if y is None else y
        self._run(_lib.ndmg_apply, self._check(x), self._check(y))
        return y

    def vcycle(self, g, z=None):
        z = self.zeros() if z is None else z
        self._run(_lib.ndmg_vcycle, self._check(g), self._check(z))
        return z

    def solve(self, b, rtol=1e-10, maxit=500, u=None, raise_on_noconv=True, warm=False):
        """u = A^{-1} b by V-cycle PCG; returns (u, iterations, relative residual), the
        last two as lists over the right-hand sides when nrhs > 1.  warm: start from the
        values in u instead of 0."""
        u = self.zeros() if u is None else u
        if warm:
            code, it, rel = self._run(_lib.ndmg_pcg_solve_warm, self._check(b), self._check(u), rtol, maxit,
                                      self.nrhs, raise_on_noconv)
            return (u, it[0], rel[0]) if self.nrhs == 1 else (u, it, rel)
        if self.nrhs == 1:
            code, it, rel = self._run(_lib.ndmg_pcg_solve, self._check(b), self._check(u), rtol,
                                      maxit, raise_on_noconv)
            return u, it, rel
        code, it, rel = self._run(_lib.ndmg_pcg_solve_batched, self._check(b), self._check(u), rtol,
                                  maxit, self.nrhs, raise_on_noconv)
        return u, it, rel

    def maxwell_step(self, f, u, v, a, dt, eps=1.0, sigma=0.0, mu=1.0, rtol=1e-10, maxit=500):
        """One average-acceleration Newmark step of eps E'' + sigma E' + curl(mu^-1 curl E) = J'
        (each step is the model problem with this solver's alpha = dt^2 / (4 mu (eps +
        sigma dt / 2)), eq. Maxwell timestep); u, v, a updated in place; f = (J', phi) at the
        new time.  Returns (iterations, relative residuals) per right-hand side."""
        return self._run(_lib.ndmg_maxwell_step, self._check(f), self._check(u), self._check(v), self._check(a),
                         dt, eps, sigma, mu, rtol, maxit, self.nrhs)

    def contraction(self, b, rtol=1e-13, maxit=200):
        """V-cycle contraction number ||E||_a = 1 - lambda_min(B A) by the Lanczos process of
        preconditioned CG started from b; returns (contraction, lambda_max(B A), steps)."""
        u = self.zeros()
        return self._run(_lib.ndmg_contraction, self._check(b), self._check(u), rtol, maxit)

    def assemble_rhs(self, f):
        """b from f sampled at the 2x2x2 Gauss points ([n^3, 8, 3] float64)."""
        f = torch.as_tensor(f, dtype=torch.float64, device=self.device).contiguous()
        if f.numel() != self.nrhs * self.n ** 3 * 24:
            raise ValueError("f must hold nrhs x n^3 x 8 x 3 values")
        b = self.zeros()
        self._run(_lib.ndmg_assemble_rhs, f.data_ptr(), self._check(b))
        return b

    def curlcurl_form(self, lam, u):
        """sum_r lam_r^T K u_r for stacked vectors [k, vec_len] (any k)."""
        lam = lam.reshape(-1, self.vec_len).contiguous()
        u = u.reshape(-1, self.vec_len).contiguous()
        if lam.shape != u.shape or lam.dtype != torch.float64 or u.dtype != torch.float64:
            raise ValueError("lam and u must be float64 of the same shape")
        return self._run(_lib.ndmg_curlcurl_form, lam.data_ptr(), u.data_ptr(), lam.shape[0])

    def level_op(self, level, op, x, out=None):
        """One step on one level (FP64 solvers): op in 'apply', 'smooth', 'restrict',
        'prolong' (out += P x, out of level `level`, x of level-1), 'coarse'."""
        ops = {"apply": 0, "smooth": 1, "restrict": 2, "prolong": 3, "coarse": 4}
        lvl = level if level >= 0 else self.levels + level
        in_level = lvl - 1 if op == "prolong" else lvl
        out_level = lvl - 1 if op == "restrict" else lvl
        ln_in = _lib.ndmg_layout(self.ctx, in_level)[3] * self.nrhs
        ln_out = _lib.ndmg_layout(self.ctx, out_level)[3] * self.nrhs
        x = x.contiguous()
        if x.numel() != ln_in or x.dtype != torch.float64:
            raise ValueError("input has the wrong length or dtype")
        if out is None:
            out = torch.zeros(ln_out, dtype=torch.float64, device=self.device)
        if out.numel() != ln_out:
            raise ValueError("output has the wrong length")
        self._run(_lib.ndmg_level_op, lvl, ops[op], x.data_ptr(), out.data_ptr())
        return out

    def export_factor(self, level, which, typ=13):
        buf, d = _lib.ndmg_export_factor(self.ctx, level, which, typ)
        return np.array(buf).reshape(d, d)


class BatchedSolver(_Context):
    """Many independent problems of uneven sizes (n[p] cubes per axis, alpha[p]) with
    nrhs right-hand sides each, solved together: every kernel covers all pairs of one
    size, sizes run concurrently, and each (problem, right-hand side) pair has its own
    CG scalars and stops on its own.  Vectors are batch vectors (see `offset`)."""

    def __init__(self, ns, alphas, nrhs=1, length=1.0, m=1, eta=None, precision="fp32",
                 boundary_patches=True, flexible=None, use_graphs=None, device="cuda:0",
                 bottom_n=None, dense_n=None, smoother="vertex", subdomain=2):
        self.ns = [int(v) for v in ns]
        self.alphas = [float(v) for v in alphas]
        self.nrhs, self.length, self.precision = int(nrhs), float(length), precision
        o = _opts(m, eta, precision, boundary_patches, flexible, use_graphs, bottom_n, dense_n,
                  smoother, subdomain)
        self.opts = o
        ws_bytes, self.total_len = _lib.ndmg_plan_batched(self.ns, self.length, self.nrhs, o)
        self._alloc(ws_bytes, device)
        self.ctx = _lib.ndmg_setup_batched(self.ns, self.length, self.alphas, self.nrhs, o,
                                           self._ws_ptr, ws_bytes, self.stream.cuda_stream)
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        self.layouts = [_lib.ndmg_batch_layout(self.ctx, p) for p in range(len(self.ns))]
        self.npairs = len(self.ns) * self.nrhs

    @property
    def nprob(self):
        return len(self.ns)

    def offset(self, p):
        """(first element, vector length, n, P, B, levels) of problem p in a batch vector."""
        return tuple(self.layouts[p])

    def zeros(self):
        return torch.zeros(self.total_len, dtype=torch.float64, device=self.device)

    def view(self, X, p):
        """The [nrhs, vec_len] block of problem p in batch vector X (a view)."""
        off, vl = self.layouts[p][0], self.layouts[p][1]
        return X[off:off + self.nrhs * vl].view(self.nrhs, vl)

    def pack(self, blocks):
        """Batch vector from a list of per-problem [nrhs, vec_len] tensors."""
        X = self.zeros()
        for p, blk in enumerate(blocks):
            self.view(X, p).copy_(blk.reshape(self.nrhs, -1))
        return X

    def _check(self, t):
        if (t.dtype != torch.float64 or t.device != self.device or not t.is_contiguous()
                or t.numel() != self.total_len):
            raise ValueError(f"batch vectors must be contiguous float64 [{self.total_len}] tensors")
        return t.data_ptr()

    def apply(self, x, y=None):
        y = self.zeros() if y is None else y
        self._run(_lib.ndmg_apply, self._check(x), self._check(y))
        return y

    def vcycle(self, g, z=None):
        z = self.zeros() if z is None else z
        self._run(_lib.ndmg_vcycle, self._check(g), self._check(z))
        return z

    def sample_len(self):
        """Length of the Gauss-point sample array of assemble_rhs: n^3 x 8 x 3 values per
        pair, pairs in batch-vector order."""
        return sum(24 * n ** 3 * self.nrhs for n in self.ns)

    def assemble_rhs(self, f):
        """Batch vector of load vectors from f sampled at the 2x2x2 Gauss points of every
        element of every pair (see sample_len; pairs ordered as in batch vectors)."""
        if (f.dtype != torch.float64 or f.device != self.device or not f.is_contiguous()
                or f.numel() != self.sample_len()):
            raise ValueError(f"f must be a contiguous float64 tensor of {self.sample_len()} values")
        b = self.zeros()
        self._run(_lib.ndmg_assemble_rhs, f.data_ptr(), self._check(b))
        return b

    def solve(self, B, rtol=1e-10, maxit=500, U=None, raise_on_noconv=True):
        """U = A_p^{-1} B for every pair; returns (U, iterations [nprob, nrhs],
        relative residuals [nprob, nrhs])."""
        U = self.zeros() if U is None else U
        code, it, rel = self._run(_lib.ndmg_pcg_solve_batched, self._check(B), self._check(U), rtol,
                                  maxit, self.npairs, raise_on_noconv)
        return (U, np.array(it, dtype=np.int64).reshape(self.nprob, self.nrhs),
                np.array(rel).reshape(self.nprob, self.nrhs))
