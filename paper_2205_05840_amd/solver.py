"""Solver: a torch-facing wrapper of one ndmg context.

PyTorch supplies device memory (the workspace and the vectors) and the stream; every
computation runs in libndmg.so.
"""
import numpy as np
import torch

from . import _lib

PRECISIONS = {"fp64": 0, "fp32": 1}


class Solver:
    """V-cycle-preconditioned CG for curl(alpha curl u) + u = f on (0, length)^3 with
    n^3 cubes, lowest-order Nedelec edge elements and zero tangential trace."""

    def __init__(self, n, alpha, length=1.0, m=1, eta=None, precision="fp64",
                 boundary_patches=True, flexible=None, use_graphs=True, device="cuda:0"):
        self.n, self.alpha, self.length = int(n), float(alpha), float(length)
        self.device = torch.device(device)
        o = _lib.ndmg_default_opts()
        o.m = int(m)
        if eta is not None:
            o.eta = float(eta)
        o.precision = PRECISIONS[precision]
        o.boundary_patches = 1 if boundary_patches else 0
        o.flexible = -1 if flexible is None else int(bool(flexible))
        o.use_graphs = 1 if use_graphs else 0
        self.opts = o
        self.precision = precision
        self.ws_bytes, self.vec_len = _lib.ndmg_plan(self.n, self.length, self.alpha, o)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        # the library works on a stream of its own (default priority; graph capture needs a
        # non-null stream); calls are ordered after the caller's current stream and the
        # caller's stream waits for them
        self.stream = torch.cuda.Stream(device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self.ctx = _lib.ndmg_setup(self.n, self.length, self.alpha, o, self._ws_ptr,
                                   self.ws_bytes, self.stream.cuda_stream)
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        info = _lib.ndmg_layout(self.ctx, -1)
        self.P, self.B, self.levels, self.ndof = info[1], info[2], info[4], info[5]

    # ---- helpers -------------------------------------------------------------------
    def zeros(self, *lead):
        return torch.zeros(*lead, self.vec_len, dtype=torch.float64, device=self.device)

    def _check(self, t):
        if t.dtype != torch.float64 or t.device != self.device or not t.is_contiguous():
            raise ValueError("vectors must be contiguous float64 tensors on the solver's device")
        if t.shape[-1] != self.vec_len:
            raise ValueError(f"vector length {t.shape[-1]} != {self.vec_len}")
        return t.data_ptr()

    def layout(self, level=-1):
        return _lib.ndmg_layout(self.ctx, level)

    def unknown_mask(self):
        """1.0 at the entries of the padded layout that are unknowns (interior edges), else 0."""
        if getattr(self, "_mask", None) is None:
            n = self.n
            r = torch.arange(n + 1, device=self.device)
            k, j, i = torch.meshgrid(r, r, r, indexing="ij")
            node = (r >= 1) & (r <= n - 1)
            cell = r < n
            m = torch.zeros(3, n + 1, n + 1, self.P, dtype=torch.float64, device=self.device)
            m[0, :, :, :n + 1] = (cell[i] & node[j] & node[k]).double()
            m[1, :, :, :n + 1] = (node[i] & cell[j] & node[k]).double()
            m[2, :, :, :n + 1] = (node[i] & node[j] & cell[k]).double()
            self._mask = m.reshape(-1)
        return self._mask

    # ---- operations -----------------------------------------------------------------
    def _run(self, fn, *args):
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        try:
            return fn(self.ctx, *args)
        finally:
            cur.wait_stream(self.stream)

    def apply(self, x, y=None):
        y = self.zeros() if y is None else y
        self._run(_lib.ndmg_apply, self._check(x), self._check(y))
        return y

    def vcycle(self, g, z=None):
        z = self.zeros() if z is None else z
        self._run(_lib.ndmg_vcycle, self._check(g), self._check(z))
        return z

    def solve(self, b, rtol=1e-10, maxit=500, u=None, raise_on_noconv=True):
        u = self.zeros() if u is None else u
        code, it, rel = self._run(_lib.ndmg_pcg_solve, self._check(b), self._check(u), rtol, maxit,
                                  raise_on_noconv)
        return u, it, rel

    def assemble_rhs(self, f):
        """b from f sampled at the 2x2x2 Gauss points ([n^3, 8, 3] float64)."""
        f = torch.as_tensor(f, dtype=torch.float64, device=self.device).contiguous()
        if f.numel() != self.n ** 3 * 24:
            raise ValueError("f must hold n^3 x 8 x 3 values")
        b = self.zeros()
        self._run(_lib.ndmg_assemble_rhs, f.data_ptr(), self._check(b))
        return b

    def curlcurl_form(self, lam, u):
        """sum_r lam_r^T K u_r for stacked vectors [nrhs, vec_len]."""
        lam = lam.reshape(-1, self.vec_len).contiguous()
        u = u.reshape(-1, self.vec_len).contiguous()
        return self._run(_lib.ndmg_curlcurl_form, self._check(lam), self._check(u), lam.shape[0])

    def level_op(self, level, op, x, out=None):
        """One step on one level (FP64 solvers): op in 'apply', 'smooth', 'restrict',
        'prolong' (out += P x, out of level `level`, x of level-1), 'coarse'."""
        ops = {"apply": 0, "smooth": 1, "restrict": 2, "prolong": 3, "coarse": 4}
        lvl = level if level >= 0 else self.levels + level
        in_level = lvl - 1 if op == "prolong" else lvl
        out_level = lvl - 1 if op == "restrict" else lvl
        ln_in = _lib.ndmg_layout(self.ctx, in_level)[3]
        ln_out = _lib.ndmg_layout(self.ctx, out_level)[3]
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
