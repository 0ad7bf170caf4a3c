"""ctypes binding of libndmg.so (the C ABI declared in include/ndmg.h).

Argument marshalling only: every step of the solver runs in the HIP library.  The
functions keep the C names; device pointers are passed as integers (for example
``tensor.data_ptr()``) and the stream as ``torch.cuda.Stream.cuda_stream``.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libndmg.so")

NDMG_OK = 0
NDMG_EINVAL = 1
NDMG_EHIP = 2
NDMG_ENOCONV = 3
NDMG_EBREAKDOWN = 4
NDMG_EWORKSPACE = 5

EXPORTED = [
    "ndmg_default_opts", "ndmg_plan", "ndmg_setup", "ndmg_layout", "ndmg_apply",
    "ndmg_vcycle", "ndmg_pcg_solve", "ndmg_assemble_rhs", "ndmg_curlcurl_form",
    "ndmg_export_factor", "ndmg_level_op", "ndmg_destroy", "ndmg_last_error",
    "ndmg_plan_batched", "ndmg_setup_batched", "ndmg_batch_layout", "ndmg_pcg_solve_batched",
    "ndmg_curlcurl_form_noalloc", "ndmg_contraction", "ndmg_pcg_solve_warm", "ndmg_maxwell_step",
    "ndmg_source_key", "ndmg_tuning_load", "ndmg_tuning_set", "ndmg_tuning_clear", "ndmg_time_stencil",
    "ndmg_stencil_shape",
]

# The autotuner's table of launch shapes (written by tune.py on the device); loaded with the
# library when its key matches the library's kernel sources.
TUNING_PATH = os.path.join(HERE, "tuning.txt")

NDMG_OP_APPLY, NDMG_OP_SMOOTH, NDMG_OP_RESTRICT, NDMG_OP_PROLONG, NDMG_OP_COARSE, NDMG_OP_PATCH = range(6)


class ndmg_opts(ctypes.Structure):
    _fields_ = [
        ("smoother", ctypes.c_int),
        ("m", ctypes.c_int),
        ("eta", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("subdomain", ctypes.c_int),
        ("boundary_patches", ctypes.c_int),
        ("flexible", ctypes.c_int),
        ("use_graphs", ctypes.c_int),
        ("bottom_n", ctypes.c_int),
        ("dense_n", ctypes.c_int),
        ("coef_r", ctypes.c_int),
        ("coef", ctypes.POINTER(ctypes.c_double)),
        ("domain", ctypes.POINTER(ctypes.c_ubyte)),
    ]


class NdmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ndmg error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libndmg.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, d, i = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_double, ctypes.c_int
    P = ctypes.POINTER
    L.ndmg_default_opts.argtypes = [P(ndmg_opts)]
    L.ndmg_default_opts.restype = None
    L.ndmg_plan.argtypes = [i, i, i, P(d), d, i, P(ndmg_opts), P(sz), P(sz)]
    L.ndmg_setup.argtypes = [P(vp), i, i, i, P(d), d, i, P(ndmg_opts), vp, sz, vp]
    L.ndmg_layout.argtypes = [vp, i, P(ctypes.c_int64)]
    L.ndmg_apply.argtypes = [vp, vp, vp]
    L.ndmg_vcycle.argtypes = [vp, vp, vp]
    L.ndmg_pcg_solve.argtypes = [vp, vp, vp, d, i, P(i), P(d)]
    L.ndmg_assemble_rhs.argtypes = [vp, vp, vp]
    L.ndmg_curlcurl_form.argtypes = [vp, vp, vp, i, P(d)]
    L.ndmg_curlcurl_form_noalloc.argtypes = [i, d, vp, vp, i, P(d), vp]
    L.ndmg_contraction.argtypes = [vp, vp, vp, d, i, P(d), P(d), P(i)]
    L.ndmg_pcg_solve_warm.argtypes = [vp, vp, vp, d, i, P(i), P(d)]
    L.ndmg_maxwell_step.argtypes = [vp, vp, vp, vp, vp, d, d, d, d, d, i, P(i), P(d)]
    L.ndmg_export_factor.argtypes = [vp, i, i, i, P(d), P(i)]
    L.ndmg_level_op.argtypes = [vp, i, i, vp, vp]
    L.ndmg_plan_batched.argtypes = [i, P(i), d, i, P(ndmg_opts), P(sz), P(sz)]
    L.ndmg_setup_batched.argtypes = [P(vp), i, P(i), d, P(d), i, P(ndmg_opts), vp, sz, vp]
    L.ndmg_batch_layout.argtypes = [vp, i, P(ctypes.c_int64)]
    L.ndmg_pcg_solve_batched.argtypes = [vp, vp, vp, d, i, P(i), P(d)]
    L.ndmg_destroy.argtypes = [vp]
    L.ndmg_last_error.argtypes = []
    L.ndmg_last_error.restype = ctypes.c_char_p
    L.ndmg_source_key.argtypes = []
    L.ndmg_source_key.restype = ctypes.c_char_p
    L.ndmg_tuning_load.argtypes = [ctypes.c_char_p]
    L.ndmg_tuning_set.argtypes = [ctypes.c_char_p]
    L.ndmg_tuning_clear.argtypes = []
    L.ndmg_time_stencil.argtypes = [i, i, i, i, i, i, vp, vp, vp, vp, vp, i, i, vp, P(d)]
    L.ndmg_stencil_shape.argtypes = [i, i, i, i, P(i), P(i)]
    for name in EXPORTED:
        if name not in ("ndmg_default_opts", "ndmg_last_error", "ndmg_source_key"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    if os.path.exists(TUNING_PATH) and L.ndmg_tuning_load(TUNING_PATH.encode()) != NDMG_OK:
        import warnings
        warnings.warn("launch-shape table not used: " + L.ndmg_last_error().decode())
    return L


def check(code):
    if code != NDMG_OK:
        raise NdmgError(code, lib().ndmg_last_error().decode())
    return code


def ndmg_default_opts():
    o = ndmg_opts()
    lib().ndmg_default_opts(ctypes.byref(o))
    return o


def _box(dims, box):
    """(nx, ny, nz) and the box lengths from an int n (cube) or a triple, and a scalar
    length or a triple."""
    dims = (int(dims),) * 3 if isinstance(dims, (int,)) or hasattr(dims, "__index__") else tuple(int(v) for v in dims)
    box = (float(box),) * 3 if isinstance(box, (int, float)) else tuple(float(v) for v in box)
    return dims, (ctypes.c_double * 3)(*box)


def ndmg_plan(dims, box, alpha, opts, levels=0):
    (nx, ny, nz), b = _box(dims, box)
    ws, vl = ctypes.c_size_t(), ctypes.c_size_t()
    check(lib().ndmg_plan(nx, ny, nz, b, alpha, int(levels), ctypes.byref(opts), ctypes.byref(ws),
                          ctypes.byref(vl)))
    return ws.value, vl.value


def ndmg_setup(dims, box, alpha, opts, d_workspace, workspace_bytes, stream, levels=0):
    (nx, ny, nz), b = _box(dims, box)
    ctx = ctypes.c_void_p()
    check(lib().ndmg_setup(ctypes.byref(ctx), nx, ny, nz, b, alpha, int(levels), ctypes.byref(opts),
                           d_workspace, workspace_bytes, stream))
    return ctx


def ndmg_layout(ctx, level=-1):
    info = (ctypes.c_int64 * 6)()
    check(lib().ndmg_layout(ctx, level, info))
    return list(info)


def ndmg_apply(ctx, d_x, d_y):
    return check(lib().ndmg_apply(ctx, d_x, d_y))


def ndmg_vcycle(ctx, d_g, d_z):
    return check(lib().ndmg_vcycle(ctx, d_g, d_z))


def ndmg_pcg_solve(ctx, d_b, d_u, rtol, maxit, raise_on_noconv=True):
    it, rel = ctypes.c_int(), ctypes.c_double()
    code = lib().ndmg_pcg_solve(ctx, d_b, d_u, rtol, maxit, ctypes.byref(it), ctypes.byref(rel))
    if code != NDMG_OK and (raise_on_noconv or code != NDMG_ENOCONV):
        check(code)
    return code, it.value, rel.value


def ndmg_contraction(ctx, d_b, d_u, rtol, maxit):
    c, lm, it = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
    check(lib().ndmg_contraction(ctx, d_b, d_u, rtol, maxit, ctypes.byref(c), ctypes.byref(lm), ctypes.byref(it)))
    return c.value, lm.value, it.value


def ndmg_pcg_solve_warm(ctx, d_b, d_u, rtol, maxit, npairs, raise_on_noconv=True):
    it = (ctypes.c_int * npairs)()
    rel = (ctypes.c_double * npairs)()
    code = lib().ndmg_pcg_solve_warm(ctx, d_b, d_u, rtol, maxit, it, rel)
    if code != NDMG_OK and (raise_on_noconv or code != NDMG_ENOCONV):
        check(code)
    return code, list(it), list(rel)


def ndmg_maxwell_step(ctx, d_f, d_u, d_v, d_a, dt, eps, sigma, mu, rtol, maxit, npairs):
    it = (ctypes.c_int * npairs)()
    rel = (ctypes.c_double * npairs)()
    check(lib().ndmg_maxwell_step(ctx, d_f, d_u, d_v, d_a, dt, eps, sigma, mu, rtol, maxit, it, rel))
    return list(it), list(rel)


def ndmg_plan_batched(ns, length, nrhs, opts):
    arr = (ctypes.c_int * len(ns))(*[int(v) for v in ns])
    ws, tl = ctypes.c_size_t(), ctypes.c_size_t()
    check(lib().ndmg_plan_batched(len(ns), arr, length, nrhs, ctypes.byref(opts), ctypes.byref(ws),
                                  ctypes.byref(tl)))
    return ws.value, tl.value


def ndmg_setup_batched(ns, length, alphas, nrhs, opts, d_workspace, workspace_bytes, stream):
    if len(alphas) != len(ns):
        raise ValueError("one alpha per problem")
    narr = (ctypes.c_int * len(ns))(*[int(v) for v in ns])
    aarr = (ctypes.c_double * len(ns))(*[float(v) for v in alphas])
    ctx = ctypes.c_void_p()
    check(lib().ndmg_setup_batched(ctypes.byref(ctx), len(ns), narr, length, aarr, nrhs,
                                   ctypes.byref(opts), d_workspace, workspace_bytes, stream))
    return ctx


def ndmg_batch_layout(ctx, prob):
    info = (ctypes.c_int64 * 6)()
    check(lib().ndmg_batch_layout(ctx, prob, info))
    return list(info)


def ndmg_pcg_solve_batched(ctx, d_b, d_u, rtol, maxit, npairs, raise_on_noconv=True,
                           raise_on_breakdown=True):
    """Returns (status, iterations, relative residuals) per pair; ENOCONV and EBREAKDOWN
    are returned instead of raised when the matching flag is False."""
    it = (ctypes.c_int * npairs)()
    rel = (ctypes.c_double * npairs)()
    code = lib().ndmg_pcg_solve_batched(ctx, d_b, d_u, rtol, maxit, it, rel)
    quiet = ((code == NDMG_ENOCONV and not raise_on_noconv)
             or (code == NDMG_EBREAKDOWN and not raise_on_breakdown))
    if code != NDMG_OK and not quiet:
        check(code)
    return code, list(it), list(rel)


def ndmg_assemble_rhs(ctx, d_f, d_b):
    return check(lib().ndmg_assemble_rhs(ctx, d_f, d_b))


def ndmg_curlcurl_form(ctx, d_lam, d_u, nrhs):
    out = ctypes.c_double()
    check(lib().ndmg_curlcurl_form(ctx, d_lam, d_u, nrhs, ctypes.byref(out)))
    return out.value


def ndmg_export_factor(ctx, level, which, typ=13):
    dims = ctypes.c_int()
    check(lib().ndmg_export_factor(ctx, level, which, typ, None, ctypes.byref(dims)))
    buf = (ctypes.c_double * (dims.value * dims.value))()
    check(lib().ndmg_export_factor(ctx, level, which, typ, buf, ctypes.byref(dims)))
    return list(buf), dims.value


def ndmg_level_op(ctx, level, op, d_in, d_out):
    return check(lib().ndmg_level_op(ctx, level, op, d_in, d_out))


def ndmg_destroy(ctx):
    return check(lib().ndmg_destroy(ctx))
