"""CPU-side checks of the C ABI: the library loads, exports every declared symbol, and
plans / validates problems without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2205_05840_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ndmg.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(ndmg_\w+)\s*\(", src, re.M)))


def test_every_declared_symbol_is_exported(lib):
    L = lib.lib()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    assert sorted(lib.EXPORTED) == names


def test_default_opts(lib):
    o = lib.ndmg_default_opts()
    assert o.m == 1 and o.eta == 0.0 and o.subdomain == 2 and o.smoother == 0   # eta 0: Sec. 5's value
    assert o.boundary_patches == 1 and o.precision == 0


@pytest.mark.parametrize("n,nl", [(2, 1), (3, 1), (4, 2), (6, 2), (8, 3), (12, 3), (64, 6),
                                  (96, 6), (128, 7)])
def test_plan_sizes(lib, n, nl):
    o = lib.ndmg_default_opts()
    ws, vl = lib.ndmg_plan(n, 1.0, 1.0, o)
    P = ((n + 1) + 7) // 8 * 8
    assert vl == 3 * (n + 1) ** 2 * P
    assert ws % 256 == 0 and ws > 4 * vl * 8


@pytest.mark.parametrize("args,code", [
    ((1, 1.0, 1.0), 1), ((8, 1.0, 0.0), 1), ((8, 1.0, -1.0), 1), ((8, 0.0, 1.0), 1),
    ((8, 1.0, float("nan")), 1), ((22, 1.0, 1.0), 1),   # coarsest 11^3 is too large
])
def test_plan_rejects(lib, args, code):
    o = lib.ndmg_default_opts()
    with pytest.raises(lib.NdmgError) as e:
        lib.ndmg_plan(*args, o)
    assert e.value.code == code
    assert lib.lib().ndmg_last_error().decode()


def test_plan_rejects_bad_options(lib):
    for field, val in (("m", 0), ("precision", 7), ("subdomain", 3), ("smoother", 5), ("subdomain", 8),
                       ("dense_n", -2), ("dense_n", 9), ("use_graphs", 2), ("use_graphs", -2)):
        o = lib.ndmg_default_opts()
        setattr(o, field, val)
        with pytest.raises(lib.NdmgError):
            lib.ndmg_plan(8, 1.0, 1.0, o)


def test_dense_default_by_class_size(lib):
    """dense_n = -1 (the default): the dense bottom from the 8^3 level for a single problem,
    from 4^3 for a class of 16 or more problems (workspace equal to dense_n 8, resp. 4)."""
    o = lib.ndmg_default_opts()
    assert o.dense_n == -1 and o.use_graphs == -1

    def ws(ns, dense):
        q = lib.ndmg_default_opts()
        q.dense_n = dense
        return lib.ndmg_plan_batched(ns, 1.0, 2, q)[0]

    assert ws([16], -1) == ws([16], 8) != ws([16], 4)
    assert ws([16] * 16, -1) == ws([16] * 16, 4) != ws([16] * 16, 8)
    assert ws([16] * 15, -1) == ws([16] * 15, 8)


def test_null_arguments(lib):
    L = lib.lib()
    assert L.ndmg_apply(None, None, None) == lib.NDMG_EINVAL
    assert L.ndmg_layout(None, 0, None) == lib.NDMG_EINVAL
    ctx = ctypes.c_void_p()
    o = lib.ndmg_default_opts()
    box = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    assert L.ndmg_setup(ctypes.byref(ctx), 8, 8, 8, box, 1.0, 0, ctypes.byref(o), None, 0, None) == \
        lib.NDMG_EINVAL
    assert L.ndmg_plan(8, 8, 8, None, 1.0, 0, ctypes.byref(o), None, None) == lib.NDMG_EINVAL
    assert L.ndmg_destroy(None) == 0


def test_product_path_does_not_import_oracle():
    """The package never imports the oracle (parity would be void otherwise)."""
    pkg = os.path.join(ROOT, "paper_2205_05840_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle", txt, re.M), f


def test_plan_batched_matches_single(lib):
    o = lib.ndmg_default_opts()
    # one problem, one right-hand side: same vector length as the single plan
    ws1, vl1 = lib.ndmg_plan(16, 1.0, 1.0, o)
    wsb, tl = lib.ndmg_plan_batched([16], 1.0, 1, o)
    assert tl == vl1 and wsb >= ws1 // 2
    # uneven sizes: the batch vector concatenates nrhs padded vectors per problem
    ns, nrhs = [8, 12, 16, 8, 24, 32, 12], 4
    ws, tl = lib.ndmg_plan_batched(ns, 1.0, nrhs, o)
    per = [3 * (n + 1) ** 2 * (((n + 1) + 7) // 8 * 8) for n in ns]
    assert tl == nrhs * sum(per)
    assert ws % 256 == 0 and ws > 4 * tl * 8


@pytest.mark.parametrize("ns,nrhs", [([8, 1], 1), ([8, 22], 1), ([8], 0), ([], 1),
                                     ([8] * 20000, 4)])
def test_plan_batched_rejects(lib, ns, nrhs):
    o = lib.ndmg_default_opts()
    with pytest.raises(lib.NdmgError) as e:
        lib.ndmg_plan_batched(ns, 1.0, nrhs, o)
    assert e.value.code == lib.NDMG_EINVAL


def test_batched_null_arguments(lib):
    L = lib.lib()
    ctx = ctypes.c_void_p()
    o = lib.ndmg_default_opts()
    n = (ctypes.c_int * 2)(8, 12)
    assert L.ndmg_setup_batched(ctypes.byref(ctx), 2, n, 1.0, None, 1, ctypes.byref(o), None, 0,
                                None) == lib.NDMG_EINVAL
    assert L.ndmg_batch_layout(None, 0, None) == lib.NDMG_EINVAL
    assert L.ndmg_pcg_solve_batched(None, None, None, 1e-10, 10, None, None) == lib.NDMG_EINVAL


@pytest.mark.parametrize("dims,box,msg", [((8, 8, 8), (1.0, 1.0, 1.5), b"must be cubes"),
                                          ((8, 8, 8), (1.0, -1.0, 1.0), b"box lengths"),
                                          ((8, 8, 1), (1.0, 1.0, 0.125), b">= 2"),
                                          ((16, 12, 8), (4.0, 3.0, 2.0), b"must divide the coarsest"),
                                          ((256, 2, 2), (128.0, 1.0, 1.0), b"too elongated")])
def test_plan_box_rejections(lib, dims, box, msg):
    """The boundary takes a box (Sec. 1) with nx x ny x nz elements; the elements must be
    cubes, and a box that is not a cube must fit the embedding cube's level hierarchy:
    anything else is refused with a message (no silent fallback)."""
    o = lib.ndmg_default_opts()
    with pytest.raises(lib.NdmgError) as e:
        lib.ndmg_plan(dims, box, 1.0, o)
    assert e.value.code == lib.NDMG_EINVAL
    assert msg in lib.lib().ndmg_last_error()


def test_plan_box_cube_equals_scalar_form(lib):
    o = lib.ndmg_default_opts()
    assert lib.ndmg_plan((16, 16, 16), (2.0, 2.0, 2.0), 1.0, o) == lib.ndmg_plan(16, 2.0, 1.0, o)


@pytest.mark.parametrize("dims,box", [((16, 8, 8), (2.0, 1.0, 1.0)), ((8, 16, 16), (1.0, 2.0, 2.0)),
                                      ((32, 16, 16), (2.0, 1.0, 1.0))])
def test_plan_box_embedded(lib, dims, box):
    """A box that is not a cube plans in the layout of the cube of max(n_d) elements (the
    same vector length as that cube), and refuses coefficient boxes of its own."""
    import numpy as np
    o = lib.ndmg_default_opts()
    n = max(dims)
    ws, vl = lib.ndmg_plan(dims, box, 1.0, o)
    _, vl_c = lib.ndmg_plan(n, max(box), 1.0, o)
    assert vl == vl_c and ws > 0
    with pytest.raises(lib.NdmgError):
        lib.ndmg_plan(dims, box, 1.0, _coef_opts(lib, 2))


@pytest.mark.parametrize("n,levels,ok", [(32, 1, False), (32, 2, False), (32, 3, False), (32, 4, True),
                                         (32, 5, True), (32, 6, False), (12, 1, False), (12, 2, True),
                                         (6, 1, True)])
def test_plan_levels(lib, n, levels, ok):
    """levels = L keeps the L finest levels n, n/2, ...; the coarsest of them is solved
    exactly, so it must have at most 1024 unknowns (8^3 has 1176: too many); more levels
    than the halving rule gives are refused."""
    o = lib.ndmg_default_opts()
    if ok:
        ws, vl = lib.ndmg_plan(n, 1.0, 1.0, o, levels)
        ws_all, vl_all = lib.ndmg_plan(n, 1.0, 1.0, o)
        assert vl == vl_all and ws <= ws_all
    else:
        with pytest.raises(lib.NdmgError) as e:
            lib.ndmg_plan(n, 1.0, 1.0, o, levels)
        assert e.value.code == lib.NDMG_EINVAL


@pytest.mark.parametrize("smoother,s,n", [(1, 2, 8), (1, 2, 16), (1, 4, 16), (0, 4, 8), (0, 4, 64),
                                          (1, 2, 12), (0, 4, 24)])
def test_plan_generic_smoothers(lib, smoother, s, n):
    """The edge smoother (eq. Preconditioner E) and 4 x 4 x 4 subdomains plan; the one-launch
    bottom is refused for them."""
    o = lib.ndmg_default_opts()
    o.smoother, o.subdomain = smoother, s
    ws, vl = lib.ndmg_plan(n, 1.0, 1.0, o)
    assert ws % 256 == 0 and vl == 3 * (n + 1) ** 2 * (((n + 1) + 7) // 8 * 8)
    o.bottom_n = 8
    with pytest.raises(lib.NdmgError):
        lib.ndmg_plan(n, 1.0, 1.0, o)


def test_plan_s4_needs_divisible_levels(lib):
    o = lib.ndmg_default_opts()
    o.subdomain = 4
    with pytest.raises(lib.NdmgError):
        lib.ndmg_plan(10, 1.0, 1.0, o)       # 10 is not divisible by min(4, 10 / 2)


def test_tuning_table(lib, tmp_path):
    """The launch-shape table: entries set by line change the operator shape the library
    picks; a file keyed to other kernel sources, or malformed, is refused and leaves the
    table as it was; clearing brings back the cost model."""
    L = lib.lib()
    v, z = ctypes.c_int(), ctypes.c_int()
    L.ndmg_tuning_clear()
    assert L.ndmg_stencil_shape(96, 0, 0, 1, ctypes.byref(v), ctypes.byref(z)) == 0
    model = (v.value, z.value)
    assert L.ndmg_tuning_set(b"stencil 96 fp64 0 0 1 12") == 0
    assert L.ndmg_stencil_shape(96, 0, 0, 1, ctypes.byref(v), ctypes.byref(z)) == 0
    assert (v.value, z.value) == (1, 12)
    # a variant that does not exist falls back to the model
    assert L.ndmg_tuning_set(b"stencil 96 fp64 0 0 7 12") == 0
    assert L.ndmg_stencil_shape(96, 0, 0, 1, ctypes.byref(v), ctypes.byref(z)) == 0
    assert (v.value, z.value) == model
    key = L.ndmg_source_key().decode()
    good = tmp_path / "good.txt"
    good.write_text(f"# comment\nkey {key}\nstencil 96 fp64 0 0 2 16\n")
    assert L.ndmg_tuning_load(str(good).encode()) == 0
    L.ndmg_stencil_shape(96, 0, 0, 1, ctypes.byref(v), ctypes.byref(z))
    assert (v.value, z.value) == (2, 16)
    stale = tmp_path / "stale.txt"
    stale.write_text("key 0000000000000000\nstencil 96 fp64 0 0 0 4\n")
    assert L.ndmg_tuning_load(str(stale).encode()) == lib.NDMG_EINVAL
    assert b"other kernel sources" in L.ndmg_last_error()
    L.ndmg_stencil_shape(96, 0, 0, 1, ctypes.byref(v), ctypes.byref(z))
    assert (v.value, z.value) == (2, 16)             # unchanged
    assert L.ndmg_tuning_set(b"stencil 96 fp64") == lib.NDMG_EINVAL
    assert L.ndmg_tuning_set(b"warp 96 fp64 0 0 1 1") == lib.NDMG_EINVAL
    # the patch products' addressing: 64-bit addresses or 32-bit buffer offsets only
    assert L.ndmg_tuning_set(b"patchaddr 64 fp32 0 0 64 1") == 0
    assert L.ndmg_tuning_set(b"patchaddr 64 fp64 0 0 32 1") == 0
    assert L.ndmg_tuning_set(b"patchaddr 64 fp32 0 0 48 1") == lib.NDMG_EINVAL
    L.ndmg_tuning_clear()
    L.ndmg_stencil_shape(96, 0, 0, 1, ctypes.byref(v), ctypes.byref(z))
    assert (v.value, z.value) == model
    if os.path.exists(lib.TUNING_PATH):   # leave the process as the binding set it up
        L.ndmg_tuning_load(lib.TUNING_PATH.encode())


def _coef_opts(lib, r, values=None, **kw):
    import numpy as np
    o = lib.ndmg_default_opts()
    for k, v in kw.items():
        setattr(o, k, v)
    if r:
        arr = np.ascontiguousarray(np.full((r, r, r), 3.0) if values is None else values, dtype=np.float64)
        o.coef_r = r
        o.coef = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        o._keep = arr
    return o


@pytest.mark.parametrize("n,r,kw,ok", [
    (8, 2, {}, True), (16, 2, {"subdomain": 4}, True), (12, 3, {}, True), (40, 5, {}, True),
    (8, 1, {"smoother": 1}, True),
    (8, 3, {}, False),                       # 3 does not divide the coarsest level (2)
    (16, 4, {}, False),                      # nor does 4
    (24, 3, {"subdomain": 4}, False),        # level 6 has subdomains of 3 cells, boxes of 2
    (8, 2, {"bottom_n": 8}, False),          # the one-launch bottom takes one alpha
])
def test_plan_coefficient_boxes(lib, n, r, kw, ok):
    """A coefficient with jumps plans when its boxes hold whole elements of every level and
    whole subdomains of every smoothed level; else it is refused with a message."""
    o = _coef_opts(lib, r, **kw)
    if ok:
        ws, vl = lib.ndmg_plan(n, 1.0, 1.0, o)
        _, vl0 = lib.ndmg_plan(n, 1.0, 1.0, _coef_opts(lib, 0, **kw))
        assert vl == vl0 and ws > 0
    else:
        with pytest.raises(lib.NdmgError) as e:
            lib.ndmg_plan(n, 1.0, 1.0, o)
        assert e.value.code == lib.NDMG_EINVAL


def test_plan_coefficient_rejects(lib):
    import numpy as np
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        vals = np.ones((2, 2, 2))
        vals[1, 0, 1] = bad
        with pytest.raises(lib.NdmgError):
            lib.ndmg_plan(8, 1.0, 1.0, _coef_opts(lib, 2, vals))
    o = lib.ndmg_default_opts()
    o.coef_r = 2                              # no array
    with pytest.raises(lib.NdmgError):
        lib.ndmg_plan(8, 1.0, 1.0, o)
    # batches of several problems take one alpha per problem
    with pytest.raises(lib.NdmgError):
        lib.ndmg_plan_batched([8, 8], 1.0, 1, _coef_opts(lib, 2))
    ws, tl = lib.ndmg_plan_batched([8], 1.0, 2, _coef_opts(lib, 2))
    assert tl > 0


def _domain_opts(lib, active, coef=None):
    import numpy as np
    o = _coef_opts(lib, active.shape[0], coef) if coef is not None else lib.ndmg_default_opts()
    d = np.ascontiguousarray(active.astype(np.uint8))
    o.coef_r = active.shape[0]
    o.domain = d.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))
    o._keep_d = d
    return o


def test_plan_domain(lib):
    """A non-box domain plans on the box grid (coef optional); it needs the grid, at least
    one kept box and a single problem."""
    import numpy as np
    fichera = np.ones((2, 2, 2), dtype=bool)
    fichera[1, 1, 1] = False
    ws, vl = lib.ndmg_plan(16, 1.0, 1.0, _domain_opts(lib, fichera))
    _, vl0 = lib.ndmg_plan(16, 1.0, 1.0, lib.ndmg_default_opts())
    assert vl == vl0 and ws > 0
    lib.ndmg_plan(16, 1.0, 1.0, _domain_opts(lib, fichera, np.full((2, 2, 2), 2.0)))
    o = _domain_opts(lib, fichera)
    o.coef_r = 0                                          # no grid
    with pytest.raises(lib.NdmgError):
        lib.ndmg_plan(16, 1.0, 1.0, o)
    with pytest.raises(lib.NdmgError):                    # keeps nothing
        lib.ndmg_plan(16, 1.0, 1.0, _domain_opts(lib, np.zeros((2, 2, 2), dtype=bool)))
    with pytest.raises(lib.NdmgError):                    # 3 does not divide the coarsest level
        lib.ndmg_plan(16, 1.0, 1.0, _domain_opts(lib, np.ones((3, 3, 3), dtype=bool)))
    with pytest.raises(lib.NdmgError):                    # one problem only
        lib.ndmg_plan_batched([16, 16], 1.0, 1, _domain_opts(lib, fichera))
