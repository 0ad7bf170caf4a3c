"""Level hierarchy, compact interior-edge numbering and subdomain index sets.

Geometry (Sec. 1, Sec. 2): a box with axis-parallel edges, meshed by n^3 congruent
cubes of side h.  An edge of direction d is addressed by an integer triple
p = (p0, p1, p2): along axis d it is a *cell* index in [0, n), along the two
other axes a *node* index in [0, n].  Edges with a transverse node index equal to
0 or n lie on the boundary and carry no unknown (zero tangential trace, eq.
H(curl) and the boundary condition of eq. model problem).

Compact numbering (oracle only): the x-, y- and z-edge blocks follow each other;
inside block d the unknowns are ordered as a C array indexed [p2][p1][p0] where the
cell axis has n entries (0..n-1) and each node axis n-1 entries (1..n-1).
"""
import numpy as np


def level_sizes(n):
    """Elements per axis of every level, coarsest first (Sec. 3.1: h_k = h_{k-1}/2).

    The finest level has n; a coarser level exists while the current one is even
    and its half is at least 2, so the coarsest level has 2 or 3 (or the odd n
    itself when n is odd).
    """
    if n < 2:
        raise ValueError("need n >= 2")
    sizes = [n]
    while sizes[-1] % 2 == 0 and sizes[-1] // 2 >= 2:
        sizes.append(sizes[-1] // 2)
    return sizes[::-1]


def block_shape(n, d):
    """Array shape (z, y, x) of the compact block of direction d."""
    return tuple(n if ax == d else n - 1 for ax in (2, 1, 0))


def ndof(n):
    """Number of interior edges, 3 n (n-1)^2."""
    return 3 * n * (n - 1) ** 2


def block_offset(n, d):
    return d * n * (n - 1) ** 2


def compact_index(n, dd, p0, p1, p2, d=None):
    """Compact index of the edge of direction dd at p; -1 where it is a boundary edge.

    dd may be None with an array ``d`` of per-entry directions instead."""
    p = [np.asarray(p0), np.asarray(p1), np.asarray(p2)]
    dirs = np.asarray(dd if dd is not None else d)
    shape = np.broadcast(*p, dirs).shape
    ok = np.ones(shape, dtype=bool)
    idx = np.full(shape, -1, dtype=np.int64)
    for dv in range(3):
        sel = np.broadcast_to(dirs == dv, shape)
        if not np.any(sel):
            continue
        q = []
        okd = np.ones(shape, dtype=bool)
        for ax in range(3):
            pa = np.broadcast_to(p[ax], shape)
            if ax == dv:
                okd &= (pa >= 0) & (pa < n)
                q.append(pa)
            else:
                okd &= (pa >= 1) & (pa <= n - 1)
                q.append(pa - 1)
        sh = block_shape(n, dv)
        val = block_offset(n, dv) + (q[2] * sh[1] + q[1]) * sh[2] + q[0]
        idx = np.where(sel, val, idx)
        ok = np.where(sel, okd, ok)
    return np.where(ok, idx, -1)


def edge_coords(n):
    """(d, p0, p1, p2) of every unknown, in compact order."""
    ds, ps = [], []
    for d in range(3):
        s = block_shape(n, d)
        g2, g1, g0 = np.meshgrid(*[np.arange(m) for m in s], indexing="ij")
        lo = [0 if ax == d else 1 for ax in range(3)]
        ps.append(np.stack([g0.ravel() + lo[0], g1.ravel() + lo[1], g2.ravel() + lo[2]], 1))
        ds.append(np.full(g0.size, d))
    return np.concatenate(ds), np.concatenate(ps, 0)


# ---------------------------------------------------------------------------
# Subdomain index sets (Sec. 3.2).  The coarse mesh T_H is the fine mesh grouped in
# s x s x s blocks of fine cells (s = 2 is T_H = T_{k-1}).  E_h^D is read as the
# fine edges lying in the *open* set D (not on its boundary) and not on the
# boundary of Omega.
# ---------------------------------------------------------------------------

def interior_set(n, s, t):
    """Compact indices of E_h^T: fine edges strictly inside coarse element t."""
    out = []
    for d in range(3):
        rng = []
        for ax in range(3):
            if ax == d:
                rng.append(np.arange(s * t[ax], s * t[ax] + s))
            else:
                rng.append(np.arange(s * t[ax] + 1, s * t[ax] + s))
        g0, g1, g2 = np.meshgrid(*rng, indexing="ij")
        out.append(compact_index(n, d, g0.ravel(), g1.ravel(), g2.ravel()))
    idx = np.concatenate(out)
    assert np.all(idx >= 0)
    return np.sort(idx)


def vertex_interface_set(n, s, v):
    """Compact indices of the interface unknowns of the vertex space N_h^V (eq. vertex space).

    For the coarse vertex at fine node (s v0, s v1, s v2): the fine edges lying in
    the interiors of the coarse faces and on the coarse edges that contain the
    vertex.  For direction d they are the edges with cell index in
    [s v_d - s, s v_d + s - 1] whose transverse node pair (a, b) satisfies
    (a = s v_a and |b - s v_b| < s) or (b = s v_b and 0 < |a - s v_a| < s).
    For a vertex on the boundary of Omega the edges on the boundary or outside
    Omega are dropped (zero tangential trace).  An interior vertex has
    6 s + 24 s (s - 1) of them (60 for s = 2).
    """
    out = []
    for d in range(3):
        ea, eb = [ax for ax in range(3) if ax != d]
        cells = np.arange(s * v[d] - s, s * v[d] + s)
        pairs = []
        for db in range(-(s - 1), s):
            pairs.append((0, db))
        for da in range(-(s - 1), s):
            if da != 0:
                pairs.append((da, 0))
        for da, db in pairs:
            p = [None, None, None]
            p[d] = cells
            p[ea] = np.full(cells.shape, s * v[ea] + da)
            p[eb] = np.full(cells.shape, s * v[eb] + db)
            out.append(compact_index(n, d, *p))
    idx = np.concatenate(out)
    return np.sort(idx[idx >= 0])


def edge_interface_set(n, s, axis, c):
    """Compact indices of the interface unknowns of the edge space N_h^E (eq. edge space).

    Coarse edge along ``axis`` from fine node c = (c0, c1, c2) (multiples of s) to
    c + s e_axis: the fine edges on it and in the interiors of the 4 coarse faces
    sharing it.
    """
    out = []
    ea, eb = [ax for ax in range(3) if ax != axis]
    # edges parallel to the coarse edge
    cells = np.arange(c[axis], c[axis] + s)
    pairs = [(0, 0)]
    for t in range(1, s):
        pairs += [(t, 0), (-t, 0), (0, t), (0, -t)]
    for da, db in pairs:
        p = [None, None, None]
        p[axis] = cells
        p[ea] = np.full(cells.shape, c[ea] + da)
        p[eb] = np.full(cells.shape, c[eb] + db)
        out.append(compact_index(n, axis, *p))
    # edges transverse to it, in the 4 faces: direction ea in the face spanned by
    # (axis, ea) at node c[eb], and direction eb in the face (axis, eb) at node c[ea]
    for d, other in ((ea, eb), (eb, ea)):
        nodes_along = np.arange(c[axis] + 1, c[axis] + s)
        cells_d = np.arange(c[d] - s, c[d] + s)
        g_ax, g_d = np.meshgrid(nodes_along, cells_d, indexing="ij")
        p = [None, None, None]
        p[axis] = g_ax.ravel()
        p[d] = g_d.ravel()
        p[other] = np.full(g_ax.size, c[other])
        out.append(compact_index(n, d, *p))
    idx = np.concatenate(out)
    return np.sort(idx[idx >= 0])


def coarse_elements(n, s):
    m = n // s
    return [(a, b, c) for c in range(m) for b in range(m) for a in range(m)]


def coarse_vertices(n, s, boundary=True):
    """Coarse vertices that carry a vertex space.

    boundary=False: the interior vertices of T_H only (the set V_H as written in
    Sec. 3.2).  boundary=True: also the vertices on the boundary of Omega, each with
    its patch cut to Omega; this is the set that reproduces the contraction numbers
    of Table 2 for k >= 2.  Vertices whose interface set is empty (the 8 corners of
    the box) are skipped.
    """
    m = n // s
    if not boundary:
        return [(a, b, c) for c in range(1, m) for b in range(1, m) for a in range(1, m)]
    out = []
    for c in range(m + 1):
        for b in range(m + 1):
            for a in range(m + 1):
                if sum(x in (0, m) for x in (a, b, c)) < 3:
                    out.append((a, b, c))
    return out


def vertex_type(n, s, v):
    """0..26: per axis 0 (on the low face), 1 (inside), 2 (on the high face)."""
    m = n // s
    t = [0 if x == 0 else (2 if x == m else 1) for x in v]
    return t[0] + 3 * t[1] + 9 * t[2]


def patch_elements(n, s, v):
    """The coarse elements around vertex v that lie inside Omega."""
    m = n // s
    out = []
    for c in (1, 0):
        for b in (1, 0):
            for a in (1, 0):
                t = (v[0] - a, v[1] - b, v[2] - c)
                if all(0 <= x < m for x in t):
                    out.append(t)
    return out


def interior_coarse_vertices(n, s):
    return coarse_vertices(n, s, boundary=False)


def coarse_edges(n, s, boundary=True):
    """(axis, fine start node) of every coarse edge carrying an edge space.

    boundary=False: interior edges of T_H only; boundary=True: also coarse edges on
    the boundary of Omega whose interface set (cut to Omega) is non-empty.
    """
    m = n // s
    out = []
    for axis in range(3):
        ea, eb = [ax for ax in range(3) if ax != axis]
        lo, hi = (1, m) if not boundary else (0, m + 1)
        for c_ax in range(m):
            for cb in range(lo, hi):
                for ca in range(lo, hi):
                    if boundary and ca in (0, m) and cb in (0, m):
                        continue
                    c = [0, 0, 0]
                    c[axis] = s * c_ax
                    c[ea] = s * ca
                    c[eb] = s * cb
                    out.append((axis, tuple(c)))
    return out


def edge_patch_elements(n, s, axis, c):
    m = n // s
    ea, eb = [ax for ax in range(3) if ax != axis]
    out = []
    for db in (1, 0):
        for da in (1, 0):
            t = [0, 0, 0]
            t[axis] = c[axis] // s
            t[ea] = c[ea] // s - da
            t[eb] = c[eb] // s - db
            if all(0 <= x < m for x in t):
                out.append(tuple(t))
    return out


# ---------------------------------------------------------------------------
# Whole-level index arrays (the same sets as above, built for all subdomains or
# vertices at once; compact indices are affine in the edge coordinates within each
# direction block, so translating a set keeps its sorted order).
# ---------------------------------------------------------------------------

def _shifted(n, rel_d, rel_p, shifts):
    """Compact indices of the edges (rel_d, rel_p + shift) for every shift (rows)."""
    P = shifts[:, None, :] + rel_p[None, :, :]
    return compact_index(n, None, P[..., 0], P[..., 1], P[..., 2], d=rel_d[None, :])


def interior_sets(n, s):
    """[n_subdomains, 3 s (s-1)^2] array; row r is interior_set(n, s, coarse_elements()[r])."""
    elems = np.array(coarse_elements(n, s))
    ref = interior_set(n, s, (0, 0, 0))
    d, p = edge_coords(n)
    rel_d, rel_p = d[ref], p[ref]
    return _shifted(n, rel_d, rel_p, s * elems)


def vertex_interface_sets(n, s, verts):
    """[len(verts), |Gamma|] for vertices of one type; rows equal vertex_interface_set."""
    verts = np.asarray(verts)
    ref = vertex_interface_set(n, s, tuple(verts[0]))
    d, p = edge_coords(n)
    rel_d, rel_p = d[ref], p[ref] - s * verts[0][None, :]
    return _shifted(n, rel_d, rel_p, s * verts)
