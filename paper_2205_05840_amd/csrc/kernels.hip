// Device kernels of the ndmg library (gfx950).
//
// Operator (Sec. 2, eq. def bilinear form): A = alpha K + M on interior edges with
//   K = h C^T M_F C,  M = h^3 M_E,
// C the face circulation of edge values (right-hand rule), M_F the Raviart-Thomas face
// mass = tridiag(1/6, 2/3, 1/6) along each face normal, M_E = the tensor product of the
// same 1-D matrix across each edge direction.  For an edge of direction a with (b, c)
// the next two axes cyclically:
//   F_b(q) = u_a(q + e_c) - u_a(q) - u_c(q + e_a) + u_c(q)       (faces of normal b)
//   F_c(q) = u_b(q + e_a) - u_b(q) - u_a(q + e_b) + u_a(q)       (faces of normal c)
//   G_b = M_F F_b along b,  G_c = M_F F_c along c,
//   (C^T G)_a(p) = G_b(p - e_c) - G_b(p) - G_c(p - e_b) + G_c(p).
// All reads of an interior edge's stencil stay inside [0, n]^3 of the padded layout and
// boundary entries are zero, so no bounds checks are needed inside the stencil.
//
// Batching: see kernels.hpp.  Grids carry the pair index in blockIdx.x (node and
// subdomain grids, as pair * blocks_per_pair + block) or in blockIdx.y (1-D grids).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "kernels.hpp"
#include "reduce.hpp"
#include "tuning.hpp"

namespace ndmg {

namespace {

__device__ __forceinline__ int64_t lin(const DGeom& g, int i, int j, int k) {
  return (int64_t)k * g.plane + (int64_t)j * g.P + i;
}

__device__ __forceinline__ int64_t vlen(const DGeom& g) { return 3 * g.B; }

// Edge of direction d at (i, j, k) is an unknown: cell index along d in [0, n),
// node indices across in [1, n-1].
__device__ __forceinline__ bool is_unknown(const DGeom& g, int d, int i, int j, int k) {
  const int o[3] = {i, j, k};
  bool ok = true;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    if (ax == d) ok = ok && (o[ax] < g.n);
    else ok = ok && (o[ax] >= 1 && o[ax] <= g.n - 1);
  }
  return ok;
}

// Workgroups go to the 8 XCDs (each with its own L2) round-robin by linear index;
// renumbered with this bijection, each XCD takes a contiguous range of logical indices,
// so neighbouring tiles, which share halo data, meet in the same L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, i = b >> 3;
  return x * q + min(x, r) + i;
}

__device__ __forceinline__ bool inactive(const Bat& bt, int pair) {
  return bt.act != nullptr && bt.act[pair] == 0;
}

// This block's coordinates in the grid, renumbered so that consecutive blocks of the
// grid's x-y-z order run on one XCD (the hardware deals blocks to the 8 XCDs in turn, and
// each XCD has its own L2): neighbouring rows of a box, which read each other's halo,
// then share an L2.
__device__ __forceinline__ int3 xcd_grid_block() {
  const int gx = gridDim.x, gy = gridDim.y;
  const int lb = xcd_block(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
  return make_int3(lb % gx, (lb / gx) % gy, lb / (gx * gy));
}

// Position (a, b, c) of this thread in a w x w x w box of work items (subdomains, or
// nodes of the transfers), for block coordinates bk (xcd_grid_block; pair bk.x / nbx):
// blocks of 64 lanes along a row (grid (nbx * pairs, w, w)), or, packed (grid (nbx *
// pairs, w)), over consecutive positions of the (a, b) plane, so that rows shorter than a
// wave leave no lane idle.  False past the row (or plane).
__device__ __forceinline__ bool box_position(const int3& bk, int w, int nbx, int packed, int& a, int& b,
                                             int& c) {
  const int t = (bk.x % nbx) * blockDim.x + threadIdx.x;
  if (packed) {
    a = t % w;
    b = t / w;
    c = bk.y;
    return t < w * w;
  }
  a = t;
  b = bk.y;
  c = bk.z;
  return t < w;
}


template <typename T>
__device__ __forceinline__ T apply_at(const T* __restrict__ u, const DGeom& g, int a, int64_t p,
                                      T ah, T h3) {
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  const int64_t st[3] = {1, (int64_t)g.P, g.plane};
  const int64_t sa = st[a], sb = st[b], sc = st[c];
  const T* __restrict__ ua = u + a * g.B;
  const T* __restrict__ ub = u + b * g.B;
  const T* __restrict__ uc = u + c * g.B;
  const T t6 = T(1) / T(6), t23 = T(2) / T(3);
  auto Fb = [&](int64_t q) { return (ua[q + sc] - ua[q]) - (uc[q + sa] - uc[q]); };
  auto Fc = [&](int64_t q) { return (ub[q + sa] - ub[q]) - (ua[q + sb] - ua[q]); };
  auto Gb = [&](int64_t q) { return t6 * (Fb(q - sb) + Fb(q + sb)) + t23 * Fb(q); };
  auto Gc = [&](int64_t q) { return t6 * (Fc(q - sc) + Fc(q + sc)) + t23 * Fc(q); };
  const T curl = (Gb(p - sc) - Gb(p)) - (Gc(p - sb) - Gc(p));
  auto row = [&](int64_t q) { return t6 * (ua[q - sc] + ua[q + sc]) + t23 * ua[q]; };
  const T mass = t6 * (row(p - sb) + row(p + sb)) + t23 * row(p);
  return ah * curl + h3 * mass;
}

// With coefficient boxes, a box of factor 0 lies outside the domain (a non-box domain,
// Sec. 6): the edge of direction d at node o is an unknown only if its (up to four)
// cells, o[d] along d and o[b] - 1 .. o[b], o[c] - 1 .. o[c] across, all lie in boxes of
// positive factor.  The caller has checked is_unknown (so the cells are inside the cube).
__device__ __forceinline__ bool edge_in_domain(const double* __restrict__ coef, int r, int n, int d, const int o[3]) {
  const int b = (d + 1) % 3, c = (d + 2) % 3, w = n / r;
  bool in = true;
#pragma unroll
  for (int db = 0; db < 2; ++db)
#pragma unroll
    for (int dc = 0; dc < 2; ++dc) {
      int q[3];
      q[d] = o[d];
      q[b] = o[b] - 1 + db;
      q[c] = o[c] - 1 + dc;
      in = in && coef[((q[2] / w) * r + q[1] / w) * r + q[0] / w] > 0.0;
    }
  return in;
}

// The same with one alpha per cell (a coefficient with jumps, Sec. 6): the curl part sums
// alpha_T K_T over the four cells T around the edge, so each face term of the RT0 mass
// takes the alphas of the two cells on either side of the face.  ah = alpha h (alpha the
// common factor), coef[(bz r + by) r + bx] the factor of each box, w = n / r cells per box.
// a00 .. a11: the factors of the cells at index o[a] along the edge and o[b] - 1 + db,
// o[c] - 1 + dc across (a_{db dc}).
template <typename T>
__device__ __forceinline__ T apply_at_cells(const T* __restrict__ u, const DGeom& g, int a, int64_t p, T ah, T h3,
                                            T a00, T a10, T a01, T a11) {
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  const int64_t st[3] = {1, (int64_t)g.P, g.plane};
  const int64_t sa = st[a], sb = st[b], sc = st[c];
  const T* __restrict__ ua = u + a * g.B;
  const T* __restrict__ ub = u + b * g.B;
  const T* __restrict__ uc = u + c * g.B;
  const T t6 = T(1) / T(6), t3 = T(1) / T(3), t23 = T(2) / T(3);
  auto Fb = [&](int64_t q) { return (ua[q + sc] - ua[q]) - (uc[q + sa] - uc[q]); };
  auto Fc = [&](int64_t q) { return (ub[q + sa] - ub[q]) - (ua[q + sb] - ua[q]); };
  // face of normal b (c) at q between the cells of alpha am (below along b (c)) and ap
  auto Gb = [&](int64_t q, T am, T ap) { return t6 * (am * Fb(q - sb) + ap * Fb(q + sb)) + t3 * (am + ap) * Fb(q); };
  auto Gc = [&](int64_t q, T am, T ap) { return t6 * (am * Fc(q - sc) + ap * Fc(q + sc)) + t3 * (am + ap) * Fc(q); };
  const T curl = (Gb(p - sc, a00, a10) - Gb(p, a01, a11)) - (Gc(p - sb, a00, a01) - Gc(p, a10, a11));
  auto row = [&](int64_t q) { return t6 * (ua[q - sc] + ua[q + sc]) + t23 * ua[q]; };
  const T mass = t6 * (row(p - sb) + row(p + sb)) + t23 * row(p);
  return ah * curl + h3 * mass;
}

template <typename T>
__device__ __forceinline__ T apply_at_coef(const T* __restrict__ u, const DGeom& g, int a, int64_t p,
                                           const int o[3], T ah, T h3, const double* __restrict__ coef,
                                           int r) {
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  const int w = g.n / r;
  auto cell = [&](int db, int dc) {
    int q[3];
    q[a] = o[a];
    q[b] = o[b] - 1 + db;
    q[c] = o[c] - 1 + dc;
    return (T)coef[((q[2] / w) * r + q[1] / w) * r + q[0] / w];
  };
  return apply_at_cells(u, g, a, p, ah, h3, cell(0, 0), cell(1, 0), cell(0, 1), cell(1, 1));
}

// ---------------------------------------------------------------------------------
// operator apply / residual (one thread per node position, small levels)
// ---------------------------------------------------------------------------------
// y (or b - A x) at the three edges of node (i, j, k)
template <typename T, int MODE>
__device__ __forceinline__ void apply_node(const T* __restrict__ x, const T* __restrict__ b,
                                           T* __restrict__ y, const DGeom& g, T ah, T h3, int i, int j,
                                           int k) {
  const int64_t p = lin(g, i, j, k);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T v = T(0);
    if (is_unknown(g, d, i, j, k)) {
      const T ax = apply_at(x, g, d, p, ah, h3);
      v = (MODE == 1) ? b[d * g.B + p] - ax : ax;
    }
    y[d * g.B + p] = v;
  }
}

// The three edges of a node share the 8 cells around it (o - 1 and o on each axis): their
// factors are looked up once (6 divisions by the box width instead of 3 per cell and
// edge).  Cells outside the cube are clamped into it; they belong to no unknown's edge.
template <typename T, int MODE>
__device__ __forceinline__ void apply_node_coef(const T* __restrict__ x, const T* __restrict__ b,
                                                T* __restrict__ y, const DGeom& g, T ah, T h3,
                                                const double* __restrict__ coef, int r, int i, int j, int k) {
  const int64_t p = lin(g, i, j, k);
  const int o[3] = {i, j, k};
  const int w = g.n / r;
  int bq[3][2];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax)
#pragma unroll
    for (int s = 0; s < 2; ++s) bq[ax][s] = min(max(o[ax] - 1 + s, 0), g.n - 1) / w;
  double cf[2][2][2];
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) cf[dz][dy][dx] = coef[(bq[2][dz] * r + bq[1][dy]) * r + bq[0][dx]];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int bb = (d + 1) % 3, cc = (d + 2) % 3;
    // the cell at o[d] along the edge and o[bb] - 1 + db, o[cc] - 1 + dc across
    auto cell = [&](int db, int dc) {
      int s[3];
      s[d] = 1;
      s[bb] = db;
      s[cc] = dc;
      return cf[s[2]][s[1]][s[0]];
    };
    const double c00 = cell(0, 0), c10 = cell(1, 0), c01 = cell(0, 1), c11 = cell(1, 1);
    T v = T(0);
    if (is_unknown(g, d, i, j, k) && c00 > 0.0 && c10 > 0.0 && c01 > 0.0 && c11 > 0.0) {
      const T ax = apply_at_cells(x, g, d, p, ah, h3, (T)c00, (T)c10, (T)c01, (T)c11);
      v = (MODE == 1) ? b[d * g.B + p] - ax : ax;
    }
    y[d * g.B + p] = v;
  }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(64) k_apply(const T* __restrict__ x, const T* __restrict__ b,
                                              T* __restrict__ y, DGeom g, Bat bt, double h, int nbx) {
  const int3 bk = xcd_grid_block();
  const int pair = bk.x / nbx;
  const int i = (bk.x % nbx) * blockDim.x + threadIdx.x;
  const int j = bk.y, k = bk.z;
  if (i > g.n || inactive(bt, pair)) return;
  const int64_t off = (int64_t)pair * vlen(g);
  x += off;
  y += off;
  if (MODE == 1) b += off;
  const T ah = (T)(bt.alpha[pair / bt.nrhs] * h), h3 = (T)(h * h * h);
  if (bt.coef)
    apply_node_coef<T, MODE>(x, b, y, g, ah, h3, bt.coef, bt.coef_r, i, j, k);
  else
    apply_node<T, MODE>(x, b, y, g, ah, h3, i, j, k);
}

// The same for rows shorter than a wave (n + 1 < 64): the lanes of a block take
// consecutive positions of the (i, j) plane (row after row) instead of one row each, so
// that no lane idles past the row's end.  blockIdx.x = pair * nbp + block of the plane,
// blockIdx.y = k.
template <typename T, int MODE>
__global__ void __launch_bounds__(64) k_apply_plane(const T* __restrict__ x, const T* __restrict__ b,
                                                    T* __restrict__ y, DGeom g, Bat bt, double h, int nbp) {
  const int pair = blockIdx.x / nbp;
  const int t = (blockIdx.x % nbp) * blockDim.x + threadIdx.x;
  const int w = g.n + 1;
  if (t >= w * w || inactive(bt, pair)) return;
  const int i = t % w, j = t / w, k = blockIdx.y;
  const int64_t off = (int64_t)pair * vlen(g);
  x += off;
  y += off;
  if (MODE == 1) b += off;
  const T ah = (T)(bt.alpha[pair / bt.nrhs] * h), h3 = (T)(h * h * h);
  if (bt.coef)
    apply_node_coef<T, MODE>(x, b, y, g, ah, h3, bt.coef, bt.coef_r, i, j, k);
  else
    apply_node<T, MODE>(x, b, y, g, ah, h3, i, j, k);
}

// ---------------------------------------------------------------------------------
// grid transfers (Sec. 3.1): per direction P0 (x) P1 (x) P1
// ---------------------------------------------------------------------------------
// gc at the three edges of coarse node (I, J, K)
template <typename T>
__device__ __forceinline__ void restrict_node(const T* __restrict__ rf, T* __restrict__ gc, const DGeom& f,
                                              const DGeom& c, int I, int J, int K,
                                              const double* __restrict__ coef = nullptr, int coef_r = 0) {
  const int64_t stf[3] = {1, (int64_t)f.P, f.plane};
  const int64_t pc = lin(c, I, J, K);
  const int64_t pf = lin(f, 2 * I, 2 * J, 2 * K);
  const int oc[3] = {I, J, K};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T v = T(0);
    if (is_unknown(c, a, I, J, K) && (coef == nullptr || edge_in_domain(coef, coef_r, c.n, a, oc))) {
      const int b = (a + 1) % 3, cc = (a + 2) % 3;
      const T* __restrict__ r = rf + a * f.B + pf;
      T acc = T(0);
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int64_t q = e * stf[a];
        const T mid = T(0.5) * (r[q - stf[cc]] + r[q + stf[cc]]) + r[q];
        const T lo = T(0.5) * (r[q - stf[b] - stf[cc]] + r[q - stf[b] + stf[cc]]) + r[q - stf[b]];
        const T hi = T(0.5) * (r[q + stf[b] - stf[cc]] + r[q + stf[b] + stf[cc]]) + r[q + stf[b]];
        acc += T(0.5) * (lo + hi) + mid;
      }
      v = acc;
    }
    gc[a * c.B + pc] = v;
  }
}

template <typename T>
__global__ void __launch_bounds__(64) k_restrict(const T* __restrict__ rf, T* __restrict__ gc,
                                                 DGeom f, DGeom c, Bat bt, int nbx, int packed) {
  const int3 bk = xcd_grid_block();
  const int pair = bk.x / nbx;
  int I, J, K;
  if (!box_position(bk, c.n, nbx, packed, I, J, K) || inactive(bt, pair)) return;
  restrict_node(rf + (int64_t)pair * vlen(f), gc + (int64_t)pair * vlen(c), f, c, I, J, K, bt.coef, bt.coef_r);
}

// zf += I_{k-1}^k ec at the three edges of fine node (i, j, k)
// Inputs of the prolongation at one fine node: per direction the 4 coarse values that
// enter and the old fine value.
template <typename T>
struct ProlongIn {
  T e[3][4];
  T old[3];
};

// branch-free: across each axis the coarse neighbour enters with weight 1/2 at an odd
// fine index, else with weight 0 and stride 0 (so its load stays in bounds).  (i, j, k) is
// an inner node, so every coarse node read lies inside the coarse grid.
template <typename T>
__device__ __forceinline__ void prolong_load(const T* __restrict__ ec, const T* zf, const DGeom& f,
                                             const DGeom& c, int i, int j, int k, ProlongIn<T>& in) {
  const int o[3] = {i, j, k};
  const int64_t stc[3] = {1, (int64_t)c.P, c.plane};
  const int64_t pf = lin(f, i, j, k);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, cc = (a + 2) % 3;
    const T* __restrict__ e = ec + a * c.B + lin(c, o[0] >> 1, o[1] >> 1, o[2] >> 1);
    const int64_t sb = (o[b] & 1) ? stc[b] : 0, sc = (o[cc] & 1) ? stc[cc] : 0;
    in.e[a][0] = e[0];
    in.e[a][1] = e[sb];
    in.e[a][2] = e[sc];
    in.e[a][3] = e[sb + sc];
    in.old[a] = zf[a * f.B + pf];
  }
}

// zf += I_{k-1}^k ec at node (i, j, k) from its loaded inputs; off the unknowns the
// increment is 0
template <typename T>
__device__ __forceinline__ void prolong_store(T* zf, const DGeom& f, int i, int j, int k,
                                              const ProlongIn<T>& in) {
  const int o[3] = {i, j, k};
  const int64_t pf = lin(f, i, j, k);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const bool on = is_unknown(f, a, i, j, k);
    const bool ob = o[(a + 1) % 3] & 1, oc = o[(a + 2) % 3] & 1;
    // scaling by 1/2 is exact: the same roundings as 0.5 (x + y) and 0.25 ((.) + (.))
    const T wb0 = ob ? T(0.5) : T(1), wb1 = ob ? T(0.5) : T(0);
    const T wc0 = oc ? T(0.5) : T(1), wc1 = oc ? T(0.5) : T(0);
    const T rowlo = wb0 * in.e[a][0] + wb1 * in.e[a][1];
    const T rowhi = wb0 * in.e[a][2] + wb1 * in.e[a][3];
    const T v = wc0 * rowlo + wc1 * rowhi;
    zf[a * f.B + pf] = on ? in.old[a] + v : in.old[a];
  }
}

template <typename T>
__device__ __forceinline__ void prolong_node(const T* __restrict__ ec, T* __restrict__ zf, const DGeom& f,
                                             const DGeom& c, int i, int j, int k) {
  ProlongIn<T> in;
  prolong_load(ec, zf, f, c, i, j, k, in);
  prolong_store(zf, f, i, j, k, in);
}

// KP consecutive planes per lane (the grid's plane coordinate counts blocks of KP
// planes), every load before any store: a fine level has few nodes per lane otherwise,
// and its waves would wait on one round trip after another.  Planes past the level
// repeat the last one (which then stores the same values twice).
template <typename T, int KP>
__global__ void __launch_bounds__(64) k_prolong_add(const T* __restrict__ ec, T* __restrict__ zf,
                                                    DGeom f, DGeom c, Bat bt, int nbx, int packed) {
  const int3 bk = xcd_grid_block();
  const int pair = bk.x / nbx;
  int i, j, kb;
  if (!box_position(bk, f.n, nbx, packed, i, j, kb) || inactive(bt, pair)) return;
  ec += (int64_t)pair * vlen(c);
  zf += (int64_t)pair * vlen(f);
  ProlongIn<T> in[KP];
#pragma unroll
  for (int q = 0; q < KP; ++q) prolong_load(ec, zf, f, c, i, j, min(KP * kb + q, f.n - 1), in[q]);
#pragma unroll
  for (int q = 0; q < KP; ++q) prolong_store(zf, f, i, j, min(KP * kb + q, f.n - 1), in[q]);
}

// ---------------------------------------------------------------------------------
// vertex-based smoother (Sec. 3.2.2), s = 2
// ---------------------------------------------------------------------------------
// Interior unknowns of the subdomain with lower fine node (2a, 2b, 2c), in the order of
// interior_dofs(2): x-edges (0,1,1), (1,1,1); y-edges (1,0,1), (1,1,1);
// z-edges (1,1,0), (1,1,1).
__device__ __forceinline__ void interior_offsets_s2(const DGeom& g, int64_t base, int64_t off[6]) {
  const int64_t sx = 1, sy = g.P, sz = g.plane;
  off[0] = 0 * g.B + base + sy + sz;
  off[1] = 0 * g.B + base + sx + sy + sz;
  off[2] = 1 * g.B + base + sx + sz;
  off[3] = 1 * g.B + base + sx + sy + sz;
  off[4] = 2 * g.B + base + sx + sy;
  off[5] = 2 * g.B + base + sx + sy + sz;
}

// zi = A_T^{-1} r on the interior unknowns of subdomain (a, b, c)
template <typename T>
__device__ __forceinline__ void interior_sub_s2(const T* __restrict__ r, T* __restrict__ zi,
                                                const T* __restrict__ ATinv, const DGeom& g, int a, int b,
                                                int c) {
  int64_t off[6];
  interior_offsets_s2(g, lin(g, 2 * a, 2 * b, 2 * c), off);
  T rv[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) rv[q] = r[off[q]];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    T s = T(0);
#pragma unroll
    for (int t = 0; t < 6; ++t) s += ATinv[q * 6 + t] * rv[t];
    zi[off[q]] = s;
  }
}


// Word 3 of a buffer descriptor on gfx9-family devices: 32-bit data format, raw
// addressing (no index, no swizzle); accesses are range-checked against the descriptor's
// byte count, loads past it return zero and stores past it are dropped.
constexpr int kBufferFlags = 0x00020000;

// Operands of the 16x16x4 MFMAs: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16].
// Result register q of lane l holds D[row(l / 16, q)][l % 16], where (measured on
// gfx950) row = 4 q + l / 16 for the f64 instruction and 4 (l / 16) + q for f32.
template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int q) { return 4 * q + lk; }
};

template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int q) { return 4 * lk + q; }
};

// Vertex patch solves on MFMA.  A workgroup (4 waves) takes 4 * gpw groups of 16 vertices
// of one segment (one patch type) of one pair (blockIdx.y); the chunk gives gpw, wave 0's
// first vertex and the vertex steps between waves and between a wave's groups (groups
// consecutive per wave, or dealt out in turn among the waves of one XCD).  S_type^{-1} is
// staged in LDS; wave w then walks its gpw groups: lane l gathers the B-operand column values
// g[slot = 4 ks + l / 16] of vertex l % 16 straight from memory (the next group's gathers
// are in flight while the current group's products run), reads the A-operand fragments
// S^{-1}[16 mb + l % 16][4 ks + l / 16] from LDS and accumulates the 16 x 16 output tile
// per mb; results go to Y (layout at y_pos: a group's 16 vertices fill one aligned run
// of each row).
// - Slots are direction-major (NG / 3 per edge direction, a multiple of 4), so the edge
//   direction of k-step ks is fixed and its block offset d B is uniform; a lane adds a
//   32-bit offset to a per-group scalar base.
// - Which slots a patch lacks depends only on its type (a vertex inside the box has every
//   slot, one on a face of the box lacks the same slots wherever it lies on that face), so
//   each lane holds one bit mask of present slots for the whole block.
// - Lanes past the segment's end take the group's first vertex: they gather and compute
//   exactly what lane 0 does and store the same values to the same places.  So every load
//   and store is issued unconditionally; predicated memory operations would make the
//   compiler's wait counters conservative, and each product would then wait for the loads
//   and stores of the groups around it.
// - S^{-1} sits in LDS fragment-major: the A operands of one lane for VE consecutive
//   k-steps are one 16-byte word, and the 64 lanes read 64 consecutive words.
// - BUF (a pair's vector and its Y rows each below 2 GB): gathers and stores address
//   through buffer descriptors with 32-bit byte offsets per lane, one add per gather
//   instead of 64-bit address arithmetic and selects; an absent slot's offset is 2^31,
//   past the descriptor's range, and a load there returns zero.  The freed registers
//   give FP32 6 waves per SIMD instead of 4 (80 registers; measured 34.1 -> 30.0 us
//   at 128^3, FP64 50.6 -> 47.4 us, results bit for bit the same).
// FP64: at least 3 waves per SIMD (168 registers), the residency patch_groups assumes;
// FP32 without BUF fits 4 waves without the bound (asking for more makes it spill).
template <typename T, int S, bool BUF>
__global__ void __launch_bounds__(256, sizeof(T) == 4 ? (BUF ? 5 : 1) : 3)
    k_sm_patch(const T* __restrict__ gg, T* __restrict__ Y, const T* __restrict__ Sinv, DGeom g, DSub sub,
               Bat bt) {
  constexpr int NG = 6 * S * (4 * S - 3);
  constexpr int NPAD = (NG + 15) / 16 * 16;
  constexpr int NKS = NPAD / 4, NMB = NPAD / 16;
  constexpr int NKE = (NG + 3) / 4;                // k-steps that hold a slot
  constexpr int KD = NG / 12;                      // k-steps per edge direction
  static_assert(NG % 12 == 0, "slots of one direction fill whole k-steps");
  constexpr int VE = 16 / (int)sizeof(T);          // elements per 16-byte word
  constexpr int NL = NPAD * NPAD / VE / 256;       // 16-byte loads of S^{-1} per thread
  constexpr int NKV = NKS / VE;                    // A words per mb and lane
  constexpr int NKVE = (NKE + VE - 1) / VE;        // of which hold a slot
  static_assert(NPAD * NPAD % (VE * 256) == 0, "S^{-1} staging shape");
  typedef T vec_t __attribute__((ext_vector_type(VE)));
  // FP32 with 60 slots: S^{-1} row i of the last row block goes to the A operand's row
  // perm_row(i) (an involution swapping 51, 55, 59 with 60, 61, 62), so that the result
  // register 3 of that block holds the 4 padding rows in every lane
  constexpr bool kPerm = sizeof(T) == 4 && NG == 60 && NPAD == 64;
  auto perm_row = [](int i) {
    if (!kPerm || i < 48) return i;
    const int lk = (i - 48) >> 2, q = (i - 48) & 3;
    if (q == 3 && lk < 3) return 60 + lk;
    if (lk == 3 && q < 3) return 51 + 4 * q;
    return i;
  };
  __shared__ vec_t sA[NMB * NKV * 64];
  __shared__ int srel[NPAD];    // node offset of the slot's edge from the vertex's node
  __shared__ int spres[NPAD];   // 1 if this patch type has the slot
  const int lb = xcd_block(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
  const int pair = lb / gridDim.x;
  const int chunk = lb - pair * gridDim.x;
  const int cw = sub.chunks[4 * chunk];
  // a right-hand-side chunk runs in the workgroups of pairs whose index within their
  // problem is a multiple of 4; wave w then takes pair + w (same problem, same S^{-1})
  const bool rhsw = (cw & kChunkRhsWaves) != 0;
  if (rhsw ? (pair % bt.nrhs) % 4 != 0 : inactive(bt, pair)) return;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const bool wact = __builtin_amdgcn_readfirstlane(
      !rhsw || ((pair % bt.nrhs) + wave < bt.nrhs && !inactive(bt, pair + wave)));
  const int wpair = __builtin_amdgcn_readfirstlane(rhsw && wact ? pair + wave : pair);
  const int64_t NVY = y_row_len(sub.nH);
  gg += (int64_t)wpair * vlen(g);
  Y += (int64_t)wpair * NVY * NPAD;
  const int seg = cw & 0xffff;
  const int gpw = (cw >> 16) & 0x3fff;   // 16-vertex groups per wave in this chunk
  const int first = sub.chunks[4 * chunk + 1];
  const int wstep = sub.chunks[4 * chunk + 2];   // wave w's first group at first + w wstep
  const int cstep = sub.chunks[4 * chunk + 3];   // its group c at that + c cstep
  // segment parameters, read once: inside the loop the compiler could not keep them
  // across the stores to Y, and a reload would wait for every load and store in flight
  const int* sg = sub.segs + 8 * seg;
  const int type = __builtin_amdgcn_readfirstlane(sg[0]);
  const int lo0 = __builtin_amdgcn_readfirstlane(sg[1]);
  const int lo1 = __builtin_amdgcn_readfirstlane(sg[2]);
  const int lo2 = __builtin_amdgcn_readfirstlane(sg[3]);
  const int d0 = __builtin_amdgcn_readfirstlane(sg[4]);
  const int d1 = __builtin_amdgcn_readfirstlane(sg[5]);
  const int ybase = __builtin_amdgcn_readfirstlane(sg[6]);
  const int count = __builtin_amdgcn_readfirstlane(sg[7]);
  const T* __restrict__ Sm = Sinv + ((int64_t)(pair / bt.nrhs) * 27 + type) * NPAD * NPAD;
  for (int e = tid; e < NPAD; e += blockDim.x) {
    int rel = 0, pres = 0;
    if (e < NG) {
      const int* sl = sub.slots + 4 * e;
      const int d = sl[0], dx = sl[1], dy = sl[2], dz = sl[3];
      rel = (int)((int64_t)dz * g.plane + (int64_t)dy * g.P + dx);
      // the edge's node must satisfy 0 <= o <= n - 1 along its direction and
      // 1 <= o <= n - 1 across it; checked at the segment's first vertex
      const int ox = S * lo0 + dx, oy = S * lo1 + dy, oz = S * lo2 + dz, nmax = g.n - 1;
      pres = (ox >= (d != 0)) & (ox <= nmax) & (oy >= (d != 1)) & (oy <= nmax) & (oz >= (d != 2)) &
             (oz <= nmax);
    }
    srel[e] = rel;
    spres[e] = pres;
  }
  // S^{-1}: all of this thread's 16-byte loads go out together, before the first gathers
  vec_t sv[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) sv[l] = reinterpret_cast<const vec_t*>(Sm)[l * 256 + tid];
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  const int wfirst = first + wave * wstep;
  int rl[NKE];
  unsigned lmask = 0;
#pragma unroll
  for (int ks = 0; ks < NKE; ++ks) {
    rl[ks] = srel[4 * ks + lk];
    lmask |= (unsigned)spres[4 * ks + lk] << ks;
  }

  // BUF: byte offsets of this lane's slots from its vertex's node (direction block
  // included), 2^31 for an absent slot; byte offsets of result register q's row within a
  // 16-row block (sp: the permuted last block)
  typedef unsigned u2_t __attribute__((ext_vector_type(2)));
  const __amdgpu_buffer_rsrc_t rg = __builtin_amdgcn_make_buffer_rsrc(
      (void*)gg, (short)0, BUF ? (int)(vlen(g) * (int64_t)sizeof(T)) : 0, kBufferFlags);
  const __amdgpu_buffer_rsrc_t ry = __builtin_amdgcn_make_buffer_rsrc(
      (void*)Y, (short)0, BUF ? (int)(NVY * NPAD * (int64_t)sizeof(T)) : 0, kBufferFlags);
  unsigned ro[BUF ? NKE : 1], so[4], sp[4];
  if constexpr (BUF) {
#pragma unroll
    for (int ks = 0; ks < NKE; ++ks)
      ro[ks] = ((lmask >> ks) & 1u) ? (unsigned)((rl[ks] + (ks / KD) * (int)g.B) * (int)sizeof(T)) : 0x80000000u;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      so[q] = (unsigned)(Mfma<T>::row(lk, q) * NVY * (int64_t)sizeof(T));
      sp[q] = kPerm && lk == 3 ? (unsigned)((3 + 4 * q) * NVY * (int64_t)sizeof(T)) : so[q];
    }
  }
  // BUF: group c's gathers; yb = byte offset of the lane's vertex in a Y row
  auto gather_buf = [&](int c, T (&bcol)[NKS], unsigned& yb) {
    const int v0 = min(wfirst + cstep * c, count - 1);
    int v = wfirst + cstep * c + lr;
    if (v >= count) v = v0;
    const int vx = lo0 + v % d0, vy = lo1 + (v / d0) % d1, vz = lo2 + v / (d0 * d1);
    const unsigned u = (unsigned)(lin(g, S * vx, S * vy, S * vz) * (int64_t)sizeof(T));
    yb = (unsigned)(((int64_t)ybase + v) * (int64_t)sizeof(T));
#pragma unroll
    for (int ks = 0; ks < NKE; ++ks) {
      if constexpr (sizeof(T) == 4)
        bcol[ks] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rg, (int)(u + ro[ks]), 0, 0));
      else
        bcol[ks] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rg, (int)(u + ro[ks]), 0, 0));
    }
#pragma unroll
    for (int ks = NKE; ks < NKS; ++ks) bcol[ks] = T(0);
  };
  auto product_store_buf = [&](const T (&bcol)[NKS], unsigned yb) {
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb) {
      __asm__ volatile("" ::: "memory");
      vec_t a[NKVE];
#pragma unroll
      for (int kv = 0; kv < NKVE; ++kv) a[kv] = sA[(mb * NKV + kv) * 64 + lane];
      typename Mfma<T>::v4 acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int ks = 0; ks < NKE; ++ks) acc = Mfma<T>::mma(a[ks / VE][ks % VE], bcol[ks], acc);
      const unsigned mbo = (unsigned)(16 * mb * NVY * (int64_t)sizeof(T));
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (sizeof(T) == 8 && 16 * mb + 4 * q >= NG) continue;
        if (kPerm && mb == NMB - 1 && q == 3) continue;
        const unsigned off = yb + mbo + ((kPerm && mb == NMB - 1) ? sp[q] : so[q]);
        // the element is copied out first: a bit cast of acc[q] itself compiled to a
        // store of element 0 for every q
        const T val = acc[q];
        if constexpr (sizeof(T) == 4) {
          unsigned bits;
          __builtin_memcpy(&bits, &val, 4);
          __builtin_amdgcn_raw_buffer_store_b32(bits, ry, (int)off, 0, 0);
        } else {
          u2_t bits;
          __builtin_memcpy(&bits, &val, 8);
          __builtin_amdgcn_raw_buffer_store_b64(bits, ry, (int)off, 0, 0);
        }
      }
    }
  };
  // group c: lane's vertex (clamped), node offset from lane 0's node, Y row offsets
  auto gather = [&](int c, T (&bcol)[NKS], int64_t& y0, int& yoff) {
    const int v0 = min(wfirst + cstep * c, count - 1);
    int v = wfirst + cstep * c + lr;
    if (v >= count) v = v0;
    const int vx = lo0 + v % d0, vy = lo1 + (v / d0) % d1, vz = lo2 + v / (d0 * d1);
    const int64_t node = lin(g, S * vx, S * vy, S * vz);
    // lane 0 holds v0, the smallest vertex of the group: the offsets are >= 0
    const int64_t node0 = __builtin_amdgcn_readfirstlane((unsigned)(node & 0xffffffff)) |
                          ((int64_t)__builtin_amdgcn_readfirstlane((int)(node >> 32)) << 32);
    y0 = (int64_t)ybase + v0;
    const int loff = (int)(node - node0);
    yoff = v - v0;
#pragma unroll
    for (int ks = 0; ks < NKE; ++ks) {
      // absent slots read entry 0 (an x-edge on the boundary: zero), so that no select
      // waits for the loaded value
      const T* gb = gg + (int64_t)(ks / KD) * g.B + node0;
      const bool ok = (lmask >> ks) & 1u;
      bcol[ks] = *(ok ? gb + (loff + rl[ks]) : gg);
    }
#pragma unroll
    for (int ks = NKE; ks < NKS; ++ks) bcol[ks] = T(0);
  };
  auto product_store = [&](const T (&bcol)[NKS], int64_t y0, int yoff) {
    T* yl = Y + y0 + yoff;
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb) {
      // keep the A fragments in LDS (read per use) instead of registers: occupancy
      __asm__ volatile("" ::: "memory");
      vec_t a[NKVE];
#pragma unroll
      for (int kv = 0; kv < NKVE; ++kv) a[kv] = sA[(mb * NKV + kv) * 64 + lane];
      typename Mfma<T>::v4 acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int ks = 0; ks < NKE; ++ks) acc = Mfma<T>::mma(a[ks / VE][ks % VE], bcol[ks], acc);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // padding rows (>= NG) are never read, so a register that holds only such rows
        // is not stored.  FP64: register q holds rows 16 mb + 4 q .. + 3 in every lane.
        // FP32 (row 4 lk + q): the last block's rows are permuted (kPerm) so that its
        // register 3 holds the padding rows, and lanes lk = 3 store slots 51 + 4 q
        if (sizeof(T) == 8 && 16 * mb + 4 * q >= NG) continue;
        if (kPerm && mb == NMB - 1 && q == 3) continue;
        int row = 16 * mb + Mfma<T>::row(lk, q);
        if (kPerm && mb == NMB - 1 && lk == 3) row = 16 * mb + 3 + 4 * q;
        yl[(int64_t)row * NVY] = acc[q];
      }
    }
  };

  int ngroups = 0;
  for (int c = 0; c < gpw; ++c)
    if (wact && wfirst + cstep * c < count) ngroups = c + 1;
  T b0[NKS], b1[NKS];
  int64_t y0a = 0, y0b = 0;
  int yoa = 0, yob = 0;
  unsigned yba = 0, ybb = 0;
  // with no group, every lane takes the segment's last vertex
  if constexpr (BUF)
    gather_buf(0, b0, yba);
  else
    gather(0, b0, y0a, yoa);
#pragma unroll
  for (int l = 0; l < NL; ++l)
#pragma unroll
    for (int u = 0; u < VE; ++u) {
      const int e = (l * 256 + tid) * VE + u;
      const int r = perm_row(e / NPAD), col = e % NPAD;
      const int ks = col / 4, ln = (col % 4) * 16 + r % 16;
      sA[((r / 16) * NKV + ks / VE) * 64 + ln][ks % VE] = sv[l][u];
    }
  __syncthreads();
  if (ngroups == 0) return;   // no barrier below
  // two buffers used in turn, so that no buffer is copied (a copy would wait for the
  // loads in flight); past the last group the gathers repeat it
  int c = 0;
  if constexpr (BUF) {
    for (; c + 2 <= ngroups; c += 2) {
      gather_buf(c + 1, b1, ybb);
      product_store_buf(b0, yba);
      gather_buf(min(c + 2, ngroups - 1), b0, yba);
      product_store_buf(b1, ybb);
    }
    if (c < ngroups) product_store_buf(b0, yba);
  } else {
    for (; c + 2 <= ngroups; c += 2) {
      gather(c + 1, b1, y0b, yob);
      product_store(b0, y0a, yoa);
      gather(min(c + 2, ngroups - 1), b0, y0a, yoa);
      product_store(b1, y0b, yob);
    }
    if (c < ngroups) product_store(b0, y0a, yoa);
  }
  // the zero run that vertices without a patch read (row `lane`): the buffer is shared
  // with the small-level kernel's layout
  if (chunk == 0 && (rhsw || wave == 0)) {   // (a right-hand-side wave: its own pair)
#pragma unroll
    for (int row = lane; row < NPAD; row += 64) {
      T* yz = Y + (int64_t)row * NVY + y_zero_run(sub.nH);
#pragma unroll
      for (int i = 0; i < 16; ++i) yz[i] = T(0);
    }
  }
}

// w = sum_V R_V^T y_V on the interface unknowns of node (i, j, k), i < n; z (assign ? =,
// +=) eta w there.  Y is slot-major ([slot][vertex], NV vertices); slut the slot lookup.
template <typename T, int S>
__device__ __forceinline__ void pull_node(const T* __restrict__ Y, T* __restrict__ w, T* __restrict__ z,
                                          const DGeom& g, const int* slut, int nv, int64_t NV, T eta,
                                          int assign, int i, int j, int k) {
  constexpr int W = 2 * S + 1;
  const int o[3] = {i, j, k};
  const int64_t p = lin(g, i, j, k);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (!is_unknown(g, d, i, j, k)) continue;
    const int b = (d + 1) % 3, c = (d + 2) % 3;
    const int rb = o[b] % S, rc = o[c] % S;
    if (rb != 0 && rc != 0) continue;
    // candidate vertices: along d two, across as dictated by the residues
    int vb0, vb1, vc0, vc1;
    if (rb == 0) { vb0 = vb1 = o[b] / S; } else { vb0 = o[b] / S; vb1 = vb0 + 1; }
    if (rc == 0) { vc0 = vc1 = o[c] / S; } else { vc0 = o[c] / S; vc1 = vc0 + 1; }
    T acc = T(0);
    const int vd0 = o[d] / S;
#pragma unroll
    for (int ed = 0; ed < 2; ++ed)
      for (int vb = vb0; vb <= vb1; ++vb)
        for (int vc = vc0; vc <= vc1; ++vc) {
          int V[3];
          V[d] = vd0 + ed;
          V[b] = vb;
          V[c] = vc;
          const int dx = o[0] - S * V[0], dy = o[1] - S * V[1], dz = o[2] - S * V[2];
          const int slot = slut[((d * W + (dx + S)) * W + (dy + S)) * W + (dz + S)];
          const int64_t row = ((int64_t)V[2] * nv + V[1]) * nv + V[0];
          if (slot >= 0) acc += Y[(int64_t)slot * NV + row];
        }
    w[d * g.B + p] = acc;
    const T old = assign ? T(0) : z[d * g.B + p];
    z[d * g.B + p] = old + eta * acc;
  }
}


// Harmonic extension into subdomain interiors and the final interior update:
// z_I (assign ? =, +=) eta (zi_I - X_T w_dT), X_T = A_T^{-1} A_{I, dT} (6 x 48 for s = 2),
// w_dT the interface correction on the 48 edges of the subdomain's boundary (zero where
// they lie on the boundary of the domain).
// z_I of subdomain (a, b, c) (assign ? =, +=) eta (zi_I - X_T w_dT); sX = X_T (6 x 48),
// sofs the offsets of the 48 boundary edges from the subdomain's lower node
template <typename T>
__device__ __forceinline__ void extend_sub_s2(const T* __restrict__ w, const T* __restrict__ zi,
                                              T* __restrict__ z, const T* sX, const int64_t* sofs,
                                              const DGeom& g, T eta, int assign, int a, int b, int c) {
  const int64_t base = lin(g, 2 * a, 2 * b, 2 * c);
  T wv[48];
#pragma unroll
  for (int e = 0; e < 48; ++e) wv[e] = w[base + sofs[e]];
  // interior unknown t: direction d = t / 2 at offset 1 across d and (t & 1) along d
  // (the order of interior_offsets_s2)
  const int64_t st[3] = {1, (int64_t)g.P, g.plane};
  const int64_t all1 = st[0] + st[1] + st[2];
#pragma unroll 1
  for (int t = 0; t < 6; ++t) {
    const int d = t >> 1;
    const int64_t off = d * g.B + base + all1 - (1 - (t & 1)) * (d == 0 ? st[0] : (d == 1 ? st[1] : st[2]));
    T q = T(0);
#pragma unroll
    for (int e = 0; e < 48; ++e) q += sX[t * 48 + e] * wv[e];
    const T old = assign ? T(0) : z[off];
    z[off] = old + eta * (zi[off] - q);
  }
}


// ---------------------------------------------------------------------------------
// coarsest level: dense inverse (one workgroup per pair)
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_coarse(const T* __restrict__ g, T* __restrict__ z,
                                                const T* __restrict__ A0inv,
                                                const int64_t* __restrict__ map, int N0, int64_t len,
                                                Bat bt) {
  __shared__ T gl[1024];
  const int pair = blockIdx.x;
  if (inactive(bt, pair)) return;
  g += (int64_t)pair * len;
  z += (int64_t)pair * len;
  A0inv += (int64_t)(pair / bt.nrhs) * N0 * N0;
  for (int i = threadIdx.x; i < N0; i += blockDim.x) gl[i] = g[map[i]];
  __syncthreads();
  for (int i = threadIdx.x; i < N0; i += blockDim.x) {
    T s = T(0);
    for (int j = 0; j < N0; ++j) s += A0inv[(int64_t)i * N0 + j] * gl[j];
    z[map[i]] = s;
  }
}

// Patches holding each boundary edge of a 2 x 2 x 2 subdomain, computed at compile time
// by the rules of the host tables (vertex_slots, boundary_dofs, boundary_patch_table),
// which setup compares against them: the boundary edges in order (direction, then z, y,
// x offsets from the lower node, x fastest); per edge the corners cx + 2 cy + 4 cz and
// patch slots of its 2 or 4 candidate vertices (two along the edge; across each
// transverse axis the one the edge lies on, or both where the offset is odd).
struct BoundaryPatches {
  int n = 0;
  int d[48] = {}, o[48][3] = {}, ncand[48] = {}, corner[48][4] = {}, slot[48][4] = {};
  bool owned[48] = {};
};

constexpr int vertex_slot_index(int d, int dx, int dy, int dz) {
  int idx = 0;
  for (int dd = 0; dd < 3; ++dd)
    for (int z = -2; z <= 2; ++z)
      for (int y = -2; y <= 2; ++y)
        for (int x = -2; x <= 2; ++x) {
          const int o[3] = {x, y, z};
          if (o[dd] < -2 || o[dd] > 1) continue;
          const int a = (dd + 1) % 3, b = (dd + 2) % 3;
          const int oa = o[a], ob = o[b];
          const bool ok = (oa == 0 && ob > -2 && ob < 2) || (ob == 0 && oa != 0 && oa > -2 && oa < 2);
          if (!ok) continue;
          if (dd == d && x == dx && y == dy && z == dz) return idx;
          ++idx;
        }
  return -1;
}

constexpr BoundaryPatches make_boundary_patches() {
  BoundaryPatches t;
  for (int d = 0; d < 3; ++d)
    for (int z = 0; z <= 2; ++z)
      for (int y = 0; y <= 2; ++y)
        for (int x = 0; x <= 2; ++x) {
          const int o[3] = {x, y, z};
          bool edge = true, interior = true;
          for (int ax = 0; ax < 3; ++ax) {
            if (ax == d) edge = edge && (o[ax] >= 0 && o[ax] < 2);
            else interior = interior && (o[ax] == 1);
          }
          if (!edge || interior) continue;
          const int e = t.n++;
          t.d[e] = d;
          t.o[e][0] = x; t.o[e][1] = y; t.o[e][2] = z;
          t.owned[e] = (x <= 1 && y <= 1 && z <= 1);
          int nc = 0;
          for (int cz = 0; cz < 2; ++cz)
            for (int cy = 0; cy < 2; ++cy)
              for (int cx = 0; cx < 2; ++cx) {
                const int c[3] = {cx, cy, cz};
                bool cand = true;
                for (int ax = 0; ax < 3; ++ax)
                  if (ax != d && o[ax] % 2 == 0 && c[ax] != o[ax] / 2) cand = false;
                if (!cand) continue;
                const int sl = vertex_slot_index(d, x - 2 * cx, y - 2 * cy, z - 2 * cz);
                if (sl < 0 || nc >= 4) continue;
                t.corner[e][nc] = cx + 2 * cy + 4 * cz;
                t.slot[e][nc] = sl;
                ++nc;
              }
          t.ncand[e] = nc;
        }
  return t;
}

constexpr BoundaryPatches kBP = make_boundary_patches();
static_assert(kBP.n == 48, "48 boundary edges of a 2 x 2 x 2 subdomain");

// The interface unknowns a subdomain owns (offsets in {0, 1} from its lower node, not
// interior), with the subdomains whose boundary holds each: T + q for q in {-1, 0}^3
// (step -1 across each transverse axis where the offset is 0, i.e. the edge lies on that
// face plane), and the edge's index among the boundary edges of T + q.
struct OwnedInterface {
  int n = 0;
  int d[18] = {}, o[18][3] = {}, nadj[18] = {}, q[18][4] = {}, e[18][4] = {};
};
constexpr OwnedInterface make_owned_interface() {
  OwnedInterface t;
  for (int e = 0; e < kBP.n; ++e) {
    if (!kBP.owned[e]) continue;
    const int k = t.n++;
    const int d = kBP.d[e];
    t.d[k] = d;
    for (int ax = 0; ax < 3; ++ax) t.o[k][ax] = kBP.o[e][ax];
    const int b = (d + 1) % 3, c = (d + 2) % 3;
    int na = 0;
    for (int sb = 0; sb < 2; ++sb)
      for (int sc = 0; sc < 2; ++sc) {
        if ((sb && kBP.o[e][b] != 0) || (sc && kBP.o[e][c] != 0)) continue;
        int qv[3] = {0, 0, 0};
        qv[b] = -sb;
        qv[c] = -sc;
        // offsets of the edge from the lower node of T + q
        const int l[3] = {kBP.o[e][0] - 2 * qv[0], kBP.o[e][1] - 2 * qv[1], kBP.o[e][2] - 2 * qv[2]};
        int idx = -1;
        for (int f = 0; f < kBP.n; ++f)
          if (kBP.d[f] == d && kBP.o[f][0] == l[0] && kBP.o[f][1] == l[1] && kBP.o[f][2] == l[2]) idx = f;
        t.q[k][na] = (-qv[0]) + 2 * (-qv[1]) + 4 * (-qv[2]);
        t.e[k][na] = idx;
        ++na;
      }
    t.nadj[k] = na;
  }
  return t;
}
constexpr OwnedInterface kOI = make_owned_interface();
static_assert(kOI.n == 18, "18 interface unknowns owned per subdomain");

// Condensed interface residual g_G = r_G - (A z_I)_G with z_I = A_T^{-1} r_I on every
// subdomain: the interior unknowns of T couple only to edges of T, so (A z_I)_e is the
// sum over the subdomains T whose boundary holds e of (X_T^T r_I(T))_e, X_T^T =
// A_{dT,I} A_T^{-1} (A_T symmetric).  One thread per subdomain T writes g on the 18
// interface unknowns T owns, from r there and the interior residuals of T and its
// neighbours T - e_x, T - e_y, T - e_z and their pairwise sums (all tables compile-time).
// Other entries of g are left untouched (never read).
// Copy n (<= 64 * R) values from global memory into LDS with one batch of loads per
// thread (a loop that stores each value before loading the next waits for every load).
template <typename T, int R>
__device__ __forceinline__ void stage_load(T (&v)[R], const T* __restrict__ src, int n) {
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = src[min((int)threadIdx.x + 64 * i, n - 1)];
}
template <typename T, int R>
__device__ __forceinline__ void stage_store(T* __restrict__ dst, const T (&v)[R], int n) {
#pragma unroll
  for (int i = 0; i < R; ++i)
    if ((int)threadIdx.x + 64 * i < n) dst[threadIdx.x + 64 * i] = v[i];
}
template <typename T, int R>
__device__ __forceinline__ void stage_lds(T* __restrict__ dst, const T* __restrict__ src, int n) {
  T v[R];
  stage_load(v, src, n);
  stage_store(dst, v, n);
}

// BUF (the pair's vector below 2 GB): the residual loads go through a buffer descriptor,
// a per-lane byte offset of the subdomain's node plus a uniform offset per slot, with no
// 64-bit address arithmetic (FP64 measured 58.5 -> 53.8 us for condensation and
// pull/extend at 128^3, FP32 unchanged; results bit for bit the same).
template <typename T, bool BUF>
__global__ void __launch_bounds__(64) k_sm_condense(const T* __restrict__ r, T* __restrict__ gg,
                                                    const T* __restrict__ XT, DGeom g, int nH, Bat bt, int nbx,
                                                    int packed) {
  constexpr int NB = 48;
  __shared__ T sX[6 * NB];
  const int3 bk = xcd_grid_block();
  const int pair = bk.x / nbx;
  if (inactive(bt, pair)) return;
  XT += (int64_t)(pair / bt.nrhs) * 6 * NB;
  // X_T's loads first, then this thread's residual loads, then X_T into LDS and the
  // barrier: the residual loads are in flight across the staging (lanes past the box
  // load subdomain 0's values and return after the barrier)
  constexpr int RX = (6 * NB + 63) / 64;
  T xv[RX];
  stage_load(xv, XT, 6 * NB);
  int a, b, c;
  const bool valid = box_position(bk, nH, nbx, packed, a, b, c);
  if (!valid) a = b = c = 0;
  const int64_t voff = (int64_t)pair * vlen(g);
  r += voff;
  gg += voff;
  // interior residuals of T - q (q = bits x, y, z; not all three: never needed), from a
  // clamped subdomain where T - q leaves the domain (those values are never used)
  T rI[8][6];
  const int64_t base = lin(g, 2 * a, 2 * b, 2 * c);
  // every owned slot is read and written (its node lies inside the grid); a slot on the
  // domain boundary gets 0, which keeps the zero there.  No branch around a load or
  // store: predicated memory operations make the compiler's wait counters conservative.
  T rO[18];
  if constexpr (BUF) {
    const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(
        (void*)r, (short)0, (int)(vlen(g) * (int64_t)sizeof(T)), kBufferFlags);
    auto ld = [&](unsigned voff, int soff) -> T {
      if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rr, (int)voff, soff, 0));
      else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rr, (int)voff, soff, 0));
    };
    // byte offsets of the interior unknowns from a subdomain's lower node (the order of
    // interior_offsets_s2), uniform
    const int es = (int)sizeof(T);
    const int io[6] = {(int)((g.P + g.plane) * es),         (int)((1 + g.P + g.plane) * es),
                       (int)((g.B + 1 + g.plane) * es),     (int)((g.B + 1 + g.P + g.plane) * es),
                       (int)((2 * g.B + 1 + g.P) * es),     (int)((2 * g.B + 1 + g.P + g.plane) * es)};
#pragma unroll
    for (int qq = 0; qq < 7; ++qq) {
      const int sa = max(a - (qq & 1), 0), sb = max(b - ((qq >> 1) & 1), 0), sc = max(c - (qq >> 2), 0);
      const unsigned vb = (unsigned)(lin(g, 2 * sa, 2 * sb, 2 * sc) * es);
#pragma unroll
      for (int t = 0; t < 6; ++t) rI[qq][t] = ld(vb, io[t]);
    }
    const unsigned vb = (unsigned)(base * es);
#pragma unroll
    for (int k = 0; k < 18; ++k)
      rO[k] = ld(vb, (int)((kOI.d[k] * g.B + lin(g, kOI.o[k][0], kOI.o[k][1], kOI.o[k][2])) * es));
  } else {
#pragma unroll
    for (int qq = 0; qq < 7; ++qq) {
      const int sa = max(a - (qq & 1), 0), sb = max(b - ((qq >> 1) & 1), 0), sc = max(c - (qq >> 2), 0);
      int64_t off[6];
      interior_offsets_s2(g, lin(g, 2 * sa, 2 * sb, 2 * sc), off);
#pragma unroll
      for (int t = 0; t < 6; ++t) rI[qq][t] = r[off[t]];
    }
#pragma unroll
    for (int k = 0; k < 18; ++k)
      rO[k] = r[kOI.d[k] * g.B + base + lin(g, kOI.o[k][0], kOI.o[k][1], kOI.o[k][2])];
  }
  stage_store(sX, xv, 6 * NB);
  __syncthreads();
  if (!valid) return;
#pragma unroll
  for (int k = 0; k < 18; ++k) {
    const int d = kOI.d[k];
    const int gi = 2 * a + kOI.o[k][0], gj = 2 * b + kOI.o[k][1], gk = 2 * c + kOI.o[k][2];
    const int64_t off = d * g.B + base + lin(g, kOI.o[k][0], kOI.o[k][1], kOI.o[k][2]);
    T acc = rO[k];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      if (m < kOI.nadj[k]) {
        const int qq = kOI.q[k][m], e = kOI.e[k][m];
#pragma unroll
        for (int t = 0; t < 6; ++t) acc -= sX[t * NB + e] * rI[qq][t];
      }
    }
    gg[off] = is_unknown(g, d, gi, gj, gk) ? acc : T(0);
  }
}

// Interface sum and harmonic extension in one pass, one thread per subdomain T: every
// edge on the boundary of T lies in the patches of corners of T only, so the thread
// forms w on its 48 boundary edges straight from the patch results of its 8 corners
// (as the interface sum takes them, kBP), then z_I (assign ? =, +=) eta (zi_I -
// X_T w_dT) on its 6 interior unknowns and z (assign ? =, +=) eta w on the interface
// unknowns it owns (offsets in {0, 1} from its lower node): every unknown of the level
// is written exactly once and w never goes to memory.  Edges on the domain boundary sum
// to zero (their slots are absent from every patch that lists them).  All table lookups
// are compile-time constants, so the 160 loads of a thread go out together.
template <typename T>
__global__ void __launch_bounds__(64) k_sm_pull_extend(const T* __restrict__ Y, const T* __restrict__ r,
                                                       T* __restrict__ z, const T* __restrict__ XT,
                                                       const T* __restrict__ ATinv, DGeom g, DSub sub, T eta,
                                                       int assign, Bat bt, int nbx, int packed) {
  constexpr int NB = 48, NPAD = 64;
  constexpr bool kInPlace = sizeof(T) == 4;
  __shared__ T lX[kInPlace ? 1 : 6 * NB];
  __shared__ T lA[kInPlace ? 1 : 36];
  const int3 bk = xcd_grid_block();
  const int pair = bk.x / nbx;
  if (inactive(bt, pair)) return;
  // FP32: X_T and A_T^{-1} are read in place (uniform, constant indices: scalar loads that
  // overlap the vector loads; no barrier in front of the patch-result loads).  FP64:
  // staged in LDS (read in place, the compiler keeps too many of them in registers).
  // (k_sm_condense stages them: its products interleave with the loads, and scalar
  // loads on demand there measured slower.)
  const T* __restrict__ gX = XT + (int64_t)(pair / bt.nrhs) * 6 * NB;
  const T* __restrict__ gA = ATinv + (int64_t)(pair / bt.nrhs) * 36;
  if constexpr (!kInPlace) {
    stage_lds<T, (6 * NB + 63) / 64>(lX, gX, 6 * NB);
    stage_lds<T, 1>(lA, gA, 36);
    __syncthreads();
  }
  auto sX = [&](int i) -> T {
    if constexpr (kInPlace) return gX[i];
    else return lX[i];
  };
  auto sA = [&](int i) -> T {
    if constexpr (kInPlace) return gA[i];
    else return lA[i];
  };
  const int nH = sub.nH;
  int a, b, c;
  if (!box_position(bk, nH, nbx, packed, a, b, c)) return;
  const int64_t NVY = y_row_len(nH);
  const int64_t voff = (int64_t)pair * vlen(g);
  r += voff;
  z += voff;
  // Y rows as a uniform base per slot plus a 32-bit byte offset per corner (corner
  // i + 2 j + 4 k at vertex (a + i, b + j, c + k)): 8 offset registers serve every load
  const char* __restrict__ Yb = reinterpret_cast<const char*>(Y + (int64_t)pair * NVY * NPAD);
  const int64_t rowb = NVY * (int64_t)sizeof(T);
  unsigned cb[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int x = a + (q & 1), y = b + ((q >> 1) & 1), zc = c + (q >> 2);
    cb[q] = (unsigned)y_pos(nH, sub.bpatch, x, y, zc) * (unsigned)sizeof(T);
  }
  const int64_t base = lin(g, 2 * a, 2 * b, 2 * c);
  int64_t ioff[6];
  interior_offsets_s2(g, base, ioff);
  // the old values of z (accumulating form) and r_I first: issued before the patch
  // results, they are in hand when those are, and no store waits for a load
  T zo[6 + NB], rI[6];
#pragma unroll
  for (int t = 0; t < 6 + NB; ++t) zo[t] = T(0);
  if (!assign) {
#pragma unroll
    for (int t = 0; t < 6; ++t) zo[t] = z[ioff[t]];
#pragma unroll
    for (int e = 0; e < NB; ++e)
      if (kBP.owned[e]) zo[6 + e] = z[kBP.d[e] * g.B + base + lin(g, kBP.o[e][0], kBP.o[e][1], kBP.o[e][2])];
  }
#pragma unroll
  for (int t = 0; t < 6; ++t) rI[t] = r[ioff[t]];
  T wv[NB];
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    T acc = T(0);
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (t < kBP.ncand[e])
        acc += *reinterpret_cast<const T*>(Yb + kBP.slot[e][t] * rowb + cb[kBP.corner[e][t]]);
    wv[e] = acc;
  }
  // interior unknowns (the order of interior_offsets_s2): z_I += eta (A_T^{-1} r_I - X_T w)
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    T q = T(0);
#pragma unroll
    for (int e = 0; e < NB; ++e) q += sX(t * NB + e) * wv[e];
    T zi = T(0);
#pragma unroll
    for (int s2 = 0; s2 < 6; ++s2) zi += sA(t * 6 + s2) * rI[s2];
    z[ioff[t]] = zo[t] + eta * (zi - q);
  }
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    if (kBP.owned[e]) {
      const int64_t off = kBP.d[e] * g.B + base + lin(g, kBP.o[e][0], kBP.o[e][1], kBP.o[e][2]);
      z[off] = zo[6 + e] + eta * wv[e];
    }
  }
}

// ---------------------------------------------------------------------------------
// the V-cycle from one level down as a dense matrix per problem
// ---------------------------------------------------------------------------------
// With z_0 = 0, MG(k, g, 0, m) (Fig. 1) is a linear map of g; its matrix over the
// unknowns of level k is built column by column from unit vectors by the recursive
// V-cycle itself and then applied instead of the recursion.

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// pair p (problem p / K, column col = j0 + p % K): g = e_col (zero when col >= N)
template <typename T>
__global__ void k_unit_cols(T* __restrict__ g, const int64_t* __restrict__ map, int N, int j0,
                            int64_t len, Bat bt) {
  const int pair = blockIdx.y;
  const int col = j0 + pair % bt.nrhs;
  const int64_t t = (col < N) ? map[col] : -1;
  g += (int64_t)pair * len;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x)
    g[e] = (e == t) ? T(1) : T(0);
}

// column col of the matrix of problem p / K: Bm[i][col] = z[map[i]] (row-major), or
// stored transposed, Bm[col][i] (colmajor)
template <typename T>
__global__ void k_gather_cols(const T* __restrict__ z, T* __restrict__ Bm, const int64_t* __restrict__ map,
                              int N, int j0, int64_t len, int colmajor, Bat bt) {
  const int pair = blockIdx.y;
  const int col = j0 + pair % bt.nrhs;
  if (col >= N) return;
  z += (int64_t)pair * len;
  Bm += (int64_t)(pair / bt.nrhs) * N * N;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    const int64_t at = colmajor ? (int64_t)col * N + i : (int64_t)i * N + col;
    Bm[at] = z[map[i]];
  }
}

// z = Bm g with the matrix stored transposed (Bt[j][i] = Bm[i][j]), for classes of many
// problems: block (x, problem), one row i per thread; the right-hand sides, RC at a time,
// are gathered into LDS and each thread runs over j with coalesced loads of Bt[j][.]
// (no cross-lane sums).  Non-unknown entries of z are not written.
template <typename T, int RC>
__global__ void __launch_bounds__(256) k_dense_vcycle_t(const T* __restrict__ g, T* __restrict__ z,
                                                        const T* __restrict__ Bt,
                                                        const int64_t* __restrict__ map, int N, int64_t len,
                                                        Bat bt) {
  extern __shared__ __align__(16) unsigned char dense_smem[];
  T* sg = reinterpret_cast<T*>(dense_smem);
  const int prob = blockIdx.y;
  const int nr = bt.nrhs;
  const T* __restrict__ Bp = Bt + (int64_t)prob * N * N;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ic = i < N ? i : 0;
  for (int rc = 0; rc < nr; rc += RC) {
    const int nrc = min(RC, nr - rc);
    bool live[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) live[r] = r < nrc && !inactive(bt, prob * nr + rc + r);
    __syncthreads();   // the previous chunk is done with sg
    for (int e = threadIdx.x; e < RC * N; e += blockDim.x) {
      const int r = e / N, j = e - r * N;
      sg[e] = live[r] ? g[(int64_t)(prob * nr + rc + r) * len + map[j]] : T(0);
    }
    __syncthreads();
    T acc[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) acc[r] = T(0);
    int j = 0;
    for (; j + 8 <= N; j += 8) {
      T b[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) b[u] = Bp[(int64_t)(j + u) * N + ic];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int r = 0; r < RC; ++r) acc[r] += b[u] * sg[r * N + j + u];
    }
    for (; j < N; ++j) {
      const T b = Bp[(int64_t)j * N + ic];
#pragma unroll
      for (int r = 0; r < RC; ++r) acc[r] += b * sg[r * N + j];
    }
    if (i < N) {
      const int64_t zi = map[i];
#pragma unroll
      for (int r = 0; r < RC; ++r)
        if (live[r]) z[(int64_t)(prob * nr + rc + r) * len + zi] = acc[r];
    }
  }
}

// z[map[i]] = sum_j Bm[i][j] g[map[j]] for every pair of a problem.  Block (x, problem):
// the problem's right-hand sides, RC at a time, are gathered into LDS; wave w takes rows
// (4 x + w) rpw .. + rpw - 1, lane l holds the entries j = l + 64 jj of a row (all its
// loads issued at once; the first row's before the gather) and the row sums are wave
// reductions, so each row of Bm is read once per RC right-hand sides.  Non-unknown
// entries of z are not written (zero by the layout contract).
template <typename T, int RC>
__global__ void __launch_bounds__(256) k_dense_vcycle(const T* __restrict__ g, T* __restrict__ z,
                                                      const T* __restrict__ Bm,
                                                      const int64_t* __restrict__ map, int N, int64_t len,
                                                      int rpw, Bat bt) {
  extern __shared__ __align__(16) unsigned char dense_smem[];
  T* sg = reinterpret_cast<T*>(dense_smem);
  constexpr int NJ = (kDenseMaxN + 63) / 64;           // row entries per lane
  constexpr int kPer = (RC * kDenseMaxN + 255) / 256;   // gathered values per thread
  const int prob = blockIdx.y;
  const int nr = bt.nrhs;
  const T* __restrict__ Bp = Bm + (int64_t)prob * N * N;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row0 = (blockIdx.x * 4 + wave) * rpw;
  // entries of row i (rows past N and entries past N read entry 0 and are masked)
  auto load_row = [&](int i, T (&bv)[NJ]) {
    const T* __restrict__ Brow = Bp + (int64_t)(i < N ? i : 0) * N;
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      const int j = lane + 64 * jj;
      bv[jj] = Brow[j < N ? j : 0];
    }
  };
  auto row_sums = [&](const T (&bv)[NJ], T (&acc)[RC]) {
#pragma unroll
    for (int r = 0; r < RC; ++r) acc[r] = T(0);
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      const int j = lane + 64 * jj;
      if (j < N) {
#pragma unroll
        for (int r = 0; r < RC; ++r) acc[r] += bv[jj] * sg[r * N + j];
      }
    }
  };
  for (int rc = 0; rc < nr; rc += RC) {
    const int nrc = min(RC, nr - rc);
    bool live[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) live[r] = r < nrc && !inactive(bt, prob * nr + rc + r);
    T bcur[NJ];
    load_row(row0, bcur);
    // offsets first, then values: each phase's loads are independent and go out together
    int64_t src[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int e = threadIdx.x + 256 * t;
      src[t] = -1;
      if (e < RC * N) {
        const int r = e / N, j = e - r * N;
        if (live[r]) src[t] = (int64_t)(prob * nr + rc + r) * len + map[j];
      }
    }
    T val[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) val[t] = (src[t] >= 0) ? g[src[t]] : T(0);
    __syncthreads();   // the previous chunk's rows are done with sg
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int e = threadIdx.x + 256 * t;
      if (e < RC * N) sg[e] = val[t];
    }
    __syncthreads();
    for (int ii = 0; ii < rpw; ++ii) {
      const int i = row0 + ii;
      if (i >= N) break;
      T bnext[NJ];
      if (ii + 1 < rpw) load_row(i + 1, bnext);
      T acc[RC];
      row_sums(bcur, acc);
      T mine = T(0);
#pragma unroll
      for (int r = 0; r < RC; ++r) {
        const T v = wave_sum(acc[r]);
        if (lane == r) mine = v;
      }
      bool w = false;
#pragma unroll
      for (int r = 0; r < RC; ++r) w = w || (lane == r && live[r]);
      if (w) z[(int64_t)(prob * nr + rc + lane) * len + map[i]] = mine;
#pragma unroll
      for (int jj = 0; jj < NJ; ++jj) bcur[jj] = bnext[jj];
    }
  }
}

template <typename T>
__global__ void k_fill_zero(T* __restrict__ y, int64_t len, Bat bt) {
  const int pair = blockIdx.y;
  if (inactive(bt, pair)) return;
  y += (int64_t)pair * len;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x)
    y[e] = T(0);
}

// ---------------------------------------------------------------------------------
// the bottom of the V-cycle in one workgroup per pair
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(512) k_vcycle_small(SmallArgs<T> a, Bat bt) {
  constexpr int NG = 60, NPAD = 64;
  __shared__ int sslot[NPAD][4];
  __shared__ int64_t soff[NPAD];
  __shared__ int slut[3 * 125];
  __shared__ T sX[6 * 48];
  __shared__ int64_t sofs[48];
  __shared__ T sg0[1024];
  const int pair = blockIdx.x;
  if (inactive(bt, pair)) return;
  const int prob = pair / bt.nrhs;
  const int tid = threadIdx.x, nth = blockDim.x;
  const T alpha = (T)bt.alpha[prob];

  // pointers of this pair / problem on level k
  struct Lv {
    DGeom g;
    T ah, h3;
    int nH, nv, bpatch;
    int64_t NV;
    T *z, *gv, *r, *zi, *gg, *w, *Y, *G;
    const T *ATinv, *Sinv, *XT, *A0inv;
    const int64_t *bofs, *map;
    const int *lut, *slots;
    int N0;
  };
  auto level = [&](int k) {
    const SmallLevel<T>& L = a.lv[k];
    Lv v;
    v.g = L.g;
    v.ah = alpha * (T)L.h;
    v.h3 = (T)(L.h * L.h * L.h);
    v.nH = L.nH;
    v.bpatch = L.bpatch;
    v.nv = L.nH + 1;
    v.NV = (int64_t)v.nv * v.nv * v.nv;
    const int64_t vo = (int64_t)pair * vlen(L.g), yo = (int64_t)pair * v.NV * NPAD;
    v.z = L.z + vo;
    v.gv = L.gv + vo;
    v.r = L.r ? L.r + vo : nullptr;
    v.zi = L.zi ? L.zi + vo : nullptr;
    v.gg = L.gg ? L.gg + vo : nullptr;
    v.w = L.w ? L.w + vo : nullptr;
    v.Y = L.Y ? L.Y + yo : nullptr;
    v.G = L.G ? L.G + yo : nullptr;
    v.ATinv = L.ATinv ? L.ATinv + (int64_t)prob * 36 : nullptr;
    v.Sinv = L.Sinv ? L.Sinv + (int64_t)prob * 27 * NPAD * NPAD : nullptr;
    v.XT = L.XT ? L.XT + (int64_t)prob * 6 * 48 : nullptr;
    v.A0inv = L.A0inv ? L.A0inv + (int64_t)prob * L.N0 * L.N0 : nullptr;
    v.bofs = L.bofs;
    v.map = L.map;
    v.lut = L.lut;
    v.slots = L.slots;
    v.N0 = L.N0;
    return v;
  };
  // y = A x (mode 0) or b - A x (mode 1) on every node of the level
  auto apply = [&](const Lv& L, const T* x, const T* b, T* y, int mode) {
    const int n1 = L.g.n + 1;
    for (int e = tid; e < n1 * n1 * n1; e += nth) {
      const int i = e % n1, j = (e / n1) % n1, k = e / (n1 * n1);
      if (mode) apply_node<T, 1>(x, b, y, L.g, L.ah, L.h3, i, j, k);
      else apply_node<T, 0>(x, b, y, L.g, L.ah, L.h3, i, j, k);
    }
    __syncthreads();
  };
  // vertex type (per axis 0 on the low face, 1 inside, 2 on the high face)
  auto vtype = [&](int nH, int vx, int vy, int vz) {
    const int tx = vx == 0 ? 0 : (vx == nH ? 2 : 1), ty = vy == 0 ? 0 : (vy == nH ? 2 : 1),
              tz = vz == 0 ? 0 : (vz == nH ? 2 : 1);
    return tx + 3 * ty + 9 * tz;
  };
  // z (assign ? =, +=) M^{-1} r, the vertex-based smoother (eq. Preconditioner P), in six
  // phases separated by workgroup barriers
  auto smooth = [&](const Lv& L, const T* r, T* z, int assign) {
    const DGeom& g = L.g;
    const int nH = L.nH, nv = L.nv;
    const T eta = (T)a.eta;
    // tables of the level (read after the first barrier below)
    for (int e = tid; e < NPAD; e += nth) {
      if (e < NG) {
        const int* sl = L.slots + 4 * e;
        sslot[e][0] = sl[0]; sslot[e][1] = sl[1]; sslot[e][2] = sl[2]; sslot[e][3] = sl[3];
        soff[e] = sl[0] * g.B + (int64_t)sl[3] * g.plane + (int64_t)sl[2] * g.P + sl[1];
      } else {
        sslot[e][0] = -1; sslot[e][1] = sslot[e][2] = sslot[e][3] = 0;
        soff[e] = 0;
      }
    }
    for (int e = tid; e < 3 * 125; e += nth) slut[e] = L.lut[e];
    for (int e = tid; e < 6 * 48; e += nth) sX[e] = L.XT[e];
    for (int e = tid; e < 48; e += nth) sofs[e] = L.bofs[e];
    // 1. interior solves
    for (int e = tid; e < nH * nH * nH; e += nth)
      interior_sub_s2(r, L.zi, L.ATinv, g, e % nH, (e / nH) % nH, e / (nH * nH));
    __syncthreads();
    // 2. condensed interface residual gg = r - A zi (zi vanishes off subdomain interiors)
    apply(L, L.zi, r, L.gg, 1);
    // 3. gather the interface residual of every vertex patch (absent slots of boundary
    //    patches are zero)
    for (int e = tid; e < L.NV * NPAD; e += nth) {
      const int v = e / NPAD, slot = e % NPAD;
      const int vx = v % nv, vy = (v / nv) % nv, vz = v / (nv * nv);
      T val = T(0);
      if (slot < NG) {
        const int d = sslot[slot][0];
        const int o[3] = {2 * vx + sslot[slot][1], 2 * vy + sslot[slot][2], 2 * vz + sslot[slot][3]};
        bool ok = true;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          if (ax == d) ok = ok && (o[ax] >= 0 && o[ax] < g.n);
          else ok = ok && (o[ax] >= 1 && o[ax] <= g.n - 1);
        }
        if (ok) val = L.gg[lin(g, 2 * vx, 2 * vy, 2 * vz) + soff[slot]];
      }
      L.G[e] = val;
    }
    __syncthreads();
    // 4. patch solves y_V = S_type^{-1} g_V (slot-major Y; no patch: zero)
    for (int e = tid; e < L.NV * NPAD; e += nth) {
      const int v = e / NPAD, row = e % NPAD;
      const int vx = v % nv, vy = (v / nv) % nv, vz = v / (nv * nv);
      const int type = vtype(nH, vx, vy, vz);
      T acc = T(0);
      if (type == 13 || L.bpatch) {
        const T* srow = L.Sinv + ((int64_t)type * NPAD + row) * NPAD;
        const T* gv = L.G + (int64_t)v * NPAD;
#pragma unroll 4
        for (int col = 0; col < NG; ++col) acc += srow[col] * gv[col];
      }
      L.Y[(int64_t)row * L.NV + v] = acc;
    }
    __syncthreads();
    // 5. interface correction w and z on the interface
    {
      const int n1 = g.n + 1;
      for (int e = tid; e < n1 * n1 * n1; e += nth) {
        const int i = e % n1, j = (e / n1) % n1, k = e / (n1 * n1);
        if (i < g.n) pull_node<T, 2>(L.Y, L.w, z, g, slut, nv, L.NV, eta, assign, i, j, k);
      }
    }
    __syncthreads();
    // 6. harmonic extension into the subdomain interiors
    for (int e = tid; e < nH * nH * nH; e += nth)
      extend_sub_s2(L.w, L.zi, z, sX, sofs, g, eta, assign, e % nH, (e / nH) % nH, e / (nH * nH));
    __syncthreads();
  };
  auto restrict_to = [&](const Lv& F, const Lv& C, const T* rf, T* gc) {
    const int n1 = C.g.n + 1;
    for (int e = tid; e < n1 * n1 * n1; e += nth)
      restrict_node(rf, gc, F.g, C.g, e % n1, (e / n1) % n1, e / (n1 * n1));
    __syncthreads();
  };
  auto prolong_add = [&](const Lv& F, const Lv& C, const T* ec, T* zf) {
    const int n1 = F.g.n + 1;
    for (int e = tid; e < n1 * n1 * n1; e += nth)
      prolong_node(ec, zf, F.g, C.g, e % n1, (e / n1) % n1, e / (n1 * n1));
    __syncthreads();
  };
  auto coarse = [&](const Lv& L) {
    for (int i = tid; i < L.N0; i += nth) sg0[i] = L.gv[L.map[i]];
    __syncthreads();
    for (int i = tid; i < L.N0; i += nth) {
      T s = T(0);
      for (int j = 0; j < L.N0; ++j) s += L.A0inv[(int64_t)i * L.N0 + j] * sg0[j];
      L.z[L.map[i]] = s;
    }
    __syncthreads();
  };

  const int top = a.top, m = a.m;
  // descend: pre-smoothing from z = 0, restriction of the residual
  for (int k = top; k >= 1; --k) {
    const Lv L = level(k);
    smooth(L, L.gv, L.z, 1);
    for (int l = 1; l < m; ++l) {
      apply(L, L.z, L.gv, L.r, 1);
      smooth(L, L.r, L.z, 0);
    }
    apply(L, L.z, L.gv, L.r, 1);
    const Lv C = level(k - 1);
    restrict_to(L, C, L.r, C.gv);
  }
  coarse(level(0));
  // ascend: prolongation of the correction, post-smoothing
  for (int k = 1; k <= top; ++k) {
    const Lv L = level(k);
    const Lv C = level(k - 1);
    prolong_add(L, C, C.z, L.z);
    for (int l = 0; l < m; ++l) {
      apply(L, L.z, L.gv, L.r, 1);
      smooth(L, L.r, L.z, 0);
    }
  }
}

template <typename Tin, typename Tout>
__global__ void k_convert(const Tin* __restrict__ in, Tout* __restrict__ out, int64_t len, Bat bt) {
  const int pair = blockIdx.y;
  if (inactive(bt, pair)) return;
  in += (int64_t)pair * len;
  out += (int64_t)pair * len;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = (Tout)in[e];
}

// ---------------------------------------------------------------------------------
// reductions (FP64)
// ---------------------------------------------------------------------------------
// Four consecutive values per access (16-byte vector loads and stores): vectors are
// padded to multiples of 8 values and start 32-byte aligned, which the launchers check.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T>
struct Quad;
template <>
struct Quad<double> {
  static __device__ __forceinline__ void load(const double* __restrict__ p, double (&v)[4]) {
    const d2v a = *reinterpret_cast<const d2v*>(p);
    const d2v b = *reinterpret_cast<const d2v*>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
  static __device__ __forceinline__ void store(double* __restrict__ p, const double (&v)[4]) {
    d2v a, b;
    a.x = v[0]; a.y = v[1]; b.x = v[2]; b.y = v[3];
    *reinterpret_cast<d2v*>(p) = a;
    *reinterpret_cast<d2v*>(p + 2) = b;
  }
};
template <>
struct Quad<float> {
  static __device__ __forceinline__ void load(const float* __restrict__ p, float (&v)[4]) {
    const f4v a = *reinterpret_cast<const f4v*>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  }
  static __device__ __forceinline__ void store(float* __restrict__ p, const float (&v)[4]) {
    f4v a;
    a.x = v[0]; a.y = v[1]; a.z = v[2]; a.w = v[3];
    *reinterpret_cast<f4v*>(p) = a;
  }
};

template <typename TA>
__global__ void __launch_bounds__(256) k_dot(const TA* __restrict__ a, const double* __restrict__ b,
                                             const double* __restrict__ c, double* __restrict__ part,
                                             int64_t pstride, int64_t len, Bat bt) {
  __shared__ double sh[8];
  const int pair = blockIdx.y;
  if (inactive(bt, pair)) return;
  a += (int64_t)pair * len;
  b += (int64_t)pair * len;
  if (c) c += (int64_t)pair * len;
  part += (int64_t)pair * pstride;
  double s1 = 0.0, s2 = 0.0;
  const int64_t n4 = len >> 2;
#pragma unroll 2
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n4;
       e += (int64_t)gridDim.x * blockDim.x) {
    TA av[4];
    double bv[4];
    Quad<TA>::load(a + 4 * e, av);
    Quad<double>::load(b + 4 * e, bv);
#pragma unroll
    for (int k = 0; k < 4; ++k) s1 += (double)av[k] * bv[k];
    if (c) {
      double cv[4];
      Quad<double>::load(c + 4 * e, cv);
#pragma unroll
      for (int k = 0; k < 4; ++k) s2 += (double)av[k] * cv[k];
    }
  }
  s1 = block_sum(s1, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s1;
  if (c) {
    s2 = block_sum(s2, sh);
    if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = s2;
  }
}

__global__ void __launch_bounds__(256) k_final(const double* __restrict__ part, int nparts,
                                               int64_t pstride, int nout, double* __restrict__ out,
                                               Bat bt) {
  __shared__ double sh[8];
  const int pair = blockIdx.x;
  if (inactive(bt, pair)) return;
  part += (int64_t)pair * pstride;
  out += (int64_t)pair * kScalStride;
  for (int o = 0; o < nout; ++o) {
    double s = 0.0;
    for (int e = threadIdx.x; e < nparts; e += blockDim.x) s += part[o * nparts + e];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[o] = s;
  }
}

// u += a p, r -= a q (a = s[i_num] / s[i_den]), partial sums of r . r; with r32 the new
// residual is also written in FP32 (input of the next mixed-precision V-cycle).  DEFER:
// u is not touched; a goes to s[kS_AL] and the update is marked pending.
template <bool DEFER>
__global__ void __launch_bounds__(256) k_cg_update(double* __restrict__ u, double* __restrict__ r,
                                                   const double* __restrict__ p,
                                                   const double* __restrict__ q,
                                                   double* __restrict__ scal, int i_num,
                                                   const double* __restrict__ pq_part, int pq_n,
                                                   float* __restrict__ r32, double* __restrict__ part,
                                                   int64_t pstride, int64_t len, Bat bt) {
  __shared__ double sh[17];
  const int pair = blockIdx.y;
  if (inactive(bt, pair)) return;
  const int64_t off = (int64_t)pair * len;
  if (!DEFER) u += off;
  r += off;
  p += off;
  q += off;
  if (r32) r32 += off;
  scal += (int64_t)pair * kScalStride;
  part += (int64_t)pair * pstride;
  // this lane's first quads do not depend on alpha: loaded before the partial sums are
  // read (index clamped, no branch), so the two latencies overlap
  const int64_t n4 = len >> 2, step = (int64_t)gridDim.x * blockDim.x;
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double u0[4] = {0.0, 0.0, 0.0, 0.0}, r0[4], p0[4], q0[4];
  {
    const int64_t ec = 4 * (e0 < n4 ? e0 : 0);
    if (!DEFER) Quad<double>::load(u + ec, u0);
    Quad<double>::load(r + ec, r0);
    if (!DEFER) Quad<double>::load(p + ec, p0);
    Quad<double>::load(q + ec, q0);
  }
  // p^T A p from the partials of the operator kernel (every block the same value)
  const double pq = reduce_partials(pq_part + (int64_t)pair * pstride, pq_n, sh);
  const double alpha = scal[i_num] / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[kS_PQ] = pq;
    if (DEFER) {
      scal[kS_AL] = alpha;
      scal[kS_PEND] = 1.0;
    }
  }
  double s = 0.0;
  auto update = [&](int64_t e, double (&uv)[4], double (&rv)[4], const double (&pv)[4],
                    const double (&qv)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (!DEFER) uv[k] += alpha * pv[k];
      rv[k] -= alpha * qv[k];
      s += rv[k] * rv[k];
    }
    if (!DEFER) Quad<double>::store(u + 4 * e, uv);
    Quad<double>::store(r + 4 * e, rv);
    if (r32) {
      float rf[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) rf[k] = (float)rv[k];
      Quad<float>::store(r32 + 4 * e, rf);
    }
  };
  if (e0 < n4) update(e0, u0, r0, p0, q0);
#pragma unroll 2
  for (int64_t e = e0 + step; e < n4; e += step) {
    double uv[4] = {0.0, 0.0, 0.0, 0.0}, rv[4], pv[4], qv[4];
    if (!DEFER) Quad<double>::load(u + 4 * e, uv);
    Quad<double>::load(r + 4 * e, rv);
    if (!DEFER) Quad<double>::load(p + 4 * e, pv);
    Quad<double>::load(q + 4 * e, qv);
    update(e, uv, rv, pv, qv);
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename TZ, bool WITHU>
__global__ void __launch_bounds__(256) k_cg_direction(double* __restrict__ p, const TZ* __restrict__ z,
                                                      double* __restrict__ u, double* __restrict__ scal,
                                                      int i_num, int i_den, int flexible, int i_zq, int i_an,
                                                      int i_ad, const double* __restrict__ dot_part, int dot_n,
                                                      int64_t pstride, int64_t len, Bat bt) {
  __shared__ double sh[17];
  const int pair = blockIdx.y;
  if (inactive(bt, pair)) return;
  p += (int64_t)pair * len;
  z += (int64_t)pair * len;
  if (WITHU) u += (int64_t)pair * len;
  scal += (int64_t)pair * kScalStride;
  // this lane's first quads of z, p (and u) do not depend on beta: their loads go out
  // before the partial sums are read, so the two latencies overlap (index clamped, no
  // branch)
  const int64_t n4 = len >> 2, step = (int64_t)gridDim.x * blockDim.x;
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  TZ z0[4];
  double p0[4], u0[4];
  Quad<TZ>::load(z + 4 * (e0 < n4 ? e0 : 0), z0);
  Quad<double>::load(p + 4 * (e0 < n4 ? e0 : 0), p0);
  if (WITHU) Quad<double>::load(u + 4 * (e0 < n4 ? e0 : 0), u0);
  // the pending update's alpha: an active pair always has one here (the update of the
  // previous iteration, or of the first step), and the update that follows in this
  // iteration marks its own as pending again
  const double al = WITHU ? scal[kS_AL] : 0.0;
  // r . z (and z . q) from the partials of the dot kernel; block 0 keeps them
  const double* dp = dot_part + (int64_t)pair * pstride;
  const double rz = reduce_partials(dp, dot_n, sh);
  const double zq = flexible ? reduce_partials(dp + dot_n, dot_n, sh) : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[i_num] = rz;
    if (flexible) scal[i_zq] = zq;
  }
  double beta;
  if (flexible) beta = -(scal[i_an] / scal[i_ad]) * zq / scal[i_den];
  else beta = rz / scal[i_den];
  if (e0 < n4) {
    if (WITHU) {
#pragma unroll
      for (int k = 0; k < 4; ++k) u0[k] += al * p0[k];
      Quad<double>::store(u + 4 * e0, u0);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) p0[k] = (double)z0[k] + beta * p0[k];
    Quad<double>::store(p + 4 * e0, p0);
  }
#pragma unroll 2
  for (int64_t e = e0 + step; e < n4; e += step) {
    TZ zv[4];
    double pv[4], uv[4];
    Quad<TZ>::load(z + 4 * e, zv);
    Quad<double>::load(p + 4 * e, pv);
    if (WITHU) {
      Quad<double>::load(u + 4 * e, uv);
#pragma unroll
      for (int k = 0; k < 4; ++k) uv[k] += al * pv[k];
      Quad<double>::store(u + 4 * e, uv);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) pv[k] = (double)zv[k] + beta * pv[k];
    Quad<double>::store(p + 4 * e, pv);
  }
}

// u += s[kS_AL] p where an update is pending; clears the flag
__global__ void __launch_bounds__(256) k_cg_finish(double* __restrict__ u, const double* __restrict__ p,
                                                   double* __restrict__ scal, int64_t len, Bat bt) {
  const int pair = blockIdx.y;
  if (inactive(bt, pair)) return;
  double* s = scal + (int64_t)pair * kScalStride;
  if (s[kS_PEND] == 0.0) return;
  const double al = s[kS_AL];
  u += (int64_t)pair * len;
  p += (int64_t)pair * len;
  const int64_t n4 = len >> 2, step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n4; e += step) {
    double uv[4], pv[4];
    Quad<double>::load(u + 4 * e, uv);
    Quad<double>::load(p + 4 * e, pv);
#pragma unroll
    for (int k = 0; k < 4; ++k) uv[k] += al * pv[k];
    Quad<double>::store(u + 4 * e, uv);
  }
}

// clears the pending flags once every block of k_cg_finish has read them
__global__ void k_cg_finish_clear(double* __restrict__ scal, int count) {
  for (int p = threadIdx.x; p < count; p += blockDim.x) scal[(int64_t)p * kScalStride + kS_PEND] = 0.0;
}

__global__ void __launch_bounds__(1024) k_pcg_init(double* __restrict__ scal, int* __restrict__ act,
                                                   int* __restrict__ iters, int* __restrict__ status,
                                                   int count, double rtol) {
  for (int p = threadIdx.x; p < count; p += blockDim.x) {
    double* s = scal + (int64_t)p * kScalStride;
    const double bb = s[kS_BB];
    s[kS_TOL] = rtol;
    s[kS_REL] = 0.0;
    s[kS_PEND] = 0.0;
    iters[p] = 0;
    if (!isfinite(bb)) {
      act[p] = 0;
      status[p] = kPairBroken;
    } else if (bb == 0.0) {
      act[p] = 0;
      status[p] = kPairDone;
    } else {
      act[p] = 1;
      status[p] = kPairRun;
    }
  }
}

__global__ void __launch_bounds__(1024) k_pcg_check(double* __restrict__ scal, int* __restrict__ act,
                                                    int* __restrict__ iters, int* __restrict__ status,
                                                    int count, int i_rz, int* __restrict__ nact,
                                                    const double* __restrict__ rr_part, int rr_n,
                                                    int64_t pstride, double* __restrict__ hist) {
  __shared__ int sh[16];
  __shared__ double shd[17];
  // r . r of each active pair from the update's partials: the block together for few
  // pairs (many partials each), one thread per pair otherwise
  if (count <= 8) {
    for (int p = 0; p < count; ++p) {
      if (act[p] == 0) continue;   // uniform over the block
      const double rr = reduce_partials(rr_part + (int64_t)p * pstride, rr_n, shd);
      if (threadIdx.x == 0) scal[(int64_t)p * kScalStride + kS_RR] = rr;
    }
    __syncthreads();
  } else {
    for (int p = threadIdx.x; p < count; p += blockDim.x) {
      if (act[p] == 0) continue;
      double rr = 0.0;
      for (int e = 0; e < rr_n; ++e) rr += rr_part[(int64_t)p * pstride + e];
      scal[(int64_t)p * kScalStride + kS_RR] = rr;
    }
  }
  int c = 0;
  for (int p = threadIdx.x; p < count; p += blockDim.x) {
    if (act[p] == 0) continue;
    double* s = scal + (int64_t)p * kScalStride;
    const double pq = s[kS_PQ], rr = s[kS_RR], rz = s[i_rz];
    if (iters[p] < kHistCap) {   // (r . z, p . A p) of this iteration: the Lanczos coefficients of CG
      hist[((int64_t)p * kHistCap + iters[p]) * 2] = rz;
      hist[((int64_t)p * kHistCap + iters[p]) * 2 + 1] = pq;
    }
    iters[p] += 1;
    const double rel = sqrt(rr) / sqrt(s[kS_BB]);
    s[kS_REL] = rel;
    if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rr) || !isfinite(rz)) {
      act[p] = 0;
      status[p] = kPairBroken;
    } else if (rel <= s[kS_TOL]) {
      act[p] = 0;
      status[p] = kPairDone;
    } else {
      ++c;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    nact[0] = t;
  }
}

__global__ void k_copy(const double* __restrict__ x, double* __restrict__ y, int64_t len, Bat bt) {
  const int pair = blockIdx.y;
  if (inactive(bt, pair)) return;
  x += (int64_t)pair * len;
  y += (int64_t)pair * len;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x)
    y[e] = x[e];
}

__global__ void k_zero(double* __restrict__ y, int64_t len, Bat bt) {
  const int pair = blockIdx.y;
  if (inactive(bt, pair)) return;
  y += (int64_t)pair * len;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x)
    y[e] = 0.0;
}

// y = c0 x0 + c1 x1 + c2 x2 per entry (x1, x2 may be null; y may alias any x)
__global__ void k_lincomb(double* y, const double* x0, double c0, const double* x1, double c1, const double* x2,
                          double c2, int64_t len, Bat bt) {
  const int pair = blockIdx.y;
  if (inactive(bt, pair)) return;
  const int64_t off = (int64_t)pair * len;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x) {
    double v = c0 * x0[off + e];
    if (x1) v += c1 * x1[off + e];
    if (x2) v += c2 * x2[off + e];
    y[off + e] = v;
  }
}

// ---------------------------------------------------------------------------------
// load vector from 2x2x2 Gauss samples
// ---------------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_assemble_rhs(const double* __restrict__ f, double* __restrict__ bv,
                                                     DGeom g, double w8, const double* __restrict__ coef,
                                                     int coef_r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y, k = blockIdx.z;
  if (i > g.n) return;
  const double x0 = 0.5 - 0.5 / 1.7320508075688772935;   // (1 - 1/sqrt 3) / 2
  const double x1 = 0.5 + 0.5 / 1.7320508075688772935;
  const double gx[2] = {x0, x1};
  const int o[3] = {i, j, k};
  const int64_t p = lin(g, i, j, k);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double v = 0.0;
    if (is_unknown(g, d, i, j, k) && (coef == nullptr || edge_in_domain(coef, coef_r, g.n, d, o))) {
      const int b = (d + 1) % 3, c = (d + 2) % 3;
      // the four elements sharing the edge: cell o[d] along d, o[b]-1+eb, o[c]-1+ec across
      for (int ec = 0; ec < 2; ++ec)
        for (int eb = 0; eb < 2; ++eb) {
          int cell[3];
          cell[d] = o[d];
          cell[b] = o[b] - 1 + eb;
          cell[c] = o[c] - 1 + ec;
          const int lb = o[b] - cell[b];   // local node offset (0 or 1) along b
          const int lc = o[c] - cell[c];
          const int64_t e = ((int64_t)cell[2] * g.n + cell[1]) * g.n + cell[0];
          const double* fe = f + e * 24;
          for (int q = 0; q < 8; ++q) {
            const int qa[3] = {q & 1, (q >> 1) & 1, (q >> 2) & 1};
            const double tb = gx[qa[b]], tc = gx[qa[c]];
            const double pb = lb ? tb : 1.0 - tb;
            const double pc = lc ? tc : 1.0 - tc;
            v += fe[q * 3 + d] * pb * pc;
          }
        }
      v *= w8;
    }
    bv[d * g.B + p] = v;
  }
}

__global__ void __launch_bounds__(64) k_curlcurl_form(const double* __restrict__ lam,
                                                      const double* __restrict__ u,
                                                      double* __restrict__ part, DGeom g, double h,
                                                      const double* __restrict__ coef, int coef_r) {
  __shared__ double sh[8];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y, k = blockIdx.z;
  double s = 0.0;
  if (i <= g.n) {
    const int64_t p = lin(g, i, j, k);
    const int o[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (is_unknown(g, d, i, j, k) && (coef == nullptr || edge_in_domain(coef, coef_r, g.n, d, o)))
        s += lam[d * g.B + p] * (coef ? apply_at_coef(u, g, d, p, o, h, 0.0, coef, coef_r)
                                      : apply_at(u, g, d, p, h, 0.0));
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0)
    part[((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
}

// node grid: x = blocks per pair * pairs, y = j, z = k
inline dim3 node_grid(const Geom& g, int nbx, int count) {
  return dim3((unsigned)(nbx * count), (unsigned)(g.n + 1), (unsigned)(g.n + 1));
}

inline int nbx64(int n) { return (n + 1 + 63) / 64; }

// Grid over the nodes [0, n)^3 only: every unknown has all coordinates below n (the
// transfers leave the other entries, zero by the layout contract, untouched).
inline dim3 inner_grid(const Geom& g, int nbx, int count) {
  return dim3((unsigned)(nbx * count), (unsigned)g.n, (unsigned)g.n);
}
inline int nbx_inner(int n) { return (n + 63) / 64; }

// the four-value vector kernels: every pair's vector starts 16-byte aligned
template <typename T>
inline bool quad_ok(int64_t len, const T* ptr) {
  return len % 4 == 0 && reinterpret_cast<uintptr_t>(ptr) % 16 == 0;
}

// blocks per pair of the grid-stride vector kernels: enough for a level, fewer for many pairs
inline unsigned vec_blocks(int64_t len, int count, unsigned cap) {
  const int64_t want = (len + 255) / 256;
  unsigned b = (unsigned)std::min<int64_t>(want, (int64_t)cap);
  if (count > 1) b = std::min<unsigned>(b, std::max<unsigned>(4u, 4096u / (unsigned)count));
  return std::max<unsigned>(b, 1u);
}

}  // namespace

// ---------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------
template <typename T>
hipError_t launch_apply(const T* x, const T* b, T* y, const Geom& g, const Bat& bt, int mode,
                        hipStream_t st) {
  // batches of four or more pairs take the plane-marching kernel from n = 17 in both
  // precisions (one position per lane up to n = 64: for the 512-problem batch FP32 165.6
  // against 182.7 ms per 2048 solves with the per-thread kernel at n = 24, 32)
  const int min_n = stencil_min_n(bt.count);
  // with a coefficient per cell the plane-marching kernel takes box grids of up to 8^3
  // (its factors in LDS); others, and the smaller levels, take the per-thread kernels
  if (g.n > min_n && g.n <= stencil_max_n()) {
    const hipError_t e = launch_stencil<T>(x, b, y, g, bt, mode, nullptr, 0, nullptr, st);
    if (e != hipErrorNotSupported) return e;   // else: the per-thread kernel below
  }
  // rows shorter than a wave: lanes packed over the plane
  if (g.n + 1 < 64) {
    const int w = g.n + 1, nbp = (w * w + 63) / 64;
    const dim3 grid((unsigned)(nbp * bt.count), (unsigned)w);
    if (mode == 0)
      hipLaunchKernelGGL((k_apply_plane<T, 0>), grid, dim3(64), 0, st, x, b, y, dgeom(g), bt, g.h, nbp);
    else
      hipLaunchKernelGGL((k_apply_plane<T, 1>), grid, dim3(64), 0, st, x, b, y, dgeom(g), bt, g.h, nbp);
    return hipGetLastError();
  }
  const int nbx = nbx64(g.n);
  if (mode == 0)
    hipLaunchKernelGGL((k_apply<T, 0>), node_grid(g, nbx, bt.count), dim3(64), 0, st, x, b, y, dgeom(g),
                       bt, g.h, nbx);
  else
    hipLaunchKernelGGL((k_apply<T, 1>), node_grid(g, nbx, bt.count), dim3(64), 0, st, x, b, y, dgeom(g),
                       bt, g.h, nbx);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(const T* rf, T* gc, const Geom& f, const Geom& c, const Bat& bt,
                           hipStream_t st) {
  // rows shorter than a wave: lanes packed over the (I, J) plane of inner nodes
  const int packed = (c.n < 64) ? 1 : 0;
  const int nbx = packed ? (c.n * c.n + 63) / 64 : nbx_inner(c.n);
  const dim3 grid = packed ? dim3((unsigned)(nbx * bt.count), (unsigned)c.n) : inner_grid(c, nbx, bt.count);
  hipLaunchKernelGGL((k_restrict<T>), grid, dim3(64), 0, st, rf, gc, dgeom(f), dgeom(c), bt, nbx, packed);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_add(const T* ec, T* zf, const Geom& f, const Geom& c, const Bat& bt,
                              hipStream_t st) {
  constexpr int KP = sizeof(T) == 4 ? 4 : 2;   // FP64: 4 planes leave 3 waves per SIMD
  const int packed = (f.n < 64) ? 1 : 0;
  const int nbx = packed ? (f.n * f.n + 63) / 64 : nbx_inner(f.n);
  const unsigned nkb = (unsigned)((f.n + KP - 1) / KP);
  const dim3 grid = packed ? dim3((unsigned)(nbx * bt.count), nkb) : dim3((unsigned)(nbx * bt.count), (unsigned)f.n, nkb);
  hipLaunchKernelGGL((k_prolong_add<T, KP>), grid, dim3(64), 0, st, ec, zf, dgeom(f), dgeom(c), bt, nbx, packed);
  return hipGetLastError();
}

// Buffer addressing for the smoother's condensation and patch products when a pair's
// vector and Y rows fit the descriptors' 31-bit ranges (offsets of 2^31 must lie past
// both), unless the table asks for 64-bit addresses at this size (which also lets a test
// compare the two forms).
bool smoother_buffers(const DGeom& dg, const DSub& sub, const Bat& bt, size_t elem) {
  constexpr int64_t NPAD = (6 * 2 * (4 * 2 - 3) + 15) / 16 * 16;
  int bits = 32, unused = 0;
  tune_lookup(kTunePatchAddr, dg.n, (int)elem, 0, bt.count, &bits, &unused);
  return bits == 32 && 3 * dg.B * (int64_t)elem < 0x7fffffffLL &&
         y_row_len(sub.nH) * NPAD * (int64_t)elem < 0x7fffffffLL;
}

template <typename T>
void launch_sm_patch(const LevelPtrs<T>& L, const DSub& sub, const DGeom& dg, const Bat& bt, hipStream_t st) {
  const bool buf = smoother_buffers(dg, sub, bt, sizeof(T));
  const dim3 grid((unsigned)sub.nchunks, (unsigned)bt.count);
  if (buf)
    hipLaunchKernelGGL((k_sm_patch<T, 2, true>), grid, dim3(256), 0, st, L.gg, L.Y, L.Sinv, dg, sub, bt);
  else
    hipLaunchKernelGGL((k_sm_patch<T, 2, false>), grid, dim3(256), 0, st, L.gg, L.Y, L.Sinv, dg, sub, bt);
}

template <typename T>
hipError_t launch_smooth(const T* r, T* z, const LevelPtrs<T>& L, const DSub& sub,
                         const Geom& g, const Bat& bt, double eta, int assign, hipStream_t st) {
  if (sub.s != 2) return hipErrorInvalidValue;
  const DGeom dg = dgeom(g);
  // condensed interface residual gg = r - A A_T^{-1} r_I on the interface unknowns
  // rows shorter than a wave: lanes packed over the subdomain plane
  const int packed = (sub.nH < 64) ? 1 : 0;
  const int nbs = packed ? (sub.nH * sub.nH + 63) / 64 : (sub.nH + 63) / 64;
  const dim3 eg((unsigned)(nbs * bt.count), (unsigned)sub.nH, packed ? 1u : (unsigned)sub.nH);
  if (smoother_buffers(dg, sub, bt, sizeof(T)))
    hipLaunchKernelGGL((k_sm_condense<T, true>), eg, dim3(64), 0, st, r, L.gg, L.XT, dg, sub.nH, bt, nbs, packed);
  else
    hipLaunchKernelGGL((k_sm_condense<T, false>), eg, dim3(64), 0, st, r, L.gg, L.XT, dg, sub.nH, bt, nbs, packed);
  if (sub.nchunks > 0) launch_sm_patch<T>(L, sub, dg, bt, st);
  hipLaunchKernelGGL((k_sm_pull_extend<T>), eg, dim3(64), 0, st, L.Y, r, z, L.XT, L.ATinv, dg, sub, (T)eta, assign,
                     bt, nbs, packed);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_patch_products(const LevelPtrs<T>& L, const DSub& sub, const Geom& g, const Bat& bt,
                                 hipStream_t st) {
  if (sub.s != 2) return hipErrorInvalidValue;
  if (sub.nchunks > 0) launch_sm_patch<T>(L, sub, dgeom(g), bt, st);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse(const T* g, T* z, const T* A0inv, const int64_t* map, int N0,
                         int64_t len, const Bat& bt, hipStream_t st) {
  if (N0 > 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_coarse<T>), dim3((unsigned)bt.count), dim3(256), 0, st, g, z, A0inv, map, N0,
                     len, bt);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_unit_cols(T* g, const int64_t* map, int N, int j0, int64_t len, const Bat& bt,
                            hipStream_t st) {
  hipLaunchKernelGGL((k_unit_cols<T>), dim3(vec_blocks(len, bt.count, 64), (unsigned)bt.count), dim3(256), 0, st,
                     g, map, N, j0, len, bt);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_cols(const T* z, T* Bm, const int64_t* map, int N, int j0, int64_t len, bool colmajor,
                              const Bat& bt, hipStream_t st) {
  hipLaunchKernelGGL((k_gather_cols<T>), dim3((unsigned)((N + 255) / 256), (unsigned)bt.count), dim3(256), 0, st,
                     z, Bm, map, N, j0, len, colmajor ? 1 : 0, bt);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dense_vcycle(const T* g, T* z, const T* Bm, const int64_t* map, int N, int64_t len,
                               const Bat& bt, bool clear, bool colmajor, hipStream_t st) {
  if (N < 1 || N > kDenseMaxN || bt.nrhs < 1 || bt.count % bt.nrhs) return hipErrorInvalidValue;
  if (clear)
    hipLaunchKernelGGL((k_fill_zero<T>), dim3(vec_blocks(len, bt.count, 2048), (unsigned)bt.count), dim3(256), 0,
                       st, z, len, bt);
  const int nprob = bt.count / bt.nrhs;
  if (colmajor) {
    const dim3 grid((unsigned)((N + 255) / 256), (unsigned)nprob);
    if (bt.nrhs == 1)
      hipLaunchKernelGGL((k_dense_vcycle_t<T, 1>), grid, dim3(256), (size_t)N * sizeof(T), st, g, z, Bm, map, N,
                         len, bt);
    else
      hipLaunchKernelGGL((k_dense_vcycle_t<T, 4>), grid, dim3(256), (size_t)4 * N * sizeof(T), st, g, z, Bm, map,
                         N, len, bt);
    return hipGetLastError();
  }
  // rows per wave: about 1024 workgroups over all problems, 1 .. 16 rows per wave
  const int64_t want = (int64_t)N * nprob / (4 * 1024);
  const int rpw = (int)std::max<int64_t>(1, std::min<int64_t>(16, want));
  const unsigned nbx = (unsigned)((N + 4 * rpw - 1) / (4 * rpw));
  if (bt.nrhs == 1) {
    hipLaunchKernelGGL((k_dense_vcycle<T, 1>), dim3(nbx, (unsigned)nprob), dim3(256), (size_t)N * sizeof(T), st, g,
                       z, Bm, map, N, len, rpw, bt);
  } else {
    hipLaunchKernelGGL((k_dense_vcycle<T, 4>), dim3(nbx, (unsigned)nprob), dim3(256), (size_t)4 * N * sizeof(T),
                       st, g, z, Bm, map, N, len, rpw, bt);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_vcycle_small(const SmallArgs<T>& a, const Bat& bt, hipStream_t st) {
  if (a.top < 0 || a.top >= kSmallMaxLevels) return hipErrorInvalidValue;
  for (int k = 1; k <= a.top; ++k)
    if (a.lv[k].g.n / 2 < 2 || a.lv[k].nH * 2 != a.lv[k].g.n) return hipErrorInvalidValue;
  if (a.lv[0].N0 > 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_vcycle_small<T>), dim3((unsigned)bt.count), dim3(512), 0, st, a, bt);
  return hipGetLastError();
}

template hipError_t launch_vcycle_small<double>(const SmallArgs<double>&, const Bat&, hipStream_t);
template hipError_t launch_vcycle_small<float>(const SmallArgs<float>&, const Bat&, hipStream_t);

template <typename Tin, typename Tout>
hipError_t launch_convert(const Tin* in, Tout* out, int64_t len, const Bat& bt, hipStream_t st) {
  hipLaunchKernelGGL((k_convert<Tin, Tout>), dim3(vec_blocks(len, bt.count, 2048), (unsigned)bt.count),
                     dim3(256), 0, st, in, out, len, bt);
  return hipGetLastError();
}

template <typename TA>
hipError_t launch_dot(const TA* a, const double* b, const double* c, double* part, int64_t pstride,
                      double* out, int64_t len, const Bat& bt, hipStream_t st) {
  if (!quad_ok(len, a) || !quad_ok(len, b) || (c && !quad_ok(len, c))) return hipErrorInvalidValue;
  const unsigned nb = vec_blocks(len, bt.count, kRedBlocks);
  if ((c ? 2 : 1) * (int64_t)nb > pstride) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_dot<TA>), dim3(nb, (unsigned)bt.count), dim3(256), 0, st, a, b, c, part, pstride,
                     len, bt);
  if (out)
    hipLaunchKernelGGL(k_final, dim3((unsigned)bt.count), dim3(256), 0, st, part, (int)nb, pstride, c ? 2 : 1,
                       out, bt);
  return hipGetLastError();
}

int dot_parts(int64_t len, int count) { return (int)vec_blocks(len, count, kRedBlocks); }

hipError_t launch_final(const double* part, int nparts, int64_t pstride, int nout, double* out,
                        const Bat& bt, hipStream_t st) {
  hipLaunchKernelGGL(k_final, dim3((unsigned)bt.count), dim3(256), 0, st, part, nparts, pstride, nout, out,
                     bt);
  return hipGetLastError();
}

hipError_t launch_cg_update(double* u, double* r, const double* p, const double* q, double* scal,
                            int i_num, const double* pq_part, int pq_n, float* r32, double* part,
                            int64_t pstride, int64_t len, const Bat& bt, hipStream_t st) {
  if ((u && !quad_ok(len, u)) || !quad_ok(len, r) || !quad_ok(len, p) || !quad_ok(len, q) ||
      (r32 && !quad_ok(len, r32)))
    return hipErrorInvalidValue;
  const unsigned nb = vec_blocks(len, bt.count, kRedBlocks);
  if ((int64_t)nb > pstride || pq_n > pstride) return hipErrorInvalidValue;
  if (u)
    hipLaunchKernelGGL(k_cg_update<false>, dim3(nb, (unsigned)bt.count), dim3(256), 0, st, u, r, p, q, scal,
                       i_num, pq_part, pq_n, r32, part, pstride, len, bt);
  else
    hipLaunchKernelGGL(k_cg_update<true>, dim3(nb, (unsigned)bt.count), dim3(256), 0, st, u, r, p, q, scal,
                       i_num, pq_part, pq_n, r32, part, pstride, len, bt);
  return hipGetLastError();
}

template <typename TZ>
hipError_t launch_cg_direction(double* p, const TZ* z, double* u, double* scal, int i_num, int i_den,
                               int flexible, int i_zq, int i_an, int i_ad, const double* dot_part, int dot_n,
                               int64_t pstride, int64_t len, const Bat& bt, hipStream_t st) {
  if (!quad_ok(len, p) || !quad_ok(len, z) || (u && !quad_ok(len, u))) return hipErrorInvalidValue;
  const dim3 grid(vec_blocks(len, bt.count, 2048), (unsigned)bt.count);
  if (u)
    hipLaunchKernelGGL((k_cg_direction<TZ, true>), grid, dim3(256), 0, st, p, z, u, scal, i_num, i_den, flexible,
                       i_zq, i_an, i_ad, dot_part, dot_n, pstride, len, bt);
  else
    hipLaunchKernelGGL((k_cg_direction<TZ, false>), grid, dim3(256), 0, st, p, z, u, scal, i_num, i_den,
                       flexible, i_zq, i_an, i_ad, dot_part, dot_n, pstride, len, bt);
  return hipGetLastError();
}

hipError_t launch_cg_finish(double* u, const double* p, double* scal, int64_t len, const Bat& bt, hipStream_t st) {
  if (!quad_ok(len, u) || !quad_ok(len, p)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cg_finish, dim3(vec_blocks(len, bt.count, 2048), (unsigned)bt.count), dim3(256), 0, st, u,
                     p, scal, len, bt);
  hipLaunchKernelGGL(k_cg_finish_clear, dim3(1), dim3(1024), 0, st, scal, bt.count);
  return hipGetLastError();
}

template hipError_t launch_dot<double>(const double*, const double*, const double*, double*, int64_t,
                                       double*, int64_t, const Bat&, hipStream_t);
template hipError_t launch_dot<float>(const float*, const double*, const double*, double*, int64_t,
                                      double*, int64_t, const Bat&, hipStream_t);
template hipError_t launch_cg_direction<double>(double*, const double*, double*, double*, int, int, int, int, int,
                                                int, const double*, int, int64_t, int64_t, const Bat&, hipStream_t);
template hipError_t launch_cg_direction<float>(double*, const float*, double*, double*, int, int, int, int, int,
                                               int, const double*, int, int64_t, int64_t, const Bat&, hipStream_t);

hipError_t launch_pcg_init(double* scal, int* act, int* iters, int* status, int count, double rtol,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_init, dim3(1), dim3(1024), 0, st, scal, act, iters, status, count, rtol);
  return hipGetLastError();
}

hipError_t launch_pcg_check(double* scal, int* act, int* iters, int* status, int count, int i_rz,
                            int* nact, const double* rr_part, int rr_n, int64_t pstride, double* hist,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_check, dim3(1), dim3(1024), 0, st, scal, act, iters, status, count, i_rz,
                     nact, rr_part, rr_n, pstride, hist);
  return hipGetLastError();
}

hipError_t launch_copy(const double* x, double* y, int64_t len, const Bat& bt, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, dim3(vec_blocks(len, bt.count, 2048), (unsigned)bt.count), dim3(256), 0, st, x,
                     y, len, bt);
  return hipGetLastError();
}

hipError_t launch_zero(double* y, int64_t len, const Bat& bt, hipStream_t st) {
  hipLaunchKernelGGL(k_zero, dim3(vec_blocks(len, bt.count, 2048), (unsigned)bt.count), dim3(256), 0, st, y,
                     len, bt);
  return hipGetLastError();
}

hipError_t launch_lincomb(double* y, const double* x0, double c0, const double* x1, double c1, const double* x2,
                          double c2, int64_t len, const Bat& bt, hipStream_t st) {
  hipLaunchKernelGGL(k_lincomb, dim3(vec_blocks(len, bt.count, 2048), (unsigned)bt.count), dim3(256), 0, st, y, x0,
                     c0, x1, c1, x2, c2, len, bt);
  return hipGetLastError();
}

hipError_t launch_assemble_rhs(const double* f, double* b, const Geom& g, hipStream_t st, const double* coef,
                               int coef_r) {
  const double w8 = g.h * g.h * g.h / 8.0;
  hipLaunchKernelGGL(k_assemble_rhs, node_grid(g, nbx64(g.n), 1), dim3(64), 0, st, f, b, dgeom(g), w8, coef,
                     coef_r);
  return hipGetLastError();
}

hipError_t launch_curlcurl_form(const double* lam, const double* u, const Geom& g,
                                double* partial, double* out, hipStream_t st, const double* coef, int coef_r) {
  const dim3 grid = node_grid(g, nbx64(g.n), 1);
  const int nparts = (int)(grid.x * grid.y * grid.z);
  hipLaunchKernelGGL(k_curlcurl_form, grid, dim3(64), 0, st, lam, u, partial, dgeom(g), g.h, coef, coef_r);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, st, partial, nparts, (int64_t)0, 1, out,
                     Bat{1, 1, nullptr, nullptr});
  return hipGetLastError();
}

// The compile-time table of the interface-sum-and-extension kernel against the host's.
bool boundary_patches_match(const std::vector<int>& tab) {
  if ((int)tab.size() != 4 * kBP.n) return false;
  for (int e = 0; e < kBP.n; ++e)
    for (int t = 0; t < 4; ++t) {
      int want = (t < kBP.ncand[e]) ? kBP.corner[e][t] + 8 * kBP.slot[e][t] : -1;
      if (t == 0 && kBP.owned[e]) want |= 1 << 30;
      if (tab[e * 4 + t] != want) return false;
    }
  return true;
}

// explicit instantiations
#define NDMG_INST(T)                                                                              \
  template hipError_t launch_apply<T>(const T*, const T*, T*, const Geom&, const Bat&, int,       \
                                      hipStream_t);                                               \
  template hipError_t launch_restrict<T>(const T*, T*, const Geom&, const Geom&, const Bat&,      \
                                         hipStream_t);                                            \
  template hipError_t launch_prolong_add<T>(const T*, T*, const Geom&, const Geom&, const Bat&,   \
                                            hipStream_t);                                         \
  template hipError_t launch_smooth<T>(const T*, T*, const LevelPtrs<T>&, const DSub&,            \
                                       const Geom&, const Bat&, double, int, hipStream_t);       \
  template hipError_t launch_patch_products<T>(const LevelPtrs<T>&, const DSub&, const Geom&,     \
                                               const Bat&, hipStream_t);                          \
  template hipError_t launch_coarse<T>(const T*, T*, const T*, const int64_t*, int, int64_t,      \
                                       const Bat&, hipStream_t);                                  \
  template hipError_t launch_unit_cols<T>(T*, const int64_t*, int, int, int64_t, const Bat&,      \
                                          hipStream_t);                                           \
  template hipError_t launch_gather_cols<T>(const T*, T*, const int64_t*, int, int, int64_t, bool, \
                                            const Bat&, hipStream_t);                             \
  template hipError_t launch_dense_vcycle<T>(const T*, T*, const T*, const int64_t*, int, int64_t, \
                                             const Bat&, bool, bool, hipStream_t);
NDMG_INST(double)
NDMG_INST(float)
#undef NDMG_INST
template hipError_t launch_convert<double, float>(const double*, float*, int64_t, const Bat&,
                                                  hipStream_t);
template hipError_t launch_convert<float, double>(const float*, double*, int64_t, const Bat&,
                                                  hipStream_t);

}  // namespace ndmg
