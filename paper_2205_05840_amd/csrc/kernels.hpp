// Device kernels of the ndmg library and their launchers (host side).
//
// Every launcher works on a batch of "pairs" (problem, right-hand side) of one size
// class: all pairs share the level geometry, their vectors follow each other with a
// stride of the level's vector length, pairs p*nrhs .. p*nrhs + nrhs - 1 belong to
// problem p and share its alpha and its local factors (which follow each other with a
// stride of one factor block).  A single solve is the batch of one pair.
#pragma once
#include <algorithm>

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "ndmg_internal.hpp"

namespace ndmg {

// Geometry passed by value to kernels.
struct DGeom {
  int n;
  int P;
  int64_t plane;
  int64_t B;
};

inline DGeom dgeom(const Geom& g) { return DGeom{g.n, g.P, g.plane, g.B}; }

// Batch description passed by value to kernels.
struct Bat {
  int count;               // pairs in the launch
  int nrhs;                // consecutive pairs per problem
  const double* alpha;     // per problem (device)
  const int* act;          // per pair, 0 = skip (converged); nullptr = all active
  const double* coef;      // coefficient boxes (device, r^3, [z][y][x]): alpha(x) = alpha *
                           // coef[box of x], 0 for a box outside the domain; nullptr =
                           // constant alpha on the cube (one problem only)
  int coef_r;              // boxes per axis (r divides every level's n)
};

inline Bat single_batch(const double* d_alpha) { return Bat{1, 1, d_alpha, nullptr}; }

// Smoother tables of one level on the device (shared by all pairs of a class).
struct DSub {
  int s, nH, nI, nG, npad, lut_w, nB;
  int bpatch;           // boundary vertices carry patches
  const int* lut;       // [3][w][w][w] slot lookup
  const int* slots;     // [nG][4]: d, dx, dy, dz
  const int* segs;      // [nseg][8]: type, lo0, lo1, lo2, d0, d1, row position of the
                        // segment's first vertex in Y (y_pos), count
  const int* chunks;    // [nchunks][4]: segment | groups per wave << 16 (| kChunkRhsWaves),
                        // first vertex of wave 0, vertex step between waves, vertex step
                        // between a wave's groups (all multiples of 16)
  int nchunks;
  const int64_t* bofs;  // nB offsets of the subdomain boundary edges from its lower node
};

// ---- Y, the vertex patch results of the large-level smoother --------------------------
// Slot-major: npad rows per pair, row `slot` holding y_V[slot] of every vertex V at
// y_pos(V).  The vertices of one patch type (inside the box, on one of its 6 faces, on
// one of its 12 edges) lie together, in the order of their segment, each type in a
// region of whole 16-entry runs: 16 consecutive vertices of a segment from a multiple of
// 16 fill one aligned run, so each store of the patch kernel writes whole cache lines.
// Vertices with no patch (the box corners; all boundary vertices when those carry none)
// share the zero run at the end of the row, which the patch kernel clears.
__host__ __device__ inline int64_t y_run16(int64_t x) { return (x + 15) / 16 * 16; }
__host__ __device__ inline int64_t y_zero_run(int nH) {
  const int64_t m = nH - 1;
  return y_run16(m * m * m) + 6 * y_run16(m * m) + 12 * y_run16(m);
}
__host__ __device__ inline int64_t y_row_len(int nH) { return y_zero_run(nH) + 16; }
// row position of vertex (x, y, z), 0 <= x, y, z <= nH.  Plain arithmetic on 0/1 flags,
// no selects between expressions: a kernel computes it between loads that it wants in
// flight together, and branches there would make it wait for them.  Row positions fit in
// 32 bits (the host checks y_row_len).
__host__ __device__ inline int y_pos(int nH, int bpatch, int x, int y, int z) {
  const int m = nH - 1;
  // per axis: inside the box (i), on its upper face (h); on the lower face otherwise
  const int ix = (x > 0) & (x < nH), iy = (y > 0) & (y < nH), iz = (z > 0) & (z < nH);
  const int hx = x == nH, hy = y == nH, hz = z == nH;
  const int nb = 3 - ix - iy - iz;   // axes on which the vertex lies on the box boundary
  // the segment's order: x fastest, then y, then z, over the axes inside the box
  const int dx = 1 + ix * (m - 1), dy = 1 + iy * (m - 1);
  const int local = ix * (x - 1) + dx * (iy * (y - 1) + dy * (iz * (z - 1)));
  const int r3 = (int)y_run16((int64_t)m * m * m), r2 = (int)y_run16((int64_t)m * m), r1 = (int)y_run16(m);
  // a face (nb = 1) by its normal axis and side: 2 axis + side
  const int f = (1 - ix) * hx + (1 - iy) * (2 + hy) + (1 - iz) * (4 + hz);
  // an edge (nb = 2) by the axis along it, then the sides of the other two, lower axis
  // first: 4 axis + 2 side1 + side2
  const int e = 4 * (iy + 2 * iz) + 2 * (ix * hy + (1 - ix) * hx) + (iz * hy + (1 - iz) * hz);
  const int base = (nb == 1) * (r3 + f * r2) + (nb == 2) * (r3 + 6 * r2 + e * r1);
  // no patch: the box corners, and every boundary vertex when those carry none
  const int none = (nb == 3) | ((nb > 0) & (bpatch == 0));
  const int pos = base + local;
  return pos + none * (r3 + 6 * r2 + 12 * r1 - pos);
}

// Patch chunk flag: the workgroup of pair p takes right-hand sides p .. p + 3 of p's
// problem, one per wave, when p's right-hand-side index is a multiple of 4 (else it
// does nothing); its segment has one group of 16 vertices.
constexpr int kChunkRhsWaves = 1 << 30;

// True when the kernels' compile-time table of the patches holding each subdomain
// boundary edge equals the host's boundary_patch_table().
bool boundary_patches_match(const std::vector<int>& tab);

template <typename T>
struct LevelPtrs {
  T* z;       // solution / correction
  T* r;       // residual scratch
  T* zi;      // interior solves (only interior-of-subdomain entries ever written)
  T* gg;      // condensed interface residual
  T* w;       // interface correction (only interface entries ever written)
  T* Y;       // vertex patch results, [npad][y_row_len(nH)] per pair (the small-level
              // kernel uses [npad][(nH+1)^3] in the same buffer)
  const T* ATinv;   // nI x nI per problem
  const T* Sinv;    // 27 x npad x npad per problem
  const T* XT;      // nI x nB per problem
};

int stencil_max_n();
int stencil_min_n(int count);   // the plane-marching kernel serves stencil_min_n(pairs) < n <= stencil_max_n()
int stencil_blocks(const Geom& g, int count);   // partial sums per pair of the dot mode
int stencil_max_blocks(const Geom& g);          // at most that many, whatever the launch shape
int stencil_variant_count(int elem, int mode, int n);   // launch variants the tuner may choose from
// the shape (variant index, planes per workgroup) a launch would take now (forced, tuned
// or from the cost model)
bool stencil_shape(int n, int elem, int mode, int count, int* variant, int* kz);
// groups of 16 vertices per wave in the patch kernel: more on large levels (fewer
// S^{-1} stagings), one on small levels (more workgroups)
// 16-vertex groups per wave of the patch kernel for a level with `groups` groups in all
// (summed over the segments and the pairs of a class): the fewest that let the whole grid
// be resident at once, given the workgroups per CU that the kernel's registers allow
// (6 in FP32 with buffer addressing, 3 in FP64 on a 256-CU MI355X), at most 8.
inline int64_t patch_resident_blocks(size_t elem) { return (elem == 4 ? 6 : 3) * 256; }
inline int patch_groups(int64_t groups, size_t elem) {
  const int64_t resident = patch_resident_blocks(elem) * 4;   // waves
  const int64_t g = (groups + resident - 1) / resident;
  return (int)std::max<int64_t>(1, std::min<int64_t>(8, g));
}

// Plane-marching operator kernel: mode 0 y = A x, 1 y = b - A x, 2 y = A x and partial
// sums of x . y per tile in part[pair * pstride + tile] (stencil_blocks(g, count) of
// them; with dot != nullptr a second small kernel reduces them into dot[pair *
// kScalStride]).  Returns hipErrorNotSupported (launching nothing) for a mode and size
// it does not serve.
template <typename T>
hipError_t launch_stencil(const T* x, const T* b, T* y, const Geom& g, const Bat& bt, int mode,
                          double* part, int64_t pstride, double* dot, hipStream_t st);

// y = A x (mode 0) or y = b - A x (mode 1); all entries of y in [0, n]^3 written.
template <typename T>
hipError_t launch_apply(const T* x, const T* b, T* y, const Geom& g, const Bat& bt, int mode,
                        hipStream_t st);

// gc = I_k^{k-1} rf (restriction, eq. F2C); all entries of gc written.
template <typename T>
hipError_t launch_restrict(const T* rf, T* gc, const Geom& f, const Geom& c, const Bat& bt,
                           hipStream_t st);

// zf += I_{k-1}^k ec (prolongation by natural injection) on interior edges.
template <typename T>
hipError_t launch_prolong_add(const T* ec, T* zf, const Geom& f, const Geom& c, const Bat& bt,
                              hipStream_t st);

// z (assign != 0: z =, else z +=) M_V^{-1} r  (vertex-based smoother, damping eta included).
template <typename T>
hipError_t launch_smooth(const T* r, T* z, const LevelPtrs<T>& L, const DSub& sub,
                         const Geom& g, const Bat& bt, double eta, int assign, hipStream_t st);

// The vertex patch products of the smoother alone (k_sm_patch): Y = S^{-1} gg per patch,
// on the level's current condensed residual (for timing the kernel in isolation).
template <typename T>
hipError_t launch_patch_products(const LevelPtrs<T>& L, const DSub& sub, const Geom& g, const Bat& bt,
                                 hipStream_t st);

// ---- the bottom of the V-cycle in one launch ---------------------------------------
// Levels 0 .. top (coarsest first) of one size class, described for the first pair and
// the first problem (pairs follow with the strides of the level vectors, of Y and of the
// factor blocks, as in the per-level launchers).
constexpr int kSmallMaxLevels = 8;

template <typename T>
struct SmallLevel {
  DGeom g;
  double h;
  int nH;                        // subdomains per axis (smoothed levels)
  int bpatch;                    // vertex spaces at boundary coarse vertices too
  T *z, *gv, *r, *zi, *gg, *w, *Y;
  T* G;                          // gathered patch inputs, vertex-major [NV][64]
  const T *ATinv, *Sinv, *XT;
  const int64_t* bofs;
  const int *lut, *slots;
  const T* A0inv;                // coarsest level
  const int64_t* map;
  int N0;
};

template <typename T>
struct SmallArgs {
  SmallLevel<T> lv[kSmallMaxLevels];
  int top;      // z_top = MG(top, g_top, 0, m) (Fig. 1), g_top and z_top in lv[top]
  int m;
  double eta;
};

// One workgroup per pair runs MG(top, g, 0, m) over the levels 0 .. top: smoothing,
// residuals, transfers and the exact coarsest solve, with workgroup barriers between the
// steps (one launch instead of a dozen per level; a single compute unit per pair is
// slower than the per-level launches on the sizes measured, so it is an option).
template <typename T>
hipError_t launch_vcycle_small(const SmallArgs<T>& a, const Bat& bt, hipStream_t st);

// z = A_0^{-1} g on the coarsest level (A0inv: N0 x N0 per problem).
template <typename T>
hipError_t launch_coarse(const T* g, T* z, const T* A0inv, const int64_t* map, int N0,
                         int64_t len, const Bat& bt, hipStream_t st);

// The V-cycle from one level down as a dense matrix per problem (MG(k, g, 0, m) is linear
// in g).  Build, per chunk of columns j0 .. j0 + K - 1 (K = bt.nrhs, pair = problem * K +
// column - j0): g = unit vectors, then the recursive V-cycle, then the results become
// columns of Bm (N x N per problem, row-major, over the unknowns listed in map).
constexpr int kDenseMaxN = 1176;   // the unknowns of an 8^3 level
template <typename T>
hipError_t launch_unit_cols(T* g, const int64_t* map, int N, int j0, int64_t len, const Bat& bt,
                            hipStream_t st);
template <typename T>
hipError_t launch_gather_cols(const T* z, T* Bm, const int64_t* map, int N, int j0, int64_t len, bool colmajor,
                              const Bat& bt, hipStream_t st);
// z = Bm g for every pair (Bm of problem pair / nrhs, stored transposed when colmajor:
// one thread per row, for classes of many problems); clear: zero all of z first (for
// output vectors whose non-unknown entries the caller may not have zeroed).
template <typename T>
hipError_t launch_dense_vcycle(const T* g, T* z, const T* Bm, const int64_t* map, int N, int64_t len,
                               const Bat& bt, bool clear, bool colmajor, hipStream_t st);

template <typename Tin, typename Tout>
hipError_t launch_convert(const Tin* in, Tout* out, int64_t len, const Bat& bt, hipStream_t st);

// ---- FP64 CG vector kernels with device-resident scalars ----------------------------
// Per pair: scalars at scal + pair * kScalStride, partial sums at part + pair * pstride.
constexpr int kRedBlocks = 512;    // partial sums per reduction per pair (single solve)
constexpr int kScalStride = 16;
// scalar slots of a pair
enum : int {
  kS_BB = 0,    // b . b
  kS_PQ = 1,    // p . A p
  kS_RR = 2,    // r . r
  kS_RZA = 3,   // r . z (even iterations)
  kS_ZQA = 4,   // z . q (flexible beta)
  kS_RZB = 5,   // r . z (odd iterations)
  kS_ZQB = 6,
  kS_TOL = 7,   // relative tolerance
  kS_REL = 8,   // ||r|| / ||b|| after the last iteration
  kS_CC = 9,    // curl-curl form
  kS_AL = 10,   // alpha of the last update, whose u += alpha p is still pending
  kS_PEND = 11, // 1 once an update has left its u += alpha p pending (the next direction
                // kernel applies it, or launch_cg_finish at the end of a solve)
};
// per-pair PCG state
enum : int { kPairRun = 0, kPairDone = 1, kPairBroken = 2 };

// Partial sums a . b (and a . c when c != nullptr) per block and pair at part[pair *
// pstride + blk] (a . c at + nparts), nparts = dot_parts(len, count); with out != nullptr
// a second small kernel also reduces them into out[pair*kScalStride + 0 (, 1)].  In the
// CG iteration the next kernel reduces the partials itself (every block in the same
// order, so all get the same value) instead of a separate launch.
template <typename TA>
hipError_t launch_dot(const TA* a, const double* b, const double* c, double* part, int64_t pstride,
                      double* out, int64_t len, const Bat& bt, hipStream_t st);
int dot_parts(int64_t len, int count);
// per pair: out[pair*kScalStride + o] = sum of nparts partials (o < nout)
hipError_t launch_final(const double* part, int nparts, int64_t pstride, int nout, double* out,
                        const Bat& bt, hipStream_t st);
// pq = sum of the pq_n partials pq_part[pair * pstride + ..] (kept in s[kS_PQ]);
// alpha = s[i_num] / pq; u += alpha p; r -= alpha q; partial sums of r . r at
// part[pair * pstride + blk] (dot_parts(len, count) of them); r32 (may be null) receives
// r in FP32
// With u == nullptr the u += a p of this update is left pending: a is kept in s[kS_AL]
// and s[kS_PEND] = 1, and the next direction kernel (or launch_cg_finish) applies it
// while it reads p anyway, which saves the update one vector read.
hipError_t launch_cg_update(double* u, double* r, const double* p, const double* q, double* scal,
                            int i_num, const double* pq_part, int pq_n, float* r32, double* part,
                            int64_t pstride, int64_t len, const Bat& bt, hipStream_t st);
// rz (and zq when flexible) = sums of the dot partials (kept in s[i_num], s[i_zq]);
// beta = rz / s[i_den] (flexible: beta = -(s[i_an] / s[i_ad]) zq / s[i_den]); with
// u != nullptr first the pending u += s[kS_AL] p (old p), then p = z + beta p
template <typename TZ>
hipError_t launch_cg_direction(double* p, const TZ* z, double* u, double* scal, int i_num, int i_den,
                               int flexible, int i_zq, int i_an, int i_ad, const double* dot_part, int dot_n,
                               int64_t pstride, int64_t len, const Bat& bt, hipStream_t st);
// u += s[kS_AL] p for every pair of bt whose update is pending (s[kS_PEND] != 0), then
// s[kS_PEND] = 0: the end of a solve.
hipError_t launch_cg_finish(double* u, const double* p, double* scal, int64_t len, const Bat& bt, hipStream_t st);
// Start of a solve: s[kS_TOL] = rtol, iters = 0; pairs with b = 0 are done, pairs with a
// non-finite b . b broken, all others active.
hipError_t launch_pcg_init(double* scal, int* act, int* iters, int* status, int count, double rtol,
                           hipStream_t st);
// End of an iteration, per active pair: s[kS_RR] = sum of the update's rr_n partials;
// (s[i_rz], s[kS_PQ]) recorded at hist[pair][iters] while iters < kHistCap; iters += 1;
// broken if s[kS_PQ] <= 0 or a scalar is not finite; done if ||r|| / ||b|| <= rtol
// (s[kS_REL] = that ratio).  *nact = pairs still active.
constexpr int kHistCap = 512;
hipError_t launch_pcg_check(double* scal, int* act, int* iters, int* status, int count, int i_rz,
                            int* nact, const double* rr_part, int rr_n, int64_t pstride, double* hist,
                            hipStream_t st);
hipError_t launch_copy(const double* x, double* y, int64_t len, const Bat& bt, hipStream_t st);
hipError_t launch_zero(double* y, int64_t len, const Bat& bt, hipStream_t st);
// y = c0 x0 + c1 x1 + c2 x2 entrywise for every pair (x1, x2 may be null; y may alias them)
hipError_t launch_lincomb(double* y, const double* x0, double c0, const double* x1, double c1, const double* x2,
                          double c2, int64_t len, const Bat& bt, hipStream_t st);

// b = load vector of f sampled at the 2x2x2 Gauss points (single problem).
hipError_t launch_assemble_rhs(const double* f, double* b, const Geom& g, hipStream_t st, const double* coef = nullptr,
                               int coef_r = 0);

// out[0] = lam . (K u) for one pair of vectors (single problem), K = dA/dalpha.
hipError_t launch_curlcurl_form(const double* lam, const double* u, const Geom& g,
                                double* part, double* out, hipStream_t st, const double* coef = nullptr, int coef_r = 0);

}  // namespace ndmg
