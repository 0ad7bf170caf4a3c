// Internal declarations of the ndmg library (not part of the C ABI).
#pragma once

#include <array>
#include <climits>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ndmg.h"

namespace ndmg {

// Geometry of one level in the padded edge layout (see ndmg.h).
struct Geom {
  int n;           // cells per axis
  int P;           // row pitch (elements)
  int64_t plane;   // (n + 1) * P
  int64_t B;       // (n + 1) * plane: one direction block
  int64_t len;     // 3 * B
  double h;        // cell size
};

Geom make_geom(int n, double length);

// Subdomain bookkeeping of a smoothed level (s x s x s fine cells per subdomain).
struct SubInfo {
  int s;           // subdomain size
  int nH;          // subdomains per axis
  int nI;          // interior unknowns per subdomain, 3 s (s-1)^2
  int nG;          // interface slots of an interior vertex patch, 6 s (4 s - 3)
  int npad;        // nG rounded up to a multiple of 16
  int lut_w;       // 2 s + 1: width of the slot lookup table per axis
};

SubInfo make_sub(int s, int n);

// One interface slot of a vertex patch: direction and (x, y, z) offset of the edge's
// (cell or node) indices from the vertex's fine node.
struct Slot {
  int d, dx, dy, dz;
};

// Slots of an interior vertex patch in their fixed order: direction, then z, y, x
// offsets lexicographically (x fastest).
std::vector<Slot> vertex_slots(int s);

// Slot lookup: index [d][dx + s][dy + s][dz + s] (width 2 s + 1) -> slot or -1.
std::vector<int> slot_lookup(int s);

// Interior unknowns of a subdomain in their fixed order: direction, then z, y, x
// (x fastest); offsets from the subdomain's lower fine node.
std::vector<Slot> interior_dofs(int s);

// Edges on the boundary of a subdomain (cell offset in [0, s) along the direction,
// node offsets in [0, s] across, not interior), same ordering: 3 (s+1)^2 s - nI of them.
std::vector<Slot> boundary_dofs(int s);

// For each boundary dof of a subdomain (order of boundary_dofs) the vertex patches that
// hold it, as the sum of the interface correction w = sum_V R_V^T y_V takes them: four
// codes per dof, corner + 8 slot (corner = cx + 2 cy + 4 cz of the subdomain's corners,
// slot in the patch order of vertex_slots), -1 where there are fewer than four; bit 30
// marks dofs the subdomain owns (local offsets all in {0, 1}: each interface unknown is
// owned by exactly one subdomain, the one at floor(o / 2)).  Subdomain size 2 only.
std::vector<int> boundary_patch_table();

// Segment of vertices sharing a patch type: a box of the vertex grid (0..nH)^3.
struct Segment {
  int type;        // tx + 3 ty + 9 tz, t = 0 low face, 1 inside, 2 high face
  int lo[3];
  int dims[3];
  int count;
};

std::vector<Segment> vertex_segments(int nH, bool boundary_patches);

// Host FP64 factors of one smoothed level.
struct LevelFactors {
  std::vector<double> ATinv;   // nI x nI
  std::vector<double> XT;      // nI x nB: A_T^{-1} A_{I, boundary of T}
  std::vector<double> Sinv;    // 27 x npad x npad (zero for absent types/slots)
};

// Build the factors for a level (h, alpha, s).  Returns false and sets err on failure.
bool build_level_factors(double h, double alpha, const SubInfo& sub, bool boundary_patches,
                         LevelFactors* out, std::string* err);
// The same, cast to T and written straight into the caller's arrays (nI x nI, nI x nB,
// 27 x npad x npad); entries of absent patch types and slots are not written, so Sinv
// must hold zeros there.  The local matrices of each (s, boundary choice) are assembled
// once per process with h and alpha factored out.
template <typename T>
bool build_level_factors_into(double h, double alpha, const SubInfo& sub, bool boundary_patches, T* ATinv,
                              T* XT, T* Sinv, std::string* err);

// Interface slots of the edge space of a coarse edge along axis a (Sec. 3.2.1), offsets
// from the edge's first node (a multiple of s per axis): s (4 s - 3) edges along a, then
// 2 s (s - 1) along each of the two other axes; s + 8 s (s - 1) in all.
std::vector<Slot> edge_slots(int s, int a);

// A_T^{-1} of an s x s x s subdomain (nI x nI, order of interior_dofs) and X_T =
// A_T^{-1} A_{I, dT} (nI x nB, columns in the order of boundary_dofs).
bool subdomain_factors(int s, double h, double alpha, std::vector<double>* ATinv, std::vector<double>* XT,
                       std::string* err);

// Inverse Schur complement of one patch (eq. AVDef / AEDef in the discrete-harmonic basis):
// cells are the fine cells of the patch (offsets from its anchor node), slots its
// interface edges, t[ax] = 0 / 2 where the anchor lies on the low / high boundary plane
// of axis ax (edges in such a plane through the anchor carry no unknown), 1 otherwise.
// out (npad x npad, row-major) receives S^{-1} on the present slots and zeros elsewhere;
// present[j] = 1 for the slots that hold an unknown.  cell_alpha, if given, holds each
// cell's own alpha (in the order of cells) in place of the common alpha; present_in, if
// given, names the present slots (a patch cut by the boundary of a non-box domain).
bool patch_inverse(const std::vector<std::array<int, 3>>& cells, const std::vector<Slot>& slots,
                   const int t[3], int s, double h, double alpha, int npad, double* out,
                   std::vector<char>* present, std::string* err,
                   const std::vector<double>* cell_alpha = nullptr,
                   const std::vector<char>* present_in = nullptr);

// Patch types of the generic smoother.  kind 0 (vertex spaces): type = tx + 3 ty + 9 tz,
// t = 0 / 1 / 2 for a vertex on the low boundary plane / inside / on the high plane of
// that axis.  kind 1 (edge spaces): type = 9 a + tb + 3 tc for a coarse edge along axis
// a, (b, c) = (a + 1, a + 2) mod 3 the axes across it; t[a] = 1.
void patch_type_axes(int kind, int type, int t[3]);
// The fine cells of a patch of that type (offsets from its anchor node): the 8 (vertex)
// or 4 (edge) subdomains around the anchor that lie in the domain.
std::vector<std::array<int, 3>> patch_cells(int kind, int type, int s);
// Slots of a patch that hold an unknown: inside the patch's cells and not in a boundary
// plane through the anchor.
std::vector<char> patch_slots_present(const std::vector<std::array<int, 3>>& cells,
                                      const std::vector<Slot>& slots, const int t[3]);

// Relative offset of a slot without an unknown (the same value as the kernels' kGenAbsent).
constexpr int64_t kGenAbsentHost = INT64_MIN;

// Device tables of one level of the generic smoother (geometry only).
// A coefficient with jumps (Sec. 6): alpha(x) = alpha * v[(bz r + by) r + bx] on an
// r x r x r grid of boxes tiling the cube; r = 0: constant.
struct CoefBoxes {
  int r = 0;
  const double* v = nullptr;
  // factor of cell (x, y, z) of a level with n cells per axis (r divides n): 1 without
  // boxes, 0 outside the domain
  double at(int n, int x, int y, int z) const {
    if (x < 0 || y < 0 || z < 0 || x >= n || y >= n || z >= n) return 0.0;
    if (r == 0) return 1.0;
    const int w = n / r;
    return v[((size_t)(z / w) * r + (size_t)(y / w)) * r + (size_t)(x / w)];
  }
  // a box of factor 0 lies outside the domain (a non-box domain): the edge of direction d
  // at node (x, y, z) is an unknown only if its four cells lie in boxes of positive factor
  bool edge_in(int n, int d, int x, int y, int z) const {
    const int o[3] = {x, y, z};
    const int b = (d + 1) % 3, c = (d + 2) % 3;
    for (int db = 0; db < 2; ++db)
      for (int dc = 0; dc < 2; ++dc) {
        int q[3];
        q[d] = o[d];
        q[b] = o[b] - 1 + db;
        q[c] = o[c] - 1 + dc;
        if (!(at(n, q[0], q[1], q[2]) > 0.0)) return false;
      }
    return true;
  }
};

struct GenTables {
  int kind = 0, s = 2, ntypes = 27;
  // subdomain types: one per box of the coefficient (one without boxes), with its factor
  int ntypesI = 1;
  std::vector<double> boxI{1.0};
  // patch types with a coefficient: the geometric type (0 .. 26) of each, and the factors
  // of the 8 cells at offsets {-1, 0}^3 from the anchor node (x fastest; 0 outside the
  // domain or the patch), one per subdomain of the patch.  Without boxes the type is the
  // geometric type and these stay empty.
  std::vector<int> geomP;
  std::vector<std::array<double, 8>> keyP;
  int nI = 0, nB = 0;
  int npadI = 0, npadB = 0, npadE = 0, npadP = 0;
  std::vector<int64_t> unitsI;         // subdomain anchors, grouped by subdomain type
  std::vector<int64_t> relI;           // [ntypesI][npadI] interior offsets
  std::vector<int64_t> relE;           // [ntypesI][npadE] interior offsets, then boundary offsets
  std::vector<int> chunksI;            // [n][4]
  std::vector<int64_t> unitsP, relP;   // patch anchors; [ntypes][npadP] slot offsets
  std::vector<int> chunksP;
  std::vector<char> presentP;          // [ntypes][npadP]
  std::vector<int> typesP;             // the types that have patches
  std::vector<int> gamma;              // interface unknowns (offsets below 2^31)
  std::vector<int> ccodes;             // [ngam][4] subdomain terms (boundary slot * units + u)
  std::vector<int> codes;              // [ngam][4] patch results (slot * units + u)
};
bool build_gen_tables(const Geom& g, int s, int kind, bool boundary, GenTables* out, std::string* err,
                      const CoefBoxes& cf = CoefBoxes{});

// Padded-layout offsets of the interior edges (the unknowns) of a level, direction-major
// and then in layout order; with coefficient boxes only those inside the domain.
std::vector<int64_t> unknown_offsets(const Geom& g, const CoefBoxes& cf = CoefBoxes{});

// Coarsest level: dense inverse of A_0 over its unknowns and the padded offset of each
// (the order of unknown_offsets).
bool build_coarse(const Geom& g, double alpha, std::vector<double>* A0inv,
                  std::vector<int64_t>* map, std::string* err, const CoefBoxes& cf = CoefBoxes{});

// 12 x 12 element matrix alpha K_T + M_T of a cube of side h (local edge order 4 d + a + 2 b).
void element_matrix(double h, double alpha, double curl_scale, double* out144);

// Dense SPD inverse via Cholesky, in place (row-major n x n).  False if not SPD.
bool spd_inverse(std::vector<double>& A, int n);

}  // namespace ndmg
