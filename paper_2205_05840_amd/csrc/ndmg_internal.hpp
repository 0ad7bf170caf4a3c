// Internal declarations of the ndmg library (not part of the C ABI).
#pragma once

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
  std::vector<double> S27;     // same layout, the Schur complements themselves
};

// Build the factors for a level (h, alpha, s).  Returns false and sets err on failure.
bool build_level_factors(double h, double alpha, const SubInfo& sub, bool boundary_patches,
                         LevelFactors* out, std::string* err);

// Padded-layout offsets of the interior edges (the unknowns) of a level, direction-major
// and then in layout order.
std::vector<int64_t> unknown_offsets(const Geom& g);

// Coarsest level: dense inverse of A_0 over its unknowns and the padded offset of each
// (the order of unknown_offsets).
bool build_coarse(const Geom& g, double alpha, std::vector<double>* A0inv,
                  std::vector<int64_t>* map, std::string* err);

// 12 x 12 element matrix alpha K_T + M_T of a cube of side h (local edge order 4 d + a + 2 b).
void element_matrix(double h, double alpha, double curl_scale, double* out144);

// Dense SPD inverse via Cholesky, in place (row-major n x n).  False if not SPD.
bool spd_inverse(std::vector<double>& A, int n);

}  // namespace ndmg
