// Host-side setup of the ndmg library: level geometry, the 12x12 Nedelec element
// matrices, local subdomain and vertex-patch matrices, and their FP64 inverses.
//
// Element matrices (Sec. 2): on a cube of side h the lowest-order Nedelec basis
// function of the x-edge at transverse offsets (a, b) is (psi_a(y) psi_b(z), 0, 0) in
// local coordinates, psi_0(t) = 1 - t, psi_1(t) = t.  Its mass matrix is h^3 times the
// tensor product of the 1-D hat mass [[1/3, 1/6], [1/6, 1/3]] over the two transverse
// axes.  The curl of the element field is a Raviart-Thomas face field whose flux through
// a face is h times the circulation of the edge values around it; the face mass along
// the face normal is the same 1-D matrix, so K_T = h C^T blockdiag(m, m, m) C with C the
// 6x12 circulation matrix.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <tuple>

#include "ndmg_internal.hpp"

namespace ndmg {

Geom make_geom(int n, double length) {
  Geom g;
  g.n = n;
  g.P = ((n + 1) + 7) / 8 * 8;
  g.plane = (int64_t)(n + 1) * g.P;
  g.B = (int64_t)(n + 1) * g.plane;
  g.len = 3 * g.B;
  g.h = length / n;
  return g;
}

SubInfo make_sub(int s, int n) {
  SubInfo si;
  si.s = s;
  si.nH = n / s;
  si.nI = 3 * s * (s - 1) * (s - 1);
  si.nG = 6 * s * (4 * s - 3);
  si.npad = (si.nG + 15) / 16 * 16;
  si.lut_w = 2 * s + 1;
  return si;
}

std::vector<Slot> vertex_slots(int s) {
  // For direction d with transverse axes (a, b): cell offset in [-s, s-1];
  // (off_a == 0 and |off_b| < s) or (off_b == 0 and 0 < |off_a| < s).
  std::vector<Slot> out;
  for (int d = 0; d < 3; ++d) {
    for (int dz = -s; dz <= s; ++dz)
      for (int dy = -s; dy <= s; ++dy)
        for (int dx = -s; dx <= s; ++dx) {
          int o[3] = {dx, dy, dz};
          if (o[d] < -s || o[d] > s - 1) continue;
          int a = (d + 1) % 3, b = (d + 2) % 3;
          int oa = o[a], ob = o[b];
          bool ok = (oa == 0 && std::abs(ob) < s) || (ob == 0 && oa != 0 && std::abs(oa) < s);
          if (ok) out.push_back({d, dx, dy, dz});
        }
  }
  return out;
}

std::vector<int> slot_lookup(int s) {
  int w = 2 * s + 1;
  std::vector<int> lut(3 * w * w * w, -1);
  auto slots = vertex_slots(s);
  for (size_t i = 0; i < slots.size(); ++i) {
    const Slot& q = slots[i];
    lut[((q.d * w + (q.dx + s)) * w + (q.dy + s)) * w + (q.dz + s)] = (int)i;
  }
  return lut;
}

std::vector<Slot> interior_dofs(int s) {
  std::vector<Slot> out;
  for (int d = 0; d < 3; ++d)
    for (int z = 0; z <= s; ++z)
      for (int y = 0; y <= s; ++y)
        for (int x = 0; x <= s; ++x) {
          int o[3] = {x, y, z};
          bool ok = true;
          for (int ax = 0; ax < 3; ++ax) {
            if (ax == d) ok &= (o[ax] >= 0 && o[ax] < s);
            else ok &= (o[ax] >= 1 && o[ax] <= s - 1);
          }
          if (ok) out.push_back({d, x, y, z});
        }
  return out;
}

std::vector<Slot> boundary_dofs(int s) {
  std::vector<Slot> out;
  for (int d = 0; d < 3; ++d)
    for (int z = 0; z <= s; ++z)
      for (int y = 0; y <= s; ++y)
        for (int x = 0; x <= s; ++x) {
          int o[3] = {x, y, z};
          bool edge = true, interior = true;
          for (int ax = 0; ax < 3; ++ax) {
            if (ax == d) edge &= (o[ax] >= 0 && o[ax] < s);
            else interior &= (o[ax] >= 1 && o[ax] <= s - 1);
          }
          if (edge && !interior) out.push_back({d, x, y, z});
        }
  return out;
}

std::vector<int> boundary_patch_table() {
  const std::vector<Slot> bd = boundary_dofs(2);
  const std::vector<int> lut = slot_lookup(2);
  std::vector<int> tab(bd.size() * 4, -1);
  for (size_t e = 0; e < bd.size(); ++e) {
    const int o[3] = {bd[e].dx, bd[e].dy, bd[e].dz};
    const int d = bd[e].d;
    int n = 0;
    // candidate vertices: two along the edge, and across each transverse axis one where
    // the offset is even (the edge lies on that plane) or two where it is odd
    for (int cz = 0; cz < 2; ++cz)
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
          const int c[3] = {cx, cy, cz};
          bool cand = true;
          for (int ax = 0; ax < 3; ++ax)
            if (ax != d && o[ax] % 2 == 0 && c[ax] != o[ax] / 2) cand = false;
          if (!cand) continue;
          const int rel[3] = {o[0] - 2 * cx, o[1] - 2 * cy, o[2] - 2 * cz};
          const int slot = lut[((d * 5 + rel[0] + 2) * 5 + rel[1] + 2) * 5 + rel[2] + 2];
          if (slot < 0) continue;
          if (n < 4) tab[e * 4 + n] = (cx + 2 * cy + 4 * cz) + 8 * slot;
          ++n;
        }
    if (o[0] <= 1 && o[1] <= 1 && o[2] <= 1) tab[e * 4] |= 1 << 30;
  }
  return tab;
}

std::vector<Segment> vertex_segments(int nH, bool boundary_patches) {
  std::vector<Segment> out;
  for (int tz = 0; tz < 3; ++tz)
    for (int ty = 0; ty < 3; ++ty)
      for (int tx = 0; tx < 3; ++tx) {
        int t[3] = {tx, ty, tz};
        int nb = (tx != 1) + (ty != 1) + (tz != 1);
        if (nb == 3) continue;                 // box corners: empty interface
        if (!boundary_patches && nb > 0) continue;
        Segment sg;
        sg.type = tx + 3 * ty + 9 * tz;
        sg.count = 1;
        for (int ax = 0; ax < 3; ++ax) {
          if (t[ax] == 0) { sg.lo[ax] = 0; sg.dims[ax] = 1; }
          else if (t[ax] == 2) { sg.lo[ax] = nH; sg.dims[ax] = 1; }
          else { sg.lo[ax] = 1; sg.dims[ax] = nH - 1; }
          sg.count *= sg.dims[ax];
        }
        if (sg.count > 0) out.push_back(sg);
      }
  return out;
}

// ---------------------------------------------------------------------------------
// Element matrix
// ---------------------------------------------------------------------------------
static inline int ledge(int d, int a, int b) { return 4 * d + a + 2 * b; }

void element_matrix(double h, double alpha, double curl_scale, double* E) {
  const double m[2][2] = {{1.0 / 3.0, 1.0 / 6.0}, {1.0 / 6.0, 1.0 / 3.0}};
  for (int i = 0; i < 144; ++i) E[i] = 0.0;
  // mass: per direction, tensor product over the transverse (a, b) offsets
  const double h3 = h * h * h;
  for (int d = 0; d < 3; ++d)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a)
        for (int b2 = 0; b2 < 2; ++b2)
          for (int a2 = 0; a2 < 2; ++a2)
            E[ledge(d, a, b) * 12 + ledge(d, a2, b2)] += h3 * m[a][a2] * m[b][b2];
  // circulation matrix C (6 faces x 12 edges): face of normal ax at local node f.
  // Right-hand rule around +ax with (p, q) the next two axes cyclically:
  //   + e_q(at p = 1) - e_q(at p = 0) - e_p(at q = 1) + e_p(at q = 0)
  // where e_q is the edge of direction q and e_p of direction p on that face.
  double C[6][12] = {{0}};
  for (int ax = 0; ax < 3; ++ax) {
    int p = (ax + 1) % 3, q = (ax + 2) % 3;
    for (int f = 0; f < 2; ++f) {
      // edge of direction dir (p or q) on this face, at node c along the third axis
      auto edge_at = [&](int dir, int c) {
        int o[3] = {0, 0, 0};
        o[ax] = f;
        o[3 - dir - ax] = c;
        int t0 = (dir == 0) ? 1 : 0;   // transverse axes of dir, ascending
        int t1 = (dir == 2) ? 1 : 2;
        return ledge(dir, o[t0], o[t1]);
      };
      int row = 2 * ax + f;
      C[row][edge_at(q, 1)] += 1.0;   // edge of direction q at p-node 1
      C[row][edge_at(q, 0)] -= 1.0;   // edge of direction q at p-node 0
      C[row][edge_at(p, 1)] -= 1.0;   // edge of direction p at q-node 1
      C[row][edge_at(p, 0)] += 1.0;   // edge of direction p at q-node 0
    }
  }
  const double kh = alpha * curl_scale * h;
  for (int ax = 0; ax < 3; ++ax)
    for (int f = 0; f < 2; ++f)
      for (int f2 = 0; f2 < 2; ++f2) {
        double w = kh * m[f][f2];
        const double* ci = C[2 * ax + f];
        const double* cj = C[2 * ax + f2];
        for (int i = 0; i < 12; ++i) {
          if (ci[i] == 0.0) continue;
          for (int j = 0; j < 12; ++j)
            if (cj[j] != 0.0) E[i * 12 + j] += w * ci[i] * cj[j];
        }
      }
}

// ---------------------------------------------------------------------------------
// Dense SPD inverse (Cholesky)
// ---------------------------------------------------------------------------------
bool spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> L(A);
  for (int j = 0; j < n; ++j) {
    double d = L[j * n + j];
    for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    L[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = L[i * n + j];
      for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = v / d;
    }
  }
  // inverse of L (lower), then A^{-1} = L^{-T} L^{-1}
  std::vector<double> Li(n * (size_t)n, 0.0);
  for (int j = 0; j < n; ++j) {
    Li[j * n + j] = 1.0 / L[j * n + j];
    for (int i = j + 1; i < n; ++i) {
      double v = 0.0;
      for (int k = j; k < i; ++k) v -= L[i * n + k] * Li[k * n + j];
      Li[i * n + j] = v / L[i * n + i];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      double v = 0.0;
      for (int k = i; k < n; ++k) v += Li[k * n + i] * Li[k * n + j];
      A[i * n + j] = v;
      A[j * n + i] = v;
    }
  return true;
}

// ---------------------------------------------------------------------------------
// Local assembly over a set of fine cells (relative integer coordinates)
// ---------------------------------------------------------------------------------
namespace {

using Key = std::tuple<int, int, int, int>;   // direction, x, y, z

struct LocalSystem {
  std::map<Key, int> index;
  std::vector<Key> keys;
  std::vector<double> A;   // dense, size N x N, filled after assembly
  int N = 0;
};

// Edge of direction d of the cell with lower corner c at transverse offsets (a, b).
Key cell_edge(const int c[3], int d, int a, int b) {
  int t0 = (d == 0) ? 1 : 0;
  int t1 = (d == 2) ? 1 : 2;
  int o[3] = {c[0], c[1], c[2]};
  o[t0] += a;
  o[t1] += b;
  return Key(d, o[0], o[1], o[2]);
}

// A_loc = sum over cells of alpha_T K_T + M_T, with alpha_T = cell_alpha[i] when given.
void assemble_cells(const std::vector<std::array<int, 3>>& cells, double h, double alpha,
                    LocalSystem* sys, const std::vector<double>* cell_alpha = nullptr) {
  for (auto& c : cells)
    for (int d = 0; d < 3; ++d)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          Key k = cell_edge(c.data(), d, a, b);
          if (!sys->index.count(k)) {
            sys->index[k] = (int)sys->keys.size();
            sys->keys.push_back(k);
          }
        }
  sys->N = (int)sys->keys.size();
  sys->A.assign((size_t)sys->N * sys->N, 0.0);
  double E[144];
  element_matrix(h, alpha, 1.0, E);
  double Ealpha = alpha;
  for (size_t ic = 0; ic < cells.size(); ++ic) {
    const auto& c = cells[ic];
    if (cell_alpha && (*cell_alpha)[ic] != Ealpha) {
      Ealpha = (*cell_alpha)[ic];
      element_matrix(h, Ealpha, 1.0, E);
    }
    int loc[12];
    for (int d = 0; d < 3; ++d)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) loc[ledge(d, a, b)] = sys->index[cell_edge(c.data(), d, a, b)];
    for (int i = 0; i < 12; ++i)
      for (int j = 0; j < 12; ++j) sys->A[(size_t)loc[i] * sys->N + loc[j]] += E[i * 12 + j];
  }
}

std::vector<double> submatrix(const LocalSystem& sys, const std::vector<int>& r,
                              const std::vector<int>& c) {
  std::vector<double> out(r.size() * c.size());
  for (size_t i = 0; i < r.size(); ++i)
    for (size_t j = 0; j < c.size(); ++j) out[i * c.size() + j] = sys.A[(size_t)r[i] * sys.N + c[j]];
  return out;
}

}  // namespace

namespace {

// The local matrices of one level, with h and alpha factored out: every element matrix
// is alpha h K1 + h^3 M1 (K1, M1 those of the unit cube), so each block below is
// assembled once per (s, boundary choice) from K1 and M1 and scaled per problem.
struct TypePattern {
  int nG = 0;                       // interface unknowns of the patch (0: no patch)
  std::vector<int> Gslot;           // slot of each
  std::vector<int> bstart;          // interior unknowns grouped by subdomain: block starts
  std::vector<double> KGG, MGG;     // nG x nG
  std::vector<double> KII, MII;     // per block b: nb x nb, stored one after another
  std::vector<double> KIG, MIG;     // per block b: nb x nG, stored one after another
};

struct LevelPattern {
  int nI = 0, nB = 0;
  std::vector<double> KII, MII, KIB, MIB;   // subdomain: nI x nI, nI x nB
  TypePattern type[27];
};

void split_km(const LocalSystem& a1, const LocalSystem& a0, const std::vector<int>& r, const std::vector<int>& c,
              std::vector<double>* K, std::vector<double>* M) {
  const std::vector<double> A1 = submatrix(a1, r, c), A0 = submatrix(a0, r, c);
  K->resize(A1.size());
  M->resize(A1.size());
  for (size_t i = 0; i < A1.size(); ++i) {
    (*M)[i] = A0[i];
    (*K)[i] = A1[i] - A0[i];
  }
}

LevelPattern make_pattern(int s, bool boundary_patches) {
  LevelPattern P;
  {
    std::vector<std::array<int, 3>> cells;
    for (int z = 0; z < s; ++z)
      for (int y = 0; y < s; ++y)
        for (int x = 0; x < s; ++x) cells.push_back({x, y, z});
    LocalSystem a1, a0;
    assemble_cells(cells, 1.0, 1.0, &a1);
    assemble_cells(cells, 1.0, 0.0, &a0);
    std::vector<int> I, Bd;
    for (auto& q : interior_dofs(s)) I.push_back(a1.index.at(Key(q.d, q.dx, q.dy, q.dz)));
    for (auto& q : boundary_dofs(s)) Bd.push_back(a1.index.at(Key(q.d, q.dx, q.dy, q.dz)));
    P.nI = (int)I.size();
    P.nB = (int)Bd.size();
    split_km(a1, a0, I, I, &P.KII, &P.MII);
    split_km(a1, a0, I, Bd, &P.KIB, &P.MIB);
  }
  const std::vector<Slot> slots = vertex_slots(s);
  for (int type = 0; type < 27; ++type) {
    const int t[3] = {type % 3, (type / 3) % 3, type / 9};
    const int nb = (t[0] != 1) + (t[1] != 1) + (t[2] != 1);
    if (nb == 3 || (!boundary_patches && nb > 0)) continue;
    int lo[3], hi[3];   // present cells [lo, hi) relative to the vertex node
    for (int ax = 0; ax < 3; ++ax) {
      lo[ax] = (t[ax] == 0) ? 0 : -s;
      hi[ax] = (t[ax] == 2) ? 0 : s;
    }
    std::vector<std::array<int, 3>> cells;
    for (int z = lo[2]; z < hi[2]; ++z)
      for (int y = lo[1]; y < hi[1]; ++y)
        for (int x = lo[0]; x < hi[0]; ++x) cells.push_back({x, y, z});
    LocalSystem a1, a0;
    assemble_cells(cells, 1.0, 1.0, &a1);
    assemble_cells(cells, 1.0, 0.0, &a0);
    // an edge is Dirichlet if it lies in a boundary plane (node coordinate 0 along a
    // boundary axis, for an axis other than its direction)
    auto dirichlet = [&](const Key& k) {
      const int d = std::get<0>(k);
      const int o[3] = {std::get<1>(k), std::get<2>(k), std::get<3>(k)};
      for (int ax = 0; ax < 3; ++ax)
        if (ax != d && t[ax] != 1 && o[ax] == 0) return true;
      return false;
    };
    auto inside_cells = [&](const Key& k) {
      const int d = std::get<0>(k);
      const int o[3] = {std::get<1>(k), std::get<2>(k), std::get<3>(k)};
      for (int ax = 0; ax < 3; ++ax) {
        if (ax == d) {
          if (o[ax] < lo[ax] || o[ax] >= hi[ax]) return false;
        } else if (o[ax] < lo[ax] || o[ax] > hi[ax]) {
          return false;
        }
      }
      return true;
    };
    TypePattern& T = P.type[type];
    std::vector<int> G;
    for (size_t si = 0; si < slots.size(); ++si) {
      const Key k(slots[si].d, slots[si].dx, slots[si].dy, slots[si].dz);
      if (!inside_cells(k) || dirichlet(k)) continue;
      G.push_back(a1.index.at(k));
      T.Gslot.push_back((int)si);
    }
    T.nG = (int)G.size();
    if (T.nG == 0) continue;
    // interior unknowns of the patch, grouped by subdomain (floor(o / s) across)
    std::map<std::array<int, 3>, std::vector<int>> blocks;
    for (int e = 0; e < a1.N; ++e) {
      const Key& k = a1.keys[e];
      const int d = std::get<0>(k);
      const int o[3] = {std::get<1>(k), std::get<2>(k), std::get<3>(k)};
      bool interior = true;
      for (int ax = 0; ax < 3; ++ax)
        if (ax != d && ((o[ax] % s) + s) % s == 0) interior = false;
      if (!interior || dirichlet(k)) continue;
      std::array<int, 3> blk;
      for (int ax = 0; ax < 3; ++ax) blk[ax] = (o[ax] - ((o[ax] % s) + s) % s) / s;
      blocks[blk].push_back(e);
    }
    split_km(a1, a0, G, G, &T.KGG, &T.MGG);
    T.bstart.push_back(0);
    for (auto& kv : blocks) {
      std::vector<double> K, M;
      split_km(a1, a0, kv.second, kv.second, &K, &M);
      T.KII.insert(T.KII.end(), K.begin(), K.end());
      T.MII.insert(T.MII.end(), M.begin(), M.end());
      split_km(a1, a0, kv.second, G, &K, &M);
      T.KIG.insert(T.KIG.end(), K.begin(), K.end());
      T.MIG.insert(T.MIG.end(), M.begin(), M.end());
      T.bstart.push_back(T.bstart.back() + (int)kv.second.size());
    }
  }
  return P;
}

// The pattern of (s, boundary choice), built on first use (thread-safe: static locals of
// the four possible keys are initialised once).
const LevelPattern& level_pattern(int s, bool boundary_patches) {
  if (s == 2) {
    if (boundary_patches) {
      static const LevelPattern p = make_pattern(2, true);
      return p;
    }
    static const LevelPattern p = make_pattern(2, false);
    return p;
  }
  if (boundary_patches) {
    static const LevelPattern p = make_pattern(4, true);
    return p;
  }
  static const LevelPattern p = make_pattern(4, false);
  return p;
}

// out = a K + b M elementwise
void combine(const double* K, const double* M, size_t n, double a, double b, double* out) {
  for (size_t i = 0; i < n; ++i) out[i] = a * K[i] + b * M[i];
}

}  // namespace

template <typename T>
bool build_level_factors_into(double h, double alpha, const SubInfo& sub, bool boundary_patches, T* ATinv_out,
                              T* XT_out, T* Sinv_out, std::string* err) {
  const int s = sub.s;
  if (s != 2 && s != 4) {
    *err = "subdomain size must be 2 or 4";
    return false;
  }
  const LevelPattern& P = level_pattern(s, boundary_patches);
  const double ka = alpha * h, mb = h * h * h;   // element matrices: alpha h K1 + h^3 M1
  // ---- subdomain interior ------------------------------------------------------------
  const int nI = P.nI, nB = P.nB;
  std::vector<double> ATinv((size_t)nI * nI);
  combine(P.KII.data(), P.MII.data(), P.KII.size(), ka, mb, ATinv.data());
  if (!spd_inverse(ATinv, nI)) {
    *err = "subdomain matrix A_T is not positive definite";
    return false;
  }
  // X_T = A_T^{-1} A_{I, dT}: maps the boundary values of T to (minus) the
  // discrete-harmonic extension into its interior
  std::vector<double> AIB((size_t)nI * nB), XT((size_t)nI * nB, 0.0);
  combine(P.KIB.data(), P.MIB.data(), AIB.size(), ka, mb, AIB.data());
  for (int i = 0; i < nI; ++i)
    for (int k = 0; k < nI; ++k) {
      const double a = ATinv[(size_t)i * nI + k];
      for (int j = 0; j < nB; ++j) XT[(size_t)i * nB + j] += a * AIB[(size_t)k * nB + j];
    }
  for (size_t i = 0; i < ATinv.size(); ++i) ATinv_out[i] = (T)ATinv[i];
  for (size_t i = 0; i < XT.size(); ++i) XT_out[i] = (T)XT[i];
  // ---- vertex patches, one per type: S = A_GG - sum over subdomain blocks of
  //      A_GI A_II^{-1} A_IG, then S^{-1}; entries of absent types and slots are left
  //      as they are (the caller's zeros) ------------------------------------------------
  const int np = sub.npad;
  std::vector<double> S, AII, AIG, X;
  for (int type = 0; type < 27; ++type) {
    const TypePattern& Tp = P.type[type];
    const int nG = Tp.nG;
    if (nG == 0) continue;
    S.resize((size_t)nG * nG);
    combine(Tp.KGG.data(), Tp.MGG.data(), S.size(), ka, mb, S.data());
    size_t oII = 0, oIG = 0;
    for (size_t b = 0; b + 1 < Tp.bstart.size(); ++b) {
      const int nb = Tp.bstart[b + 1] - Tp.bstart[b];
      AII.resize((size_t)nb * nb);
      AIG.resize((size_t)nb * nG);
      combine(Tp.KII.data() + oII, Tp.MII.data() + oII, AII.size(), ka, mb, AII.data());
      combine(Tp.KIG.data() + oIG, Tp.MIG.data() + oIG, AIG.size(), ka, mb, AIG.data());
      oII += AII.size();
      oIG += AIG.size();
      if (!spd_inverse(AII, nb)) {
        *err = "patch interior matrix is not positive definite";
        return false;
      }
      // X = A_II^{-1} A_IG, S -= A_IG^T X
      X.assign((size_t)nb * nG, 0.0);
      for (int i = 0; i < nb; ++i)
        for (int k = 0; k < nb; ++k) {
          const double a = AII[(size_t)i * nb + k];
          for (int j = 0; j < nG; ++j) X[(size_t)i * nG + j] += a * AIG[(size_t)k * nG + j];
        }
      for (int i = 0; i < nG; ++i)
        for (int k = 0; k < nb; ++k) {
          const double a = AIG[(size_t)k * nG + i];
          if (a == 0.0) continue;
          for (int j = 0; j < nG; ++j) S[(size_t)i * nG + j] -= a * X[(size_t)k * nG + j];
        }
    }
    for (int i = 0; i < nG; ++i)     // symmetrise against rounding
      for (int j = 0; j < i; ++j) {
        const double v = 0.5 * (S[(size_t)i * nG + j] + S[(size_t)j * nG + i]);
        S[(size_t)i * nG + j] = S[(size_t)j * nG + i] = v;
      }
    if (!spd_inverse(S, nG)) {
      *err = "vertex Schur complement is not positive definite";
      return false;
    }
    T* dst = Sinv_out + (size_t)type * np * np;
    for (int i = 0; i < nG; ++i)
      for (int j = 0; j < nG; ++j) dst[(size_t)Tp.Gslot[i] * np + Tp.Gslot[j]] = (T)S[(size_t)i * nG + j];
  }
  return true;
}

template bool build_level_factors_into<double>(double, double, const SubInfo&, bool, double*, double*, double*,
                                               std::string*);
template bool build_level_factors_into<float>(double, double, const SubInfo&, bool, float*, float*, float*,
                                              std::string*);

bool build_level_factors(double h, double alpha, const SubInfo& sub, bool boundary_patches,
                         LevelFactors* out, std::string* err) {
  const int nI = sub.nI;
  const int nB = 3 * (sub.s + 1) * (sub.s + 1) * sub.s - nI;
  out->ATinv.assign((size_t)nI * nI, 0.0);
  out->XT.assign((size_t)nI * nB, 0.0);
  out->Sinv.assign((size_t)27 * sub.npad * sub.npad, 0.0);
  return build_level_factors_into<double>(h, alpha, sub, boundary_patches, out->ATinv.data(), out->XT.data(),
                                          out->Sinv.data(), err);
}

// ---------------------------------------------------------------------------------
// Generic patches (any subdomain size; vertex and edge spaces)
// ---------------------------------------------------------------------------------
std::vector<Slot> edge_slots(int s, int a) {
  // Sec. 3.2.1, eq. (edge space): the fine edges on the coarse edge from the anchor node
  // to anchor + s e_a and in the interiors of the 4 coarse faces containing it.
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  std::vector<Slot> out;
  auto push = [&](int d, int oa, int ob, int oc) {
    int o[3];
    o[a] = oa;
    o[b] = ob;
    o[c] = oc;
    out.push_back({d, o[0], o[1], o[2]});
  };
  std::vector<std::pair<int, int>> pairs{{0, 0}};
  for (int t = 1; t < s; ++t) {
    pairs.push_back({t, 0});
    pairs.push_back({-t, 0});
    pairs.push_back({0, t});
    pairs.push_back({0, -t});
  }
  for (auto& pq : pairs)
    for (int ca = 0; ca < s; ++ca) push(a, ca, pq.first, pq.second);
  // edges across it: direction b in the face (a, b) at c-node 0, direction c in the
  // face (a, c) at b-node 0; node offsets 1 .. s-1 along a, cells -s .. s-1 across
  for (int na = 1; na < s; ++na)
    for (int cb = -s; cb < s; ++cb) push(b, na, cb, 0);
  for (int na = 1; na < s; ++na)
    for (int cc = -s; cc < s; ++cc) push(c, na, 0, cc);
  return out;
}

bool subdomain_factors(int s, double h, double alpha, std::vector<double>* ATinv, std::vector<double>* XT,
                       std::string* err) {
  std::vector<std::array<int, 3>> cells;
  for (int z = 0; z < s; ++z)
    for (int y = 0; y < s; ++y)
      for (int x = 0; x < s; ++x) cells.push_back({x, y, z});
  LocalSystem sys;
  assemble_cells(cells, h, alpha, &sys);
  std::vector<int> I, Bd;
  for (auto& q : interior_dofs(s)) I.push_back(sys.index.at(Key(q.d, q.dx, q.dy, q.dz)));
  for (auto& q : boundary_dofs(s)) Bd.push_back(sys.index.at(Key(q.d, q.dx, q.dy, q.dz)));
  *ATinv = submatrix(sys, I, I);
  const int nI = (int)I.size(), nB = (int)Bd.size();
  if (!spd_inverse(*ATinv, nI)) {
    *err = "subdomain matrix A_T is not positive definite";
    return false;
  }
  const std::vector<double> AIB = submatrix(sys, I, Bd);
  XT->assign((size_t)nI * nB, 0.0);
  for (int i = 0; i < nI; ++i)
    for (int k = 0; k < nI; ++k) {
      const double a = (*ATinv)[(size_t)i * nI + k];
      for (int j = 0; j < nB; ++j) (*XT)[(size_t)i * nB + j] += a * AIB[(size_t)k * nB + j];
    }
  return true;
}

namespace {

// An edge (direction d, offsets o from the anchor) lies on the boundary of the domain if
// it is in a boundary plane through the anchor: node offset 0 along an axis on which the
// anchor lies on the boundary (t[ax] != 1).
bool in_boundary_plane(const int t[3], int d, const int o[3]) {
  for (int ax = 0; ax < 3; ++ax)
    if (ax != d && t[ax] != 1 && o[ax] == 0) return true;
  return false;
}

}  // namespace

std::vector<char> patch_slots_present(const std::vector<std::array<int, 3>>& cells,
                                      const std::vector<Slot>& slots, const int t[3]) {
  int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
  for (auto& c : cells)
    for (int ax = 0; ax < 3; ++ax) {
      lo[ax] = std::min(lo[ax], c[ax]);
      hi[ax] = std::max(hi[ax], c[ax] + 1);
    }
  std::vector<char> present(slots.size(), 0);
  for (size_t j = 0; j < slots.size(); ++j) {
    const int d = slots[j].d;
    const int o[3] = {slots[j].dx, slots[j].dy, slots[j].dz};
    bool in = true;
    for (int ax = 0; ax < 3; ++ax) {
      if (ax == d) in &= (o[ax] >= lo[ax] && o[ax] < hi[ax]);
      else in &= (o[ax] >= lo[ax] && o[ax] <= hi[ax]);
    }
    present[j] = in && !in_boundary_plane(t, d, o);
  }
  return present;
}

std::vector<std::array<int, 3>> patch_cells(int kind, int type, int s) {
  int t[3];
  patch_type_axes(kind, type, t);
  int lo[3], hi[3];
  const int a = type / 9;   // the edge's axis (edge patches)
  for (int ax = 0; ax < 3; ++ax) {
    if (kind == 1 && ax == a) {
      lo[ax] = 0;
      hi[ax] = s;
    } else {
      lo[ax] = (t[ax] == 0) ? 0 : -s;
      hi[ax] = (t[ax] == 2) ? 0 : s;
    }
  }
  std::vector<std::array<int, 3>> cells;
  for (int z = lo[2]; z < hi[2]; ++z)
    for (int y = lo[1]; y < hi[1]; ++y)
      for (int x = lo[0]; x < hi[0]; ++x) cells.push_back({x, y, z});
  return cells;
}

void patch_type_axes(int kind, int type, int t[3]) {
  if (kind == 0) {
    t[0] = type % 3;
    t[1] = (type / 3) % 3;
    t[2] = type / 9;
  } else {
    const int a = type / 9, b = (a + 1) % 3, c = (a + 2) % 3;
    t[a] = 1;
    t[b] = type % 3;
    t[c] = (type / 3) % 3;
  }
}

bool patch_inverse(const std::vector<std::array<int, 3>>& cells, const std::vector<Slot>& slots,
                   const int t[3], int s, double h, double alpha, int npad, double* out,
                   std::vector<char>* present, std::string* err, const std::vector<double>* cell_alpha,
                   const std::vector<char>* present_in) {
  LocalSystem sys;
  assemble_cells(cells, h, alpha, &sys, cell_alpha);
  auto dirichlet = [&](int d, const int o[3]) { return in_boundary_plane(t, d, o); };
  if (present_in)
    *present = *present_in;
  else
    *present = patch_slots_present(cells, slots, t);
  std::vector<int> G, Gslot;
  for (size_t j = 0; j < slots.size(); ++j) {
    if (!(*present)[j]) continue;
    G.push_back(sys.index.at(Key(slots[j].d, slots[j].dx, slots[j].dy, slots[j].dz)));
    Gslot.push_back((int)j);
  }
  for (int i = 0; i < npad * npad; ++i) out[i] = 0.0;
  if (G.empty()) return true;
  // interior unknowns of the subdomains in the patch, grouped by subdomain: A_II is block
  // diagonal over subdomains (each block A_T of its subdomain's alpha)
  std::map<std::array<int, 3>, std::vector<int>> blocks;
  for (int e = 0; e < sys.N; ++e) {
    const Key& k = sys.keys[e];
    const int d = std::get<0>(k);
    const int o[3] = {std::get<1>(k), std::get<2>(k), std::get<3>(k)};
    bool interior = true;
    for (int ax = 0; ax < 3; ++ax)
      if (ax != d && ((o[ax] % s) + s) % s == 0) interior = false;
    if (!interior || dirichlet(d, o)) continue;
    std::array<int, 3> blk;
    for (int ax = 0; ax < 3; ++ax) blk[ax] = (o[ax] - ((o[ax] % s) + s) % s) / s;   // floor(o / s)
    blocks[blk].push_back(e);
  }
  const int nG = (int)G.size();
  std::vector<double> S = submatrix(sys, G, G);
  for (auto& kv : blocks) {
    const std::vector<int>& I = kv.second;
    const int nI = (int)I.size();
    std::vector<double> AII = submatrix(sys, I, I);
    if (!spd_inverse(AII, nI)) {
      *err = "patch interior block is not positive definite";
      return false;
    }
    std::vector<double> AIG = submatrix(sys, I, G);
    std::vector<double> X((size_t)nI * nG, 0.0);   // A_II^{-1} A_IG
    for (int i = 0; i < nI; ++i)
      for (int k = 0; k < nI; ++k) {
        const double a = AII[(size_t)i * nI + k];
        for (int j = 0; j < nG; ++j) X[(size_t)i * nG + j] += a * AIG[(size_t)k * nG + j];
      }
    for (int i = 0; i < nG; ++i)
      for (int k = 0; k < nI; ++k) {
        const double a = AIG[(size_t)k * nG + i];
        if (a == 0.0) continue;
        for (int j = 0; j < nG; ++j) S[(size_t)i * nG + j] -= a * X[(size_t)k * nG + j];
      }
  }
  for (int i = 0; i < nG; ++i)
    for (int j = 0; j < i; ++j) {
      const double v = 0.5 * (S[(size_t)i * nG + j] + S[(size_t)j * nG + i]);
      S[(size_t)i * nG + j] = S[(size_t)j * nG + i] = v;
    }
  if (!spd_inverse(S, nG)) {
    *err = "patch Schur complement is not positive definite";
    return false;
  }
  for (int i = 0; i < nG; ++i)
    for (int j = 0; j < nG; ++j) out[(size_t)Gslot[i] * npad + Gslot[j]] = S[(size_t)i * nG + j];
  return true;
}

bool build_gen_tables(const Geom& g, int s, int kind, bool boundary, GenTables* out, std::string* err,
                      const CoefBoxes& cf) {
  const int n = g.n, nH = n / s;
  const bool jumps = cf.r > 0;
  if (jumps && (n % cf.r || (n / cf.r) % s)) {
    *err = "every subdomain must lie in one box of the coefficient: n_k / r must be a multiple of the "
           "subdomain size on every smoothed level";
    return false;
  }
  GenTables& tb = *out;
  tb = GenTables{};
  tb.kind = kind;
  tb.s = s;
  tb.ntypes = 27;
  const std::vector<Slot> idofs = interior_dofs(s), bdofs = boundary_dofs(s);
  tb.nI = (int)idofs.size();
  tb.nB = (int)bdofs.size();
  tb.npadI = (tb.nI + 15) / 16 * 16;
  tb.npadB = (tb.nB + 15) / 16 * 16;
  tb.npadE = (tb.nI + tb.nB + 15) / 16 * 16;
  auto rel_of = [&](const Slot& q) { return q.d * g.B + (int64_t)q.dz * g.plane + (int64_t)q.dy * g.P + q.dx; };
  auto anchor = [&](int x, int y, int z) { return (int64_t)z * g.plane + (int64_t)y * g.P + x; };
  // subdomains: one type per box of the coefficient (one type without boxes); every
  // boundary edge of a subdomain lies in [0, n] (those on the boundary of the domain are
  // zero in every vector read there)
  tb.ntypesI = jumps ? cf.r * cf.r * cf.r : 1;
  tb.boxI.assign(tb.ntypesI, 1.0);
  if (jumps)
    for (int b = 0; b < tb.ntypesI; ++b) tb.boxI[b] = cf.v[b];
  tb.relI.assign((size_t)tb.ntypesI * tb.npadI, kGenAbsentHost);
  tb.relE.assign((size_t)tb.ntypesI * tb.npadE, kGenAbsentHost);
  for (int t = 0; t < tb.ntypesI; ++t) {
    for (int j = 0; j < tb.nI; ++j)
      tb.relI[(size_t)t * tb.npadI + j] = tb.relE[(size_t)t * tb.npadE + j] = rel_of(idofs[j]);
    for (int j = 0; j < tb.nB; ++j) tb.relE[(size_t)t * tb.npadE + tb.nI + j] = rel_of(bdofs[j]);
  }
  {
    std::vector<std::vector<int64_t>> byType(tb.ntypesI);
    const int w = jumps ? n / cf.r : n;
    for (int c = 0; c < nH; ++c)
      for (int b = 0; b < nH; ++b)
        for (int a = 0; a < nH; ++a) {
          const int t = jumps ? ((s * c / w) * cf.r + s * b / w) * cf.r + s * a / w : 0;
          if (jumps && !(cf.v[t] > 0.0)) continue;   // a box outside the domain
          byType[t].push_back(anchor(s * a, s * b, s * c));
        }
    for (int t = 0; t < tb.ntypesI; ++t) {
      const size_t first = tb.unitsI.size();
      tb.unitsI.insert(tb.unitsI.end(), byType[t].begin(), byType[t].end());
      for (size_t u = first; u < tb.unitsI.size(); u += 64) {
        tb.chunksI.push_back(t);
        tb.chunksI.push_back((int)u);
        tb.chunksI.push_back((int)std::min<size_t>(64, tb.unitsI.size() - u));
        tb.chunksI.push_back(0);
      }
    }
  }
  // patches, grouped by type
  const int nslots = kind == 0 ? 6 * s * (4 * s - 3) : s + 8 * s * (s - 1);
  tb.npadP = (nslots + 15) / 16 * 16;
  auto positions = [&](int t, int cells_axis, std::vector<int>* pos) {
    // coarse coordinates of the given type along one axis: node axes 0 / inside / nH,
    // the edge's own axis its cells 0 .. nH - 1
    pos->clear();
    if (cells_axis) {
      for (int i = 0; i < nH; ++i) pos->push_back(i);
    } else if (t == 0) {
      pos->push_back(0);
    } else if (t == 2) {
      pos->push_back(nH);
    } else {
      for (int i = 1; i < nH; ++i) pos->push_back(i);
    }
  };
  // per geometric type: present slots and their offsets; the anchors of each type
  std::vector<std::vector<char>> gpres(27);
  std::vector<std::vector<int64_t>> grel(27);
  std::vector<std::vector<int64_t>> byType;     // anchors per type
  std::map<std::pair<int, std::array<double, 8>>, int> keyIndex;
  std::vector<std::vector<char>> presByType;   // with boxes: slots present per type
  std::vector<char> hasSlots;
  if (!jumps) byType.assign(27, {});
  for (int type = 0; type < 27; ++type) {
    int t[3];
    patch_type_axes(kind, type, t);
    const int nb = (t[0] != 1) + (t[1] != 1) + (t[2] != 1);
    if (kind == 0 && nb == 3) continue;       // box corners: no interface unknowns
    if (kind == 1 && nb == 2) continue;       // coarse edges on the box's edges: none either
    if (!boundary && nb > 0) continue;
    const std::vector<Slot> slots = kind == 0 ? vertex_slots(s) : edge_slots(s, type / 9);
    if ((int)slots.size() != nslots) {
      *err = "internal: slot count";
      return false;
    }
    const std::vector<char> pres = patch_slots_present(patch_cells(kind, type, s), slots, t);
    bool any = false;
    gpres[type].assign(tb.npadP, 0);
    grel[type].assign(tb.npadP, kGenAbsentHost);
    for (int j = 0; j < nslots; ++j) {
      gpres[type][j] = pres[j];
      if (pres[j]) {
        grel[type][j] = rel_of(slots[j]);
        any = true;
      }
    }
    if (!any) continue;
    std::vector<int> px, py, pz;
    const int a = type / 9;
    positions(t[0], kind == 1 && a == 0, &px);
    positions(t[1], kind == 1 && a == 1, &py);
    positions(t[2], kind == 1 && a == 2, &pz);
    for (int z : pz)
      for (int y : py)
        for (int x : px) {
          if (!jumps) {
            byType[type].push_back(anchor(s * x, s * y, s * z));
            continue;
          }
          // the patch's subdomains by their cells next to the anchor; for an edge patch
          // only those on the edge's side of the anchor along its axis
          std::array<double, 8> key;
          for (int o = 0; o < 8; ++o) {
            const int oc[3] = {(o & 1) - 1, ((o >> 1) & 1) - 1, ((o >> 2) & 1) - 1};
            key[o] = (kind == 1 && oc[a] < 0) ? 0.0 : cf.at(n, s * x + oc[0], s * y + oc[1], s * z + oc[2]);
          }
          const auto k = std::make_pair(type, key);
          auto it = keyIndex.find(k);
          if (it == keyIndex.end()) {
            // slots present: those of the geometric type whose edge lies in the domain
            // (the same for every patch of the key: the edge's cells are the patch's)
            std::vector<char> pres(tb.npadP, 0);
            bool anyp = false;
            for (int j = 0; j < nslots; ++j) {
              const Slot& q = slots[j];
              pres[j] = gpres[type][j] && cf.edge_in(n, q.d, s * x + q.dx, s * y + q.dy, s * z + q.dz);
              anyp = anyp || pres[j];
            }
            it = keyIndex.emplace(k, (int)tb.geomP.size()).first;
            tb.geomP.push_back(type);
            tb.keyP.push_back(key);
            presByType.push_back(pres);
            byType.emplace_back();
            hasSlots.push_back(anyp);
          }
          if (hasSlots[it->second]) byType[it->second].push_back(anchor(s * x, s * y, s * z));
        }
  }
  tb.ntypes = jumps ? (int)tb.geomP.size() : 27;
  tb.relP.assign((size_t)tb.ntypes * tb.npadP, kGenAbsentHost);
  tb.presentP.assign((size_t)tb.ntypes * tb.npadP, 0);
  for (int ti = 0; ti < tb.ntypes; ++ti) {
    const int geom = jumps ? tb.geomP[ti] : ti;
    if (byType[ti].empty() || gpres[geom].empty()) continue;
    for (int j = 0; j < tb.npadP; ++j) {
      const char pr = jumps ? presByType[ti][j] : gpres[geom][j];
      tb.relP[(size_t)ti * tb.npadP + j] = pr ? grel[geom][j] : kGenAbsentHost;
      tb.presentP[(size_t)ti * tb.npadP + j] = pr;
    }
    const size_t first = tb.unitsP.size();
    tb.unitsP.insert(tb.unitsP.end(), byType[ti].begin(), byType[ti].end());
    tb.typesP.push_back(ti);
    for (size_t u = first; u < tb.unitsP.size(); u += 64) {
      tb.chunksP.push_back(ti);
      tb.chunksP.push_back((int)u);
      tb.chunksP.push_back((int)std::min<size_t>(64, tb.unitsP.size() - u));
      tb.chunksP.push_back(0);
    }
  }
  if ((int64_t)tb.unitsP.size() * tb.npadP >= (int64_t)1 << 31) {
    *err = "level too large for the patch result indices";
    return false;
  }
  // interface unknowns (not inside a subdomain), grouped by blocks of 16^3 nodes (layout
  // order inside a block), and the patch results summed on each, in the order of the
  // patches.  The kernels that pull per unknown then find the patch results and
  // subdomain terms of one block in cache: a patch's row of results is consumed by
  // unknowns of at most a few neighbouring blocks.  (The order of each unknown's own sum
  // does not depend on this order.)
  std::vector<int> gpos((size_t)g.len, -1);
  if (g.len >= (int64_t)1 << 31) {
    *err = "level too large for the interface offsets";
    return false;
  }
  {
    constexpr int kBlk = 16;
    const int nbk = (g.n + 1 + kBlk - 1) / kBlk;
    std::vector<int64_t> list;
    std::vector<int> blk;
    for (int64_t e : unknown_offsets(g, cf)) {
      const int d = (int)(e / g.B);
      int64_t r = e - d * g.B;
      const int z = (int)(r / g.plane);
      r -= (int64_t)z * g.plane;
      const int y = (int)(r / g.P), x = (int)(r - (int64_t)y * g.P);
      const int o[3] = {x, y, z};
      bool interior = true;
      for (int ax = 0; ax < 3; ++ax)
        if (ax != d && o[ax] % s == 0) interior = false;
      if (interior) continue;
      list.push_back(e);
      blk.push_back(((z / kBlk) * nbk + y / kBlk) * nbk + x / kBlk);
    }
    // stable counting sort by block
    std::vector<int64_t> start((size_t)nbk * nbk * nbk + 1, 0);
    for (int b : blk) ++start[(size_t)b + 1];
    for (size_t b = 1; b < start.size(); ++b) start[b] += start[b - 1];
    tb.gamma.assign(list.size(), 0);
    for (size_t i = 0; i < list.size(); ++i) {
      const int64_t k = start[(size_t)blk[i]]++;
      tb.gamma[(size_t)k] = (int)list[i];
      gpos[(size_t)list[i]] = (int)k;
    }
  }
  // subdomain terms of the condensation on each interface unknown
  tb.ccodes.assign(tb.gamma.size() * 4, -1);
  {
    std::vector<int> cfill(tb.gamma.size(), 0);
    if ((int64_t)tb.unitsI.size() * tb.npadB >= (int64_t)1 << 31) {
      *err = "level too large for the condensation indices";
      return false;
    }
    for (size_t u = 0; u < tb.unitsI.size(); ++u)
      for (int b = 0; b < tb.nB; ++b) {
        const int64_t e = tb.unitsI[u] + tb.relE[tb.nI + b];
        if (e < 0 || e >= g.len) {
          *err = "internal: a subdomain boundary edge outside the level";
          return false;
        }
        const int k = gpos[(size_t)e];
        if (k < 0) continue;   // on the boundary of the domain
        if (cfill[k] == 4) {
          *err = "internal: more than 4 subdomains hold an interface unknown";
          return false;
        }
        tb.ccodes[(size_t)k * 4 + cfill[k]++] = b * (int)tb.unitsI.size() + (int)u;
      }
  }
  tb.codes.assign(tb.gamma.size() * 4, -1);
  std::vector<int> fill(tb.gamma.size(), 0);
  for (size_t c = 0; c < tb.chunksP.size(); c += 4) {
    const int type = tb.chunksP[c], u0 = tb.chunksP[c + 1], cnt = tb.chunksP[c + 2];
    for (int u = u0; u < u0 + cnt; ++u)
      for (int j = 0; j < tb.npadP; ++j) {
        const int64_t ro = tb.relP[(size_t)type * tb.npadP + j];
        if (ro == kGenAbsentHost) continue;
        const int64_t e = tb.unitsP[u] + ro;
        if (e < 0 || e >= g.len || gpos[(size_t)e] < 0) {
          *err = "internal: a patch slot is not an interface unknown";
          return false;
        }
        const int k = gpos[(size_t)e];
        if (fill[k] == 4) {
          *err = "internal: more than 4 patches hold an interface unknown";
          return false;
        }
        tb.codes[(size_t)k * 4 + fill[k]++] = j * (int)tb.unitsP.size() + u;
      }
  }
  return true;
}

std::vector<int64_t> unknown_offsets(const Geom& g, const CoefBoxes& cf) {
  const int n = g.n;
  std::vector<int64_t> off;
  off.reserve((size_t)3 * n * (n - 1) * (n - 1));
  for (int d = 0; d < 3; ++d)
    for (int z = 0; z <= n; ++z)
      for (int y = 0; y <= n; ++y)
        for (int x = 0; x <= n; ++x) {
          const int o[3] = {x, y, z};
          bool ok = true;
          for (int ax = 0; ax < 3; ++ax) {
            if (ax == d) ok &= (o[ax] < n);
            else ok &= (o[ax] >= 1 && o[ax] <= n - 1);
          }
          if (ok && cf.r > 0) ok = cf.edge_in(n, d, x, y, z);
          if (ok) off.push_back(d * g.B + (int64_t)z * g.plane + (int64_t)y * g.P + x);
        }
  return off;
}

bool build_coarse(const Geom& g, double alpha, std::vector<double>* A0inv,
                  std::vector<int64_t>* map, std::string* err, const CoefBoxes& cf) {
  const int n = g.n;
  // unknowns: interior edges (inside the domain) in padded-layout order
  *map = unknown_offsets(g, cf);
  std::map<Key, int> idx;
  for (size_t u = 0; u < map->size(); ++u) {
    int64_t r = (*map)[u];
    const int d = (int)(r / g.B);
    r -= d * g.B;
    const int z = (int)(r / g.plane);
    r -= (int64_t)z * g.plane;
    const int y = (int)(r / g.P);
    const int x = (int)(r - (int64_t)y * g.P);
    idx[Key(d, x, y, z)] = (int)u;
  }
  const int N = (int)map->size();
  if (N > 1024) {
    *err = "coarsest level too large for the dense solve (over 1024 unknowns)";
    return false;
  }
  A0inv->assign((size_t)N * N, 0.0);
  double E[144];
  element_matrix(g.h, alpha, 1.0, E);
  double Ealpha = alpha;
  for (int z = 0; z < n; ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        const double fac = cf.at(n, x, y, z);
        if (!(fac > 0.0)) continue;   // outside the domain
        const double ac = alpha * fac;
        if (ac != Ealpha) {
          Ealpha = ac;
          element_matrix(g.h, Ealpha, 1.0, E);
        }
        int c[3] = {x, y, z};
        int loc[12];
        for (int d = 0; d < 3; ++d)
          for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
              auto it = idx.find(cell_edge(c, d, a, b));
              loc[ledge(d, a, b)] = (it == idx.end()) ? -1 : it->second;
            }
        for (int i = 0; i < 12; ++i)
          for (int j = 0; j < 12; ++j)
            if (loc[i] >= 0 && loc[j] >= 0) (*A0inv)[(size_t)loc[i] * N + loc[j]] += E[i * 12 + j];
      }
  if (!spd_inverse(*A0inv, N)) {
    *err = "coarsest matrix is not positive definite";
    return false;
  }
  return true;
}

}  // namespace ndmg
