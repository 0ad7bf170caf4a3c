// The substructuring smoother for any subdomain size and either interface space (vertex
// or edge patches): device-side description of one level and its launchers.
#pragma once

#include <cstdint>

#include "kernels.hpp"

namespace ndmg {

// Relative offset of a slot that holds no unknown for a patch type (never read).
constexpr int64_t kGenAbsent = INT64_MIN;

enum : int { kGemmToVector = 0, kGemmToY = 1 };

// out = M_type x|gathered for units of 64 (subdomains or patches).  Unit u has the anchor
// offset units[u] (its lower / vertex / edge-start node in the padded layout); input
// slot k of type t is read at units[u] + relIn[t npadK + k] (kGenAbsent: no unknown, read
// as 0), from x for k < ksplit and from x2 otherwise.  M holds, per type, the matrix with
// rows r and columns k stored k-major: M[(t npadK + k) npadR + r].  chunks[c] = {type,
// first unit, unit count <= 64, 0}.  To a vector (kGemmToVector): out (=, +=) scale times
// row r at units[u] + relOut[t npadR + r]; to Y (kGemmToY): row r at Y[u npadR + r].
template <typename T>
struct GemmArgs {
  const T* x;
  const T* x2;          // slots k >= ksplit (may equal x)
  int ksplit;
  T* out;
  const T* M;           // per problem, stride mstride
  int64_t mstride;
  const int* chunks;
  int nchunks;
  const int64_t* units;
  const int64_t* relIn;
  const int64_t* relOut;
  int npadK, npadR;     // multiples of 16
  int nrb;              // ceil(npadR / 64)
  int64_t vlen;         // vector length per pair
  int64_t ylen;         // Y length per pair
  int64_t nunits;       // units of the level (Y is row-major over them: row r of unit u at r * nunits + u)
  T scale;
  int assign;
};

template <typename T>
struct GenLevel {
  GemmArgs<T> cond;       // C_T = X_T^T r_I over the subdomains
  GemmArgs<T> patch;      // y_P = S_P^{-1} g|Gamma_P over the patches
  GemmArgs<T> ext;        // z_I = eta [A_T^{-1} | -X_T] [r_I ; w_dT] over the subdomains
  T *C, *gg, *Y, *w;
  const int* gamma;       // interface unknowns (padded offsets)
  const int* ccodes;      // [ngam][4] indices into C of the subdomain terms at each (-1: none)
  const int* codes;       // [ngam][4] indices into Y of the patch results at each (-1: none)
  int64_t ngam;
  int64_t clen;           // C length per pair
};

// z (assign ? = : +=) M^{-1} r, damping eta included.
template <typename T>
hipError_t launch_smooth_generic(const T* r, T* z, const GenLevel<T>& L, const Geom& g, const Bat& bt, double eta,
                                 int assign, hipStream_t st);

// The patch products alone on the level's condensed residual (timing).
template <typename T>
hipError_t launch_patch_generic(const GenLevel<T>& L, const Bat& bt, hipStream_t st);

}  // namespace ndmg
