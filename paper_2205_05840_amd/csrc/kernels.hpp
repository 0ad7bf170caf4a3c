// Device kernels of the ndmg library and their launchers (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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

// Smoother tables of one level on the device.
struct DSub {
  int s, nH, nI, nG, npad, lut_w;
  const int* lut;       // [3][w][w][w] slot lookup
  const int* slots;     // [nG][4]: d, dx, dy, dz
  const int* segs;      // [nseg][8]: type, lo0, lo1, lo2, d0, d1, d2, count
  const int* chunks;    // [nchunks][2]: segment, first vertex
  int nchunks;
  int gpw;              // 16-vertex groups per wave in the patch kernel
};

template <typename T>
struct LevelPtrs {
  T* z;       // solution / correction
  T* r;       // residual scratch
  T* zi;      // interior solves (only interior-of-subdomain entries ever written)
  T* gg;      // condensed interface residual
  T* w;       // interface correction (only interface entries ever written)
  T* Y;       // vertex patch results, slot-major [npad][(nH+1)^3]
  const T* ATinv;   // nI x nI
  const T* Sinv;    // 27 x npad x npad
  const T* XT;      // nI x nB
  const int64_t* bofs;   // nB offsets of the subdomain boundary edges from its lower node
};

// Plane-marching operator kernel: mode 0 y = A x, 1 y = b - A x, 2 y = A x and
// part[block] = partial sums of x . y (then k_final over stencil_blocks(g) partials).
template <typename T>
hipError_t launch_stencil(const T* x, const T* b, T* y, const Geom& g, double alpha, int mode,
                          double* part, int* nparts, hipStream_t st);
int stencil_max_n();
int stencil_min_n();   // the plane-marching kernel serves stencil_min_n() < n <= stencil_max_n()
// groups of 16 vertices per wave in the patch kernel: more on large levels (fewer
// S^{-1} stagings), one on small levels (more workgroups)
inline int patch_groups(int nH) { return nH >= 48 ? 4 : (nH >= 24 ? 2 : 1); }
int stencil_blocks(const Geom& g);
hipError_t launch_final(const double* part, int nparts, int nout, double* out, hipStream_t st);

// y = A x (mode 0) or y = b - A x (mode 1); all entries of y written.
template <typename T>
hipError_t launch_apply(const T* x, const T* b, T* y, const Geom& g, double alpha, int mode,
                        hipStream_t st);

// gc = I_k^{k-1} rf (restriction, eq. F2C); all entries of gc written.
template <typename T>
hipError_t launch_restrict(const T* rf, T* gc, const Geom& f, const Geom& c, hipStream_t st);

// zf += I_{k-1}^k ec (prolongation by natural injection) on interior edges.
template <typename T>
hipError_t launch_prolong_add(const T* ec, T* zf, const Geom& f, const Geom& c, hipStream_t st);

// z (assign != 0: z =, else z +=) eta * M_V^{-1} r  (vertex-based smoother).
template <typename T>
hipError_t launch_smooth(const T* r, T* z, const LevelPtrs<T>& L, const DSub& sub,
                         const Geom& g, double alpha, double eta, int assign, hipStream_t st);

// z = A_0^{-1} g on the coarsest level.
template <typename T>
hipError_t launch_coarse(const T* g, T* z, const T* A0inv, const int64_t* map, int N0,
                         hipStream_t st);

template <typename Tin, typename Tout>
hipError_t launch_convert(const Tin* in, Tout* out, int64_t len, hipStream_t st);

// ---- FP64 CG vector kernels with device-resident scalars ----------------------------
constexpr int kRedBlocks = 512;   // partial sums per reduction

// out[0] = a . b (and out[1] = a . c when c != nullptr); deterministic two-stage sum.
hipError_t launch_dot(const double* a, const double* b, const double* c, double* partial,
                      double* out, int64_t len, hipStream_t st);
// alpha = s[i_num] / s[i_den]; u += alpha p; r -= alpha q; out = r . r
hipError_t launch_cg_update(double* u, double* r, const double* p, const double* q,
                            const double* scal, int i_num, int i_den, double* partial,
                            double* out, int64_t len, hipStream_t st);
// beta = s[i_num] / s[i_den] (flexible: beta = -alpha s[i_zq] / s[i_den] with alpha =
// s[i_an]/s[i_ad]); p = z + beta p
hipError_t launch_cg_direction(double* p, const double* z, const double* scal, int i_num,
                               int i_den, int flexible, int i_zq, int i_an, int i_ad,
                               int64_t len, hipStream_t st);
// y = x (copy) and y = 0
hipError_t launch_copy(const double* x, double* y, int64_t len, hipStream_t st);
hipError_t launch_zero(double* y, int64_t len, hipStream_t st);

// b = load vector of f sampled at the 2x2x2 Gauss points.
hipError_t launch_assemble_rhs(const double* f, double* b, const Geom& g, hipStream_t st);

// partial sums of lam . (K u) for one pair; accumulates into out[0] via final stage.
hipError_t launch_curlcurl_form(const double* lam, const double* u, const Geom& g,
                                double* partial, double* out, hipStream_t st);

}  // namespace ndmg
