// Plane-marching kernel for the operator A = alpha K + M (Sec. 2, eq. def bilinear form)
// on the padded edge layout.
//
// Factorised form (see kernels.hip): with face circulations
//   F_x(p) = z(p+e_y) - z(p) - y(p+e_z) + y(p)
//   F_y(p) = x(p+e_z) - x(p) - z(p+e_x) + z(p)
//   F_z(p) = y(p+e_x) - y(p) - x(p+e_y) + x(p)
// and face masses G_d = T F_d along the face normal d (T = tridiag(1/6, 2/3, 1/6)),
//   (A u)_x = ah [G_y(p-e_z) - G_y(p) - G_z(p-e_y) + G_z(p)] + h3 (T_y T_z x)(p)
//   (A u)_y = ah [G_z(p-e_x) - G_z(p) - G_x(p-e_z) + G_x(p)] + h3 (T_x T_z y)(p)
//   (A u)_z = ah [G_x(p-e_y) - G_x(p) - G_y(p-e_x) + G_y(p)] + h3 (T_x T_y z)(p)
// with ah = alpha h, h3 = h^3.
//
// Mapping: a workgroup has NW waves; wave w owns row j = j0 - 1 + w of the (i, j)
// plane (rows j0 - 1 and j0 + NW - 2 are halo rows whose outputs are not written).
// Lane l owns positions i = R l + r, r < R, so one wave spans a row of up to 64 R
// positions; neighbours along x come from the same lane or from lanes l -+ 1 through
// DPP wave shifts (lanes outside the wave read zero, which is the boundary value).
// Neighbours along y go through LDS; along z the wave keeps a few planes in
// registers and marches k.  Step s loads plane s + 1 and emits the outputs of plane
// s - 1.  All inputs outside [0, n)^3 are zero (boundary or padding).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace ndmg {

namespace {

constexpr int kWaveShr1 = 0x138;   // DPP: lane l receives lane l - 1
constexpr int kWaveShl1 = 0x130;   // DPP: lane l receives lane l + 1

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}

template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xffffffffull), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// value at position i - 1 / i + 1 for each of the R positions of the lane
template <typename T, int R>
__device__ __forceinline__ void shr1(const T (&v)[R], T (&o)[R]) {
  o[0] = dpp<kWaveShr1>(v[R - 1]);
#pragma unroll
  for (int r = 1; r < R; ++r) o[r] = v[r - 1];
}

template <typename T, int R>
__device__ __forceinline__ void shl1(const T (&v)[R], T (&o)[R]) {
#pragma unroll
  for (int r = 0; r < R - 1; ++r) o[r] = v[r + 1];
  o[R - 1] = dpp<kWaveShl1>(v[0]);
}

template <typename T, int R>
__device__ __forceinline__ void tri_x(const T (&v)[R], T (&o)[R]) {
  T m[R], p[R];
  shr1<T, R>(v, m);
  shl1<T, R>(v, p);
  const T t6 = T(1) / T(6), t23 = T(2) / T(3);
#pragma unroll
  for (int r = 0; r < R; ++r) o[r] = t6 * (m[r] + p[r]) + t23 * v[r];
}

template <typename T, int R>
struct Plane {
  T v[R];
};

// Load R consecutive values of row (j, k) starting at i0 = R * lane, zero outside [0, n)^3.
template <typename T, int R>
__device__ __forceinline__ void load_row(const T* __restrict__ base, const DGeom& g, int i0, int j,
                                         int k, T (&o)[R]) {
  const bool row_ok = (j >= 0 && j < g.n && k >= 0 && k < g.n);
  const T* p = base + (int64_t)k * g.plane + (int64_t)j * g.P + i0;
#pragma unroll
  for (int r = 0; r < R; ++r) o[r] = (row_ok && i0 + r < g.n) ? p[r] : T(0);
}

template <typename T, int R, int NW, int MODE>
__global__ void __launch_bounds__(64 * NW) k_stencil(const T* __restrict__ x, const T* __restrict__ bv,
                                                     T* __restrict__ y, DGeom g, Bat bt, double h,
                                                     int KZ, int ntj, int ntiles,
                                                     double* __restrict__ part, int64_t pstride) {
  constexpr int TJ = NW - 2;
  constexpr int W = 64 * R;
  // LDS: phase A (x, z of the current plane), phase B (F_y, G_z, G_x, Tz x, Tx z)
  __shared__ T sA[2][NW][W];
  __shared__ T sB[5][NW][W];
  __shared__ double sred[NW];

  const int pair = blockIdx.y;
  if (bt.act != nullptr && bt.act[pair] == 0) return;
  {
    const int64_t off = (int64_t)pair * 3 * g.B;
    x += off;
    y += off;
    if (MODE == 1) bv += off;
  }
  const T ah = (T)(bt.alpha[pair / bt.nrhs] * h), h3 = (T)(h * h * h);
  // XCD-aware tile order: blocks b, b + 8, b + 16, ... run on one XCD, so give them
  // consecutive tiles (neighbouring j-tiles share halo rows in that XCD's L2).
  const int nb = gridDim.x;
  const int per = (nb + 7) / 8;
  const int tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
  const bool active = tile < ntiles;
  const int tj = active ? tile % ntj : 0;
  const int tk = active ? tile / ntj : 0;
  const int j0 = tj * TJ;
  const int k0 = tk * KZ;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = j0 - 1 + wave;
  const int i0 = R * lane;
  const bool out_row = active && wave >= 1 && wave <= TJ && j <= g.n;
  const T t6 = T(1) / T(6), t23 = T(2) / T(3);
  const T* __restrict__ X = x;
  const T* __restrict__ Yc = x + g.B;
  const T* __restrict__ Zc = x + 2 * g.B;

  // registers: x, y at planes s-2, s-1, s (index 0, 1, 2) and the new plane s+1 (3)
  T xp[4][R], yp[4][R], zp[2][R];   // z at s-1, s
  T fz[2][R];                       // F_z at s-2, s-1
  T gy[2][R];                       // G_y at s-2, s-1
  T gx[2][R];                       // G_x at s-2, s-1
#pragma unroll
  for (int r = 0; r < R; ++r) {
    xp[0][r] = xp[1][r] = T(0);
    yp[0][r] = yp[1][r] = T(0);
    zp[0][r] = T(0);
    fz[0][r] = fz[1][r] = gy[0][r] = gy[1][r] = gx[0][r] = gx[1][r] = T(0);
  }
  const int kstart = k0 - 1;
  load_row<T, R>(X, g, i0, j, kstart, xp[2]);
  load_row<T, R>(Yc, g, i0, j, kstart, yp[2]);
  load_row<T, R>(Zc, g, i0, j, kstart, zp[1]);
  // software pipeline: plane s + 2 (and b of plane s) is requested during step s
  T xn[R], yn[R], zn[R], bn[3][R];
  load_row<T, R>(X, g, i0, j, kstart + 1, xn);
  load_row<T, R>(Yc, g, i0, j, kstart + 1, yn);
  load_row<T, R>(Zc, g, i0, j, kstart + 1, zn);
#pragma unroll
  for (int r = 0; r < R; ++r) bn[0][r] = bn[1][r] = bn[2][r] = T(0);
  double dot = 0.0;
  const int kend = min(k0 + KZ, g.n + 1);   // output planes [k0, kend)

  for (int s = kstart; s <= kend; ++s) {
    T znew[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      xp[3][r] = xn[r];
      yp[3][r] = yn[r];
      znew[r] = zn[r];
    }
    T bcur[3][R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      bcur[0][r] = bn[0][r];
      bcur[1][r] = bn[1][r];
      bcur[2][r] = bn[2][r];
    }
    if (s + 1 <= kend) {
      load_row<T, R>(X, g, i0, j, s + 2, xn);
      load_row<T, R>(Yc, g, i0, j, s + 2, yn);
      load_row<T, R>(Zc, g, i0, j, s + 2, zn);
    }
    if (MODE == 1 && out_row && s >= k0 && s < kend) {
      // b of output plane s, used in step s + 1 (rows and planes up to n are in the array)
      const T* pb = bv + (int64_t)s * g.plane + (int64_t)j * g.P + i0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool ok = i0 + r <= g.n;
        bn[0][r] = ok ? pb[r] : T(0);
        bn[1][r] = ok ? pb[g.B + r] : T(0);
        bn[2][r] = ok ? pb[2 * g.B + r] : T(0);
      }
    }
    // ---- phase A: x(s), z(s) across rows
#pragma unroll
    for (int r = 0; r < R; ++r) {
      sA[0][wave][i0 + r] = xp[2][r];
      sA[1][wave][i0 + r] = zp[1][r];
    }
    __syncthreads();
    T xj[R], zj[R];   // x(j+1, s), z(j+1, s); the last wave has no row above: zero
#pragma unroll
    for (int r = 0; r < R; ++r) {
      xj[r] = (wave + 1 < NW) ? sA[0][wave + 1][i0 + r] : T(0);
      zj[r] = (wave + 1 < NW) ? sA[1][wave + 1][i0 + r] : T(0);
    }
    T zi1[R], yi1[R];
    shl1<T, R>(zp[1], zi1);
    shl1<T, R>(yp[2], yi1);
    T Fx[R], Fy[R], Fz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      Fx[r] = (zj[r] - zp[1][r]) - (yp[3][r] - yp[2][r]);
      Fy[r] = (xp[3][r] - xp[2][r]) - (zi1[r] - zp[1][r]);
      Fz[r] = (yi1[r] - yp[2][r]) - (xj[r] - xp[2][r]);
    }
    T Gx[R];
    tri_x<T, R>(Fx, Gx);
    T Gz1[R], Tzx[R], Tzy[R];   // at plane s-1
#pragma unroll
    for (int r = 0; r < R; ++r) {
      Gz1[r] = t6 * (fz[0][r] + Fz[r]) + t23 * fz[1][r];
      Tzx[r] = t6 * (xp[0][r] + xp[2][r]) + t23 * xp[1][r];
      Tzy[r] = t6 * (yp[0][r] + yp[2][r]) + t23 * yp[1][r];
    }
    T massy[R], Txz[R];
    tri_x<T, R>(Tzy, massy);
    tri_x<T, R>(zp[0], Txz);
    // ---- phase B
#pragma unroll
    for (int r = 0; r < R; ++r) {
      sB[0][wave][i0 + r] = Fy[r];
      sB[1][wave][i0 + r] = Gz1[r];
      sB[2][wave][i0 + r] = gx[1][r];   // G_x(s-1)
      sB[3][wave][i0 + r] = Tzx[r];
      sB[4][wave][i0 + r] = Txz[r];
    }
    __syncthreads();
    T Gy[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const T fyl = (wave > 0) ? sB[0][wave - 1][i0 + r] : T(0);
      const T fyh = (wave + 1 < NW) ? sB[0][wave + 1][i0 + r] : T(0);
      Gy[r] = t6 * (fyl + fyh) + t23 * Fy[r];
    }
    const int ko = s - 1;   // output plane
    if (out_row && ko >= k0 && ko < kend) {
      T gzl[R], gyl[R];
      shr1<T, R>(Gz1, gzl);
      shr1<T, R>(gy[1], gyl);
      const int64_t rowoff = (int64_t)ko * g.plane + (int64_t)j * g.P + i0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = i0 + r;
        // wave > 0 here, so rows j-1 exist in LDS
        const T gzjm = sB[1][wave - 1][i];
        const T gxjm = sB[2][wave - 1][i];
        const T mx = t6 * (sB[3][wave - 1][i] + sB[3][wave + 1][i]) + t23 * Tzx[r];
        const T mz = t6 * (sB[4][wave - 1][i] + sB[4][wave + 1][i]) + t23 * Txz[r];
        T ox = ah * ((gy[0][r] - gy[1][r]) - (gzjm - Gz1[r])) + h3 * mx;
        T oy = ah * ((gzl[r] - Gz1[r]) + (gx[1][r] - gx[0][r])) + h3 * massy[r];
        T oz = ah * ((gxjm - gx[1][r]) + (gy[1][r] - gyl[r])) + h3 * mz;
        // unknown masks: x-edge: i < n, 1 <= j,k <= n-1; y-edge: j < n, 1 <= i,k <= n-1; ...
        const bool iin = (i >= 1 && i <= g.n - 1), jin = (j >= 1 && j <= g.n - 1),
                   kin = (ko >= 1 && ko <= g.n - 1);
        const bool ux = (i < g.n) && jin && kin;
        const bool uy = iin && (j < g.n) && kin;
        const bool uz = iin && jin && (ko < g.n);
        if (i <= g.n) {
          if (MODE == 1) {
            ox = ux ? bcur[0][r] - ox : T(0);
            oy = uy ? bcur[1][r] - oy : T(0);
            oz = uz ? bcur[2][r] - oz : T(0);
          } else {
            ox = ux ? ox : T(0);
            oy = uy ? oy : T(0);
            oz = uz ? oz : T(0);
          }
          y[rowoff + r] = ox;
          y[g.B + rowoff + r] = oy;
          y[2 * g.B + rowoff + r] = oz;
          if (MODE == 2) {
            dot += (double)ox * (double)xp[1][r] + (double)oy * (double)yp[1][r] +
                   (double)oz * (double)zp[0][r];
          }
        }
      }
      // the position i = n of a row falls outside the lanes when n = 64 R: zero it
      if (lane == 63 && i0 + R == g.n) {
        y[rowoff + R] = T(0);
        y[g.B + rowoff + R] = T(0);
        y[2 * g.B + rowoff + R] = T(0);
      }
    }
    // rotate the plane window
#pragma unroll
    for (int r = 0; r < R; ++r) {
      xp[0][r] = xp[1][r]; xp[1][r] = xp[2][r]; xp[2][r] = xp[3][r];
      yp[0][r] = yp[1][r]; yp[1][r] = yp[2][r]; yp[2][r] = yp[3][r];
      zp[0][r] = zp[1][r]; zp[1][r] = znew[r];
      fz[0][r] = fz[1][r]; fz[1][r] = Fz[r];
      gy[0][r] = gy[1][r]; gy[1][r] = Gy[r];
      gx[0][r] = gx[1][r]; gx[1][r] = Gx[r];
    }
  }
  if (MODE == 2) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dot += __shfl_down(dot, off, 64);
    if (lane == 0) sred[wave] = dot;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < NW; ++w) t += sred[w];
      part[(int64_t)pair * pstride + blockIdx.x] = t;
    }
  }
}

struct Tiling {
  int ntj, KZ, ntiles, nblocks;
};

Tiling tiling(int n, int NW) {
  Tiling t;
  const int TJ = NW - 2;
  t.ntj = (n + 1 + TJ - 1) / TJ;
  t.KZ = 8;
  const int ntk = (n + 1 + t.KZ - 1) / t.KZ;
  t.ntiles = t.ntj * ntk;
  t.nblocks = (t.ntiles + 7) / 8 * 8;   // the XCD remap permutes [0, nblocks)
  return t;
}

int waves_for(int n) { return (n <= 128) ? 8 : 4; }

template <typename T, int R, int NW>
hipError_t launch_r(const T* x, const T* b, T* y, const Geom& g, const Bat& bt, int mode,
                    double* part, int64_t pstride, hipStream_t st) {
  const Tiling tl = tiling(g.n, NW);
  const int ntj = tl.ntj, KZ = tl.KZ, ntiles = tl.ntiles, nbr = tl.nblocks;
  const DGeom dg = dgeom(g);
  const dim3 grid((unsigned)nbr, (unsigned)bt.count);
  if (mode == 0)
    hipLaunchKernelGGL((k_stencil<T, R, NW, 0>), grid, dim3(64 * NW), 0, st, x, b, y, dg, bt, g.h, KZ, ntj,
                       ntiles, part, pstride);
  else if (mode == 1)
    hipLaunchKernelGGL((k_stencil<T, R, NW, 1>), grid, dim3(64 * NW), 0, st, x, b, y, dg, bt, g.h, KZ, ntj,
                       ntiles, part, pstride);
  else
    hipLaunchKernelGGL((k_stencil<T, R, NW, 2>), grid, dim3(64 * NW), 0, st, x, b, y, dg, bt, g.h, KZ, ntj,
                       ntiles, part, pstride);
  return hipGetLastError();
}

}  // namespace

int stencil_max_n() { return 256; }
int stencil_min_n() { return 64; }

int stencil_blocks(const Geom& g) { return tiling(g.n, waves_for(g.n)).nblocks; }

template <typename T>
hipError_t launch_stencil(const T* x, const T* b, T* y, const Geom& g, const Bat& bt, int mode,
                          double* part, int64_t pstride, hipStream_t st) {
  if (g.n <= 64) return launch_r<T, 1, 8>(x, b, y, g, bt, mode, part, pstride, st);
  if (g.n <= 128) return launch_r<T, 2, 8>(x, b, y, g, bt, mode, part, pstride, st);
  if (g.n <= 256) return launch_r<T, 4, 4>(x, b, y, g, bt, mode, part, pstride, st);
  return hipErrorInvalidValue;
}

template hipError_t launch_stencil<double>(const double*, const double*, double*, const Geom&,
                                           const Bat&, int, double*, int64_t, hipStream_t);
template hipError_t launch_stencil<float>(const float*, const float*, float*, const Geom&, const Bat&,
                                          int, double*, int64_t, hipStream_t);

}  // namespace ndmg
