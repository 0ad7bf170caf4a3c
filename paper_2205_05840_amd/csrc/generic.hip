// Substructuring smoother for any subdomain size and either kind of interface space:
// the vertex spaces of eq. (Preconditioner P) with s x s x s subdomains (s = 4 here; the
// s = 2 vertex smoother has its own fused kernels) and the edge spaces of eq.
// (Preconditioner E) (Sec. 3.2.1).  One smoothing step z (=, +=) M^{-1} r is evaluated
// through the global condensation (A_II is block diagonal over subdomains, and every
// coupling of an interface edge of a patch to interior edges stays inside that patch),
// with X_T = A_T^{-1} A_{I,dT} built in FP64 at setup, so that no step cancels the large
// curl part of A on discrete gradients in the working precision:
//   C_T = X_T^T r_I on every subdomain T                      (gathered product)
//   g_Gamma = r_Gamma - sum_{T} C_T  (the subdomains whose boundary holds the unknown)
//   y_P = S_P^{-1} g|Gamma_P on every patch P                  (gathered product)
//   w = sum_P R_P^T y_P on the interface unknowns; z_Gamma (=, +=) eta w
//   z_I (=, +=) eta (A_T^{-1} r_I - X_T w_dT) on every subdomain   (gathered product)
// The last line is eta (z_I + w_I): the interior solve plus the discrete-harmonic
// extension of the interface correction.  Sums over subdomains and patches are pulled per
// unknown in a fixed order (no atomics): the result does not depend on the launch shape.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "generic.hpp"

namespace ndmg {

namespace {

__device__ __forceinline__ bool pair_inactive(const Bat& bt, int pair) { return bt.act && bt.act[pair] == 0; }

// 16 x 16 x 4 MFMA: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; result register
// q of lane l holds D[row(l / 16, q)][l % 16] (row = 4 q + l / 16 for the f64 instruction,
// 4 (l / 16) + q for f32, as the vertex patch kernel measured on gfx950).
template <typename T>
struct GMfma;
template <>
struct GMfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int q) { return 4 * q + lk; }
};
template <>
struct GMfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int q) { return 4 * lk + q; }
};

// Units of 64 per block along x (a chunk of one patch type, or of subdomains), blocks of
// 64 result rows: wave w of the block takes rows rb 64 + 16 w .. + 15 for the 64 units
// (lane = unit).  The k dimension goes in chunks of 32: the block stages the gathered
// inputs (32 x 64 units) and the chunk of M for its 64 rows (32 x 64, k-major, coalesced
// rows of M) in LDS, every load issued before any is waited for (an absent slot reads the
// unit's own anchor and is zeroed after the load, so no load sits behind a branch); the
// next chunk's loads are in flight while the current one is multiplied, as 16 x 16 x 4
// MFMA tiles (A from the staged M, B from the staged inputs), accumulated in k order (the
// order of the sum does not depend on the launch shape; measured bit for bit equal to
// sequential fused multiply-adds in k order, in FP64 and FP32).
template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs<T> a, Bat bt) {
  constexpr int KC = 32;               // k per chunk
  constexpr int VX = KC * 64 / 256;    // gathered inputs per thread and chunk (8)
  constexpr int VM = KC * 64 / 256;    // values of M per thread and chunk (8)
  static_assert(KC == 256 / 8 && VM == 8, "M staging: 8 threads of 8 values per k-row of 64 rows");
  const int pair = blockIdx.y;
  if (pair_inactive(bt, pair)) return;
  const int chunk = blockIdx.x / a.nrb, rb = blockIdx.x - chunk * a.nrb;
  const int type = a.chunks[4 * chunk], u0 = a.chunks[4 * chunk + 1], cnt = a.chunks[4 * chunk + 2];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool valid = lane < cnt;
  const int64_t base = a.units[u0 + (valid ? lane : 0)];
  const T* __restrict__ x = a.x + (int64_t)pair * a.vlen;
  const T* __restrict__ x2 = a.x2 + (int64_t)pair * a.vlen;
  const T* __restrict__ M = a.M + (int64_t)(pair / bt.nrhs) * a.mstride + (int64_t)type * a.npadK * a.npadR;
  const int64_t* __restrict__ rin = a.relIn + (int64_t)type * a.npadK;
  __shared__ T Xs[KC][64];
  __shared__ __attribute__((aligned(16))) T Ms[KC][64];
  // M staging: thread tid copies rows mr0 .. mr0 + 7 of k-row mk (8 consecutive values)
  const int mk = tid >> 3, mr0 = (tid & 7) * 8;
  const int rowb = rb * 64;
  const int nrows = min(64, a.npadR - rowb);   // a multiple of 16
  T xr[VX], mrg[VM];
  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int i = 0; i < VX; ++i) {
      const int j = k0 + wave * VX + i;                 // uniform
      const int jj = j < a.npadK ? j : 0;
      const int64_t ro = rin[jj];
      const bool ok = j < a.npadK && ro != kGenAbsent;
      const T* __restrict__ src = j < a.ksplit ? x : x2;
      const T v = src[base + (ok ? ro : 0)];
      xr[i] = ok ? v : T(0);
    }
    const int k = k0 + mk;
    const bool mok = k < a.npadK && mr0 < nrows;
    const T* __restrict__ mp = M + (int64_t)(mok ? k : 0) * a.npadR + rowb + (mok ? mr0 : 0);
#pragma unroll
    for (int i = 0; i < VM; ++i) mrg[i] = mp[i];
#pragma unroll
    for (int i = 0; i < VM; ++i) mrg[i] = mok ? mrg[i] : T(0);
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int i = 0; i < VX; ++i) Xs[wave * VX + i][lane] = xr[i];
#pragma unroll
    for (int i = 0; i < VM; ++i) Ms[mk][mr0 + i] = mrg[i];
  };
  // wave w: 4 MFMA tiles of rows r0 .. r0 + 15 against units 16 t .. 16 t + 15
  const int lr = lane & 15, lk = lane >> 4;
  typename GMfma<T>::v4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = {T(0), T(0), T(0), T(0)};
  const int r0 = wave * 16;   // within the block's rows
  const bool rows_ok = r0 < nrows;
  load_chunk(0);
  for (int k0 = 0; k0 < a.npadK; k0 += KC) {
    store_chunk();
    __syncthreads();
    if (k0 + KC < a.npadK) load_chunk(k0 + KC);   // in flight during the products
    if (rows_ok) {
      const int nks = min(KC, a.npadK - k0) / 4;   // npadK is a multiple of 16
      for (int ks = 0; ks < nks; ++ks) {
        const T av = Ms[4 * ks + lk][r0 + lr];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = GMfma<T>::mma(av, Xs[4 * ks + lk][16 * t + lr], acc[t]);
      }
    }
    __syncthreads();
  }
  if (!rows_ok) return;
  const int rg = rowb + r0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int unit = 16 * t + lr;
    if (unit >= cnt) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = GMfma<T>::row(lk, q);
      const T val = acc[t][q];   // copied out before use as a scalar
      if (MODE == kGemmToY) {
        a.out[(int64_t)pair * a.ylen + (int64_t)(rg + row) * a.nunits + u0 + unit] = val;
      } else {
        const int64_t ro = a.relOut[(int64_t)type * a.npadR + rg + row];
        if (ro == kGenAbsent) continue;
        T* __restrict__ o = a.out + (int64_t)pair * a.vlen + a.units[u0 + unit] + ro;
        const T v = a.scale * val;
        *o = a.assign ? v : *o + v;
      }
    }
  }
}

// Sum of up to four entries of src listed in codes (-1: none), in the listed order.
template <typename T>
__device__ __forceinline__ T pull4(const T* __restrict__ src, const int4 c) {
  T acc = T(0);
  if (c.x >= 0) acc += src[c.x];
  if (c.y >= 0) acc += src[c.y];
  if (c.z >= 0) acc += src[c.z];
  if (c.w >= 0) acc += src[c.w];
  return acc;
}

// g_Gamma = r_Gamma - sum_T C_T on every interface unknown.
template <typename T>
__global__ void __launch_bounds__(256) k_gen_condense(const T* __restrict__ C, const T* __restrict__ r,
                                                      const int* __restrict__ gamma, const int4* __restrict__ codes,
                                                      int64_t ngam, T* __restrict__ gg, int64_t vlen, int64_t clen,
                                                      Bat bt) {
  const int pair = blockIdx.y;
  if (pair_inactive(bt, pair)) return;
  C += (int64_t)pair * clen;
  r += (int64_t)pair * vlen;
  gg += (int64_t)pair * vlen;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ngam; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = gamma[k];
    gg[e] = r[e] - pull4(C, codes[k]);
  }
}

// w = sum_P R_P^T y_P on every interface unknown, and z (=, +=) eta w there.
template <typename T>
__global__ void __launch_bounds__(256) k_gen_pull(const T* __restrict__ Y, const int* __restrict__ gamma,
                                                  const int4* __restrict__ codes, int64_t ngam, T* __restrict__ w,
                                                  T* __restrict__ z, T eta, int assign, int64_t vlen, int64_t ylen,
                                                  Bat bt) {
  const int pair = blockIdx.y;
  if (pair_inactive(bt, pair)) return;
  Y += (int64_t)pair * ylen;
  w += (int64_t)pair * vlen;
  z += (int64_t)pair * vlen;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ngam; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = gamma[k];
    const T acc = pull4(Y, codes[k]);
    w[e] = acc;
    z[e] = assign ? eta * acc : z[e] + eta * acc;
  }
}

template <typename T, int MODE>
hipError_t gemm(const GemmArgs<T>& a, const Bat& bt, hipStream_t st) {
  if (a.nchunks <= 0) return hipSuccess;
  if (a.npadK % 16 || a.npadR % 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_gemm<T, MODE>), dim3((unsigned)(a.nchunks * a.nrb), (unsigned)bt.count), dim3(256), 0, st,
                     a, bt);
  return hipGetLastError();
}

unsigned list_blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

}  // namespace

template <typename T>
hipError_t launch_smooth_generic(const T* r, T* z, const GenLevel<T>& L, const Geom& g, const Bat& bt, double eta,
                                 int assign, hipStream_t st) {
  hipError_t e;
  // C_T = X_T^T r_I
  GemmArgs<T> ac = L.cond;
  ac.x = ac.x2 = r;
  ac.out = L.C;
  if ((e = gemm<T, kGemmToY>(ac, bt, st)) != hipSuccess) return e;
  // g_Gamma = r_Gamma - sum_T C_T
  if (L.ngam > 0) {
    hipLaunchKernelGGL((k_gen_condense<T>), dim3(list_blocks(L.ngam), (unsigned)bt.count), dim3(256), 0, st, L.C, r,
                       L.gamma, reinterpret_cast<const int4*>(L.ccodes), L.ngam, L.gg, g.len, L.clen, bt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // patch products
  if ((e = launch_patch_generic<T>(L, bt, st)) != hipSuccess) return e;
  // interface sum and z_Gamma
  if (L.ngam > 0) {
    hipLaunchKernelGGL((k_gen_pull<T>), dim3(list_blocks(L.ngam), (unsigned)bt.count), dim3(256), 0, st, L.Y,
                       L.gamma, reinterpret_cast<const int4*>(L.codes), L.ngam, L.w, z, (T)eta, assign, g.len,
                       L.patch.ylen, bt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // z_I (=, +=) eta (A_T^{-1} r_I - X_T w_dT)
  GemmArgs<T> ax = L.ext;
  ax.x = r;
  ax.x2 = L.w;
  ax.out = z;
  ax.scale = (T)eta;
  ax.assign = assign;
  return gemm<T, kGemmToVector>(ax, bt, st);
}

template <typename T>
hipError_t launch_patch_generic(const GenLevel<T>& L, const Bat& bt, hipStream_t st) {
  GemmArgs<T> ap = L.patch;
  ap.x = ap.x2 = L.gg;
  ap.out = L.Y;
  return gemm<T, kGemmToY>(ap, bt, st);
}

template hipError_t launch_smooth_generic<double>(const double*, double*, const GenLevel<double>&, const Geom&,
                                                  const Bat&, double, int, hipStream_t);
template hipError_t launch_smooth_generic<float>(const float*, float*, const GenLevel<float>&, const Geom&,
                                                 const Bat&, double, int, hipStream_t);
template hipError_t launch_patch_generic<double>(const GenLevel<double>&, const Bat&, hipStream_t);
template hipError_t launch_patch_generic<float>(const GenLevel<float>&, const Bat&, hipStream_t);

}  // namespace ndmg
