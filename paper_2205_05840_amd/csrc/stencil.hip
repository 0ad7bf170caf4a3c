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
// The workgroup marches k over its planes.  Step s emits the outputs of plane s - 1.
//
// Input planes stream through a ring of D plane slots in LDS, filled by direct
// global-to-LDS loads (16 bytes per lane) D - 1 steps ahead: each wave copies its own
// row of x, y and z of plane s + D - 1 at step s, so the loads of D - 2 steps are in
// flight while a step computes, without holding registers.  Rows of plane s + 1 (own)
// and s (the row above, for the y differences) are read from the ring; every other
// y-neighbour goes through a second LDS area.  Synchronisation: each step waits for
// its own ring loads with an explicit vmcnt (every vector-memory operation of a step is
// issued unconditionally, so the count of operations issued after a given load is
// fixed) and then meets the workgroup at a barrier.  Rows and planes outside [0, n) are
// read from row (0, 0) of plane 0, which is zero (boundary), as is every non-unknown
// entry of the layout, so no mask is applied; positions at or beyond the row pitch
// (when 64 R exceeds it) hold copies of in-row values and only feed outputs at i >= n,
// which are written as zero.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <type_traits>

#include "kernels.hpp"
#include "tuning.hpp"
#include "reduce.hpp"

namespace ndmg {

namespace {

typedef __attribute__((address_space(3))) void* lds_ptr_t;

constexpr int kWaveShr1 = 0x138;   // DPP: lane l receives lane l - 1
constexpr int kWaveShl1 = 0x130;   // DPP: lane l receives lane l + 1

// s_waitcnt immediates: vmcnt in bits 3:0 and 15:14, expcnt in 6:4, lgkmcnt in 11:8
constexpr int waitcnt_vm(int n) { return (n & 0xF) | (0x7 << 4) | (0xF << 8) | ((n >> 4) << 14); }
constexpr int waitcnt_vm_lds(int n) { return (n & 0xF) | (0x7 << 4) | ((n >> 4) << 14); }
constexpr int kWaitLgkm0 = 0xF | (0x7 << 4) | (0x3 << 14);

__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

template <int N>
__device__ __forceinline__ void wait_vm() {
  compiler_fence();
  __builtin_amdgcn_s_waitcnt(waitcnt_vm(N));
  compiler_fence();
}

// vmcnt <= N and every LDS access of this wave complete
template <int N>
__device__ __forceinline__ void wait_vm_lds() {
  compiler_fence();
  __builtin_amdgcn_s_waitcnt(waitcnt_vm_lds(N));
  compiler_fence();
}

__device__ __forceinline__ void wait_lds() {
  compiler_fence();
  __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
  compiler_fence();
}

__device__ __forceinline__ void wg_barrier() {
  compiler_fence();
  __builtin_amdgcn_s_barrier();
  compiler_fence();
}

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

// Ring geometry: one slot holds, per wave, the x, y and z rows of one plane, and in the
// residual mode also the rows of b (ROWS = 6).
template <typename T, int R, int ROWS>
struct RingGeo {
  static constexpr int W = 64 * R;                             // positions per row
  static constexpr int RB = W * (int)sizeof(T);                // bytes per row
  static constexpr int CH = (ROWS * RB + 1023) / 1024 * 1024;  // bytes per wave and slot
  static constexpr int NQ = CH / 1024;                         // 16-byte-per-lane loads per chunk
  static constexpr int VE = 16 / (int)sizeof(T);               // elements per lane and load
};

// R consecutive values of a row (one vector access per lane).
template <typename T, int R>
struct RowVec {
  typedef T type __attribute__((ext_vector_type(R)));
};

template <typename T, int R>
__device__ __forceinline__ void ring_row(const unsigned char* chunk, int dir, int i0, T (&o)[R]) {
  typedef typename RowVec<T, R>::type V;
  const V v = *reinterpret_cast<const V*>(chunk + dir * (64 * R * (int)sizeof(T)) + i0 * (int)sizeof(T));
#pragma unroll
  for (int r = 0; r < R; ++r) o[r] = v[r];
}

// Compile-time unrolling: f(integral_constant<I>, s + I) for I < U.
template <int U, int I = 0>
struct Unroll {
  template <typename F>
  __device__ __forceinline__ static void run(F& f, int s) {
    f(std::integral_constant<int, I>(), s + I);
    Unroll<U, I + 1>::run(f, s);
  }
};
template <int U>
struct Unroll<U, U> {
  template <typename F>
  __device__ __forceinline__ static void run(F&, int) {}
};

// COEF: alpha per cell from the r^3 box factors (bt.coef, r <= kCoefMaxR): each face's
// term of the RT0 mass takes the factors of the two cells on either side (the per-cell
// form of the per-thread kernels), and an edge is written only where its four cells
// have a positive factor (a domain inside the cube).  The factors sit in LDS.  Every
// mode, the dot mode's p^T A p included, takes the per-cell form.
constexpr int kCoefMaxR = 8;

template <typename T, int R, int NW, int D, int MODE, int SYNC, bool COEF>
__global__ void __launch_bounds__(64 * NW) k_stencil(const T* __restrict__ x, const T* __restrict__ bv,
                                                     T* __restrict__ y, DGeom g, Bat bt, double h,
                                                     int KZ, int ntj, int ntiles,
                                                     double* __restrict__ part, int64_t pstride,
                                                     int opaque0) {
  constexpr int ROWS = (MODE == 1) ? 6 : 3;
  using RG = RingGeo<T, R, ROWS>;
  constexpr int TJ = NW - 2;
  constexpr int CH = RG::CH, NQ = RG::NQ, VE = RG::VE;
  static_assert(D == 3 || D == 4, "ring depth 3 or 4");
  // steps are unrolled by U = D so that every ring slot index is static
  constexpr int U = D;
  // before a step reads plane s + 1, the vector-memory operations issued after that
  // plane's ring loads (issued D - 2 steps earlier) are the ring loads of D - 3 steps
  // (and stores, which only make the wait stricter)
  constexpr int NWAIT = (D - 3) * NQ;
  static_assert(NWAIT < 64, "vmcnt holds at most 63");
  // one LDS array per ring slot: a slot being read and a slot being filled are distinct
  // objects to the compiler, so its own waits for the direct loads do not cover the reads
  __shared__ __attribute__((aligned(16))) unsigned char ring0[NW * CH];
  __shared__ __attribute__((aligned(16))) unsigned char ring1[NW * CH];
  __shared__ __attribute__((aligned(16))) unsigned char ring2[NW * CH];
  __shared__ __attribute__((aligned(16))) unsigned char ring3[D == 4 ? NW * CH : 16];
  // y-neighbour exchange: F_y, G_z, G_x, T_z x, T_x z of the current step.  SYNC = 1:
  // two copies used by step parity, and one barrier per step (see the step); SYNC = 2:
  // one copy, and a second barrier per step before it is overwritten.
  typedef typename RowVec<T, R>::type V;
  constexpr bool kOneBarrier = SYNC == 1;
  static_assert(SYNC == 1 || SYNC == 2, "one or two barriers per step");
  static_assert(!kOneBarrier || D * NW * CH + 2 * 5 * NW * 64 * (int)sizeof(V) + 1024 <= 160 * 1024,
                "two copies of the exchange area must fit the LDS");
  constexpr int kCoefN = COEF ? kCoefMaxR * kCoefMaxR * kCoefMaxR : 1;
  static_assert(!COEF || D * NW * CH + (kOneBarrier ? 2 : 1) * 5 * NW * 64 * (int)sizeof(V) +
                                 kCoefN * (int)sizeof(T) + 1024 <= 160 * 1024,
                "the box factors must fit the LDS beside the ring");
  __shared__ V sBuf[kOneBarrier ? 2 : 1][5][NW][64];
  __shared__ T sCoef[kCoefN];

  const int pair = blockIdx.y;
  if (bt.act != nullptr && bt.act[pair] == 0) return;
  {
    const int64_t off = (int64_t)pair * 3 * g.B;
    x += off;
    y += off;
    if (MODE == 1) bv += off;
  }
  const T ah = (T)(bt.alpha[pair / bt.nrhs] * h), h3 = (T)(h * h * h);
  // box factors into LDS (read from the first computing step on, which starts with a
  // barrier)
  const int rc = COEF ? bt.coef_r : 1;
  if constexpr (COEF) {
    for (int e = threadIdx.x; e < rc * rc * rc; e += blockDim.x) sCoef[e] = (T)bt.coef[e];
  }
  // XCD-aware tile order: blocks b, b + 8, b + 16, ... run on one XCD, so give them
  // consecutive tiles (neighbouring j-tiles share halo rows in that XCD's L2).
  const int nb = gridDim.x;
  const int per = (nb + 7) / 8;
  const int tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= ntiles) return;   // padding block of the XCD remap (the whole workgroup)
  const bool active = true;
  const int tj = tile % ntj;
  const int tk = tile / ntj;
  const int j0 = tj * TJ;
  const int k0 = tk * KZ;
  // output planes [k0, kend); the last tile also writes the boundary plane k = n (zero)
  const int kend = (k0 + KZ >= g.n) ? g.n + 1 : k0 + KZ;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = j0 - 1 + wave;
  const int i0 = R * lane;
  // ring reads start at i0 + opaque0 (opaque0 = 0 from the host): an offset the compiler
  // cannot bound makes every read of a slot overlap that slot's direct loads, so the waits
  // it adds for them are the ones for the slot's own (already completed) loads
  const int ir = i0 + opaque0;
  // output rows: j0 .. j0 + TJ - 1, plus the boundary row j = n (all zero) when it is the
  // top halo row of the last tile (tiles cover rows 0 .. n - 1)
  const bool zero_row = (wave == NW - 1 && j == g.n);
  const bool out_row = active && j <= g.n && ((wave >= 1 && wave <= TJ) || zero_row);
  const bool row_ok = (j >= 0 && j < g.n);
  const T t6 = T(1) / T(6), t23 = T(2) / T(3), t3 = T(1) / T(3);
  // COEF: box of a cell index (clamped into the cube: a clamped cell only meets faces
  // whose flux is zero and edges that are not written), boxes of cells i0 - 1 + q along
  // the row and of cells j - 1, j across it
  const int cwid = COEF ? g.n / rc : 1;
  auto cbox = [&](int c) { return min(max(c, 0), g.n - 1) / cwid; };
  int bxq[R + 1];
#pragma unroll
  for (int q = 0; q <= R; ++q) bxq[q] = COEF ? cbox(i0 - 1 + q) : 0;
  const int byl = COEF ? cbox(j - 1) : 0, by0 = COEF ? cbox(j) : 0;
  auto cf = [&](int bx, int by, int bz) -> T { return sCoef[(bz * rc + by) * rc + bx]; };

  // ring loads of this lane: source (x rows 0-2, b rows 3-5; direction block + clamped
  // position) of the 16 bytes it copies in each of the NQ loads of a chunk; lanes past
  // the rows copy the vector's first bytes into the chunk's padding
  const T* src_base[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int o = q * 1024 + 16 * lane;
    const int d = o / RG::RB;
    const int p = min((o % RG::RB) / (int)sizeof(T), g.P - VE);
    if (d < 3) src_base[q] = x + (int64_t)d * g.B + p;
    else if (MODE == 1 && d < 6) src_base[q] = bv + (int64_t)(d - 3) * g.B + p;
    else src_base[q] = x;
  }
  auto slot_base = [&](auto SL) -> unsigned char* {
    constexpr int sl = decltype(SL)::value;
    if constexpr (sl == 0) return ring0;
    else if constexpr (sl == 1) return ring1;
    else if constexpr (sl == 2) return ring2;
    else return ring3;
  };
  // ring loads of plane p into slot SL.  Only planes k0 - 1 .. kend feed written outputs;
  // loads of other planes (and of rows outside [0, n)) read row (0, 0) of plane 0, which
  // is zero and stays cached, so they cost no memory traffic
  auto issue_plane = [&](auto SL, int p) {
    const bool ok = row_ok && p >= 0 && p < g.n && p >= k0 - 1 && p <= kend;
    const int64_t roff = ok ? (int64_t)p * g.plane + (int64_t)j * g.P : 0;
    unsigned char* dst = slot_base(SL) + wave * CH;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      __builtin_amdgcn_global_load_lds((const void*)(src_base[q] + roff), (lds_ptr_t)(dst + q * 1024), 16,
                                       0, 0);
  };
  // registers: x, y at planes s-2, s-1, s (index 0, 1, 2) and the new plane s+1 (3)
  T xp[4][R], yp[4][R], zp[2][R];   // z at s-1, s
  T fz[2][R];                       // F_z at s-2, s-1
  T gy[2][R];                       // G_y at s-2, s-1
  T gx[2][R];                       // G_x at s-2, s-1
#pragma unroll
  for (int r = 0; r < R; ++r) {
    xp[0][r] = xp[1][r] = xp[2][r] = T(0);
    yp[0][r] = yp[1][r] = yp[2][r] = T(0);
    zp[0][r] = zp[1][r] = T(0);
    fz[0][r] = fz[1][r] = gy[0][r] = gy[1][r] = gx[0][r] = gx[1][r] = T(0);
  }
  double dot = 0.0;
  const int kstart = k0 - 1;
  const int s0 = kstart - D;                // first step: ring loads only

  // one step; PH = (s - s0) mod U.  Plane s0 + m lives in slot m mod D, so plane s + a is
  // in slot (PH + D + a) mod D.  The first D - 1 steps only start ring loads (COMPUTE
  // false).  A step holds no branch between its ring loads and its ring reads: the
  // compiler then keeps track of which slot each direct load fills and adds no wait of
  // its own.
  auto step = [&](auto PH, auto COMPUTE, int s) {
    constexpr int ph = decltype(PH)::value;
    constexpr bool compute = decltype(COMPUTE)::value;
    constexpr int sl_prev = (ph + D - 1) % D;   // plane s - 1, refilled with plane s + D - 1
    constexpr int sl_cur = ph % D;              // plane s
    constexpr int sl_next = (ph + 1) % D;       // plane s + 1
    T bcur[3][R];   // b of the output plane s - 1 (residual mode)
    // this step's copy of the exchange area
    V(*sB)[NW][64] = sBuf[kOneBarrier ? (s & 1) : 0];
    if constexpr (compute) {
      wait_vm_lds<NWAIT>();
      // plane s + 1 is in the ring; every wave is done with step s - 1.  With two copies
      // of the exchange area only the first step needs this barrier: afterwards the
      // barrier in the middle of step s - 1 already orders what it would (every wave had
      // waited for its loads of plane s and finished reading plane s - 1 from the ring,
      // whose slot this step refills, and a wave can only reach this step's exchange
      // writes after every wave has finished reading the copy of step s - 2)
      if (!kOneBarrier || s == kstart - 1) wg_barrier();
      if constexpr (MODE == 1) {
        // b rows of plane s - 1, before its slot is refilled
        const unsigned char* prev = slot_base(std::integral_constant<int, sl_prev>()) + wave * CH;
#pragma unroll
        for (int d = 0; d < 3; ++d) ring_row<T, R>(prev, 3 + d, ir, bcur[d]);
        wait_lds();
      }
    }
    issue_plane(std::integral_constant<int, sl_prev>(), s + D - 1);
    compiler_fence();
    if constexpr (compute) {
      const unsigned char* own = slot_base(std::integral_constant<int, sl_next>()) + wave * CH;
      T znew[R];
      ring_row<T, R>(own, 0, ir, xp[3]);
      ring_row<T, R>(own, 1, ir, yp[3]);
      ring_row<T, R>(own, 2, ir, znew);
      // x(j+1, s), z(j+1, s); the last wave has no row above (its values only feed the
      // halo row's outputs, which are not written)
      T xj[R], zj[R];
      {
        const unsigned char* up =
            slot_base(std::integral_constant<int, sl_cur>()) + (wave + 1 < NW ? wave + 1 : wave) * CH;
        ring_row<T, R>(up, 0, ir, xj);
        ring_row<T, R>(up, 2, ir, zj);
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
      // COEF: boxes of the cell planes s - 2, s - 1 and s
      const int bz2 = COEF ? cbox(s - 2) : 0, bz1 = COEF ? cbox(s - 1) : 0, bz0 = COEF ? cbox(s) : 0;
      T Gx[R];
      if constexpr (COEF) {
        // x-faces of plane s between cells i - 1 and i (row j)
        T Fm[R], Fp[R];
        shr1<T, R>(Fx, Fm);
        shl1<T, R>(Fx, Fp);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const T am = cf(bxq[r], by0, bz0), a0 = cf(bxq[r + 1], by0, bz0);
          Gx[r] = t6 * (am * Fm[r] + a0 * Fp[r]) + t3 * (am + a0) * Fx[r];
        }
      } else {
        tri_x<T, R>(Fx, Gx);
      }
      T Gz1[R], Tzx[R], Tzy[R];   // at plane s-1
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (COEF) {
          // z-face at plane s - 1 between cells s - 2 and s - 1
          const T a2 = cf(bxq[r + 1], by0, bz2), a1 = cf(bxq[r + 1], by0, bz1);
          Gz1[r] = t6 * (a2 * fz[0][r] + a1 * Fz[r]) + t3 * (a2 + a1) * fz[1][r];
        } else {
          Gz1[r] = t6 * (fz[0][r] + Fz[r]) + t23 * fz[1][r];
        }
        Tzx[r] = t6 * (xp[0][r] + xp[2][r]) + t23 * xp[1][r];
        Tzy[r] = t6 * (yp[0][r] + yp[2][r]) + t23 * yp[1][r];
      }
      T massy[R], Txz[R];
      tri_x<T, R>(Tzy, massy);
      tri_x<T, R>(zp[0], Txz);
      {
        V v0, v1, v2, v3, v4;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          v0[r] = Fy[r];
          v1[r] = Gz1[r];
          v2[r] = gx[1][r];   // G_x(s-1)
          v3[r] = Tzx[r];
          v4[r] = Txz[r];
        }
        sB[0][wave][lane] = v0;
        sB[1][wave][lane] = v1;
        sB[2][wave][lane] = v2;
        sB[3][wave][lane] = v3;
        sB[4][wave][lane] = v4;
      }
      wait_lds();
      wg_barrier();
      // rows j - 1 and j + 1 (the first and last wave have none: their values only feed
      // the halo rows, whose outputs are not written)
      const int wl = wave > 0 ? wave - 1 : wave, wh = wave + 1 < NW ? wave + 1 : wave;
      T Gy[R];
      {
        const V fyl = sB[0][wl][lane], fyh = sB[0][wh][lane];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if constexpr (COEF) {
            // y-face of row j between cells j - 1 and j (plane s)
            const T al = cf(bxq[r + 1], byl, bz0), a0 = cf(bxq[r + 1], by0, bz0);
            Gy[r] = t6 * (al * fyl[r] + a0 * fyh[r]) + t3 * (al + a0) * Fy[r];
          } else {
            Gy[r] = t6 * (fyl[r] + fyh[r]) + t23 * Fy[r];
          }
        }
      }
      const int ko = s - 1;   // output plane
      // a lane stores its R positions when they lie inside the row (positions > n of the
      // row are padding and receive zero)
      const bool lane_in_row = i0 + R <= g.P;
      if (out_row && zero_row && ko >= k0 && ko < kend) {
        const int64_t rowoff = (int64_t)ko * g.plane + (int64_t)j * g.P + i0;
        const V zv = V(T(0));
        if (lane_in_row) {
#pragma unroll
          for (int d = 0; d < 3; ++d) *reinterpret_cast<V*>(y + d * g.B + rowoff) = zv;
        }
        if (lane == 63 && i0 + R == g.n) {
#pragma unroll
          for (int d = 0; d < 3; ++d) y[d * g.B + rowoff + R] = T(0);
        }
      } else if (out_row && ko >= k0 && ko < kend) {
        T gzl[R], gyl[R];
        shr1<T, R>(Gz1, gzl);
        shr1<T, R>(gy[1], gyl);
        const int64_t rowoff = (int64_t)ko * g.plane + (int64_t)j * g.P + i0;
        // wave > 0 and wave + 1 < NW here
        const V gzjmv = sB[1][wave - 1][lane], gxjmv = sB[2][wave - 1][lane];
        const V txl = sB[3][wave - 1][lane], txh = sB[3][wave + 1][lane];
        const V tzl = sB[4][wave - 1][lane], tzh = sB[4][wave + 1][lane];
        V oxv, oyv, ozv;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = i0 + r;
          const T gzjm = gzjmv[r];
          const T gxjm = gxjmv[r];
          const T mx = t6 * (txl[r] + txh[r]) + t23 * Tzx[r];
          const T mz = t6 * (tzl[r] + tzh[r]) + t23 * Txz[r];
          T ox = ah * ((gy[0][r] - gy[1][r]) - (gzjm - Gz1[r])) + h3 * mx;
          T oy = ah * ((gzl[r] - Gz1[r]) + (gx[1][r] - gx[0][r])) + h3 * massy[r];
          T oz = ah * ((gxjm - gx[1][r]) + (gy[1][r] - gyl[r])) + h3 * mz;
          // unknown masks: x-edge: i < n, 1 <= j,k <= n-1; y-edge: j < n, 1 <= i,k <= n-1; ...
          const bool iin = (i >= 1 && i <= g.n - 1), jin = (j >= 1 && j <= g.n - 1),
                     kin = (ko >= 1 && ko <= g.n - 1);
          bool ux = (i < g.n) && jin && kin;
          bool uy = iin && (j < g.n) && kin;
          bool uz = iin && jin && (ko < g.n);
          if constexpr (COEF) {
            // the four cells of each edge (planes ko - 1 = s - 2 and ko = s - 1)
            const T p00 = cf(bxq[r + 1], byl, bz2), p01 = cf(bxq[r + 1], byl, bz1),
                    p10 = cf(bxq[r + 1], by0, bz2), p11 = cf(bxq[r + 1], by0, bz1);
            const T m10 = cf(bxq[r], by0, bz2), m11 = cf(bxq[r], by0, bz1), m01 = cf(bxq[r], byl, bz1);
            ux = ux && p00 > T(0) && p01 > T(0) && p10 > T(0) && p11 > T(0);
            uy = uy && m10 > T(0) && m11 > T(0) && p10 > T(0) && p11 > T(0);
            uz = uz && m01 > T(0) && m11 > T(0) && p01 > T(0) && p11 > T(0);
          }
          if (MODE == 1) {
            ox = ux ? bcur[0][r] - ox : T(0);
            oy = uy ? bcur[1][r] - oy : T(0);
            oz = uz ? bcur[2][r] - oz : T(0);
          } else {
            ox = ux ? ox : T(0);
            oy = uy ? oy : T(0);
            oz = uz ? oz : T(0);
          }
          oxv[r] = ox;
          oyv[r] = oy;
          ozv[r] = oz;
          if (MODE == 2 && i <= g.n) {
            dot += (double)ox * (double)xp[1][r] + (double)oy * (double)yp[1][r] +
                   (double)oz * (double)zp[0][r];
          }
        }
        if (lane_in_row) {
          *reinterpret_cast<V*>(y + rowoff) = oxv;
          *reinterpret_cast<V*>(y + g.B + rowoff) = oyv;
          *reinterpret_cast<V*>(y + 2 * g.B + rowoff) = ozv;
        }
        // the position i = n of a row falls outside the lanes when n = 64 R: zero it
        if (lane == 63 && i0 + R == g.n) {
#pragma unroll
          for (int d = 0; d < 3; ++d) y[d * g.B + rowoff + R] = T(0);
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
  };
  auto prologue = [&](auto I, int s) { step(I, std::false_type(), s); };
  Unroll<D - 1>::run(prologue, s0);
  // steps kstart - 1 .. kend, padded to a multiple of U (trailing steps write nothing)
  auto main_step = [&](auto I, int s) {
    step(std::integral_constant<int, (D - 1 + decltype(I)::value) % U>(), std::true_type(), s);
  };
  const int nmain = (kend - kstart + 2 + U - 1) / U * U;
  for (int s = kstart - 1; s < kstart - 1 + nmain; s += U) Unroll<U>::run(main_step, s);
  // no ring load may be left in flight when the workgroup ends
  wait_vm<0>();
  if (MODE == 2) {
    // partial sum of this tile (indexed by tile: padding workgroups write none)
    __shared__ double sh[NW];
    const double t = block_sum(dot, sh);
    if (threadIdx.x == 0) part[(int64_t)pair * pstride + tile] = t;
  }
}

struct Tiling {
  int ntj, KZ, ntiles, nblocks;
};

// Tiles cover rows and planes 0 .. n - 1 (the boundary row and plane n ride along with
// the last tiles).
Tiling tiling(int n, int NW, int KZ) {
  Tiling t;
  const int TJ = NW - 2;
  t.ntj = (n + TJ - 1) / TJ;
  t.KZ = KZ;
  const int ntk = (n + KZ - 1) / KZ;
  t.ntiles = t.ntj * ntk;
  t.nblocks = (t.ntiles + 7) / 8 * 8;   // the XCD remap permutes [0, nblocks)
  return t;
}

template <typename T, int R, int NW, int D, int MODE, int SYNC = 2>
hipError_t launch_m(const T* x, const T* b, T* y, const Geom& g, const Bat& bt, int KZ, double* part,
                    int64_t pstride, double* dot, hipStream_t st) {
  const Tiling tl = tiling(g.n, NW, KZ);
  if (MODE == 2 && (part == nullptr || tl.ntiles > pstride)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)tl.nblocks, (unsigned)bt.count);
  if (bt.coef != nullptr) {
    if (bt.coef_r < 1 || bt.coef_r > kCoefMaxR || g.n % bt.coef_r) return hipErrorNotSupported;
    hipLaunchKernelGGL((k_stencil<T, R, NW, D, MODE, SYNC, true>), grid, dim3(64 * NW), 0, st, x, b, y, dgeom(g),
                       bt, g.h, tl.KZ, tl.ntj, tl.ntiles, part, pstride, 0);
    if (MODE == 2 && dot != nullptr) return launch_final(part, tl.ntiles, pstride, 1, dot, bt, st);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_stencil<T, R, NW, D, MODE, SYNC, false>), grid, dim3(64 * NW), 0, st, x, b, y, dgeom(g),
                     bt, g.h, tl.KZ, tl.ntj, tl.ntiles, part, pstride, 0);
  if (MODE == 2 && dot != nullptr) return launch_final(part, tl.ntiles, pstride, 1, dot, bt, st);
  return hipGetLastError();
}

// Launch variants: waves per workgroup, ring depth and barriers per step (2, or 1 with
// two copies of the exchange area where they fit), each fitting the 160 KB of LDS of a
// compute unit with one workgroup per unit (the residual mode carries b in the ring,
// twice the bytes per slot).  One barrier measured faster at 64^3 (FP32 residual 10.1 ->
// 9.0 us, FP64 apply 11.1 -> 10.5 us) and slower for the FP64 apply at 128^3 (29.3 ->
// 31.8 us): the tuner's table picks per size.
struct Variant {
  int nw, d, sync;
};

int compute_units() {
  static int cus = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
      v = 256;
    return v;
  }();
  return cus;
}

// Planes per workgroup for a variant, from a cost model: workgroups run one per compute
// unit, so the time is the number of rounds of workgroups times the steps of one
// workgroup (KZ + 3 padded to the ring depth, plus D - 1 steps that only start loads)
// times its waves (the work of a step).
struct Choice {
  int kz;
  int64_t cost;
};

Choice choose_kz(int n, int count, Variant v) {
  const int tj = v.nw - 2, ntj = (n + tj - 1) / tj;
  Choice best{n, INT64_MAX};
  for (int kz = 2; kz <= n; ++kz) {
    const int ntk = (n + kz - 1) / kz;
    const int64_t blocks = (int64_t)ntj * ntk * count;
    const int64_t rounds = (blocks + compute_units() - 1) / compute_units();
    const int steps = (kz + 3 + v.d - 1) / v.d * v.d + v.d - 1;
    const int64_t cost = rounds * steps * v.nw;
    if (cost < best.cost) best = Choice{kz, cost};
  }
  return best;
}

// Candidate variants per precision, row length and mode (index 0 or 1 of the
// instantiated pair below); returns the chosen one and its KZ.
template <typename T, int R>
void variants(int mode, Variant (&vs)[4], int* nv) {
  constexpr bool f64 = std::is_same<T, double>::value;
  if (R == 1) {
    // rows of 64 positions: half the ring bytes of R = 2, so the FP64 residual fits more
    // waves and a deeper ring
    if (f64) {
      if (mode == 1) { vs[0] = {6, 3, 2}; vs[1] = {10, 3, 2}; vs[2] = {8, 4, 2}; vs[3] = {8, 4, 1}; *nv = 4; }
      else { vs[0] = {10, 3, 2}; vs[1] = {8, 4, 2}; vs[2] = {6, 4, 2}; vs[3] = {6, 4, 1}; *nv = 4; }
    } else {
      if (mode == 1) { vs[0] = {10, 3, 2}; vs[1] = {8, 4, 2}; vs[2] = {10, 3, 1}; vs[3] = {8, 4, 1}; *nv = 4; }
      else { vs[0] = {10, 4, 2}; vs[1] = {8, 4, 2}; vs[2] = {10, 4, 1}; vs[3] = {8, 4, 1}; *nv = 4; }
    }
  } else if (R == 2) {
    if (f64) {
      if (mode == 1) { vs[0] = {6, 3, 2}; *nv = 1; }
      else { vs[0] = {10, 3, 2}; vs[1] = {8, 4, 2}; vs[2] = {6, 4, 2}; vs[3] = {6, 4, 1}; *nv = 4; }
    } else {
      if (mode == 1) { vs[0] = {10, 3, 2}; vs[1] = {8, 4, 2}; vs[2] = {10, 3, 1}; vs[3] = {8, 4, 1}; *nv = 4; }
      else { vs[0] = {10, 4, 2}; vs[1] = {8, 4, 2}; vs[2] = {10, 4, 1}; vs[3] = {8, 4, 1}; *nv = 4; }
    }
  } else {
    if (f64 && mode == 1) { *nv = 0; }   // does not fit: the caller falls back
    else { vs[0] = {4, 4, 2}; *nv = 1; }
  }
}

// The shape of a launch: a shape forced by the tuner's timing calls, else the tuned
// table's entry, else the cost model.
template <typename T, int R>
bool pick(int n, int count, int mode, int* which, int* kz, Variant* var) {
  Variant vs[4];
  int nv = 0;
  variants<T, R>(mode, vs, &nv);
  if (nv == 0) return false;
  int w = -1, z = 0;
  if (tune_forced_stencil(&w, &z) ||
      tune_lookup(kTuneStencil, n, (int)sizeof(T), mode, count, &w, &z)) {
    if (w >= 0 && w < nv && z >= 2 && z <= n) {
      *which = w;
      *kz = z;
      *var = vs[w];
      return true;
    }
  }
  int64_t best = INT64_MAX;
  for (int i = 0; i < nv; ++i) {
    const Choice c = choose_kz(n, count, vs[i]);
    if (c.cost < best) {
      best = c.cost;
      *which = i;
      *kz = c.kz;
      *var = vs[i];
    }
  }
  return true;
}

template <typename T, int R, int MODE>
hipError_t launch_mode(const T* x, const T* b, T* y, const Geom& g, const Bat& bt, double* part,
                       int64_t pstride, double* dot, hipStream_t st) {
  constexpr bool f64 = std::is_same<T, double>::value;
  int which = 0, kz = 8;
  Variant var{};
  if (!pick<T, R>(g.n, bt.count, MODE, &which, &kz, &var)) return hipErrorNotSupported;
  if constexpr (R == 1) {
    if constexpr (f64 && MODE == 1) {
      if (which == 0) return launch_m<T, R, 6, 3, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
      if (which == 1) return launch_m<T, R, 10, 3, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
      if (which == 2) return launch_m<T, R, 8, 4, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
      return launch_m<T, R, 8, 4, MODE, 1>(x, b, y, g, bt, kz, part, pstride, dot, st);
    }
    if constexpr (f64 && MODE != 1) {
      if (which == 0) return launch_m<T, R, 10, 3, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
      if (which == 1) return launch_m<T, R, 8, 4, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
      if (which == 2) return launch_m<T, R, 6, 4, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
      return launch_m<T, R, 6, 4, MODE, 1>(x, b, y, g, bt, kz, part, pstride, dot, st);
    }
    if constexpr (!f64 && MODE == 1) {
      if (which == 0) return launch_m<T, R, 10, 3, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
      if (which == 1) return launch_m<T, R, 8, 4, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
      if (which == 2) return launch_m<T, R, 10, 3, MODE, 1>(x, b, y, g, bt, kz, part, pstride, dot, st);
      return launch_m<T, R, 8, 4, MODE, 1>(x, b, y, g, bt, kz, part, pstride, dot, st);
    }
    if constexpr (!f64 && MODE != 1) {
      if (which == 0) return launch_m<T, R, 10, 4, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
      if (which == 1) return launch_m<T, R, 8, 4, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
      if (which == 2) return launch_m<T, R, 10, 4, MODE, 1>(x, b, y, g, bt, kz, part, pstride, dot, st);
      return launch_m<T, R, 8, 4, MODE, 1>(x, b, y, g, bt, kz, part, pstride, dot, st);
    }
  } else if constexpr (R == 2) {
    if constexpr (f64 && MODE == 1) return launch_m<T, R, 6, 3, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
    if constexpr (f64 && MODE != 1) {
      if (which == 0) return launch_m<T, R, 10, 3, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
      if (which == 1) return launch_m<T, R, 8, 4, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
      if (which == 2) return launch_m<T, R, 6, 4, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
      return launch_m<T, R, 6, 4, MODE, 1>(x, b, y, g, bt, kz, part, pstride, dot, st);
    }
    if constexpr (!f64 && MODE == 1) {
      if (which == 0) return launch_m<T, R, 10, 3, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
      if (which == 1) return launch_m<T, R, 8, 4, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
      if (which == 2) return launch_m<T, R, 10, 3, MODE, 1>(x, b, y, g, bt, kz, part, pstride, dot, st);
      return launch_m<T, R, 8, 4, MODE, 1>(x, b, y, g, bt, kz, part, pstride, dot, st);
    }
    if constexpr (!f64 && MODE != 1) {
      if (which == 0) return launch_m<T, R, 10, 4, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
      if (which == 1) return launch_m<T, R, 8, 4, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
      if (which == 2) return launch_m<T, R, 10, 4, MODE, 1>(x, b, y, g, bt, kz, part, pstride, dot, st);
      return launch_m<T, R, 8, 4, MODE, 1>(x, b, y, g, bt, kz, part, pstride, dot, st);
    }
  } else {
    if constexpr (!(f64 && MODE == 1)) return launch_m<T, R, 4, 4, MODE>(x, b, y, g, bt, kz, part, pstride, dot, st);
  }
  return hipErrorNotSupported;
}

template <typename T, int R>
hipError_t launch_r(const T* x, const T* b, T* y, const Geom& g, const Bat& bt, int mode,
                    double* part, int64_t pstride, double* dot, hipStream_t st) {
  if (mode == 0) return launch_mode<T, R, 0>(x, b, y, g, bt, part, pstride, dot, st);
  if (mode == 1) return launch_mode<T, R, 1>(x, b, y, g, bt, part, pstride, dot, st);
  return launch_mode<T, R, 2>(x, b, y, g, bt, part, pstride, dot, st);
}

}  // namespace

int stencil_max_n() { return 256; }
// Below this size the one-thread-per-node kernel is used: n <= 32 for a single pair (the
// plane kernel's few tiles lose to its launch there), n <= 16 for batches of four or more
// pairs, where the tiles of all pairs fill the chip.
int stencil_min_n(int count) { return count >= 4 ? 16 : 32; }

// partial sums per pair of the dot mode (FP64): one per tile of the chosen launch
int stencil_blocks(const Geom& g, int count) {
  if (g.n <= stencil_min_n(count) || g.n > stencil_max_n()) return 0;
  int which = 0, kz = 8;
  Variant var{};
  const bool ok = (g.n <= 64)    ? pick<double, 1>(g.n, count, 2, &which, &kz, &var)
                  : (g.n <= 128) ? pick<double, 2>(g.n, count, 2, &which, &kz, &var)
                                 : pick<double, 4>(g.n, count, 2, &which, &kz, &var);
  return ok ? tiling(g.n, var.nw, kz).ntiles : 0;
}

// room for the partial sums of any launch shape (any variant, at least 2 planes per
// workgroup): a tuned shape never overflows a buffer sized by it
int stencil_max_blocks(const Geom& g) {
  if (g.n > stencil_max_n()) return 0;
  return tiling(g.n, 4, 2).ntiles;
}

bool stencil_shape(int n, int elem, int mode, int count, int* variant, int* kz) {
  Variant var{};
  if (n <= 64) {
    if (elem == 8) return pick<double, 1>(n, count, mode, variant, kz, &var);
    return pick<float, 1>(n, count, mode, variant, kz, &var);
  }
  if (n <= 128) {
    if (elem == 8) return pick<double, 2>(n, count, mode, variant, kz, &var);
    return pick<float, 2>(n, count, mode, variant, kz, &var);
  }
  if (elem == 8) return pick<double, 4>(n, count, mode, variant, kz, &var);
  return pick<float, 4>(n, count, mode, variant, kz, &var);
}

int stencil_variant_count(int elem, int mode, int n) {
  Variant vs[4];
  int nv = 0;
  if (n <= 64) {
    if (elem == 8) variants<double, 1>(mode, vs, &nv);
    else variants<float, 1>(mode, vs, &nv);
  } else if (n <= 128) {
    if (elem == 8) variants<double, 2>(mode, vs, &nv);
    else variants<float, 2>(mode, vs, &nv);
  } else {
    if (elem == 8) variants<double, 4>(mode, vs, &nv);
    else variants<float, 4>(mode, vs, &nv);
  }
  return nv;
}

template <typename T>
hipError_t launch_stencil(const T* x, const T* b, T* y, const Geom& g, const Bat& bt, int mode,
                          double* part, int64_t pstride, double* dot, hipStream_t st) {
  // rows span 64 R positions: R = 1 up to n = 64 (the position i = n of a row of 65 is
  // written separately), R = 2 up to 128, R = 4 up to 256
  if (g.n <= stencil_min_n(bt.count)) return hipErrorInvalidValue;
  if (g.n <= 64) return launch_r<T, 1>(x, b, y, g, bt, mode, part, pstride, dot, st);
  if (g.n <= 128) return launch_r<T, 2>(x, b, y, g, bt, mode, part, pstride, dot, st);
  if (g.n <= 256) return launch_r<T, 4>(x, b, y, g, bt, mode, part, pstride, dot, st);
  return hipErrorInvalidValue;
}

template hipError_t launch_stencil<double>(const double*, const double*, double*, const Geom&,
                                           const Bat&, int, double*, int64_t, double*, hipStream_t);
template hipError_t launch_stencil<float>(const float*, const float*, float*, const Geom&, const Bat&,
                                          int, double*, int64_t, double*, hipStream_t);

}  // namespace ndmg
