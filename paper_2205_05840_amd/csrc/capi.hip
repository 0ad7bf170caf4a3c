// C ABI of the ndmg library: planning, setup, the symmetric V-cycle MG(k, g, z0, m)
// (Sec. 3.3, Fig. 1) and preconditioned conjugate gradients around it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/ndmg.h"
#include "kernels.hpp"
#include "ndmg_internal.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define NDMG_HIP(expr)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(NDMG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Scalar slots of the CG driver (device array of doubles).
enum { S_BB = 0, S_PQ = 1, S_RR = 2, S_RZA = 3, S_ZQA = 4, S_RZB = 5, S_ZQB = 6, S_CC = 8, S_N = 16 };

struct LevelHost {
  ndmg::Geom g;
  bool smoothed = false;
  ndmg::SubInfo sub{};
  std::vector<ndmg::Segment> segs;
  std::vector<int> chunks;             // (segment, first) pairs
  ndmg::LevelFactors fac;              // FP64 host copies (smoothed levels)
  std::vector<double> A0inv;           // coarsest level
  std::vector<int64_t> map;
  // offsets into the workspace
  size_t o_z = 0, o_r = 0, o_zi = 0, o_gg = 0, o_w = 0, o_g = 0, o_Y = 0;
  size_t o_ATinv = 0, o_Sinv = 0, o_lut = 0, o_slots = 0, o_segs = 0, o_chunks = 0;
  size_t o_XT = 0, o_bofs = 0;
  int nB = 0;
  size_t o_A0 = 0, o_map = 0;
  size_t nY = 0;
};

struct Plan {
  int n = 0;
  double length = 1.0, alpha = 1.0;
  ndmg_opts opts{};
  std::vector<LevelHost> lv;   // coarsest first
  size_t elem = 8;             // bytes of the V-cycle scalar type
  size_t o_pr = 0, o_pz = 0, o_pp = 0, o_pq = 0, o_part = 0, o_scal = 0;
  size_t npart = 0;
  size_t bytes = 0;
};

}  // namespace

struct ndmg_ctx {
  Plan plan;
  char* ws = nullptr;
  hipStream_t st = nullptr;
  double* host_scal = nullptr;   // pinned
  hipGraphExec_t gexec[2] = {nullptr, nullptr};   // CG iteration body, by scalar-slot parity
  double* graph_u = nullptr;                       // solution pointer the graphs were captured with
};

namespace {

int make_plan(int n, double length, double alpha, const ndmg_opts* o_in, Plan* pl) {
  ndmg_opts o;
  ndmg_default_opts(&o);
  if (o_in) o = *o_in;
  if (n < 2) return fail(NDMG_EINVAL, "n must be >= 2");
  if (!(length > 0.0) || !std::isfinite(length)) return fail(NDMG_EINVAL, "length must be > 0");
  if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(NDMG_EINVAL, "alpha must be > 0");
  if (o.smoother != NDMG_SMOOTHER_VERTEX) return fail(NDMG_EINVAL, "unsupported smoother");
  if (o.m < 1 || o.m > 64) return fail(NDMG_EINVAL, "m must be in [1, 64]");
  if (o.precision != NDMG_PREC_FP64 && o.precision != NDMG_PREC_FP32)
    return fail(NDMG_EINVAL, "unsupported precision");
  if (o.subdomain != 2) return fail(NDMG_EINVAL, "subdomain size must be 2");
  if (o.eta <= 0.0) o.eta = 1.0 / 9.0;
  if (n > 2048) return fail(NDMG_EINVAL, "n too large");
  pl->n = n;
  pl->length = length;
  pl->alpha = alpha;
  pl->opts = o;
  pl->elem = (o.precision == NDMG_PREC_FP32) ? 4 : 8;
  std::vector<int> sizes{n};
  while (sizes.back() % 2 == 0 && sizes.back() / 2 >= 2) sizes.push_back(sizes.back() / 2);
  std::reverse(sizes.begin(), sizes.end());
  pl->lv.clear();
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o2 = off;
    off = align_up(off + bytes);
    return o2;
  };
  for (size_t k = 0; k < sizes.size(); ++k) {
    LevelHost L;
    L.g = ndmg::make_geom(sizes[k], length);
    const size_t vb = (size_t)L.g.len * pl->elem;
    L.o_z = take(vb);
    L.o_g = take(vb);
    if (k == 0) {
      const int nc = sizes[k];
      const int64_t N0 = 3LL * nc * (nc - 1) * (nc - 1);
      if (N0 > 1024)
        return fail(NDMG_EINVAL, "coarsest level has more than 1024 unknowns; choose n = c 2^j "
                                 "with c <= 7");
      L.o_A0 = take((size_t)N0 * N0 * pl->elem);
      L.o_map = take((size_t)N0 * sizeof(int64_t));
    } else {
      const int s = std::min(o.subdomain, sizes[k] / 2);
      if (sizes[k] % s) return fail(NDMG_EINVAL, "level not divisible by the subdomain size");
      L.smoothed = true;
      L.sub = ndmg::make_sub(s, sizes[k]);
      L.segs = ndmg::vertex_segments(L.sub.nH, o.boundary_patches != 0);
      L.chunks.clear();
      for (size_t si = 0; si < L.segs.size(); ++si)
        for (int f = 0; f < L.segs[si].count; f += 64 * ndmg::patch_groups(L.sub.nH)) {
          L.chunks.push_back((int)si);
          L.chunks.push_back(f);
        }
      L.o_r = take(vb);
      L.o_zi = take(vb);
      L.o_gg = take(vb);
      L.o_w = take(vb);
      const size_t nv = (size_t)(L.sub.nH + 1);
      L.nY = nv * nv * nv * (size_t)L.sub.npad;
      L.o_Y = take(L.nY * pl->elem);
      L.o_ATinv = take((size_t)L.sub.nI * L.sub.nI * pl->elem);
      L.nB = (int)ndmg::boundary_dofs(L.sub.s).size();
      L.o_XT = take((size_t)L.sub.nI * L.nB * pl->elem);
      L.o_bofs = take((size_t)L.nB * sizeof(int64_t));
      L.o_Sinv = take((size_t)27 * L.sub.npad * L.sub.npad * pl->elem);
      L.o_lut = take((size_t)3 * L.sub.lut_w * L.sub.lut_w * L.sub.lut_w * sizeof(int));
      L.o_slots = take((size_t)L.sub.nG * 4 * sizeof(int));
      L.o_segs = take(std::max<size_t>(1, L.segs.size()) * 8 * sizeof(int));
      L.o_chunks = take(std::max<size_t>(1, L.chunks.size()) * sizeof(int));
    }
    pl->lv.push_back(std::move(L));
  }
  const ndmg::Geom& gf = pl->lv.back().g;
  const size_t v8 = (size_t)gf.len * sizeof(double);
  pl->o_pr = take(v8);
  pl->o_pz = take(v8);
  pl->o_pp = take(v8);
  pl->o_pq = take(v8);
  const size_t cc_parts = (size_t)((gf.n + 1 + 63) / 64) * (gf.n + 1) * (gf.n + 1);
  pl->npart = std::max<size_t>(std::max<size_t>(2 * ndmg::kRedBlocks, cc_parts),
                               (size_t)ndmg::stencil_blocks(gf));
  pl->o_part = take(pl->npart * sizeof(double));
  pl->o_scal = take(S_N * sizeof(double));
  pl->bytes = off;
  return NDMG_OK;
}

template <typename T>
T* at(ndmg_ctx* c, size_t off) {
  return reinterpret_cast<T*>(c->ws + off);
}

template <typename T>
ndmg::LevelPtrs<T> level_ptrs(ndmg_ctx* c, const LevelHost& L) {
  ndmg::LevelPtrs<T> p;
  p.z = at<T>(c, L.o_z);
  p.r = at<T>(c, L.o_r);
  p.zi = at<T>(c, L.o_zi);
  p.gg = at<T>(c, L.o_gg);
  p.w = at<T>(c, L.o_w);
  p.Y = at<T>(c, L.o_Y);
  p.ATinv = at<T>(c, L.o_ATinv);
  p.Sinv = at<T>(c, L.o_Sinv);
  p.XT = at<T>(c, L.o_XT);
  p.bofs = at<int64_t>(c, L.o_bofs);
  return p;
}

ndmg::DSub level_dsub(ndmg_ctx* c, const LevelHost& L) {
  ndmg::DSub d;
  d.s = L.sub.s;
  d.nH = L.sub.nH;
  d.nI = L.sub.nI;
  d.nG = L.sub.nG;
  d.npad = L.sub.npad;
  d.lut_w = L.sub.lut_w;
  d.lut = at<int>(c, L.o_lut);
  d.slots = at<int>(c, L.o_slots);
  d.segs = at<int>(c, L.o_segs);
  d.chunks = at<int>(c, L.o_chunks);
  d.nchunks = (int)(L.chunks.size() / 2);
  d.gpw = ndmg::patch_groups(L.sub.nH);
  return d;
}

template <typename T>
std::vector<T> cast_vec(const std::vector<double>& v) {
  return std::vector<T>(v.begin(), v.end());
}

template <typename T>
int upload_factors(ndmg_ctx* c) {
  Plan& pl = c->plan;
  std::vector<std::vector<char>> keep;
  auto put = [&](size_t off, const void* src, size_t bytes) -> int {
    if (bytes == 0) return NDMG_OK;
    keep.emplace_back((const char*)src, (const char*)src + bytes);
    NDMG_HIP(hipMemcpyAsync(c->ws + off, keep.back().data(), bytes, hipMemcpyHostToDevice, c->st));
    return NDMG_OK;
  };
  for (auto& L : pl.lv) {
    int rc;
    if (!L.smoothed) {
      auto a = cast_vec<T>(L.A0inv);
      if ((rc = put(L.o_A0, a.data(), a.size() * sizeof(T)))) return rc;
      if ((rc = put(L.o_map, L.map.data(), L.map.size() * sizeof(int64_t)))) return rc;
      continue;
    }
    auto at_ = cast_vec<T>(L.fac.ATinv);
    auto si = cast_vec<T>(L.fac.Sinv);
    auto xt = cast_vec<T>(L.fac.XT);
    if ((rc = put(L.o_ATinv, at_.data(), at_.size() * sizeof(T)))) return rc;
    if ((rc = put(L.o_XT, xt.data(), xt.size() * sizeof(T)))) return rc;
    {
      auto bd = ndmg::boundary_dofs(L.sub.s);
      std::vector<int64_t> bo;
      for (auto& q : bd)
        bo.push_back(q.d * L.g.B + (int64_t)q.dz * L.g.plane + (int64_t)q.dy * L.g.P + q.dx);
      if ((rc = put(L.o_bofs, bo.data(), bo.size() * sizeof(int64_t)))) return rc;
    }
    if ((rc = put(L.o_Sinv, si.data(), si.size() * sizeof(T)))) return rc;
    auto lut = ndmg::slot_lookup(L.sub.s);
    if ((rc = put(L.o_lut, lut.data(), lut.size() * sizeof(int)))) return rc;
    auto slots = ndmg::vertex_slots(L.sub.s);
    std::vector<int> sl;
    for (auto& q : slots) {
      sl.push_back(q.d);
      sl.push_back(q.dx);
      sl.push_back(q.dy);
      sl.push_back(q.dz);
    }
    if ((rc = put(L.o_slots, sl.data(), sl.size() * sizeof(int)))) return rc;
    std::vector<int> sg;
    for (auto& q : L.segs) {
      sg.push_back(q.type);
      for (int a = 0; a < 3; ++a) sg.push_back(q.lo[a]);
      for (int a = 0; a < 3; ++a) sg.push_back(q.dims[a]);
      sg.push_back(q.count);
    }
    if ((rc = put(L.o_segs, sg.data(), sg.size() * sizeof(int)))) return rc;
    if ((rc = put(L.o_chunks, L.chunks.data(), L.chunks.size() * sizeof(int)))) return rc;
  }
  NDMG_HIP(hipStreamSynchronize(c->st));   // host staging buffers die with `keep`
  return NDMG_OK;
}

// z = MG(k, g, 0, m) (Fig. 1).
template <typename T>
int vcycle_rec(ndmg_ctx* c, int k, const T* g, T* z) {
  Plan& pl = c->plan;
  LevelHost& L = pl.lv[k];
  if (k == 0) {
    NDMG_HIP(ndmg::launch_coarse<T>(g, z, at<T>(c, L.o_A0), at<int64_t>(c, L.o_map),
                                    (int)L.map.size(), c->st));
    return NDMG_OK;
  }
  const int m = pl.opts.m;
  const double eta = pl.opts.eta, alpha = pl.alpha;
  auto P = level_ptrs<T>(c, L);
  auto D = level_dsub(c, L);
  LevelHost& Lc = pl.lv[k - 1];
  // z_1 .. z_m: pre-smoothing from z_0 = 0
  NDMG_HIP(ndmg::launch_smooth<T>(g, z, P, D, L.g, alpha, eta, 1, c->st));
  for (int l = 1; l < m; ++l) {
    NDMG_HIP(ndmg::launch_apply<T>(z, g, P.r, L.g, alpha, 1, c->st));
    NDMG_HIP(ndmg::launch_smooth<T>(P.r, z, P, D, L.g, alpha, eta, 0, c->st));
  }
  // gbar = I_k^{k-1} (g - A z_m)
  NDMG_HIP(ndmg::launch_apply<T>(z, g, P.r, L.g, alpha, 1, c->st));
  NDMG_HIP(ndmg::launch_restrict<T>(P.r, at<T>(c, Lc.o_g), L.g, Lc.g, c->st));
  int rc = vcycle_rec<T>(c, k - 1, at<T>(c, Lc.o_g), at<T>(c, Lc.o_z));
  if (rc) return rc;
  // z_{m+1} = z_m + I_{k-1}^k MG(k-1, gbar, 0, m)
  NDMG_HIP(ndmg::launch_prolong_add<T>(at<T>(c, Lc.o_z), z, L.g, Lc.g, c->st));
  // post-smoothing
  for (int l = 0; l < m; ++l) {
    NDMG_HIP(ndmg::launch_apply<T>(z, g, P.r, L.g, alpha, 1, c->st));
    NDMG_HIP(ndmg::launch_smooth<T>(P.r, z, P, D, L.g, alpha, eta, 0, c->st));
  }
  return NDMG_OK;
}

// B g for FP64 vectors of the finest level, in the context's precision.
int precondition(ndmg_ctx* c, const double* g, double* z) {
  Plan& pl = c->plan;
  const int J = (int)pl.lv.size() - 1;
  LevelHost& L = pl.lv[J];
  if (pl.opts.precision == NDMG_PREC_FP64) {
    if (J == 0) {
      NDMG_HIP(ndmg::launch_coarse<double>(g, z, at<double>(c, L.o_A0), at<int64_t>(c, L.o_map),
                                           (int)L.map.size(), c->st));
      return NDMG_OK;
    }
    return vcycle_rec<double>(c, J, g, z);
  }
  float* gf = at<float>(c, L.o_g);
  float* zf = at<float>(c, L.o_z);
  NDMG_HIP((ndmg::launch_convert<double, float>(g, gf, L.g.len, c->st)));
  int rc = vcycle_rec<float>(c, J, gf, zf);
  if (rc) return rc;
  NDMG_HIP((ndmg::launch_convert<float, double>(zf, z, L.g.len, c->st)));
  return NDMG_OK;
}

// q = A p with p^T q (slot S_PQ), then u += alpha p, r -= alpha q (alpha = s[num] / s[PQ])
// and r . r (slot S_RR).
int cg_apply_update(ndmg_ctx* c, double* u, int num) {
  Plan& pl = c->plan;
  const ndmg::Geom& g = pl.lv.back().g;
  const int64_t len = g.len;
  double* r = at<double>(c, pl.o_pr);
  double* p = at<double>(c, pl.o_pp);
  double* q = at<double>(c, pl.o_pq);
  double* part = at<double>(c, pl.o_part);
  double* sc = at<double>(c, pl.o_scal);
  if (g.n > ndmg::stencil_min_n() && g.n <= ndmg::stencil_max_n()) {
    int np = 0;
    NDMG_HIP(ndmg::launch_stencil<double>(p, nullptr, q, g, pl.alpha, 2, part, &np, c->st));
    NDMG_HIP(ndmg::launch_final(part, np, 1, sc + S_PQ, c->st));
  } else {
    NDMG_HIP(ndmg::launch_apply<double>(p, nullptr, q, g, pl.alpha, 0, c->st));
    NDMG_HIP(ndmg::launch_dot(p, q, nullptr, part, sc + S_PQ, len, c->st));
  }
  NDMG_HIP(ndmg::launch_cg_update(u, r, p, q, sc, num, S_PQ, part, sc + S_RR, len, c->st));
  return NDMG_OK;
}

// One CG iteration after the first: z = B r; s[nxt] = r . z (and s[nxt+1] = z . q for the
// flexible beta); p = z + beta p; then cg_apply_update with alpha = s[nxt] / p^T A p.
int cg_body_eager(ndmg_ctx* c, double* u, int cur, int nxt) {
  Plan& pl = c->plan;
  const int64_t len = pl.lv.back().g.len;
  double* r = at<double>(c, pl.o_pr);
  double* z = at<double>(c, pl.o_pz);
  double* p = at<double>(c, pl.o_pp);
  double* q = at<double>(c, pl.o_pq);
  double* part = at<double>(c, pl.o_part);
  double* sc = at<double>(c, pl.o_scal);
  const bool flexible =
      pl.opts.flexible > 0 || (pl.opts.flexible < 0 && pl.opts.precision == NDMG_PREC_FP32);
  int rc = precondition(c, r, z);
  if (rc) return rc;
  NDMG_HIP(ndmg::launch_dot(z, r, flexible ? q : nullptr, part, sc + nxt, len, c->st));
  NDMG_HIP(ndmg::launch_cg_direction(p, z, sc, nxt, cur, flexible ? 1 : 0, nxt + 1, cur, S_PQ, len,
                                     c->st));
  return cg_apply_update(c, u, nxt);
}

void drop_graphs(ndmg_ctx* c) {
  for (int i = 0; i < 2; ++i)
    if (c->gexec[i]) {
      (void)hipGraphExecDestroy(c->gexec[i]);
      c->gexec[i] = nullptr;
    }
  c->graph_u = nullptr;
}

int cg_body(ndmg_ctx* c, double* u, int cur, int nxt) {
  if (!c->plan.opts.use_graphs || c->st == nullptr) return cg_body_eager(c, u, cur, nxt);
  if (c->graph_u != u) drop_graphs(c);
  const int par = (cur == S_RZA) ? 0 : 1;
  if (!c->gexec[par]) {
    hipGraph_t graph = nullptr;
    NDMG_HIP(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
    int rc = cg_body_eager(c, u, cur, nxt);
    hipError_t e = hipStreamEndCapture(c->st, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail(NDMG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&c->gexec[par], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      c->gexec[par] = nullptr;
      return fail(NDMG_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    c->graph_u = u;
  }
  NDMG_HIP(hipGraphLaunch(c->gexec[par], c->st));
  return NDMG_OK;
}

int check_ctx(const ndmg_ctx* c) {
  if (!c) return fail(NDMG_EINVAL, "null context");
  return NDMG_OK;
}

}  // namespace

extern "C" {

void ndmg_default_opts(ndmg_opts* o) {
  if (!o) return;
  o->smoother = NDMG_SMOOTHER_VERTEX;
  o->m = 1;
  o->eta = 1.0 / 9.0;
  o->precision = NDMG_PREC_FP64;
  o->subdomain = 2;
  o->boundary_patches = 1;
  o->flexible = -1;
  o->use_graphs = 1;
}

const char* ndmg_last_error(void) { return g_err.c_str(); }

int ndmg_plan(int n, double length, double alpha, const ndmg_opts* opts, size_t* workspace_bytes,
              size_t* vec_len) {
  Plan pl;
  int rc = make_plan(n, length, alpha, opts, &pl);
  if (rc) return rc;
  if (workspace_bytes) *workspace_bytes = pl.bytes;
  if (vec_len) *vec_len = (size_t)pl.lv.back().g.len;
  return NDMG_OK;
}

int ndmg_setup(ndmg_ctx** out, int n, double length, double alpha, const ndmg_opts* opts,
               void* d_workspace, size_t workspace_bytes, void* stream) {
  if (!out) return fail(NDMG_EINVAL, "null output pointer");
  *out = nullptr;
  std::unique_ptr<ndmg_ctx> c(new ndmg_ctx());
  int rc = make_plan(n, length, alpha, opts, &c->plan);
  if (rc) return rc;
  if (!d_workspace) return fail(NDMG_EINVAL, "null workspace");
  if (workspace_bytes < c->plan.bytes)
    return fail(NDMG_EWORKSPACE, "workspace smaller than ndmg_plan reports");
  if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign)
    return fail(NDMG_EWORKSPACE, "workspace must be 256-byte aligned");
  c->ws = static_cast<char*>(d_workspace);
  c->st = static_cast<hipStream_t>(stream);
  Plan& pl = c->plan;
  std::string err;
  for (auto& L : pl.lv) {
    if (!L.smoothed) {
      if (!ndmg::build_coarse(L.g, alpha, &L.A0inv, &L.map, &err)) return fail(NDMG_EINVAL, err);
      continue;
    }
    if (!ndmg::build_level_factors(L.g.h, alpha, L.sub, pl.opts.boundary_patches != 0, &L.fac, &err))
      return fail(NDMG_EINVAL, err);
  }
  NDMG_HIP(hipMemsetAsync(c->ws, 0, pl.bytes, c->st));
  rc = (pl.elem == 8) ? upload_factors<double>(c.get()) : upload_factors<float>(c.get());
  if (rc) return rc;
  NDMG_HIP(hipHostMalloc((void**)&c->host_scal, S_N * sizeof(double), hipHostMallocDefault));
  *out = c.release();
  return NDMG_OK;
}

int ndmg_layout(const ndmg_ctx* c, int level, int64_t info[6]) {
  if (int rc = check_ctx(c)) return rc;
  if (!info) return fail(NDMG_EINVAL, "null info");
  const int nl = (int)c->plan.lv.size();
  if (level < 0) level += nl;
  if (level < 0 || level >= nl) return fail(NDMG_EINVAL, "level out of range");
  const ndmg::Geom& g = c->plan.lv[level].g;
  info[0] = g.n;
  info[1] = g.P;
  info[2] = g.B;
  info[3] = g.len;
  info[4] = nl;
  info[5] = 3LL * g.n * (g.n - 1) * (g.n - 1);
  return NDMG_OK;
}

int ndmg_apply(ndmg_ctx* c, const double* x, double* y) {
  if (int rc = check_ctx(c)) return rc;
  if (!x || !y) return fail(NDMG_EINVAL, "null vector");
  NDMG_HIP(ndmg::launch_apply<double>(x, nullptr, y, c->plan.lv.back().g, c->plan.alpha, 0, c->st));
  return NDMG_OK;
}

int ndmg_vcycle(ndmg_ctx* c, const double* g, double* z) {
  if (int rc = check_ctx(c)) return rc;
  if (!g || !z) return fail(NDMG_EINVAL, "null vector");
  return precondition(c, g, z);
}

int ndmg_pcg_solve(ndmg_ctx* c, const double* b, double* u, double rtol, int maxit, int* iters,
                   double* relres) {
  if (int rc = check_ctx(c)) return rc;
  if (!b || !u) return fail(NDMG_EINVAL, "null vector");
  if (!(rtol >= 0.0) || maxit < 1) return fail(NDMG_EINVAL, "bad rtol or maxit");
  Plan& pl = c->plan;
  const ndmg::Geom& g = pl.lv.back().g;
  const int64_t len = g.len;
  double* r = at<double>(c, pl.o_pr);
  double* z = at<double>(c, pl.o_pz);
  double* p = at<double>(c, pl.o_pp);
  double* part = at<double>(c, pl.o_part);
  double* sc = at<double>(c, pl.o_scal);
  if (iters) *iters = 0;
  if (relres) *relres = 0.0;
  NDMG_HIP(ndmg::launch_copy(b, r, len, c->st));
  NDMG_HIP(ndmg::launch_zero(u, len, c->st));
  NDMG_HIP(ndmg::launch_dot(b, b, nullptr, part, sc + S_BB, len, c->st));
  NDMG_HIP(hipMemcpyAsync(c->host_scal, sc, S_N * sizeof(double), hipMemcpyDeviceToHost, c->st));
  NDMG_HIP(hipStreamSynchronize(c->st));
  const double bb = c->host_scal[S_BB];
  if (!std::isfinite(bb)) return fail(NDMG_EBREAKDOWN, "non-finite right-hand side");
  if (bb == 0.0) return NDMG_OK;
  const double bnorm = std::sqrt(bb);
  int rc = precondition(c, r, z);
  if (rc) return rc;
  int cur = S_RZA, nxt = S_RZB;
  NDMG_HIP(ndmg::launch_dot(r, z, nullptr, part, sc + cur, len, c->st));
  NDMG_HIP(ndmg::launch_copy(z, p, len, c->st));
  if ((rc = cg_apply_update(c, u, cur))) return rc;
  for (int it = 1; it <= maxit; ++it) {
    if (it > 1) {
      // z = B r, rz_new, p = z + beta p, q = A p, u += alpha p, r -= alpha q, r . r:
      // replayed from a captured graph when the stream allows it
      if ((rc = cg_body(c, u, cur, nxt))) return rc;
      std::swap(cur, nxt);
    }
    NDMG_HIP(hipMemcpyAsync(c->host_scal, sc, S_N * sizeof(double), hipMemcpyDeviceToHost, c->st));
    NDMG_HIP(hipStreamSynchronize(c->st));
    const double pq = c->host_scal[S_PQ], rr = c->host_scal[S_RR], rz = c->host_scal[cur];
    if (!(pq > 0.0) || !std::isfinite(pq) || !std::isfinite(rr) || !std::isfinite(rz)) {
      if (iters) *iters = it;
      if (relres) *relres = std::sqrt(rr) / bnorm;
      return fail(NDMG_EBREAKDOWN, "PCG breakdown (p^T A p <= 0 or non-finite scalar)");
    }
    const double rel = std::sqrt(rr) / bnorm;
    if (iters) *iters = it;
    if (relres) *relres = rel;
    if (rel <= rtol) return NDMG_OK;
  }
  return fail(NDMG_ENOCONV, "PCG reached maxit");
}

int ndmg_assemble_rhs(ndmg_ctx* c, const double* f, double* b) {
  if (int rc = check_ctx(c)) return rc;
  if (!f || !b) return fail(NDMG_EINVAL, "null pointer");
  NDMG_HIP(ndmg::launch_assemble_rhs(f, b, c->plan.lv.back().g, c->st));
  return NDMG_OK;
}

int ndmg_curlcurl_form(ndmg_ctx* c, const double* lam, const double* u, int nrhs, double* out) {
  if (int rc = check_ctx(c)) return rc;
  if (!lam || !u || !out || nrhs < 0) return fail(NDMG_EINVAL, "bad arguments");
  Plan& pl = c->plan;
  const ndmg::Geom& g = pl.lv.back().g;
  double* part = at<double>(c, pl.o_part);
  double* sc = at<double>(c, pl.o_scal);
  double total = 0.0;
  for (int r = 0; r < nrhs; ++r) {
    NDMG_HIP(ndmg::launch_curlcurl_form(lam + (int64_t)r * g.len, u + (int64_t)r * g.len, g, part,
                                        sc + S_CC, c->st));
    NDMG_HIP(hipMemcpyAsync(c->host_scal, sc, S_N * sizeof(double), hipMemcpyDeviceToHost, c->st));
    NDMG_HIP(hipStreamSynchronize(c->st));
    total += c->host_scal[S_CC];
  }
  *out = total;
  return NDMG_OK;
}

int ndmg_export_factor(const ndmg_ctx* c, int level, int which, int type, double* buf, int* dims) {
  if (int rc = check_ctx(c)) return rc;
  if (!dims) return fail(NDMG_EINVAL, "null dims");
  const int nl = (int)c->plan.lv.size();
  if (level < 0) level += nl;
  if (level < 1 || level >= nl) return fail(NDMG_EINVAL, "level must be a smoothed level");
  const LevelHost& L = c->plan.lv[level];
  if (which == 0) {
    dims[0] = L.sub.nI;
    if (buf) std::memcpy(buf, L.fac.ATinv.data(), L.fac.ATinv.size() * sizeof(double));
    return NDMG_OK;
  }
  if (which == 1) {
    if (type < 0 || type > 26) return fail(NDMG_EINVAL, "type out of range");
    const int np = L.sub.npad;
    dims[0] = np;
    if (buf)
      std::memcpy(buf, L.fac.Sinv.data() + (size_t)type * np * np, (size_t)np * np * sizeof(double));
    return NDMG_OK;
  }
  return fail(NDMG_EINVAL, "which must be 0 or 1");
}

int ndmg_level_op(ndmg_ctx* c, int level, int op, const double* in, double* out) {
  if (int rc = check_ctx(c)) return rc;
  if (!in || !out) return fail(NDMG_EINVAL, "null vector");
  Plan& pl = c->plan;
  if (pl.elem != 8) return fail(NDMG_EINVAL, "level operations need an FP64 context");
  const int nl = (int)pl.lv.size();
  if (level < 0) level += nl;
  if (level < 0 || level >= nl) return fail(NDMG_EINVAL, "level out of range");
  LevelHost& L = pl.lv[level];
  switch (op) {
    case NDMG_OP_APPLY:
      NDMG_HIP(ndmg::launch_apply<double>(in, nullptr, out, L.g, pl.alpha, 0, c->st));
      return NDMG_OK;
    case NDMG_OP_SMOOTH: {
      if (!L.smoothed) return fail(NDMG_EINVAL, "the coarsest level has no smoother");
      auto P = level_ptrs<double>(c, L);
      auto D = level_dsub(c, L);
      NDMG_HIP(ndmg::launch_smooth<double>(in, out, P, D, L.g, pl.alpha, pl.opts.eta, 1, c->st));
      return NDMG_OK;
    }
    case NDMG_OP_RESTRICT:
      if (level < 1) return fail(NDMG_EINVAL, "restriction needs level >= 1");
      NDMG_HIP(ndmg::launch_restrict<double>(in, out, L.g, pl.lv[level - 1].g, c->st));
      return NDMG_OK;
    case NDMG_OP_PROLONG:
      if (level < 1) return fail(NDMG_EINVAL, "prolongation needs level >= 1");
      NDMG_HIP(ndmg::launch_prolong_add<double>(in, out, L.g, pl.lv[level - 1].g, c->st));
      return NDMG_OK;
    case NDMG_OP_COARSE:
      if (level != 0) return fail(NDMG_EINVAL, "coarse solve needs level 0");
      NDMG_HIP(ndmg::launch_coarse<double>(in, out, at<double>(c, L.o_A0), at<int64_t>(c, L.o_map),
                                           (int)L.map.size(), c->st));
      return NDMG_OK;
    default:
      return fail(NDMG_EINVAL, "unknown operation");
  }
}

int ndmg_destroy(ndmg_ctx* c) {
  if (!c) return NDMG_OK;
  drop_graphs(c);
  if (c->host_scal) (void)hipHostFree(c->host_scal);
  delete c;
  return NDMG_OK;
}

}  // extern "C"
