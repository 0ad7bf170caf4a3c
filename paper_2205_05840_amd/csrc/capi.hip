// C ABI of the ndmg library: planning, setup, the symmetric V-cycle MG(k, g, z0, m)
// (Sec. 3.3, Fig. 1) and preconditioned conjugate gradients around it, for one problem
// or for a batch of problems of uneven sizes with several right-hand sides each.
//
// A context holds one or more size classes (all problems with the same n).  Every
// kernel of a class works on all its (problem, right-hand side) pairs at once; the
// classes run on forked streams, and a CG iteration of the whole batch is captured as
// one HIP graph.  Each pair carries its own CG scalars and an active flag on the device:
// a converged pair drops out of every kernel of the following iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ndmg.h"
#include "generic.hpp"
#include "kernels.hpp"
#include "tuning.hpp"
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

#define NDMG_TRY(expr)          \
  do {                          \
    int rc_ = (expr);           \
    if (rc_ != NDMG_OK) return rc_; \
  } while (0)

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

using ndmg::kS_BB;
using ndmg::kS_CC;
using ndmg::kS_PQ;
using ndmg::kS_REL;
using ndmg::kS_RR;
using ndmg::kS_RZA;
using ndmg::kS_RZB;
using ndmg::kScalStride;

struct LevelHost {
  ndmg::Geom g;
  bool smoothed = false;
  ndmg::SubInfo sub{};
  std::vector<ndmg::Segment> segs;
  std::vector<int> chunks;             // per chunk: segment | gpw << 16, first, wave step, group step
  int gpw = 1;                         // 16-vertex groups per wave of the patch kernel
  std::vector<int64_t> map;            // coarsest level: padded offset of each unknown
  int nB = 0;
  // workspace offsets; per-pair arrays hold `count` copies, factors `nprob` copies
  size_t o_z = 0, o_g = 0, o_r = 0, o_zi = 0, o_gg = 0, o_w = 0, o_Y = 0;
  size_t o_ATinv = 0, o_XT = 0, o_Sinv = 0, o_A0 = 0, o_G = 0;
  size_t o_lut = 0, o_slots = 0, o_segs = 0, o_chunks = 0, o_bofs = 0, o_map = 0;
  size_t nY = 0;
  size_t blk_ATinv = 0, blk_XT = 0, blk_Sinv = 0, blk_A0 = 0;   // elements per problem
  size_t o_Bd = 0, blk_Bd = 0;         // dense V-cycle matrix of the level (dense level only)
  int Nd = 0;                          // its unknowns
  // generic smoother (edge spaces, or subdomains of size 4): tables and factors
  bool gen = false;
  ndmg::GenTables gt;
  size_t o_C = 0, o_gX = 0, o_gE = 0, o_gS = 0, blk_gX = 0, blk_gE = 0, blk_gS = 0;
  size_t o_guI = 0, o_grI = 0, o_grE = 0, o_gcI = 0, o_guP = 0, o_grP = 0, o_gcP = 0, o_ggam = 0, o_gcc = 0,
         o_gcodes = 0;
  int64_t ylenG = 0, clenG = 0;
};

struct Cls {
  int n = 0, nprob = 0, nrhs = 1, count = 0;
  int small_top = -1;              // levels 0 .. small_top run as one launch
  int dense_k = -1;                // MG(dense_k, ., 0, m) applied as a dense matrix (-1: none)
  int dense_K = 1;                 // matrix columns per problem built per V-cycle launch
  bool dense_t = false;            // matrices stored transposed (classes of many problems)
  std::vector<int> probs;          // problem indices, input order
  std::vector<double> alpha;       // per problem
  std::vector<LevelHost> lv;       // coarsest first
  int64_t vlen = 0;                // vector length of the finest level (per pair)
  int64_t vec_off = 0;             // first element of the class in a batch vector
  int64_t pstride = 0;             // partial sums per pair
  size_t o_pr = 0, o_pz = 0, o_pp = 0, o_pq = 0, o_part = 0, o_scal = 0;
  size_t o_alpha = 0, o_act = 0, o_iters = 0, o_status = 0;
  size_t o_hist = 0;               // per pair: (r . z, p . A p) of the first kHistCap iterations
  size_t o_tw = 0, o_tb = 0;       // time stepping: predictor and right-hand side (FP64, per pair)
  size_t o_alpha0 = 0;             // zeros: alpha = 0 turns the operator into the mass matrix
  size_t o_coef = 0;               // coefficient boxes (r^3 doubles), if any
};

struct Plan {
  double length = 1.0;
  int levels = 0;                  // 0: every level down to 2^3 or 3^3; else this many
  ndmg_opts opts{};                // (opts.coef cleared: the values live in coef below)
  std::vector<double> coef;        // coefficient boxes (Sec. 6), r^3 factors; empty: constant
  ndmg::CoefBoxes boxes() const { return coef.empty() ? ndmg::CoefBoxes{} : ndmg::CoefBoxes{opts.coef_r, coef.data()}; }
  size_t elem = 8;                 // bytes of the V-cycle scalar type
  int nprob = 0, nrhs = 1;
  std::vector<Cls> cls;            // ascending n
  std::vector<int> prob_cls, prob_pos;
  int64_t total_len = 0;           // batch vector length
  int npairs = 0;
  size_t bytes = 0;
};

}  // namespace

struct ndmg_ctx {
  Plan plan;
  char* ws = nullptr;
  hipStream_t st = nullptr;
  std::vector<hipStream_t> side;           // class i >= 1 runs on side[i - 1]
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  int* host_nact = nullptr;                // pinned (coherent, mapped), two sets of one per class
  int* dev_nact = nullptr;                 // its device address: the convergence kernel writes it
  hipEvent_t ev_nact[2] = {nullptr, nullptr};   // recorded after the writes of each set
  double* host_scal = nullptr;             // pinned, kScalStride per pair
  int* host_int = nullptr;                 // pinned, iters and status per pair
  hipGraphExec_t gexec[2] = {nullptr, nullptr};   // CG iteration body, by scalar-slot parity
  double* graph_u = nullptr;                       // solution pointer the graphs were captured with
};

namespace {

int check_opts(const ndmg_opts* o_in, ndmg_opts* o) {
  ndmg_default_opts(o);
  if (o_in) *o = *o_in;
  if (o->smoother != NDMG_SMOOTHER_VERTEX && o->smoother != NDMG_SMOOTHER_EDGE)
    return fail(NDMG_EINVAL, "unsupported smoother");
  if (o->m < 1 || o->m > 64) return fail(NDMG_EINVAL, "m must be in [1, 64]");
  if (o->precision != NDMG_PREC_FP64 && o->precision != NDMG_PREC_FP32)
    return fail(NDMG_EINVAL, "unsupported precision");
  if (o->subdomain != 2 && o->subdomain != 4) return fail(NDMG_EINVAL, "subdomain size must be 2 or 4");
  if (!(o->eta > 0.0)) o->eta = (o->smoother == NDMG_SMOOTHER_EDGE) ? 1.0 / 13.0 : 1.0 / 9.0;
  if (o->bottom_n > 0 && (o->smoother == NDMG_SMOOTHER_EDGE || o->subdomain != 2))
    return fail(NDMG_EINVAL, "the one-launch bottom (bottom_n) serves the vertex smoother with subdomain 2 only");
  if (o->bottom_n < 0 || o->bottom_n > 64) return fail(NDMG_EINVAL, "bottom_n must be in [0, 64]");
  if (o->dense_n < -1 || o->dense_n > 8) return fail(NDMG_EINVAL, "dense_n must be -1 or in [0, 8]");
  if (o->use_graphs < -1 || o->use_graphs > 1) return fail(NDMG_EINVAL, "use_graphs must be -1, 0 or 1");
  if (o->coef_r < 0 || o->coef_r > 64) return fail(NDMG_EINVAL, "coef_r must be in [0, 64]");
  if (o->domain && o->coef_r == 0) return fail(NDMG_EINVAL, "a domain needs the box grid: coef_r > 0");
  if (o->coef_r > 0) {
    if (!o->coef && !o->domain) return fail(NDMG_EINVAL, "coef_r > 0 needs the coef array or a domain");
    if (o->bottom_n > 0) return fail(NDMG_EINVAL, "the one-launch bottom (bottom_n) takes a constant alpha on the cube");
    const size_t nb = (size_t)o->coef_r * o->coef_r * o->coef_r;
    size_t inside = 0;
    for (size_t b = 0; b < nb; ++b) {
      if (o->coef && (!(o->coef[b] > 0.0) || !std::isfinite(o->coef[b])))
        return fail(NDMG_EINVAL, "coef values must be > 0");
      inside += (!o->domain || o->domain[b]) ? 1 : 0;
    }
    if (inside == 0) return fail(NDMG_EINVAL, "the domain keeps no box");
  }
  return NDMG_OK;
}

// Workspace layout of one size class; `take` hands out aligned offsets.
template <typename Take>
int plan_class(Cls& C, const Plan& pl, Take&& take) {
  const int n = C.n;
  std::vector<int> sizes{n};
  while (sizes.back() % 2 == 0 && sizes.back() / 2 >= 2) sizes.push_back(sizes.back() / 2);
  if (pl.levels > 0) {
    if (pl.levels > (int)sizes.size())
      return fail(NDMG_EINVAL, "n = " + std::to_string(n) + " has at most " + std::to_string(sizes.size()) +
                                   " levels (halving while a level is even and its half >= 2)");
    sizes.resize(pl.levels);
  }
  std::reverse(sizes.begin(), sizes.end());
  const size_t np = (size_t)C.nprob, el = pl.elem;
  const ndmg::CoefBoxes cf = pl.boxes();
  if (cf.r > 0 && sizes[0] % cf.r)
    return fail(NDMG_EINVAL, "coef_r = " + std::to_string(cf.r) + " must divide the coarsest level's n (" +
                                 std::to_string(sizes[0]) + "), so that every element of every level lies in one box");
  // dense bottom: the finest level with n_k <= dense_n, if above the coarsest.  -1: 8 for
  // classes of fewer than 16 problems, 4 for larger ones (whose build, nprob N_k V-cycles
  // on unit vectors, then costs 0.01 instead of 0.2 s for 512 problems, and whose solves
  // measured as fast: the bottom levels of many problems share each launch)
  const int dense_n = pl.opts.dense_n >= 0 ? pl.opts.dense_n : (C.nprob >= 16 ? 4 : 8);
  C.dense_k = -1;
  for (size_t k = 1; k < sizes.size(); ++k)
    if (sizes[k] <= dense_n) C.dense_k = (int)k;
  int64_t Nd = 0;
  if (C.dense_k >= 1) {
    const int64_t nk = sizes[C.dense_k];
    Nd = cf.r > 0 ? (int64_t)ndmg::unknown_offsets(ndmg::make_geom((int)nk, pl.length), cf).size()
                  : 3 * nk * (nk - 1) * (nk - 1);
    if (Nd > ndmg::kDenseMaxN) return fail(NDMG_EINVAL, "dense level too large");
    // the level vectors at and below the dense level serve the build at setup (nprob x
    // dense_K pairs, dense_K unit columns per problem and recursion pass); at run time only
    // its g and z are used, by count pairs.  Classes of many problems take up to 2048
    // columns in all per pass (at most a few hundred MB of level vectors): with 4 the
    // 512-problem batch spent 0.6 s of its 0.7 s setup in 1108 passes of eager launches
    // (16384 columns per pass measured no faster than 2048)
    const int64_t budget = C.nprob >= 16 ? 2048 : 256;
    C.dense_K = (int)std::max<int64_t>(C.nrhs, std::min<int64_t>(Nd, budget / C.nprob));
    // many problems: one thread per row over the transposed matrix (coalesced, no
    // cross-lane sums); few: waves over rows, more workgroups per problem
    C.dense_t = C.nprob >= 8;
  } else {
    C.dense_K = C.nrhs;
  }
  C.lv.clear();
  for (size_t k = 0; k < sizes.size(); ++k) {
    LevelHost L;
    L.g = ndmg::make_geom(sizes[k], pl.length);
    const size_t cnt = ((int)k <= C.dense_k) ? np * (size_t)C.dense_K : (size_t)C.count;
    const size_t vb = (size_t)L.g.len * el * cnt;
    L.o_z = take(vb);
    L.o_g = take(vb);
    if (k == 0) {
      const int nc = sizes[k];
      const int64_t N0 = cf.r > 0 ? (int64_t)ndmg::unknown_offsets(L.g, cf).size() : 3LL * nc * (nc - 1) * (nc - 1);
      if (N0 > 1024)
        return fail(NDMG_EINVAL, "n = " + std::to_string(n) + ": the coarsest level (" + std::to_string(nc) +
                                     "^3, solved exactly) has " + std::to_string(N0) +
                                     " unknowns, more than 1024; choose n = c 2^j with c <= 7, or more levels");
      L.blk_A0 = (size_t)N0 * N0;
      L.o_A0 = take(L.blk_A0 * el * np);
      L.o_map = take((size_t)N0 * sizeof(int64_t));
    } else {
      const int s = std::min(pl.opts.subdomain, sizes[k] / 2);
      if (sizes[k] % s) return fail(NDMG_EINVAL, "level not divisible by the subdomain size");
      L.smoothed = true;
      L.sub = ndmg::make_sub(s, sizes[k]);
      if (pl.opts.smoother == NDMG_SMOOTHER_EDGE || s != 2 || cf.r > 0) {
        // the generic smoother: gathered products over subdomains and patches (also every
        // level of a coefficient with jumps: its factors differ from box to box)
        L.gen = true;
        std::string err;
        if (!ndmg::build_gen_tables(L.g, s, pl.opts.smoother == NDMG_SMOOTHER_EDGE ? 1 : 0,
                                    pl.opts.boundary_patches != 0, &L.gt, &err, cf))
          return fail(NDMG_EINVAL, err);
        L.o_r = take(vb);
        L.o_gg = take(vb);
        L.o_w = take(vb);
        L.ylenG = (int64_t)L.gt.unitsP.size() * L.gt.npadP;
        L.clenG = (int64_t)L.gt.unitsI.size() * L.gt.npadB;
        L.o_Y = take((size_t)L.ylenG * el * cnt);
        L.o_C = take((size_t)L.clenG * el * cnt);
        L.blk_gX = (size_t)L.gt.ntypesI * L.gt.npadI * L.gt.npadB;
        L.blk_gE = (size_t)L.gt.ntypesI * L.gt.npadE * L.gt.npadI;
        L.blk_gS = (size_t)L.gt.ntypes * L.gt.npadP * L.gt.npadP;
        L.o_gX = take(L.blk_gX * el * np);
        L.o_gE = take(L.blk_gE * el * np);
        L.o_gS = take(L.blk_gS * el * np);
        L.o_guI = take(L.gt.unitsI.size() * sizeof(int64_t));
        L.o_grI = take(L.gt.relI.size() * sizeof(int64_t));
        L.o_grE = take(L.gt.relE.size() * sizeof(int64_t));
        L.o_gcI = take(std::max<size_t>(1, L.gt.chunksI.size()) * sizeof(int));
        L.o_guP = take(std::max<size_t>(1, L.gt.unitsP.size()) * sizeof(int64_t));
        L.o_grP = take(L.gt.relP.size() * sizeof(int64_t));
        L.o_gcP = take(std::max<size_t>(1, L.gt.chunksP.size()) * sizeof(int));
        L.o_ggam = take(std::max<size_t>(1, L.gt.gamma.size()) * sizeof(int));
        L.o_gcc = take(std::max<size_t>(1, L.gt.ccodes.size()) * sizeof(int));
        L.o_gcodes = take(std::max<size_t>(1, L.gt.codes.size()) * sizeof(int));
        if ((int)k == C.dense_k) {
          L.Nd = (int)Nd;
          L.blk_Bd = (size_t)Nd * Nd;
          L.o_Bd = take(L.blk_Bd * el * np);
          L.o_map = take((size_t)Nd * sizeof(int64_t));
        }
        C.lv.push_back(std::move(L));
        continue;
      }
      L.segs = ndmg::vertex_segments(L.sub.nH, pl.opts.boundary_patches != 0);
      L.chunks.clear();
      int64_t groups = 0;
      for (const auto& sg : L.segs) groups += (sg.count + 15) / 16;
      L.gpw = ndmg::patch_groups(groups * C.count, el);
      int tuned_i = 0, tuned_b = 0;
      const bool tuned = ndmg::tune_lookup(ndmg::kTunePatch, sizes[k], (int)el, 0, C.count, &tuned_i, &tuned_b) &&
                         tuned_i >= 1 && tuned_i <= 8 && tuned_b >= 1 && tuned_b <= 8;
      if (tuned) L.gpw = tuned_i;
      // Boundary-type segments check every slot against the domain, so their groups cost
      // more: they get the fewest groups per wave that still let the whole grid be
      // resident at once (else as many as the interior), so that they do not finish last.
      auto nchunks_with = [&](int gb) {
        int64_t nch = 0;
        for (const auto& sg : L.segs) nch += (sg.count + 64 * (sg.type == 13 ? L.gpw : gb) - 1) / (64 * (sg.type == 13 ? L.gpw : gb));
        return nch * C.count;
      };
      int gpw_b = L.gpw;
      for (int gb = 1; gb < L.gpw; ++gb)
        if (nchunks_with(gb) <= ndmg::patch_resident_blocks(el)) { gpw_b = gb; break; }
      if (tuned) gpw_b = tuned_b;
      for (size_t si = 0; si < L.segs.size(); ++si) {
        // and no more per wave than spreads a small segment over the 4 waves of one chunk
        const int gseg = (L.segs[si].count + 15) / 16;
        const int gs = std::max(1, std::min(L.segs[si].type == 13 ? L.gpw : gpw_b, (gseg + 3) / 4));
        // A segment of one group (a short edge of the box) in a class of several
        // right-hand sides: one workgroup per 4 right-hand sides of a problem, one per
        // wave (they share S^{-1}), instead of a workgroup per pair with 3 idle waves.
        if (C.nrhs > 1 && gseg == 1) {
          L.chunks.push_back((int)si | 1 << 16 | ndmg::kChunkRhsWaves);
          L.chunks.push_back(0);
          L.chunks.push_back(0);
          L.chunks.push_back(16);
          continue;
        }
        for (int f = 0; f < L.segs[si].count; f += 64 * gs) {
          L.chunks.push_back((int)si | gs << 16);
          L.chunks.push_back(f);
          L.chunks.push_back(16 * gs);   // wave w starts at f + w * 16 gs
          L.chunks.push_back(16);        // and takes consecutive groups
        }
      }
      // One pair: the interior segment's chunks that run on one XCD (the kernel numbers
      // blocks with xcd_block: XCD x takes a contiguous range of chunks) share their
      // vertex range with the groups dealt out in turn, wave after wave, so that at any
      // time the XCD's waves work on one band of vertices whose gathered entries fit its
      // L2, instead of each wave on its own stretch across the XCD's whole range.
      if (C.count == 1) {
        const int nch = (int)(L.chunks.size() / 4);
        int c0 = -1, c1 = -1;
        for (int j = 0; j < nch; ++j)
          if (L.segs[L.chunks[4 * j] & 0xffff].type == 13) {   // (no right-hand-side chunks: one pair)
            if (c0 < 0) c0 = j;
            c1 = j + 1;
          }
        const int q = nch / 8, rem = nch % 8;
        for (int x = 0; x < 8 && c0 >= 0; ++x) {
          const int s0 = x * q + std::min(x, rem), s1 = s0 + q + (x < rem ? 1 : 0);
          const int j0 = std::max(c0, s0), j1 = std::min(c1, s1);
          if (j1 - j0 < 2) continue;
          const int start = L.chunks[4 * j0 + 1], nw = 4 * (j1 - j0);
          for (int j = j0; j < j1; ++j) {
            L.chunks[4 * j + 1] = start + 64 * (j - j0);
            L.chunks[4 * j + 2] = 16;
            L.chunks[4 * j + 3] = 16 * nw;
          }
        }
      }
      L.o_r = take(vb);
      L.o_zi = take(vb);
      L.o_gg = take(vb);
      L.o_w = take(vb);
      const size_t nv = (size_t)(L.sub.nH + 1);
      // row positions in bytes fit in 32 bits (the smoother's reads of Y assume it)
      if (ndmg::y_row_len(L.sub.nH) * 8 > UINT32_MAX) return fail(NDMG_EINVAL, "level too large for the patch result rows");
      L.nY = std::max<size_t>(nv * nv * nv, (size_t)ndmg::y_row_len(L.sub.nH)) * (size_t)L.sub.npad;
      L.o_Y = take(L.nY * el * cnt);
      // gathered patch inputs of the one-launch bottom of the V-cycle (small levels)
      if (sizes[k] <= pl.opts.bottom_n) L.o_G = take(L.nY * el * cnt);
      L.nB = (int)ndmg::boundary_dofs(L.sub.s).size();
      L.blk_ATinv = (size_t)L.sub.nI * L.sub.nI;
      L.blk_XT = (size_t)L.sub.nI * L.nB;
      L.blk_Sinv = (size_t)27 * L.sub.npad * L.sub.npad;
      L.o_ATinv = take(L.blk_ATinv * el * np);
      L.o_XT = take(L.blk_XT * el * np);
      L.o_Sinv = take(L.blk_Sinv * el * np);
      L.o_bofs = take((size_t)L.nB * sizeof(int64_t));
      L.o_lut = take((size_t)3 * L.sub.lut_w * L.sub.lut_w * L.sub.lut_w * sizeof(int));
      L.o_slots = take((size_t)L.sub.nG * 4 * sizeof(int));
      L.o_segs = take(std::max<size_t>(1, L.segs.size()) * 8 * sizeof(int));
      L.o_chunks = take(std::max<size_t>(1, L.chunks.size()) * sizeof(int));
      if ((int)k == C.dense_k) {
        L.Nd = (int)Nd;
        L.blk_Bd = (size_t)Nd * Nd;
        L.o_Bd = take(L.blk_Bd * el * np);
        L.o_map = take((size_t)Nd * sizeof(int64_t));
      }
    }
    C.lv.push_back(std::move(L));
  }
  {
    const int bn = pl.opts.bottom_n;
    C.small_top = -1;
    for (size_t k = 0; k < C.lv.size(); ++k)
      if (C.lv[k].g.n <= bn && C.lv[k].g.n <= 64 && (int)k < ndmg::kSmallMaxLevels) C.small_top = (int)k;
  }
  const ndmg::Geom& gf = C.lv.back().g;
  C.vlen = gf.len;
  const size_t cnt = (size_t)C.count;
  const size_t v8 = (size_t)gf.len * sizeof(double) * cnt;
  C.o_pr = take(v8);
  C.o_pz = take(v8);
  C.o_pp = take(v8);
  C.o_pq = take(v8);
  const int64_t cc_parts = (int64_t)((gf.n + 1 + 63) / 64) * (gf.n + 1) * (gf.n + 1);
  C.pstride = std::max<int64_t>(std::max<int64_t>(2 * ndmg::kRedBlocks, cc_parts),
                                (int64_t)ndmg::stencil_max_blocks(gf));
  // three regions of partial sums per pair (dot, operator p^T A p, update r . r): each
  // is read by the kernel after its producer, so none overwrites another still unread
  C.o_part = take((size_t)3 * C.pstride * sizeof(double) * cnt);
  C.o_scal = take((size_t)kScalStride * sizeof(double) * cnt);
  C.o_alpha = take(np * sizeof(double));
  C.o_act = take(cnt * sizeof(int));
  C.o_iters = take(cnt * sizeof(int));
  C.o_status = take(cnt * sizeof(int));
  C.o_hist = take(cnt * (size_t)ndmg::kHistCap * 2 * sizeof(double));
  // time stepping: the predictor and the right-hand side of a step; alpha = 0 for the mass
  C.o_tw = take(v8);
  C.o_tb = take(v8);
  C.o_alpha0 = take(np * sizeof(double));
  if (cf.r > 0) C.o_coef = take(pl.coef.size() * sizeof(double));
  return NDMG_OK;
}

int make_plan(int nprob, const int* ns, double length, int nrhs, const ndmg_opts* o_in, Plan* pl,
              int levels = 0) {
  if (nprob < 1) return fail(NDMG_EINVAL, "nprob must be >= 1");
  if (levels < 0) return fail(NDMG_EINVAL, "levels must be >= 0 (0: all)");
  pl->levels = levels;
  if (!ns) return fail(NDMG_EINVAL, "null size array");
  if (nrhs < 1 || nrhs > 4096) return fail(NDMG_EINVAL, "nrhs must be in [1, 4096]");
  if ((int64_t)nprob * nrhs > 65535) return fail(NDMG_EINVAL, "more than 65535 (problem, rhs) pairs");
  if (!(length > 0.0) || !std::isfinite(length)) return fail(NDMG_EINVAL, "length must be > 0");
  NDMG_TRY(check_opts(o_in, &pl->opts));
  pl->coef.clear();
  if (pl->opts.coef_r > 0) {
    if (nprob != 1) return fail(NDMG_EINVAL, "a coefficient with jumps or a domain (coef_r > 0) serves a single problem");
    const size_t nb = (size_t)pl->opts.coef_r * pl->opts.coef_r * pl->opts.coef_r;
    // box factors, 0 for the boxes outside the domain
    pl->coef.assign(nb, 1.0);
    for (size_t b = 0; b < nb; ++b) {
      if (pl->opts.coef) pl->coef[b] = pl->opts.coef[b];
      if (pl->opts.domain && !pl->opts.domain[b]) pl->coef[b] = 0.0;
    }
  }
  pl->opts.coef = nullptr;
  pl->opts.domain = nullptr;
  for (int p = 0; p < nprob; ++p) {
    if (ns[p] < 2) return fail(NDMG_EINVAL, "n must be >= 2");
    if (ns[p] > 2048) return fail(NDMG_EINVAL, "n too large");
  }
  pl->length = length;
  pl->nprob = nprob;
  pl->nrhs = nrhs;
  pl->elem = (pl->opts.precision == NDMG_PREC_FP32) ? 4 : 8;
  std::vector<int> distinct(ns, ns + nprob);
  std::sort(distinct.begin(), distinct.end());
  distinct.erase(std::unique(distinct.begin(), distinct.end()), distinct.end());
  pl->cls.assign(distinct.size(), Cls{});
  pl->prob_cls.assign(nprob, 0);
  pl->prob_pos.assign(nprob, 0);
  for (size_t ci = 0; ci < distinct.size(); ++ci) pl->cls[ci].n = distinct[ci];
  for (int p = 0; p < nprob; ++p) {
    const int ci = (int)(std::lower_bound(distinct.begin(), distinct.end(), ns[p]) - distinct.begin());
    Cls& C = pl->cls[ci];
    pl->prob_cls[p] = ci;
    pl->prob_pos[p] = C.nprob++;
    C.probs.push_back(p);
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o2 = off;
    off = align_up(off + bytes);
    return o2;
  };
  int64_t voff = 0;
  pl->npairs = 0;
  for (auto& C : pl->cls) {
    C.nrhs = nrhs;
    C.count = C.nprob * nrhs;
    NDMG_TRY(plan_class(C, *pl, take));
    C.vec_off = voff;
    voff += (int64_t)C.count * C.vlen;
    pl->npairs += C.count;
  }
  pl->total_len = voff;
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
  d.nB = L.nB;
  d.bpatch = c->plan.opts.boundary_patches != 0;
  d.lut = at<int>(c, L.o_lut);
  d.slots = at<int>(c, L.o_slots);
  d.segs = at<int>(c, L.o_segs);
  d.chunks = at<int>(c, L.o_chunks);
  d.nchunks = (int)(L.chunks.size() / 4);
  d.bofs = at<int64_t>(c, L.o_bofs);
  return d;
}

// All pairs of a class, or only its active ones.
ndmg::Bat class_batch(ndmg_ctx* c, const Cls& C, bool masked) {
  const bool jumps = !c->plan.coef.empty();
  return ndmg::Bat{C.count, C.nrhs, at<double>(c, C.o_alpha), masked ? at<int>(c, C.o_act) : nullptr,
                   jumps ? at<double>(c, C.o_coef) : nullptr, jumps ? c->plan.opts.coef_r : 0};
}

// Host staging of everything uploaded at setup; freed after the stream has synchronised.
// A host array left uninitialised at allocation: the threads that fill it touch (and
// zero) their own parts first, so that the page faults and the zeroing of the large
// factor arrays run in parallel.
template <typename T>
struct HostArray {
  std::unique_ptr<T[]> p;
  size_t n = 0;
  void alloc(size_t count) {
    p.reset(count ? new T[count] : nullptr);
    n = count;
  }
  T* data() { return p.get(); }
};

// Host-to-device uploads on the context's stream; the sources stay alive until the
// caller synchronises the stream and drops the staging.
struct Staging {
  std::vector<std::vector<char>> keep;
  std::vector<std::shared_ptr<void>> owned;
  int put(ndmg_ctx* c, size_t off, const void* src, size_t bytes) {
    if (bytes == 0) return NDMG_OK;
    keep.emplace_back((const char*)src, (const char*)src + bytes);
    NDMG_HIP(hipMemcpyAsync(c->ws + off, keep.back().data(), bytes, hipMemcpyHostToDevice, c->st));
    return NDMG_OK;
  }
  template <typename V>
  int put_vec(ndmg_ctx* c, size_t off, const V& v) {
    return put(c, off, v.data(), v.size() * sizeof(typename V::value_type));
  }
  // uploads a large array without copying it: the staging takes it over
  template <typename T>
  int put_owned(ndmg_ctx* c, size_t off, HostArray<T>& a) {
    if (a.n == 0) return NDMG_OK;
    T* raw = a.p.release();
    owned.emplace_back(raw, [](void* q) { delete[] static_cast<T*>(q); });
    NDMG_HIP(hipMemcpyAsync(c->ws + off, raw, a.n * sizeof(T), hipMemcpyHostToDevice, c->st));
    a.n = 0;
    return NDMG_OK;
  }
};

// FP64 factors of one problem on a level of the generic smoother, cast to T, each stored
// k-major (column k of the matrix is a contiguous row of the array):
//   xc: X_T^T (rows: the nB boundary edges of a subdomain; columns: its nI interior
//       unknowns), [npadI][npadB];
//   ex: [A_T^{-1} | -X_T] (rows: interior unknowns; columns: interior, then boundary),
//       [npadE][npadI];
//   sp: S_P^{-1} of every patch type (symmetric), [ntypes][npadP][npadP], zero for
//       absent types and slots.
// With a coefficient (boxes), xc and ex hold one block per subdomain type (box) and each
// patch type has its own subdomain alphas.  The slots present in each patch factor must
// be those of the level's gather tables.
template <typename T>
bool build_gen_factors(const LevelHost& L, double alpha, T* xc, T* ex, T* sp, std::string* err) {
  const ndmg::GenTables& tb = L.gt;
  const int s = tb.s, nI = tb.nI, nB = tb.nB;
  std::vector<double> ai, xt;
  for (int tI = 0; tI < tb.ntypesI; ++tI) {
    if (!ndmg::subdomain_factors(s, L.g.h, alpha * tb.boxI[tI], &ai, &xt, err)) return false;
    T* xcb = xc + (size_t)tI * tb.npadI * tb.npadB;
    T* exb = ex + (size_t)tI * tb.npadE * tb.npadI;
    for (int k = 0; k < nI; ++k)
      for (int r = 0; r < nB; ++r) xcb[(size_t)k * tb.npadB + r] = (T)xt[(size_t)k * nB + r];
    for (int r = 0; r < nI; ++r) {
      for (int k = 0; k < nI; ++k) exb[(size_t)k * tb.npadI + r] = (T)ai[(size_t)r * nI + k];
      for (int b = 0; b < nB; ++b) exb[(size_t)(nI + b) * tb.npadI + r] = (T)(-xt[(size_t)r * nB + b]);
    }
  }
  std::vector<double> buf((size_t)tb.npadP * tb.npadP);
  std::vector<char> present;
  std::vector<double> cell_alpha;
  for (int type : tb.typesP) {
    const bool jumps = !tb.geomP.empty();
    const int geom = jumps ? tb.geomP[type] : type;
    int t[3];
    ndmg::patch_type_axes(tb.kind, geom, t);
    const std::vector<ndmg::Slot> slots = tb.kind == 0 ? ndmg::vertex_slots(s) : ndmg::edge_slots(s, geom / 9);
    const std::vector<std::array<int, 3>> cells = ndmg::patch_cells(tb.kind, geom, s);
    std::vector<std::array<int, 3>> kept;
    std::vector<char> pres_in;
    if (jumps) {   // each cell takes the alpha of its subdomain (offset floor(o / s) in {-1, 0});
                   // cells of subdomains outside the domain (factor 0) are left out
      cell_alpha.clear();
      for (const auto& c : cells) {
        int o = 0;
        for (int ax = 0; ax < 3; ++ax) o |= (c[ax] >= 0 ? 1 : 0) << ax;
        if (!(tb.keyP[type][o] > 0.0)) continue;
        kept.push_back(c);
        cell_alpha.push_back(alpha * tb.keyP[type][o]);
      }
      pres_in.assign(tb.presentP.begin() + (size_t)type * tb.npadP,
                     tb.presentP.begin() + (size_t)type * tb.npadP + slots.size());
    }
    if (!ndmg::patch_inverse(jumps ? kept : cells, slots, t, s, L.g.h, alpha, tb.npadP, buf.data(), &present, err,
                             jumps ? &cell_alpha : nullptr, jumps ? &pres_in : nullptr))
      return false;
    for (size_t j = 0; j < slots.size(); ++j)
      if (present[j] != tb.presentP[(size_t)type * tb.npadP + j]) {
        *err = "internal: patch slots differ from the gather tables";
        return false;
      }
    T* dst = sp + (size_t)type * tb.npadP * tb.npadP;
    for (size_t i = 0; i < buf.size(); ++i) dst[i] = (T)buf[i];
  }
  return true;
}

template <typename T>
ndmg::GenLevel<T> gen_level(ndmg_ctx* c, const LevelHost& L) {
  ndmg::GenLevel<T> G{};
  const ndmg::GenTables& tb = L.gt;
  auto common = [&](ndmg::GemmArgs<T>& a) {
    a.vlen = L.g.len;
    a.scale = T(1);
    a.assign = 1;
  };
  auto& Cd = G.cond;   // C_T = X_T^T r_I
  common(Cd);
  Cd.M = at<T>(c, L.o_gX);
  Cd.mstride = (int64_t)L.blk_gX;
  Cd.chunks = at<int>(c, L.o_gcI);
  Cd.nchunks = (int)(tb.chunksI.size() / 4);
  Cd.units = at<int64_t>(c, L.o_guI);
  Cd.relIn = at<int64_t>(c, L.o_grI);
  Cd.relOut = nullptr;
  Cd.ksplit = tb.npadI;
  Cd.npadK = tb.npadI;
  Cd.npadR = tb.npadB;
  Cd.nrb = (tb.npadB + 63) / 64;
  Cd.ylen = L.clenG;
  Cd.nunits = (int64_t)tb.unitsI.size();
  auto& Ex = G.ext;    // z_I = eta [A_T^{-1} | -X_T] [r_I ; w_dT]
  common(Ex);
  Ex.M = at<T>(c, L.o_gE);
  Ex.mstride = (int64_t)L.blk_gE;
  Ex.chunks = Cd.chunks;
  Ex.nchunks = Cd.nchunks;
  Ex.units = Cd.units;
  Ex.relIn = at<int64_t>(c, L.o_grE);
  Ex.relOut = at<int64_t>(c, L.o_grI);
  Ex.ksplit = tb.nI;
  Ex.npadK = tb.npadE;
  Ex.npadR = tb.npadI;
  Ex.nrb = (tb.npadI + 63) / 64;
  Ex.ylen = 0;
  auto& P = G.patch;   // y_P = S_P^{-1} g|Gamma_P
  common(P);
  P.M = at<T>(c, L.o_gS);
  P.mstride = (int64_t)L.blk_gS;
  P.chunks = at<int>(c, L.o_gcP);
  P.nchunks = (int)(tb.chunksP.size() / 4);
  P.units = at<int64_t>(c, L.o_guP);
  P.relIn = at<int64_t>(c, L.o_grP);
  P.relOut = nullptr;
  P.ksplit = tb.npadP;
  P.npadK = tb.npadP;
  P.npadR = tb.npadP;
  P.nrb = (tb.npadP + 63) / 64;
  P.ylen = L.ylenG;
  P.nunits = (int64_t)tb.unitsP.size();
  G.C = at<T>(c, L.o_C);
  G.gg = at<T>(c, L.o_gg);
  G.Y = at<T>(c, L.o_Y);
  G.w = at<T>(c, L.o_w);
  G.gamma = at<int>(c, L.o_ggam);
  G.ccodes = at<int>(c, L.o_gcc);
  G.codes = at<int>(c, L.o_gcodes);
  G.ngam = (int64_t)tb.gamma.size();
  G.clen = L.clenG;
  return G;
}

// One smoothing step z (assign ? = : +=) M^{-1} r on a smoothed level.
template <typename T>
int smooth_level(ndmg_ctx* c, const Cls& C, const LevelHost& L, const T* r, T* z, const ndmg::Bat& bt, int assign,
                 hipStream_t st) {
  const double eta = c->plan.opts.eta;
  if (L.gen) {
    NDMG_HIP(ndmg::launch_smooth_generic<T>(r, z, gen_level<T>(c, L), L.g, bt, eta, assign, st));
  } else {
    NDMG_HIP(ndmg::launch_smooth<T>(r, z, level_ptrs<T>(c, L), level_dsub(c, L), L.g, bt, eta, assign, st));
  }
  return NDMG_OK;
}

// Local factors of every (problem, level) of a class, built on host threads in FP64 and
// cast to the working precision (Sec. 3.2: A_T of eq. ATDef, A_V of eq. AVDef; coarsest
// level exact).
template <typename T>
int build_class_factors(ndmg_ctx* c, Cls& C, Staging& stg) {
  Plan& pl = c->plan;
  const int nl = (int)C.lv.size();
  // per level, problem p's blocks at p * blk of each array (zeroed by the thread that
  // builds problem p, then filled)
  std::vector<HostArray<T>> ATinv(nl), XT(nl), Sinv(nl), A0(nl);
  std::vector<size_t> bE(nl, 0), bX(nl, 0), bS(nl, 0), b0(nl, 0);
  for (int k = 0; k < nl; ++k) {
    LevelHost& L = C.lv[k];
    if (L.gen) {
      bE[k] = L.blk_gE, bX[k] = L.blk_gX, bS[k] = L.blk_gS;
    } else if (L.smoothed) {
      bE[k] = L.blk_ATinv, bX[k] = L.blk_XT, bS[k] = L.blk_Sinv;
    } else {
      b0[k] = L.blk_A0;
    }
    ATinv[k].alloc(bE[k] * C.nprob);
    XT[k].alloc(bX[k] * C.nprob);
    Sinv[k].alloc(bS[k] * C.nprob);
    A0[k].alloc(b0[k] * C.nprob);
  }
  const bool bp = pl.opts.boundary_patches != 0;
  unsigned hw = std::thread::hardware_concurrency();
  const int nth = std::max(1, std::min<int>(C.nprob, std::min<int>(16, hw ? (int)hw : 4)));
  std::vector<std::string> errs(nth);
  std::vector<std::vector<int64_t>> maps(nth);
  auto work = [&](int t) {
    for (int p = t; p < C.nprob; p += nth) {
      const double a = C.alpha[p];
      for (int k = 0; k < nl; ++k) {
        std::fill_n(ATinv[k].data() + p * bE[k], bE[k], T(0));
        std::fill_n(XT[k].data() + p * bX[k], bX[k], T(0));
        std::fill_n(Sinv[k].data() + p * bS[k], bS[k], T(0));
        std::fill_n(A0[k].data() + p * b0[k], b0[k], T(0));
      }
      for (int k = 0; k < nl; ++k) {
        LevelHost& L = C.lv[k];
        std::string err;
        if (!L.smoothed) {
          std::vector<double> inv;
          std::vector<int64_t> map;
          if (!ndmg::build_coarse(L.g, a, &inv, &map, &err, pl.boxes())) {
            errs[t] = err;
            return;
          }
              std::copy(inv.begin(), inv.end(), A0[k].data() + (size_t)p * L.blk_A0);
          if (maps[t].empty()) maps[t] = map;
          continue;
        }
        if (L.gen) {
          if (!build_gen_factors(L, a, XT[k].data() + (size_t)p * L.blk_gX, ATinv[k].data() + (size_t)p * L.blk_gE,
                                 Sinv[k].data() + (size_t)p * L.blk_gS, &err)) {
            errs[t] = err;
            return;
          }
          continue;
        }
        if (!ndmg::build_level_factors_into<T>(L.g.h, a, L.sub, bp, ATinv[k].data() + (size_t)p * L.blk_ATinv,
                                               XT[k].data() + (size_t)p * L.blk_XT,
                                               Sinv[k].data() + (size_t)p * L.blk_Sinv, &err)) {
          errs[t] = err;
          return;
        }
      }
    }
  };
  if (nth == 1) {
    work(0);
  } else {
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t) th.emplace_back(work, t);
    for (auto& x : th) x.join();
  }
  for (auto& e : errs)
    if (!e.empty()) return fail(NDMG_EINVAL, e);
  for (int k = 0; k < nl; ++k) {
    LevelHost& L = C.lv[k];
    if (!L.smoothed) {
      L.map = maps[0];
      NDMG_TRY(stg.put_owned(c, L.o_A0, A0[k]));
      NDMG_TRY(stg.put_vec(c, L.o_map, L.map));
      continue;
    }
    if (L.gen) {
      NDMG_TRY(stg.put_owned(c, L.o_gE, ATinv[k]));
      NDMG_TRY(stg.put_owned(c, L.o_gX, XT[k]));
      NDMG_TRY(stg.put_owned(c, L.o_gS, Sinv[k]));
      NDMG_TRY(stg.put_vec(c, L.o_guI, L.gt.unitsI));
      NDMG_TRY(stg.put_vec(c, L.o_grI, L.gt.relI));
      NDMG_TRY(stg.put_vec(c, L.o_grE, L.gt.relE));
      NDMG_TRY(stg.put_vec(c, L.o_gcI, L.gt.chunksI));
      NDMG_TRY(stg.put_vec(c, L.o_guP, L.gt.unitsP));
      NDMG_TRY(stg.put_vec(c, L.o_grP, L.gt.relP));
      NDMG_TRY(stg.put_vec(c, L.o_gcP, L.gt.chunksP));
      NDMG_TRY(stg.put_vec(c, L.o_ggam, L.gt.gamma));
      NDMG_TRY(stg.put_vec(c, L.o_gcc, L.gt.ccodes));
      NDMG_TRY(stg.put_vec(c, L.o_gcodes, L.gt.codes));
      if (k == C.dense_k) {
        L.map = ndmg::unknown_offsets(L.g, pl.boxes());
        if ((int)L.map.size() != L.Nd) return fail(NDMG_EINVAL, "internal: dense level size mismatch");
        NDMG_TRY(stg.put_vec(c, L.o_map, L.map));
      }
      continue;
    }
    NDMG_TRY(stg.put_owned(c, L.o_ATinv, ATinv[k]));
    NDMG_TRY(stg.put_owned(c, L.o_XT, XT[k]));
    NDMG_TRY(stg.put_owned(c, L.o_Sinv, Sinv[k]));
    {
      std::vector<int64_t> bo;
      for (auto& q : ndmg::boundary_dofs(L.sub.s))
        bo.push_back(q.d * L.g.B + (int64_t)q.dz * L.g.plane + (int64_t)q.dy * L.g.P + q.dx);
      NDMG_TRY(stg.put_vec(c, L.o_bofs, bo));
    }
    NDMG_TRY(stg.put_vec(c, L.o_lut, ndmg::slot_lookup(L.sub.s)));
    if (!ndmg::boundary_patches_match(ndmg::boundary_patch_table()))
      return fail(NDMG_EINVAL, "internal: subdomain boundary patch table differs from the kernels'");
    std::vector<int> sl;
    for (auto& q : ndmg::vertex_slots(L.sub.s)) {
      sl.push_back(q.d);
      sl.push_back(q.dx);
      sl.push_back(q.dy);
      sl.push_back(q.dz);
    }
    NDMG_TRY(stg.put_vec(c, L.o_slots, sl));
    std::vector<int> sg;
    for (auto& q : L.segs) {
      sg.push_back(q.type);
      for (int a = 0; a < 3; ++a) sg.push_back(q.lo[a]);
      for (int a = 0; a < 2; ++a) sg.push_back(q.dims[a]);
      const int nH = L.sub.nH;
      const int yb = ndmg::y_pos(nH, c->plan.opts.boundary_patches != 0, q.lo[0], q.lo[1], q.lo[2]);
      if (yb % 16) return fail(NDMG_EINVAL, "internal: patch result region not on a 16-entry run");
      sg.push_back((int)yb);
      sg.push_back(q.count);
    }
    NDMG_TRY(stg.put_vec(c, L.o_segs, sg));
    NDMG_TRY(stg.put_vec(c, L.o_chunks, L.chunks));
    if (k == C.dense_k) {
      L.map = ndmg::unknown_offsets(L.g);
      if ((int)L.map.size() != L.Nd) return fail(NDMG_EINVAL, "internal: dense level size mismatch");
      NDMG_TRY(stg.put_vec(c, L.o_map, L.map));
    }
  }
  NDMG_TRY(stg.put_vec(c, C.o_alpha, C.alpha));
  if (!pl.coef.empty()) NDMG_TRY(stg.put_vec(c, C.o_coef, pl.coef));
  return NDMG_OK;
}

// Levels 0 .. top of a class for the one-launch bottom of the V-cycle.
template <typename T>
ndmg::SmallArgs<T> small_args(ndmg_ctx* c, Cls& C, int top) {
  ndmg::SmallArgs<T> a{};
  a.top = top;
  a.m = c->plan.opts.m;
  a.eta = c->plan.opts.eta;
  for (int k = 0; k <= top; ++k) {
    LevelHost& L = C.lv[k];
    ndmg::SmallLevel<T>& s = a.lv[k];
    s.g = ndmg::dgeom(L.g);
    s.h = L.g.h;
    s.z = at<T>(c, L.o_z);
    s.gv = at<T>(c, L.o_g);
    if (L.smoothed) {
      s.nH = L.sub.nH;
      s.bpatch = c->plan.opts.boundary_patches != 0;
      s.r = at<T>(c, L.o_r);
      s.zi = at<T>(c, L.o_zi);
      s.gg = at<T>(c, L.o_gg);
      s.w = at<T>(c, L.o_w);
      s.Y = at<T>(c, L.o_Y);
      s.G = at<T>(c, L.o_G);
      s.ATinv = at<T>(c, L.o_ATinv);
      s.Sinv = at<T>(c, L.o_Sinv);
      s.XT = at<T>(c, L.o_XT);
      s.bofs = at<int64_t>(c, L.o_bofs);
      s.lut = at<int>(c, L.o_lut);
      s.slots = at<int>(c, L.o_slots);
    } else {
      s.A0inv = at<T>(c, L.o_A0);
      s.map = at<int64_t>(c, L.o_map);
      s.N0 = (int)L.map.size();
    }
  }
  return a;
}

// z = MG(k, g, 0, m) (Fig. 1) for the pairs of a class.
template <typename T>
int vcycle_rec(ndmg_ctx* c, Cls& C, int k, const T* g, T* z, const ndmg::Bat& bt, hipStream_t st) {
  Plan& pl = c->plan;
  LevelHost& L = C.lv[k];
  if (k <= C.small_top) {
    ndmg::SmallArgs<T> a = small_args<T>(c, C, k);
    a.lv[k].gv = const_cast<T*>(g);
    a.lv[k].z = z;
    NDMG_HIP(ndmg::launch_vcycle_small<T>(a, bt, st));
    return NDMG_OK;
  }
  if (k == 0) {
    NDMG_HIP(ndmg::launch_coarse<T>(g, z, at<T>(c, L.o_A0), at<int64_t>(c, L.o_map), (int)L.map.size(),
                                    L.g.len, bt, st));
    return NDMG_OK;
  }
  if (k == C.dense_k) {
    // z may be a caller's vector at the finest level: clear its non-unknown entries
    const bool top = (k == (int)C.lv.size() - 1);
    NDMG_HIP(ndmg::launch_dense_vcycle<T>(g, z, at<T>(c, L.o_Bd), at<int64_t>(c, L.o_map), L.Nd, L.g.len, bt,
                                          top, C.dense_t, st));
    return NDMG_OK;
  }
  const int m = pl.opts.m;
  auto P = level_ptrs<T>(c, L);
  LevelHost& Lc = C.lv[k - 1];
  // z_1 .. z_m: pre-smoothing from z_0 = 0
  NDMG_TRY(smooth_level<T>(c, C, L, g, z, bt, 1, st));
  for (int l = 1; l < m; ++l) {
    NDMG_HIP(ndmg::launch_apply<T>(z, g, P.r, L.g, bt, 1, st));
    NDMG_TRY(smooth_level<T>(c, C, L, P.r, z, bt, 0, st));
  }
  // gbar = I_k^{k-1} (g - A z_m)
  NDMG_HIP(ndmg::launch_apply<T>(z, g, P.r, L.g, bt, 1, st));
  NDMG_HIP(ndmg::launch_restrict<T>(P.r, at<T>(c, Lc.o_g), L.g, Lc.g, bt, st));
  NDMG_TRY(vcycle_rec<T>(c, C, k - 1, at<T>(c, Lc.o_g), at<T>(c, Lc.o_z), bt, st));
  // z_{m+1} = z_m + I_{k-1}^k MG(k-1, gbar, 0, m)
  NDMG_HIP(ndmg::launch_prolong_add<T>(at<T>(c, Lc.o_z), z, L.g, Lc.g, bt, st));
  // post-smoothing
  for (int l = 0; l < m; ++l) {
    NDMG_HIP(ndmg::launch_apply<T>(z, g, P.r, L.g, bt, 1, st));
    NDMG_TRY(smooth_level<T>(c, C, L, P.r, z, bt, 0, st));
  }
  return NDMG_OK;
}

// Matrix of MG(dense_k, ., 0, m) for every problem of a class: columns from the recursive
// V-cycle applied to unit vectors, dense_K columns per problem per pass.
template <typename T>
int build_dense(ndmg_ctx* c, Cls& C) {
  const int kd = C.dense_k;
  if (kd < 1) return NDMG_OK;
  LevelHost& L = C.lv[kd];
  const int N = L.Nd, K = C.dense_K;
  ndmg::Bat bt = class_batch(c, C, false);   // alpha and coefficient of the class
  bt.count = C.nprob * K;
  bt.nrhs = K;
  T* g = at<T>(c, L.o_g);
  T* z = at<T>(c, L.o_z);
  const int64_t* map = at<int64_t>(c, L.o_map);
  T* Bm = at<T>(c, L.o_Bd);
  C.dense_k = -1;   // the recursion, not the matrix being built
  int rc = NDMG_OK;
  for (int j0 = 0; j0 < N && rc == NDMG_OK; j0 += K) {
    hipError_t e = ndmg::launch_unit_cols<T>(g, map, N, j0, L.g.len, bt, c->st);
    if (e != hipSuccess) {
      rc = fail(NDMG_EHIP, std::string("dense build: ") + hipGetErrorString(e));
      break;
    }
    rc = vcycle_rec<T>(c, C, kd, g, z, bt, c->st);
    if (rc != NDMG_OK) break;
    e = ndmg::launch_gather_cols<T>(z, Bm, map, N, j0, L.g.len, C.dense_t, bt, c->st);
    if (e != hipSuccess) rc = fail(NDMG_EHIP, std::string("dense build: ") + hipGetErrorString(e));
  }
  C.dense_k = kd;
  return rc;
}

// z = B g for FP64 vectors of the finest level of a class, in the context's precision.
int precondition(ndmg_ctx* c, Cls& C, const double* g, double* z, const ndmg::Bat& bt, hipStream_t st) {
  Plan& pl = c->plan;
  const int J = (int)C.lv.size() - 1;
  LevelHost& L = C.lv[J];
  if (pl.opts.precision == NDMG_PREC_FP64) return vcycle_rec<double>(c, C, J, g, z, bt, st);
  float* gf = at<float>(c, L.o_g);
  float* zf = at<float>(c, L.o_z);
  NDMG_HIP((ndmg::launch_convert<double, float>(g, gf, L.g.len, bt, st)));
  NDMG_TRY(vcycle_rec<float>(c, C, J, gf, zf, bt, st));
  NDMG_HIP((ndmg::launch_convert<float, double>(zf, z, L.g.len, bt, st)));
  return NDMG_OK;
}

// In the CG driver the V-cycle reads the FP64 residual r (FP64 contexts) or its FP32 copy
// in the finest level's g (mixed precision: written by the update that produced r), and
// its result z stays in the V-cycle's precision (the finest level's z when FP32).
bool mixed(const Plan& pl) { return pl.opts.precision == NDMG_PREC_FP32; }

float* r32_of(ndmg_ctx* c, Cls& C) { return mixed(c->plan) ? at<float>(c, C.lv.back().o_g) : nullptr; }

int precondition_cg(ndmg_ctx* c, Cls& C, const ndmg::Bat& bt, hipStream_t st) {
  const int J = (int)C.lv.size() - 1;
  LevelHost& L = C.lv[J];
  if (!mixed(c->plan)) return vcycle_rec<double>(c, C, J, at<double>(c, C.o_pr), at<double>(c, C.o_pz), bt, st);
  return vcycle_rec<float>(c, C, J, at<float>(c, L.o_g), at<float>(c, L.o_z), bt, st);
}

// q = A p with p^T q (slot PQ), then u += a p, r -= a q (a = s[num] / s[PQ]) and r . r
// (and the FP32 copy of r when mixed).
// Regions of partial sums of a class: 0 the dot products, 1 p^T A p, 2 r . r; stride
// part_stride per pair.
double* part_region(ndmg_ctx* c, const Cls& C, int region) {
  return at<double>(c, C.o_part) + region * C.pstride;
}
int64_t part_stride(const Cls& C) { return 3 * C.pstride; }

// q = A p with partial sums of p^T q, then (reducing them) r -= a q (a = s[num] / p^T q)
// with partial sums of r . r (and the FP32 copy of r when mixed).  u += a p is left
// pending (a in s[kS_AL]): the next direction kernel applies it while it reads p, or
// finish_solution at the end of the solve.
int cg_apply_update(ndmg_ctx* c, Cls& C, int num, const ndmg::Bat& bt, hipStream_t st) {
  const ndmg::Geom& g = C.lv.back().g;
  const int64_t len = g.len;
  double* r = at<double>(c, C.o_pr);
  double* p = at<double>(c, C.o_pp);
  double* q = at<double>(c, C.o_pq);
  double* sc = at<double>(c, C.o_scal);
  double* pq_part = part_region(c, C, 1);
  const int64_t ps = part_stride(C);
  int pq_n = 0;
  // q = A p with the partials of p^T A p from the operator kernel, else (small meshes,
  // box grids beyond what the kernel's per-cell form holds) apply then dot
  hipError_t e = hipErrorNotSupported;
  if (g.n > ndmg::stencil_min_n(bt.count) && g.n <= ndmg::stencil_max_n())
    e = ndmg::launch_stencil<double>(p, nullptr, q, g, bt, 2, pq_part, ps, nullptr, st);
  if (e == hipSuccess) {
    pq_n = ndmg::stencil_blocks(g, bt.count);
  } else if (e == hipErrorNotSupported) {
    NDMG_HIP(ndmg::launch_apply<double>(p, nullptr, q, g, bt, 0, st));
    NDMG_HIP(ndmg::launch_dot<double>(p, q, nullptr, pq_part, ps, nullptr, len, bt, st));
    pq_n = ndmg::dot_parts(len, bt.count);
  } else {
    NDMG_HIP(e);
  }
  NDMG_HIP(ndmg::launch_cg_update(nullptr, r, p, q, sc, num, pq_part, pq_n, r32_of(c, C), part_region(c, C, 2), ps,
                                  len, bt, st));
  return NDMG_OK;
}

bool flexible_beta(const Plan& pl) {
  return pl.opts.flexible > 0 || (pl.opts.flexible < 0 && pl.opts.precision == NDMG_PREC_FP32);
}

// The convergence test of an iteration; its count of active pairs goes straight to host
// set `set` (iterations alternate between the two sets).
int pcg_check(ndmg_ctx* c, size_t ci, int i_rz, int set, hipStream_t st) {
  Cls& C = c->plan.cls[ci];
  NDMG_HIP(ndmg::launch_pcg_check(at<double>(c, C.o_scal), at<int>(c, C.o_act), at<int>(c, C.o_iters),
                                  at<int>(c, C.o_status), C.count, i_rz,
                                  c->dev_nact + set * c->plan.cls.size() + ci, part_region(c, C, 2),
                                  ndmg::dot_parts(C.vlen, C.count), part_stride(C), at<double>(c, C.o_hist), st));
  return NDMG_OK;
}

// Start of a solve for one class: r = b, u = 0, b . b, per-pair state, z = B r,
// s[cur] = r . z, p = z and the first update.
int pcg_prologue(ndmg_ctx* c, size_t ci, const double* b, double* u, double rtol, hipStream_t st, bool warm) {
  Cls& C = c->plan.cls[ci];
  const int64_t len = C.vlen;
  double* r = at<double>(c, C.o_pr);
  double* z = at<double>(c, C.o_pz);
  double* p = at<double>(c, C.o_pp);
  double* part = part_region(c, C, 0);
  const int64_t ps = part_stride(C);
  double* sc = at<double>(c, C.o_scal);
  const ndmg::Bat all = class_batch(c, C, false), act = class_batch(c, C, true);
  if (warm) {   // r = b - A u from the caller's u
    NDMG_HIP(ndmg::launch_apply<double>(u, b, r, C.lv.back().g, all, 1, st));
  } else {
    NDMG_HIP(ndmg::launch_copy(b, r, len, all, st));
    NDMG_HIP(ndmg::launch_zero(u, len, all, st));
  }
  NDMG_HIP(ndmg::launch_dot<double>(b, b, nullptr, part, ps, sc + kS_BB, len, all, st));
  NDMG_HIP(ndmg::launch_pcg_init(sc, at<int>(c, C.o_act), at<int>(c, C.o_iters), at<int>(c, C.o_status),
                                 C.count, rtol, st));
  if (mixed(c->plan)) NDMG_HIP((ndmg::launch_convert<double, float>(r, r32_of(c, C), len, act, st)));
  NDMG_TRY(precondition_cg(c, C, act, st));
  if (mixed(c->plan)) {
    const float* zf = at<float>(c, C.lv.back().o_z);
    NDMG_HIP(ndmg::launch_dot<float>(zf, r, nullptr, part, ps, sc + kS_RZA, len, act, st));
    NDMG_HIP((ndmg::launch_convert<float, double>(zf, p, len, act, st)));
  } else {
    NDMG_HIP(ndmg::launch_dot<double>(z, r, nullptr, part, ps, sc + kS_RZA, len, act, st));
    NDMG_HIP(ndmg::launch_copy(z, p, len, act, st));
  }
  NDMG_TRY(cg_apply_update(c, C, kS_RZA, act, st));
  return pcg_check(c, ci, kS_RZA, 0, st);
}

// One CG iteration after the first for one class: z = B r; s[nxt] = r . z (and
// s[nxt + 1] = z . q for the flexible beta); p = z + beta p; the update with
// a = s[nxt] / p^T A p; the convergence test.
int pcg_body(ndmg_ctx* c, size_t ci, double* u, int cur, int nxt, hipStream_t st) {
  Cls& C = c->plan.cls[ci];
  const int64_t len = C.vlen;
  double* r = at<double>(c, C.o_pr);
  double* z = at<double>(c, C.o_pz);
  double* p = at<double>(c, C.o_pp);
  double* q = at<double>(c, C.o_pq);
  double* part = part_region(c, C, 0);
  const int64_t ps = part_stride(C);
  const int nd = ndmg::dot_parts(len, C.count);
  double* sc = at<double>(c, C.o_scal);
  const bool flex = flexible_beta(c->plan);
  const ndmg::Bat act = class_batch(c, C, true);
  NDMG_TRY(precondition_cg(c, C, act, st));
  // dot partials; the direction kernel reduces them (s[nxt] = r . z, s[nxt + 1] = z . q)
  if (mixed(c->plan)) {
    const float* zf = at<float>(c, C.lv.back().o_z);
    NDMG_HIP(ndmg::launch_dot<float>(zf, r, flex ? q : nullptr, part, ps, nullptr, len, act, st));
    NDMG_HIP(ndmg::launch_cg_direction<float>(p, zf, u, sc, nxt, cur, flex ? 1 : 0, nxt + 1, cur, kS_PQ, part, nd,
                                              ps, len, act, st));
  } else {
    NDMG_HIP(ndmg::launch_dot<double>(z, r, flex ? q : nullptr, part, ps, nullptr, len, act, st));
    NDMG_HIP(ndmg::launch_cg_direction<double>(p, z, u, sc, nxt, cur, flex ? 1 : 0, nxt + 1, cur, kS_PQ, part,
                                               nd, ps, len, act, st));
  }
  NDMG_TRY(cg_apply_update(c, C, nxt, act, st));
  return pcg_check(c, ci, nxt, cur == kS_RZA ? 1 : 0, st);
}

// Run fn(ci, stream) for every class: class 0 on the context's stream, class i >= 1 on
// a side stream forked from it and joined back.
template <typename F>
int for_classes(ndmg_ctx* c, F&& fn) {
  const size_t nc = c->plan.cls.size();
  if (nc == 1) return fn((size_t)0, c->st);
  NDMG_HIP(hipEventRecord(c->ev_fork, c->st));
  for (size_t i = 1; i < nc; ++i) NDMG_HIP(hipStreamWaitEvent(c->side[i - 1], c->ev_fork, 0));
  int rc = NDMG_OK;
  for (size_t i = 0; i < nc && rc == NDMG_OK; ++i) rc = fn(i, i == 0 ? c->st : c->side[i - 1]);
  // join every side stream, also after a failure, so that none is left forked
  for (size_t i = 1; i < nc; ++i) {
    hipError_t e = hipEventRecord(c->ev_join[i - 1], c->side[i - 1]);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->st, c->ev_join[i - 1], 0);
    if (e != hipSuccess && rc == NDMG_OK)
      rc = fail(NDMG_EHIP, std::string("stream join: ") + hipGetErrorString(e));
  }
  return rc;
}

int body_all_eager(ndmg_ctx* c, double* u, int cur, int nxt) {
  return for_classes(c, [&](size_t ci, hipStream_t st) {
    return pcg_body(c, ci, u + c->plan.cls[ci].vec_off, cur, nxt, st);
  });
}

void drop_graphs(ndmg_ctx* c) {
  for (int i = 0; i < 2; ++i)
    if (c->gexec[i]) {
      (void)hipGraphExecDestroy(c->gexec[i]);
      c->gexec[i] = nullptr;
    }
  c->graph_u = nullptr;
}

// Graphs for the CG iterations: as asked, or (use_graphs -1) unless one size class with a
// finest level of n >= 80 makes each iteration long enough for eager launches to keep
// ahead of the device.
bool use_graphs(const Plan& pl) {
  if (pl.opts.use_graphs >= 0) return pl.opts.use_graphs != 0;
  return !(pl.cls.size() == 1 && pl.cls[0].lv.back().g.n >= 80);
}

int body_all(ndmg_ctx* c, double* u, int cur, int nxt) {
  if (!use_graphs(c->plan) || c->st == nullptr) return body_all_eager(c, u, cur, nxt);
  if (c->graph_u != u) drop_graphs(c);
  const int par = (cur == kS_RZA) ? 0 : 1;
  if (!c->gexec[par]) {
    hipGraph_t graph = nullptr;
    NDMG_HIP(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
    int rc = body_all_eager(c, u, cur, nxt);
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

// Marks the end of the writes of host set `set` (the counts of active pairs, one per
// class, written by the convergence test of the iteration just enqueued).
int post_active(ndmg_ctx* c, int set) {
  NDMG_HIP(hipEventRecord(c->ev_nact[set], c->st));
  return NDMG_OK;
}

// Pairs still active in host set `set`, summed over the classes (waits for its event).
int active_pairs(ndmg_ctx* c, int set, int* out) {
  const size_t nc = c->plan.cls.size();
  NDMG_HIP(hipEventSynchronize(c->ev_nact[set]));
  int t = 0;
  for (size_t i = 0; i < nc; ++i) t += c->host_nact[set * nc + i];
  *out = t;
  return NDMG_OK;
}

// Whole PCG over all pairs; per-pair results in problem order (p * nrhs + rhs).
int pcg_all(ndmg_ctx* c, const double* b, double* u, double rtol, int maxit, int* iters,
            double* relres, bool warm = false) {
  Plan& pl = c->plan;
  NDMG_TRY(for_classes(c, [&](size_t ci, hipStream_t st) {
    const Cls& C = pl.cls[ci];
    return pcg_prologue(c, ci, b + C.vec_off, u + C.vec_off, rtol, st, warm);
  }));
  // Iteration it is enqueued before the host reads the count after iteration it - 1, so
  // the device never waits for the host; when that count is zero, iteration it runs with
  // every pair inactive (each kernel returns at once) and the loop ends.
  NDMG_TRY(post_active(c, 0));
  int cur = kS_RZA, nxt = kS_RZB;
  for (int it = 2, set = 0;; ++it, set ^= 1) {
    const bool launch = it <= maxit;
    if (launch) {
      NDMG_TRY(body_all(c, u, cur, nxt));
      std::swap(cur, nxt);
      NDMG_TRY(post_active(c, set ^ 1));
    }
    int nact = 0;
    NDMG_TRY(active_pairs(c, set, &nact));
    if (!launch || nact == 0) break;
  }
  // the last update's u += a p of every pair
  NDMG_TRY(for_classes(c, [&](size_t ci, hipStream_t st) {
    Cls& C = pl.cls[ci];
    NDMG_HIP(ndmg::launch_cg_finish(u + C.vec_off, at<double>(c, C.o_pp), at<double>(c, C.o_scal), C.vlen,
                                    class_batch(c, C, false), st));
    return NDMG_OK;
  }));
  // per-pair results
  int nbroken = 0, nrun = 0, first_bad = -1;
  for (const Cls& C : pl.cls) {
    NDMG_HIP(hipMemcpyAsync(c->host_scal, at<double>(c, C.o_scal), (size_t)C.count * kScalStride * 8,
                            hipMemcpyDeviceToHost, c->st));
    NDMG_HIP(hipMemcpyAsync(c->host_int, at<int>(c, C.o_iters), (size_t)C.count * sizeof(int),
                            hipMemcpyDeviceToHost, c->st));
    NDMG_HIP(hipMemcpyAsync(c->host_int + C.count, at<int>(c, C.o_status), (size_t)C.count * sizeof(int),
                            hipMemcpyDeviceToHost, c->st));
    NDMG_HIP(hipStreamSynchronize(c->st));
    for (int j = 0; j < C.nprob; ++j)
      for (int r = 0; r < C.nrhs; ++r) {
        const int pair = j * C.nrhs + r;
        const int out = C.probs[j] * pl.nrhs + r;
        if (iters) iters[out] = c->host_int[pair];
        if (relres) relres[out] = c->host_scal[(size_t)pair * kScalStride + kS_REL];
        const int stt = c->host_int[C.count + pair];
        if (stt == ndmg::kPairBroken) {
          ++nbroken;
          if (first_bad < 0) first_bad = out;
        } else if (stt == ndmg::kPairRun) {
          ++nrun;
        }
      }
  }
  if (nbroken)
    return fail(NDMG_EBREAKDOWN, "PCG breakdown (p^T A p <= 0 or non-finite scalar) in " +
                                     std::to_string(nbroken) + " pair(s), first (problem*nrhs+rhs) " +
                                     std::to_string(first_bad));
  if (nrun) return fail(NDMG_ENOCONV, "PCG reached maxit in " + std::to_string(nrun) + " pair(s)");
  return NDMG_OK;
}

int check_ctx(const ndmg_ctx* c) {
  if (!c) return fail(NDMG_EINVAL, "null context");
  return NDMG_OK;
}

int one_class(const ndmg_ctx* c) {
  if (c->plan.cls.size() != 1)
    return fail(NDMG_EINVAL, "this call needs a context with a single problem size");
  return NDMG_OK;
}

void release(ndmg_ctx* c) {
  drop_graphs(c);
  for (auto s : c->side)
    if (s) (void)hipStreamDestroy(s);
  c->side.clear();
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  c->ev_fork = nullptr;
  for (auto e : c->ev_join)
    if (e) (void)hipEventDestroy(e);
  c->ev_join.clear();
  for (auto& e : c->ev_nact)
    if (e) {
      (void)hipEventDestroy(e);
      e = nullptr;
    }
  if (c->host_nact) (void)hipHostFree(c->host_nact);
  if (c->host_scal) (void)hipHostFree(c->host_scal);
  if (c->host_int) (void)hipHostFree(c->host_int);
  c->host_nact = nullptr;
  c->dev_nact = nullptr;
  c->host_scal = nullptr;
  c->host_int = nullptr;
}

struct CtxDeleter {
  void operator()(ndmg_ctx* c) const {
    release(c);
    delete c;
  }
};

int setup_common(ndmg_ctx** out, int nprob, const int* ns, double length, const double* alpha,
                 int nrhs, const ndmg_opts* opts, void* d_workspace, size_t workspace_bytes,
                 void* stream, int levels = 0) {
  if (!out) return fail(NDMG_EINVAL, "null output pointer");
  *out = nullptr;
  if (!alpha) return fail(NDMG_EINVAL, "null alpha array");
  std::unique_ptr<ndmg_ctx, CtxDeleter> c(new ndmg_ctx());
  NDMG_TRY(make_plan(nprob, ns, length, nrhs, opts, &c->plan, levels));
  for (int p = 0; p < nprob; ++p)
    if (!(alpha[p] > 0.0) || !std::isfinite(alpha[p])) return fail(NDMG_EINVAL, "alpha must be > 0");
  if (!d_workspace) return fail(NDMG_EINVAL, "null workspace");
  if (workspace_bytes < c->plan.bytes)
    return fail(NDMG_EWORKSPACE, "workspace smaller than the planned size");
  if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign)
    return fail(NDMG_EWORKSPACE, "workspace must be 256-byte aligned");
  c->ws = static_cast<char*>(d_workspace);
  c->st = static_cast<hipStream_t>(stream);
  Plan& pl = c->plan;
  for (auto& C : pl.cls) {
    C.alpha.clear();
    for (int p : C.probs) C.alpha.push_back(alpha[p]);
  }
  NDMG_HIP(hipMemsetAsync(c->ws, 0, pl.bytes, c->st));
  {
    Staging stg;
    for (auto& C : pl.cls)
      NDMG_TRY(pl.elem == 8 ? build_class_factors<double>(c.get(), C, stg)
                            : build_class_factors<float>(c.get(), C, stg));
    NDMG_HIP(hipStreamSynchronize(c->st));   // staging buffers die with stg
  }
  for (auto& C : pl.cls)
    NDMG_TRY(pl.elem == 8 ? build_dense<double>(c.get(), C) : build_dense<float>(c.get(), C));
  NDMG_HIP(hipStreamSynchronize(c->st));
  const size_t nc = pl.cls.size();
  for (size_t i = 1; i < nc; ++i) {
    hipStream_t s = nullptr;
    NDMG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    c->side.push_back(s);
    hipEvent_t e = nullptr;
    NDMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->ev_join.push_back(e);
  }
  if (nc > 1) NDMG_HIP(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  int maxcount = 0;
  for (auto& C : pl.cls) maxcount = std::max(maxcount, C.count);
  NDMG_HIP(hipHostMalloc((void**)&c->host_nact, 2 * nc * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent));
  NDMG_HIP(hipHostGetDevicePointer((void**)&c->dev_nact, c->host_nact, 0));
  for (auto& e : c->ev_nact) NDMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  NDMG_HIP(hipHostMalloc((void**)&c->host_scal, (size_t)maxcount * kScalStride * sizeof(double),
                         hipHostMallocDefault));
  NDMG_HIP(hipHostMalloc((void**)&c->host_int, (size_t)maxcount * 2 * sizeof(int), hipHostMallocDefault));
  *out = c.release();
  return NDMG_OK;
}

// The box (0, box[0]) x (0, box[1]) x (0, box[2]) with nx x ny x nz elements (Sec. 1: a
// box with axis-parallel edges, meshed by congruent cubes): the elements must be cubes.  A
// cube is served directly.  Another box is the domain, inside the cube of n = max(n_d)
// elements per axis, made of the boxes of g = gcd(nx, ny, nz) elements per axis that it
// covers (the grid of ndmg_opts.domain with r = n / g): every vector lives in that cube's
// layout with zeros outside the box.  *opts_out then holds the caller's options with that
// domain (pointing into *mask, which must outlive the plan or setup call).
int check_box(int nx, int ny, int nz, const double* box, const ndmg_opts* opts, int* n, double* length,
              ndmg_opts* opts_out, std::vector<unsigned char>* mask, const ndmg_opts** use) {
  if (!box) return fail(NDMG_EINVAL, "null box");
  if (nx < 2 || ny < 2 || nz < 2) return fail(NDMG_EINVAL, "nx, ny, nz must be >= 2");
  for (int d = 0; d < 3; ++d)
    if (!(box[d] > 0.0) || !std::isfinite(box[d])) return fail(NDMG_EINVAL, "box lengths must be > 0");
  const double h[3] = {box[0] / nx, box[1] / ny, box[2] / nz};
  for (int d = 1; d < 3; ++d)
    if (std::fabs(h[d] - h[0]) > 1e-12 * h[0])
      return fail(NDMG_EINVAL, "the elements must be cubes: box[d] / n_d must be equal");
  *use = opts;
  const int nd[3] = {nx, ny, nz};
  const int nmax = std::max(nx, std::max(ny, nz));
  *n = nmax;
  *length = h[0] * nmax;
  if (nx == ny && ny == nz) return NDMG_OK;
  if (opts && (opts->coef_r > 0 || opts->domain))
    return fail(NDMG_EINVAL, "a box that is not a cube is served as a domain inside a cube and takes no "
                             "coefficient boxes or domain of its own (give those on the embedding cube)");
  int g = nx;
  for (int d = 1; d < 3; ++d) {
    int a = g, b = nd[d];
    while (b) {
      const int t = a % b;
      a = b;
      b = t;
    }
    g = a;
  }
  const int r = nmax / g;
  if (r > 64) return fail(NDMG_EINVAL, "box too elongated: max(n_d) / gcd(n_d) must be at most 64");
  mask->assign((size_t)r * r * r, 0);
  for (int bz = 0; bz < r; ++bz)
    for (int by = 0; by < r; ++by)
      for (int bx = 0; bx < r; ++bx)
        (*mask)[((size_t)bz * r + by) * r + bx] = (bx * g < nx && by * g < ny && bz * g < nz) ? 1 : 0;
  if (opts)
    *opts_out = *opts;
  else
    ndmg_default_opts(opts_out);
  opts_out->coef_r = r;
  opts_out->coef = nullptr;
  opts_out->domain = mask->data();
  *use = opts_out;
  return NDMG_OK;
}

}  // namespace

extern "C" {

void ndmg_default_opts(ndmg_opts* o) {
  if (!o) return;
  o->smoother = NDMG_SMOOTHER_VERTEX;
  o->m = 1;
  o->eta = 0.0;
  o->precision = NDMG_PREC_FP64;
  o->subdomain = 2;
  o->boundary_patches = 1;
  o->flexible = -1;
  o->use_graphs = -1;
  o->bottom_n = 0;
  o->dense_n = -1;
  o->coef_r = 0;
  o->coef = nullptr;
  o->domain = nullptr;
}

const char* ndmg_last_error(void) { return g_err.c_str(); }

int ndmg_plan(int nx, int ny, int nz, const double box[3], double alpha, int levels,
              const ndmg_opts* opts, size_t* workspace_bytes, size_t* vec_len) {
  int n = 0;
  double length = 0.0;
  ndmg_opts embed;
  std::vector<unsigned char> mask;
  const ndmg_opts* use = nullptr;
  NDMG_TRY(check_box(nx, ny, nz, box, opts, &n, &length, &embed, &mask, &use));
  if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(NDMG_EINVAL, "alpha must be > 0");
  Plan pl;
  NDMG_TRY(make_plan(1, &n, length, 1, use, &pl, levels));
  if (workspace_bytes) *workspace_bytes = pl.bytes;
  if (vec_len) *vec_len = (size_t)pl.total_len;
  return NDMG_OK;
}

int ndmg_setup(ndmg_ctx** out, int nx, int ny, int nz, const double box[3], double alpha, int levels,
               const ndmg_opts* opts, void* d_workspace, size_t workspace_bytes, void* stream) {
  if (!out) return fail(NDMG_EINVAL, "null output pointer");
  *out = nullptr;
  int n = 0;
  double length = 0.0;
  ndmg_opts embed;
  std::vector<unsigned char> mask;
  const ndmg_opts* use = nullptr;
  NDMG_TRY(check_box(nx, ny, nz, box, opts, &n, &length, &embed, &mask, &use));
  return setup_common(out, 1, &n, length, &alpha, 1, use, d_workspace, workspace_bytes, stream, levels);
}

int ndmg_plan_batched(int nprob, const int* n, double length, int nrhs, const ndmg_opts* opts,
                      size_t* workspace_bytes, size_t* total_len) {
  Plan pl;
  NDMG_TRY(make_plan(nprob, n, length, nrhs, opts, &pl));
  if (workspace_bytes) *workspace_bytes = pl.bytes;
  if (total_len) *total_len = (size_t)pl.total_len;
  return NDMG_OK;
}

int ndmg_setup_batched(ndmg_ctx** out, int nprob, const int* n, double length, const double* alpha,
                       int nrhs, const ndmg_opts* opts, void* d_workspace, size_t workspace_bytes,
                       void* stream) {
  return setup_common(out, nprob, n, length, alpha, nrhs, opts, d_workspace, workspace_bytes, stream);
}

int ndmg_batch_layout(const ndmg_ctx* c, int prob, int64_t info[6]) {
  if (int rc = check_ctx(c)) return rc;
  if (!info) return fail(NDMG_EINVAL, "null info");
  const Plan& pl = c->plan;
  if (prob < 0 || prob >= pl.nprob) return fail(NDMG_EINVAL, "problem index out of range");
  const Cls& C = pl.cls[pl.prob_cls[prob]];
  const ndmg::Geom& g = C.lv.back().g;
  info[0] = C.vec_off + (int64_t)pl.prob_pos[prob] * C.nrhs * C.vlen;
  info[1] = C.vlen;
  info[2] = g.n;
  info[3] = g.P;
  info[4] = g.B;
  info[5] = (int64_t)C.lv.size();
  return NDMG_OK;
}

int ndmg_layout(const ndmg_ctx* c, int level, int64_t info[6]) {
  if (int rc = check_ctx(c)) return rc;
  if (int rc = one_class(c)) return rc;
  if (!info) return fail(NDMG_EINVAL, "null info");
  const Cls& C = c->plan.cls[0];
  const int nl = (int)C.lv.size();
  if (level < 0) level += nl;
  if (level < 0 || level >= nl) return fail(NDMG_EINVAL, "level out of range");
  const ndmg::Geom& g = C.lv[level].g;
  info[0] = g.n;
  info[1] = g.P;
  info[2] = g.B;
  info[3] = g.len;
  info[4] = nl;
  info[5] = c->plan.coef.empty() ? 3LL * g.n * (g.n - 1) * (g.n - 1)
                                 : (int64_t)ndmg::unknown_offsets(g, c->plan.boxes()).size();
  return NDMG_OK;
}

int ndmg_apply(ndmg_ctx* c, const double* x, double* y) {
  if (int rc = check_ctx(c)) return rc;
  if (!x || !y) return fail(NDMG_EINVAL, "null vector");
  return for_classes(c, [&](size_t ci, hipStream_t st) {
    Cls& C = c->plan.cls[ci];
    NDMG_HIP(ndmg::launch_apply<double>(x + C.vec_off, nullptr, y + C.vec_off, C.lv.back().g,
                                        class_batch(c, C, false), 0, st));
    return NDMG_OK;
  });
}

int ndmg_vcycle(ndmg_ctx* c, const double* g, double* z) {
  if (int rc = check_ctx(c)) return rc;
  if (!g || !z) return fail(NDMG_EINVAL, "null vector");
  return for_classes(c, [&](size_t ci, hipStream_t st) {
    Cls& C = c->plan.cls[ci];
    return precondition(c, C, g + C.vec_off, z + C.vec_off, class_batch(c, C, false), st);
  });
}

int ndmg_pcg_solve(ndmg_ctx* c, const double* b, double* u, double rtol, int maxit, int* iters,
                   double* relres) {
  if (int rc = check_ctx(c)) return rc;
  if (c->plan.npairs != 1)
    return fail(NDMG_EINVAL, "the context holds several right-hand sides; use ndmg_pcg_solve_batched");
  return ndmg_pcg_solve_batched(c, b, u, rtol, maxit, iters, relres);
}

}  // extern "C"

namespace {

int pcg_entry(ndmg_ctx* c, const double* b, double* u, double rtol, int maxit, int* iters, double* relres,
              bool warm) {
  if (int rc = check_ctx(c)) return rc;
  if (!b || !u) return fail(NDMG_EINVAL, "null vector");
  if (reinterpret_cast<uintptr_t>(b) % 16 || reinterpret_cast<uintptr_t>(u) % 16)
    return fail(NDMG_EINVAL, "d_b and d_u must be 16-byte aligned");
  if (!(rtol >= 0.0) || maxit < 1) return fail(NDMG_EINVAL, "bad rtol or maxit");
  const int np = c->plan.npairs;
  if (iters) std::fill(iters, iters + np, 0);
  if (relres) std::fill(relres, relres + np, 0.0);
  return pcg_all(c, b, u, rtol, maxit, iters, relres, warm);
}

}  // namespace

extern "C" {

int ndmg_pcg_solve_batched(ndmg_ctx* c, const double* b, double* u, double rtol, int maxit,
                           int* iters, double* relres) {
  return pcg_entry(c, b, u, rtol, maxit, iters, relres, false);
}

int ndmg_pcg_solve_warm(ndmg_ctx* c, const double* b, double* u, double rtol, int maxit, int* iters,
                        double* relres) {
  return pcg_entry(c, b, u, rtol, maxit, iters, relres, true);
}

int ndmg_maxwell_step(ndmg_ctx* c, const double* f, double* u, double* v, double* a, double dt, double eps,
                      double sigma, double mu, double rtol, int maxit, int* iters, double* relres) {
  if (int rc = check_ctx(c)) return rc;
  if (int rc = one_class(c)) return rc;
  if (!f || !u || !v || !a) return fail(NDMG_EINVAL, "null vector");
  if (!(dt > 0.0) || !(eps >= 0.0) || !(sigma >= 0.0) || !(mu > 0.0) || !(eps + 0.5 * sigma * dt > 0.0) ||
      !std::isfinite(dt) || !std::isfinite(eps) || !std::isfinite(sigma) || !std::isfinite(mu))
    return fail(NDMG_EINVAL, "need dt > 0, mu > 0, eps >= 0, sigma >= 0 and eps + sigma dt / 2 > 0");
  Cls& C = c->plan.cls[0];
  const double d = eps + 0.5 * sigma * dt;
  const double want = dt * dt / (4.0 * mu * d);
  for (double al : C.alpha)
    if (std::fabs(al - want) > 1e-12 * want)
      return fail(NDMG_EINVAL, "the context's alpha must be dt^2 / (4 mu (eps + sigma dt / 2)) = " +
                                   std::to_string(want));
  const ndmg::Geom& g = C.lv.back().g;
  const int64_t len = g.len;
  const ndmg::Bat all = class_batch(c, C, false);
  // the mass matrix: the operator at alpha = 0 (with coefficient boxes, on the same domain)
  const ndmg::Bat mass{C.count, C.nrhs, at<double>(c, C.o_alpha0), nullptr, all.coef, all.coef_r};
  double* w = at<double>(c, C.o_tw);
  double* rhs = at<double>(c, C.o_tb);
  double* t = at<double>(c, C.o_pz);   // CG vectors, free outside the solve
  hipStream_t st = c->st;
  const double h2 = 0.25 * dt * dt;
  // predictor w = u + dt v + dt^2/4 a
  NDMG_HIP(ndmg::launch_lincomb(w, u, 1.0, v, dt, a, h2, len, all, st));
  // rhs = (dt^2/4 f + M (eps w + sigma (dt/2 u + dt^2/4 v))) / (eps + sigma dt/2)
  NDMG_HIP(ndmg::launch_lincomb(t, w, eps, u, sigma * 0.5 * dt, v, sigma * h2, len, all, st));
  NDMG_HIP(ndmg::launch_apply<double>(t, nullptr, rhs, g, mass, 0, st));
  NDMG_HIP(ndmg::launch_lincomb(rhs, rhs, 1.0 / d, f, h2 / d, nullptr, 0.0, len, all, st));
  // u_{n+1}: the model problem with alpha = dt^2 / (4 mu d), started from the predictor
  NDMG_HIP(ndmg::launch_copy(w, u, len, all, st));
  const int rc = pcg_entry(c, rhs, u, rtol, maxit, iters, relres, true);
  if (rc != NDMG_OK) return rc;
  // a_{n+1} = 4 / dt^2 (u_{n+1} - w);  v_{n+1} = v_n + dt/2 (a_n + a_{n+1})
  NDMG_HIP(ndmg::launch_lincomb(t, u, 1.0 / h2, w, -1.0 / h2, nullptr, 0.0, len, all, st));
  NDMG_HIP(ndmg::launch_lincomb(v, v, 1.0, a, 0.5 * dt, t, 0.5 * dt, len, all, st));
  NDMG_HIP(ndmg::launch_copy(t, a, len, all, st));
  NDMG_HIP(hipStreamSynchronize(st));
  return NDMG_OK;
}

}  // extern "C"

namespace {

// Eigenvalues of the symmetric tridiagonal matrix (diagonal a, off-diagonal b) below x:
// the negative pivots of its LDL^T factorisation (Sturm sequence count).
int count_below(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double q = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    const double bb = i ? b[i - 1] * b[i - 1] : 0.0;
    q = (a[i] - x) - (i ? bb / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// Smallest (which = 0) or largest (which = 1) eigenvalue by bisection on the Sturm count
// within the Gershgorin interval.
double tridiag_extreme(const std::vector<double>& a, const std::vector<double>& b, int which) {
  double lo = a[0], hi = a[0];
  for (size_t i = 0; i < a.size(); ++i) {
    const double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < a.size() ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  const int target = which == 0 ? 1 : (int)a.size();   // the first x with count_below >= target
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (count_below(a, b, mid) >= target) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace

extern "C" {

int ndmg_contraction(ndmg_ctx* c, const double* b, double* u, double rtol, int maxit, double* contraction,
                     double* lam_max, int* iters) {
  if (int rc = check_ctx(c)) return rc;
  if (!contraction) return fail(NDMG_EINVAL, "null output");
  const Plan& pl = c->plan;
  if (pl.npairs != 1) return fail(NDMG_EINVAL, "the contraction needs a context with one right-hand side");
  if (pl.opts.precision != NDMG_PREC_FP64 || flexible_beta(pl))
    return fail(NDMG_EINVAL, "the contraction needs the FP64 V-cycle and the standard CG beta");
  if (maxit < 1 || maxit > ndmg::kHistCap) return fail(NDMG_EINVAL, "maxit must be in [1, 512]");
  int it = 0;
  double rel = 0.0;
  const int rc = ndmg_pcg_solve_batched(c, b, u, rtol, maxit, &it, &rel);
  if (rc != NDMG_OK && rc != NDMG_ENOCONV && rc != NDMG_EBREAKDOWN) return rc;
  const Cls& C = pl.cls[0];
  const int k = std::min(it, ndmg::kHistCap);
  if (k < 1) return fail(NDMG_EINVAL, "no CG iteration ran (zero right-hand side?)");
  std::vector<double> h((size_t)2 * k);
  NDMG_HIP(hipMemcpy(h.data(), at<double>(c, C.o_hist), h.size() * sizeof(double), hipMemcpyDeviceToHost));
  // CG with preconditioner B is the Lanczos process for B A: alpha_j = r_j.z_j / p_j.A p_j,
  // beta_j = r_{j+1}.z_{j+1} / r_j.z_j give its tridiagonal matrix T with diagonal
  // 1/alpha_j + beta_{j-1}/alpha_{j-1} and off-diagonal sqrt(beta_j)/alpha_j.  The process
  // is scale-free, so CG may run past the convergence of u; the matrix ends at a breakdown
  // (scalars not finite and positive) or once r.z has fallen below 1e-200 of its first
  // value, before the products of the shrinking vectors reach the subnormal range.
  std::vector<double> alpha, beta;
  const double rz0 = h[0];
  auto usable = [&](int j) {
    const double rz = h[2 * j], pq = h[2 * j + 1];
    return rz > 0.0 && pq > 0.0 && std::isfinite(rz) && std::isfinite(pq) && rz >= 1e-200 * rz0 &&
           pq >= 1e-200 * h[1];
  };
  for (int j = 0; j < k && usable(j); ++j) {
    alpha.push_back(h[2 * j] / h[2 * j + 1]);
    if (j + 1 < k && usable(j + 1)) beta.push_back(h[2 * j + 2] / h[2 * j]);
  }
  const size_t m = alpha.size();
  if (m < 1) return fail(NDMG_EBREAKDOWN, "no usable CG iteration");
  std::vector<double> d(m), e(m > 1 ? m - 1 : 0);
  for (size_t j = 0; j < m; ++j) d[j] = 1.0 / alpha[j] + (j ? beta[j - 1] / alpha[j - 1] : 0.0);
  for (size_t j = 0; j + 1 < m; ++j) e[j] = std::sqrt(beta[j]) / alpha[j];
  *contraction = 1.0 - tridiag_extreme(d, e, 0);
  if (lam_max) *lam_max = tridiag_extreme(d, e, 1);
  if (iters) *iters = (int)m;
  return NDMG_OK;
}

const char* ndmg_source_key(void) { return ndmg::source_key(); }

int ndmg_tuning_load(const char* path) {
  if (!path) return fail(NDMG_EINVAL, "null path");
  std::string err;
  if (!ndmg::tune_load(path, &err)) return fail(NDMG_EINVAL, err);
  return NDMG_OK;
}

int ndmg_tuning_set(const char* line) {
  if (!line) return fail(NDMG_EINVAL, "null line");
  std::string err;
  if (!ndmg::tune_set_line(line, &err)) return fail(NDMG_EINVAL, err);
  return NDMG_OK;
}

int ndmg_tuning_clear(void) {
  ndmg::tune_clear();
  return NDMG_OK;
}

int ndmg_stencil_shape(int n, int precision, int mode, int count, int* variant, int* kz) {
  if (!variant || !kz) return fail(NDMG_EINVAL, "null pointer");
  if (precision != NDMG_PREC_FP64 && precision != NDMG_PREC_FP32) return fail(NDMG_EINVAL, "bad precision");
  if (n <= ndmg::stencil_min_n(count) || n > ndmg::stencil_max_n())
    return fail(NDMG_EINVAL, "n outside the sizes of the plane-marching kernel");
  if (!ndmg::stencil_shape(n, precision == NDMG_PREC_FP64 ? 8 : 4, mode, count, variant, kz))
    return fail(NDMG_EINVAL, "no launch variant for this precision and mode");
  return NDMG_OK;
}

int ndmg_time_stencil(int n, int precision, int mode, int count, int variant, int kz, const void* x,
                      const void* b, void* y, double* part, const double* alpha, int reps, int nrot, void* stream,
                      double* avg_us) {
  if (!x || !y || !part || !alpha || !avg_us || (mode == 1 && !b)) return fail(NDMG_EINVAL, "null pointer");
  if (nrot < 1) return fail(NDMG_EINVAL, "nrot must be >= 1");
  if (precision != NDMG_PREC_FP64 && precision != NDMG_PREC_FP32) return fail(NDMG_EINVAL, "bad precision");
  if (mode < 0 || mode > 2 || (mode == 2 && precision != NDMG_PREC_FP64)) return fail(NDMG_EINVAL, "bad mode");
  if (count < 1 || reps < 1) return fail(NDMG_EINVAL, "bad count or reps");
  if (n <= ndmg::stencil_min_n(count) || n > ndmg::stencil_max_n())
    return fail(NDMG_EINVAL, "n outside the sizes of the plane-marching kernel");
  const int elem = precision == NDMG_PREC_FP64 ? 8 : 4;
  if (variant < 0 || variant >= ndmg::stencil_variant_count(elem, mode, n))
    return fail(NDMG_EINVAL, "no such launch variant");
  if (kz < 2 || kz > n) return fail(NDMG_EINVAL, "kz must be in [2, n]");
  const ndmg::Geom g = ndmg::make_geom(n, 1.0);
  const ndmg::Bat bt{count, count, alpha, nullptr};
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t ps = ndmg::stencil_max_blocks(g);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  NDMG_HIP(hipEventCreate(&e0));
  NDMG_HIP(hipEventCreate(&e1));
  // set r of the nrot rotating vector sets starts r count vectors after the first
  const int64_t set = (int64_t)count * g.len * elem;
  auto launch = [&](int r) -> hipError_t {
    const int64_t o = (int64_t)(r % nrot) * set;
    const char* xr = static_cast<const char*>(x) + o;
    const char* br = b ? static_cast<const char*>(b) + o : nullptr;
    char* yr = static_cast<char*>(y) + o;
    if (elem == 8)
      return ndmg::launch_stencil<double>((const double*)xr, (const double*)br, (double*)yr, g, bt, mode, part, ps,
                                          nullptr, st);
    return ndmg::launch_stencil<float>((const float*)xr, (const float*)br, (float*)yr, g, bt, mode, nullptr, 0,
                                       nullptr, st);
  };
  ndmg::tune_force_stencil(variant, kz);
  hipError_t e = hipSuccess;
  for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch(r);
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch(r);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  ndmg::tune_force_stencil(-1, -1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(NDMG_EHIP, std::string("stencil timing: ") + hipGetErrorString(e));
  *avg_us = 1e3 * ms / reps;
  return NDMG_OK;
}

int ndmg_assemble_rhs(ndmg_ctx* c, const double* f, double* b) {
  if (int rc = check_ctx(c)) return rc;
  if (!f || !b) return fail(NDMG_EINVAL, "null pointer");
  const Plan& pl = c->plan;
  for (const Cls& C : pl.cls) {
    const ndmg::Geom& g = C.lv.back().g;
    const int64_t flen = 24LL * g.n * g.n * g.n;
    // f follows the pair order of the batch vectors
    const int64_t f0 = [&] {
      int64_t s = 0;
      for (const Cls& D : pl.cls) {
        if (&D == &C) break;
        s += 24LL * D.n * D.n * D.n * D.count;
      }
      return s;
    }();
    for (int pr = 0; pr < C.count; ++pr)
      NDMG_HIP(ndmg::launch_assemble_rhs(f + f0 + pr * flen, b + C.vec_off + pr * C.vlen, g, c->st,
                                         pl.coef.empty() ? nullptr : at<double>(c, C.o_coef), pl.opts.coef_r));
  }
  return NDMG_OK;
}

int ndmg_curlcurl_form(ndmg_ctx* c, const double* lam, const double* u, int nrhs, double* out) {
  if (int rc = check_ctx(c)) return rc;
  if (int rc = one_class(c)) return rc;
  if (!lam || !u || !out || nrhs < 0) return fail(NDMG_EINVAL, "bad arguments");
  Cls& C = c->plan.cls[0];
  const ndmg::Geom& g = C.lv.back().g;
  double* part = at<double>(c, C.o_part);
  double* sc = at<double>(c, C.o_scal);
  double total = 0.0;
  for (int r = 0; r < nrhs; ++r) {
    const bool jumps = !c->plan.coef.empty();
    NDMG_HIP(ndmg::launch_curlcurl_form(lam + (int64_t)r * g.len, u + (int64_t)r * g.len, g, part,
                                        sc + kS_CC, c->st, jumps ? at<double>(c, C.o_coef) : nullptr,
                                        jumps ? c->plan.opts.coef_r : 0));
    NDMG_HIP(hipMemcpyAsync(c->host_scal, sc, kScalStride * sizeof(double), hipMemcpyDeviceToHost, c->st));
    NDMG_HIP(hipStreamSynchronize(c->st));
    total += c->host_scal[kS_CC];
  }
  *out = total;
  return NDMG_OK;
}

}  // extern "C"

namespace {

// Scratch of the allocation-free curl-curl form: 256 bytes for its result slot, then
// one partial sum per block of the form kernel.  Each GPU the library runs on holds its
// own copy until the process ends; every call on a GPU reuses that GPU's copy.
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
constexpr size_t kNoAllocResultBytes = 256;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};   // device address of `scratch`, per device

// Device address of `scratch` on the current device, looked up once per device with that
// device current (host code never passes the array's own name to a kernel: on the host
// it stands in for the device copy and is not a device address).
int scratch_on_current_device(void** out) {
  int dev = -1;
  NDMG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(NDMG_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    NDMG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(NDMG_EHIP, "hipGetSymbolAddress returned a null address");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return NDMG_OK;
}

}  // namespace

extern "C" {

int ndmg_curlcurl_form_noalloc(int n, double length, const double* lam, const double* u, int nrhs,
                               double* out, void* stream) {
  if (n < 2 || n > 2048) return fail(NDMG_EINVAL, "n must be in [2, 2048]");
  if (!(length > 0.0) || !std::isfinite(length)) return fail(NDMG_EINVAL, "length must be > 0");
  if (!lam || !u || !out || nrhs < 0) return fail(NDMG_EINVAL, "bad arguments");
  const ndmg::Geom g = ndmg::make_geom(n, length);
  // one partial per block of the form kernel's grid: ceil((n + 1) / 64) x (n + 1)^2
  const size_t nparts = (size_t)((n + 1 + 63) / 64) * (size_t)(n + 1) * (size_t)(n + 1);
  const size_t need = kNoAllocResultBytes + nparts * sizeof(double);
  if (need > kNoAllocScratchBytes)
    return fail(NDMG_EINVAL, "n = " + std::to_string(n) + " needs " + std::to_string(need) +
                                 " bytes of scratch, more than the fixed " +
                                 std::to_string(kNoAllocScratchBytes) + " of the allocation-free form");
  void* base = nullptr;
  NDMG_TRY(scratch_on_current_device(&base));
  double* res = static_cast<double*>(base);
  double* part = reinterpret_cast<double*>(static_cast<char*>(base) + kNoAllocResultBytes);
  hipStream_t st = static_cast<hipStream_t>(stream);
  double total = 0.0;
  for (int r = 0; r < nrhs; ++r) {
    // the form kernel writes every partial and the final sum writes the result slot, so
    // nothing left by an earlier call is read
    NDMG_HIP(ndmg::launch_curlcurl_form(lam + (int64_t)r * g.len, u + (int64_t)r * g.len, g, part, res, st));
    double v = 0.0;
    NDMG_HIP(hipMemcpyAsync(&v, res, sizeof(double), hipMemcpyDeviceToHost, st));
    NDMG_HIP(hipStreamSynchronize(st));
    total += v;
  }
  *out = total;
  return NDMG_OK;
}

int ndmg_export_factor(const ndmg_ctx* c, int level, int which, int type, double* buf, int* dims) {
  if (int rc = check_ctx(c)) return rc;
  if (int rc = one_class(c)) return rc;
  if (!dims) return fail(NDMG_EINVAL, "null dims");
  const Cls& C = c->plan.cls[0];
  const int nl = (int)C.lv.size();
  if (level < 0) level += nl;
  if (level < 1 || level >= nl) return fail(NDMG_EINVAL, "level must be a smoothed level");
  if (which != 0 && which != 1) return fail(NDMG_EINVAL, "which must be 0 or 1");
  if (which == 1 && (type < 0 || type > 26)) return fail(NDMG_EINVAL, "type out of range");
  const LevelHost& L = C.lv[level];
  if (!c->plan.coef.empty()) return fail(NDMG_EINVAL, "with a coefficient (coef_r > 0) the factors differ by box: not exported");
  if (L.gen) {
    const ndmg::GenTables& tb = L.gt;
    if (which == 1 && std::find(tb.typesP.begin(), tb.typesP.end(), type) == tb.typesP.end())
      return fail(NDMG_EINVAL, "no patch of that type on this level");
    dims[0] = which == 0 ? L.sub.nI : tb.npadP;
    if (!buf) return NDMG_OK;
    std::vector<double> xc((size_t)tb.npadI * tb.npadB), ex((size_t)tb.npadE * tb.npadI),
        sp((size_t)tb.ntypes * tb.npadP * tb.npadP);
    std::string err;
    if (!build_gen_factors<double>(L, C.alpha[0], xc.data(), ex.data(), sp.data(), &err))
      return fail(NDMG_EINVAL, err);
    if (which == 0) {   // A_T^{-1}: columns k of ex below nI (symmetric)
      for (int i = 0; i < L.sub.nI; ++i)
        for (int j = 0; j < L.sub.nI; ++j) buf[(size_t)i * L.sub.nI + j] = ex[(size_t)j * tb.npadI + i];
    } else {
      std::memcpy(buf, sp.data() + (size_t)type * tb.npadP * tb.npadP, (size_t)tb.npadP * tb.npadP * sizeof(double));
    }
    return NDMG_OK;
  }
  dims[0] = which == 0 ? L.sub.nI : L.sub.npad;
  if (!buf) return NDMG_OK;
  // rebuilt in FP64 for the first problem (the device copy is in the working precision)
  ndmg::LevelFactors fac;
  std::string err;
  if (!ndmg::build_level_factors(L.g.h, C.alpha[0], L.sub, c->plan.opts.boundary_patches != 0, &fac, &err))
    return fail(NDMG_EINVAL, err);
  if (which == 0) {
    std::memcpy(buf, fac.ATinv.data(), fac.ATinv.size() * sizeof(double));
  } else {
    const int np = L.sub.npad;
    std::memcpy(buf, fac.Sinv.data() + (size_t)type * np * np, (size_t)np * np * sizeof(double));
  }
  return NDMG_OK;
}

}  // extern "C"

namespace {

// One step on one level in the V-cycle's precision T.  in and out are the operation's
// input and output in T (for FP32 contexts: the level buffers holding the converted
// vectors).
template <typename T>
int level_op_t(ndmg_ctx* c, Cls& C, int level, int op, const T* in, T* out, const ndmg::Bat& bt) {
  LevelHost& L = C.lv[level];
  switch (op) {
    case NDMG_OP_APPLY:
      NDMG_HIP(ndmg::launch_apply<T>(in, nullptr, out, L.g, bt, 0, c->st));
      return NDMG_OK;
    case NDMG_OP_SMOOTH:
      return smooth_level<T>(c, C, L, in, out, bt, 1, c->st);
    case NDMG_OP_RESTRICT:
      NDMG_HIP(ndmg::launch_restrict<T>(in, out, L.g, C.lv[level - 1].g, bt, c->st));
      return NDMG_OK;
    case NDMG_OP_PROLONG:
      NDMG_HIP(ndmg::launch_prolong_add<T>(in, out, L.g, C.lv[level - 1].g, bt, c->st));
      return NDMG_OK;
    case NDMG_OP_PATCH:
      if (L.gen) {
        NDMG_HIP(ndmg::launch_patch_generic<T>(gen_level<T>(c, L), bt, c->st));
      } else {
        NDMG_HIP(ndmg::launch_patch_products<T>(level_ptrs<T>(c, L), level_dsub(c, L), L.g, bt, c->st));
      }
      return NDMG_OK;
    default:   // NDMG_OP_COARSE
      NDMG_HIP(ndmg::launch_coarse<T>(in, out, at<T>(c, L.o_A0), at<int64_t>(c, L.o_map), (int)L.map.size(),
                                      L.g.len, bt, c->st));
      return NDMG_OK;
  }
}

}  // namespace

extern "C" {

int ndmg_level_op(ndmg_ctx* c, int level, int op, const double* in, double* out) {
  if (int rc = check_ctx(c)) return rc;
  if (int rc = one_class(c)) return rc;
  if (!in || !out) return fail(NDMG_EINVAL, "null vector");
  Plan& pl = c->plan;
  Cls& C = pl.cls[0];
  const int nl = (int)C.lv.size();
  if (level < 0) level += nl;
  if (level < 0 || level >= nl) return fail(NDMG_EINVAL, "level out of range");
  if (op < NDMG_OP_APPLY || op > NDMG_OP_PATCH) return fail(NDMG_EINVAL, "unknown operation");
  if ((op == NDMG_OP_SMOOTH || op == NDMG_OP_PATCH) && !C.lv[level].smoothed)
    return fail(NDMG_EINVAL, "the coarsest level has no smoother");
  if ((op == NDMG_OP_RESTRICT || op == NDMG_OP_PROLONG) && level < 1)
    return fail(NDMG_EINVAL, "transfers need level >= 1");
  if (op == NDMG_OP_COARSE && level != 0) return fail(NDMG_EINVAL, "coarse solve needs level 0");
  const ndmg::Bat bt = class_batch(c, C, false);
  if (pl.elem == 8) return level_op_t<double>(c, C, level, op, in, out, bt);
  if (op == NDMG_OP_PATCH) return level_op_t<float>(c, C, level, op, nullptr, nullptr, bt);
  // FP32 context: the FP64 input is rounded into a level buffer of the input's level,
  // the step runs in FP32 into a buffer of the output's level (holding the rounded old
  // output for the accumulating prolongation), and the result is widened into out.
  const int lin = op == NDMG_OP_PROLONG ? level - 1 : level;
  const int lout = op == NDMG_OP_RESTRICT ? level - 1 : level;
  LevelHost& Li = C.lv[lin];
  LevelHost& Lo = C.lv[lout];
  float* fin = at<float>(c, Li.o_g);
  float* fout = at<float>(c, Lo.o_z);
  NDMG_HIP((ndmg::launch_convert<double, float>(in, fin, Li.g.len, bt, c->st)));
  if (op == NDMG_OP_PROLONG) NDMG_HIP((ndmg::launch_convert<double, float>(out, fout, Lo.g.len, bt, c->st)));
  NDMG_TRY(level_op_t<float>(c, C, level, op, fin, fout, bt));
  NDMG_HIP((ndmg::launch_convert<float, double>(fout, out, Lo.g.len, bt, c->st)));
  return NDMG_OK;
}

int ndmg_destroy(ndmg_ctx* c) {
  if (!c) return NDMG_OK;
  release(c);
  delete c;
  return NDMG_OK;
}

}  // extern "C"
