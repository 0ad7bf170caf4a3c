/*
 * ndmg: V-cycle multigrid for the lowest-order hexahedral Nedelec discretisation of
 *        curl(alpha curl u) + u = f in a box (this version: a cube), u x n = 0 on its
 *        boundary,
 *        with the nonoverlapping substructuring smoothers of Oh, "Multigrid methods for
 *        3D H(curl) problems with nonoverlapping domain decomposition smoothers"
 *        (arXiv 2205.05840), used as a preconditioner inside conjugate gradients.
 *
 * C ABI.  Every pointer argument named d_* is a device (HIP, gfx950) pointer owned by
 * the caller; every other pointer is a host pointer owned by the caller.  The library
 * allocates no device memory: the caller passes a device workspace of the size
 * ndmg_plan (or ndmg_plan_batched) reports (the one fixed array of the library's image,
 * used by ndmg_curlcurl_form_noalloc, is the exception).  A context owns host metadata, a few pinned
 * host words for the convergence test and, when it holds several problem sizes, one
 * side stream and event per extra size.  All device work is enqueued on the stream
 * given at setup (work of extra sizes forks from it and joins back before a call
 * returns its last enqueued operation).  A context must not be used from two threads
 * at once.  Functions return NDMG_OK or one of the error codes below and never abort
 * or throw; ndmg_last_error() then describes the failure (per thread).
 *
 * Vector layout ("padded edge layout").  The mesh has n^3 cubes of side h = length/n.
 * An edge of direction d (0 = x, 1 = y, 2 = z) is addressed by (i, j, k): along axis
 * d a cell index in [0, n), along the other two axes a node index in [0, n].  A
 * vector holds one value per edge (the edge average of the tangential component,
 * Sec. 2, eq. NDdof) at offset
 *        d * B + (k * (n + 1) + j) * P + i,    P = pitch, B = (n + 1)^2 * P,
 * total length 3 * B (ndmg_layout reports n, P, B).  Only interior edges (transverse
 * node indices in [1, n-1]) are unknowns (zero tangential trace, Sec. 1).  Every other
 * entry (boundary edges, the unused i = n of x-edges etc., the row padding) must be 0
 * on input and is written as 0 (or left untouched, where stated) on output.
 * Floating-point vectors at the boundary are always double (FP64).
 *
 * Batches.  A batched context (ndmg_setup_batched) holds nprob independent problems,
 * each with its own n and alpha, with nrhs right-hand sides each.  A "batch vector"
 * concatenates one padded vector per (problem, right-hand side) pair; ndmg_batch_layout
 * gives the offset of each problem's first vector (its nrhs vectors follow each other).
 * ndmg_apply and ndmg_vcycle act on batch vectors; a single-problem context is the
 * batch of one pair, whose batch vector is the plain padded vector.
 */
#ifndef NDMG_H
#define NDMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------- */
#define NDMG_OK 0
#define NDMG_EINVAL 1      /* invalid argument (sizes, alpha <= 0, null pointer, ...) */
#define NDMG_EHIP 2        /* a HIP runtime call failed                               */
#define NDMG_ENOCONV 3     /* PCG reached maxit; u, iters and relres are still written */
#define NDMG_EBREAKDOWN 4  /* PCG breakdown: p^T A p <= 0 or a non-finite scalar        */
#define NDMG_EWORKSPACE 5  /* workspace too small or misaligned                         */

/* ---- options ----------------------------------------------------------------------- */
#define NDMG_SMOOTHER_VERTEX 0   /* vertex-based smoother, eq. (Preconditioner P)       */
#define NDMG_SMOOTHER_EDGE 1     /* edge-based smoother, eq. (Preconditioner E)         */
#define NDMG_PREC_FP64 0         /* V-cycle in FP64                                     */
#define NDMG_PREC_FP32 1         /* V-cycle in FP32 inside FP64 CG (mixed precision)    */

typedef struct ndmg_opts {
  int smoother;         /* NDMG_SMOOTHER_VERTEX (default) or NDMG_SMOOTHER_EDGE       */
  int m;                /* smoothing steps m of MG(k, g, z0, m) (Fig. 1); default 1   */
  double eta;           /* damping of the whole smoother sum; <= 0 (default) selects
                           the value of Sec. 5: 1/9 (vertex), 1/13 (edge)             */
  int precision;        /* NDMG_PREC_FP64 or NDMG_PREC_FP32                           */
  int subdomain;        /* s: subdomains are s x s x s fine cells (min(s, n_k / 2) on
                           level k); 2 (= T_{k-1}, Sec. 3.2; default) or 4             */
  int boundary_patches; /* 1: vertex (edge) spaces also at coarse vertices (edges) on
                           the boundary, cut to the domain (default; reproduces
                           Table 2); 0: interior coarse vertices (edges) only         */
  int flexible;         /* 1: Polak-Ribiere beta in PCG (default for FP32)          */
  int use_graphs;       /* 1: replay each CG iteration from a captured HIP graph when
                           the stream is not the null stream; 0: eager launches;
                           -1 (default): graphs unless the context holds one size
                           class whose finest level has n >= 80 (there the host
                           queues an iteration's launches faster than the device
                           runs them, and eager launches measured 1-4 % faster;
                           below, graphs 8-9 % faster)                               */
  int bottom_n;         /* levels with n_k <= bottom_n (at most 64) and the coarsest
                           solve run as one launch with one workgroup per (problem,
                           right-hand side); 0 (default): every level launches its
                           own kernels (faster on MI355X for every size measured).
                           Vertex smoother with subdomain 2 only.                   */
  int dense_n;          /* with z_0 = 0 the V-cycle MG(k, g, 0, m) of Fig. 1 is a
                           linear map of g: from the finest level with n_k <= dense_n
                           (at most 8, i.e. at most 1176 unknowns) down, it is applied
                           as one dense matrix per problem, built at setup by the
                           recursive V-cycle on unit vectors (the same map, rounded
                           differently; the matrices take nprob N_k^2 scalars of the
                           workspace).  0: the recursion all the way down.  -1
                           (default): 8 for a size class of fewer than 16 problems, 4
                           for larger classes (the build costs nprob N_k V-cycles). */
  int coef_r;           /* a coefficient with jumps (Sec. 6, the first extension the
                           paper names): alpha(x) = alpha * coef[(bz r + by) r + bx] on
                           the r x r x r grid of equal boxes tiling the cube (x fastest),
                           r = coef_r.  0 (default): alpha constant.  r must divide the
                           coarsest level's n, and n_k / r must be a multiple of the
                           subdomain size on every smoothed level, so that every element
                           and every subdomain lies in one box: each level is then the
                           cell-by-cell form of eq. (fem) with its cell's alpha, the coarse
                           forms are the Galerkin restrictions of the fine one, and every
                           subdomain and patch gets the factors of its own alphas (any
                           smoother and subdomain size; the gathered-product smoother on
                           every level).  Single problems only (ndmg_setup, or one problem
                           in ndmg_setup_batched); bottom_n must be 0; ndmg_export_factor
                           is refused.  ndmg_curlcurl_form then returns lam^T K_c u with
                           K_c = sum_T coef_T K_T, the derivative of A in alpha.          */
  const double* coef;   /* the r^3 box factors (> 0), host memory, read during ndmg_plan /
                           ndmg_setup only (the context keeps a copy); NULL when r = 0,
                           or all factors 1 when a domain is given                       */
  const unsigned char* domain; /* a non-box domain (Sec. 6 names nonconvex domains as an
                           extension): the boxes of the coef_r grid that Omega keeps
                           (r^3 flags, nonzero = in Omega, same order as coef), for
                           instance the cube less one octant.  The unknowns are the edges
                           whose four cells all lie in Omega (zero tangential trace on
                           its boundary); every vector keeps zeros at the other edges,
                           and ndmg_layout's info[5] counts Omega's unknowns.  Same
                           conditions as coef_r; NULL (default): the whole cube.  Read
                           during ndmg_plan / ndmg_setup only.                          */
} ndmg_opts;

/* Fill *o with the defaults above. */
void ndmg_default_opts(ndmg_opts* o);

/* ---- planning and setup ---------------------------------------------------------------
 * ndmg_plan: validate a problem and report the device workspace size in bytes and the
 * vector length (in elements) of the padded edge layout of the finest level.
 * The domain is the box (0, box[0]) x (0, box[1]) x (0, box[2]) (Sec. 1: a box with
 * axis-parallel edges) meshed by nx x ny x nz congruent cubes (box[d] / n_d equal; the
 * uniform refinement of Sec. 3.1 keeps them cubes).  A cube (nx = ny = nz = n >= 2) is
 * served directly.  Another box is served as a non-box domain (see ndmg_opts.domain)
 * inside the cube of n = max(n_d) elements per axis and side n h, made of the boxes of
 * gcd(nx, ny, nz) elements per axis that it covers: vectors, load samples and
 * ndmg_layout then refer to that cube (zeros outside the box), n / gcd must divide the
 * coarsest level, and opts may not carry coefficient boxes or a domain of their own.
 * alpha: the constant of
 * eq. (model problem) (> 0).  levels: 0 for all levels n, n/2, ... while a level is even
 * and its half is >= 2 (Sec. 3.1, h_k = h_{k-1}/2), else the number of levels kept from
 * the finest down (1 = the exact solve alone); the coarsest is solved exactly and must
 * have at most 1024 unknowns.  Every smoothed level must be divisible by min(s, n_k / 2).
 * Either output pointer may be NULL.  Errors: NDMG_EINVAL.
 */
int ndmg_plan(int nx, int ny, int nz, const double box[3], double alpha, int levels,
              const ndmg_opts* opts, size_t* workspace_bytes, size_t* vec_len);

/* Opaque solver context. */
typedef struct ndmg_ctx ndmg_ctx;

/* ndmg_setup: for the problem of ndmg_plan (same box, alpha and levels), build the
 * level hierarchy and the local factors of every level (the
 * subdomain matrices A_T of eq. ATDef and the vertex-space matrices A_V of eq. AVDef,
 * inverted in FP64 on the host), lay out the caller's workspace (d_workspace, at
 * least the planned size, 256-byte aligned), clear it and upload the factors.
 * stream: a hipStream_t (NULL = default stream).  opts may be NULL (defaults).
 * On success *out owns host metadata only; release it with ndmg_destroy.
 * Errors: NDMG_EINVAL, NDMG_EWORKSPACE, NDMG_EHIP.
 */
int ndmg_setup(ndmg_ctx** out, int nx, int ny, int nz, const double box[3], double alpha, int levels,
               const ndmg_opts* opts, void* d_workspace, size_t workspace_bytes, void* stream);

/* ndmg_layout: describe the padded edge layout of a level (level 0 = coarsest,
 * level -1 = finest) of a context with a single problem size.  info[0] = n,
 * info[1] = P (row pitch), info[2] = B (block length), info[3] = vector length 3 B,
 * info[4] = number of levels, info[5] = number of unknowns 3 n (n-1)^2.
 * Errors: NDMG_EINVAL.
 */
int ndmg_layout(const ndmg_ctx* ctx, int level, int64_t info[6]);

/* ---- batches (Sec. 2 problem statement per problem; Sec. 3.3 V-cycle; CG per pair) ---
 * ndmg_plan_batched: validate nprob problems on cubes of side `length` with n[p]
 * elements per axis (host array) and nrhs right-hand sides each, and report the
 * workspace size in bytes and the batch vector length in elements.  Problems with the
 * same n form one size class; every kernel launch covers all pairs of a class.
 * Limits: nprob * nrhs <= 65535.  Either output pointer may be NULL.
 * Errors: NDMG_EINVAL. */
int ndmg_plan_batched(int nprob, const int* n, double length, int nrhs, const ndmg_opts* opts,
                      size_t* workspace_bytes, size_t* total_len);

/* ndmg_setup_batched: as ndmg_setup for every problem p with alpha[p] (host array, all
 * > 0); the local factors of each (problem, level) are built in FP64 on host threads.
 * Errors: NDMG_EINVAL, NDMG_EWORKSPACE, NDMG_EHIP. */
int ndmg_setup_batched(ndmg_ctx** out, int nprob, const int* n, double length,
                       const double* alpha, int nrhs, const ndmg_opts* opts, void* d_workspace,
                       size_t workspace_bytes, void* stream);

/* ndmg_batch_layout: info[0] = offset (elements) of problem `prob`'s first vector in a
 * batch vector, info[1] = its padded vector length 3 B, info[2] = n, info[3] = P,
 * info[4] = B, info[5] = number of levels.  Errors: NDMG_EINVAL. */
int ndmg_batch_layout(const ndmg_ctx* ctx, int prob, int64_t info[6]);

/* Solve A_p u = b for every (problem p, right-hand side) pair of the context as in
 * ndmg_pcg_solve, each pair with its own CG scalars and stopping test: a pair that has
 * converged (or broken down) is left out of every later kernel.  d_b and d_u are batch
 * vectors.  iters and relres (host, may be NULL) receive nprob * nrhs entries, entry
 * p * nrhs + r for right-hand side r of problem p.  The host waits once per iteration
 * for the count of pairs still active after the previous iteration, with the next
 * iteration already enqueued (so one iteration with every pair inactive, whose kernels
 * return at once, follows the last convergence); with use_graphs one iteration of the
 * whole batch (all sizes) is replayed from one captured graph.  d_b and d_u must be 16-byte aligned.
 * Errors: NDMG_EINVAL, NDMG_EHIP, NDMG_ENOCONV (some pair reached maxit; every output
 * still written), NDMG_EBREAKDOWN (some pair broke down). */
int ndmg_pcg_solve_batched(ndmg_ctx* ctx, const double* d_b, double* d_u, double rtol, int maxit,
                           int* iters, double* relres);

/* ---- operations (all FP64 vectors in the padded layout of the finest level) -------- */

/* y = A x with A the matrix of a(., .) on N_h (eq. def bilinear form, eq. fem):
 * y = alpha K x + M x.  d_x and d_y must not overlap.  Errors: NDMG_EINVAL, NDMG_EHIP. */
int ndmg_apply(ndmg_ctx* ctx, const double* d_x, double* d_y);

/* z = MG(J, g, 0, m): one symmetric V-cycle (Fig. 1) with the vertex-based smoother of
 * eq. (Preconditioner P) and the grid transfers of eq. (F2C), in the context's
 * precision.  d_g and d_z must not overlap.  Errors: NDMG_EINVAL, NDMG_EHIP. */
int ndmg_vcycle(ndmg_ctx* ctx, const double* d_g, double* d_z);

/* Solve A u = b (eq. fem) by conjugate gradients preconditioned with the V-cycle,
 * from u = 0, until ||b - A u||_2 <= rtol ||b||_2 (recursive residual) or maxit
 * iterations.  iters and relres (host pointers, may be NULL) receive the iteration
 * count and the final relative residual ||r|| / ||b|| (computed on the device, the
 * value the stopping test used).  The context must hold one pair (one problem, one
 * right-hand side).  The host waits once per iteration for the convergence test of the
 * previous iteration while the next one is already enqueued.  With use_graphs, the
 * iterations after the first
 * are replayed from two HIP graphs captured on first use (and again whenever d_u
 * changes); the stream must then not be the null stream and must not be captured by
 * the caller.  d_b and d_u must be 16-byte aligned (the CG vector kernels move four
 * values per access).
 * Errors: NDMG_EINVAL, NDMG_EHIP, NDMG_ENOCONV (u still written), NDMG_EBREAKDOWN. */
int ndmg_pcg_solve(ndmg_ctx* ctx, const double* d_b, double* d_u, double rtol, int maxit,
                   int* iters, double* relres);

/* As ndmg_pcg_solve_batched, but every pair starts from the vector the caller put in d_u
 * (its non-unknown entries must be 0): r_0 = b - A u_0, and the stopping test is still
 * ||b - A u|| <= rtol ||b||.  For sequences of related right-hand sides (time stepping):
 * a good initial guess saves iterations.  Errors: as ndmg_pcg_solve_batched. */
int ndmg_pcg_solve_warm(ndmg_ctx* ctx, const double* d_b, double* d_u, double rtol, int maxit,
                        int* iters, double* relres);

/* One implicit time step of Maxwell's equations (Sec. 1): with H eliminated, the electric
 * field solves eps E'' + sigma E' + curl(mu^{-1} curl E) = J' (all coefficients constant).
 * The average-acceleration Newmark scheme (beta = 1/4, gamma = 1/2; the trapezoidal rule,
 * which conserves the discrete energy when sigma = 0) asks in each step for
 *   (dt^2 / 4) curl(mu^{-1} curl E_{n+1}) + (eps + sigma dt / 2) E_{n+1} = R.H.S.,
 * the equation of eq. (Maxwell timestep), i.e. the model problem with alpha =
 * dt^2 / (4 mu (eps + sigma dt / 2)), which must be the context's alpha (relative 1e-12).
 * In the discrete setting (M the mass matrix, K the curl-curl matrix, padded layout):
 *   w = u + dt v + dt^2/4 a                                  (predictor)
 *   A u' = (dt^2/4 f + M (eps w + sigma (dt/2 u + dt^2/4 v))) / (eps + sigma dt/2)
 *   a' = 4 / dt^2 (u' - w),   v' = v + dt/2 (a + a')
 * with f = (J', phi_e) the load vector of the current's time derivative at the new time,
 * and the solve by V-cycle PCG started from w (ndmg_pcg_solve_warm; rtol and maxit as
 * there).  d_u, d_v, d_a (field, its rate and its second rate) are updated in place; every
 * (problem, right-hand side) pair of a single-size context steps at once.  Waits for the
 * step before returning.  Errors: NDMG_EINVAL, NDMG_EHIP, NDMG_ENOCONV, NDMG_EBREAKDOWN. */
int ndmg_maxwell_step(ndmg_ctx* ctx, const double* d_f, double* d_u, double* d_v, double* d_a, double dt,
                      double eps, double sigma, double mu, double rtol, int maxit, int* iters, double* relres);

/* Contraction number ||E_J||_a of the V-cycle (Sec. 4.2: E = I - B A with B = MG(J, ., 0,
 * m) is a-symmetric positive semidefinite, so ||E||_a = 1 - lambda_min(B A); the quantity
 * of Sec. 5, Tables 1-2), estimated by the Lanczos process of V-cycle-preconditioned CG:
 * CG on A u = b from u = 0 (d_b any vector with components along every eigenvector, e.g.
 * random; d_u receives the iterate and must be 16-byte aligned like d_b) runs for maxit
 * iterations (at most 512) or until ||r|| <= rtol ||b||, and its coefficients give the
 * tridiagonal Lanczos matrix T of B A, whose extreme eigenvalues (Sturm bisection on the
 * host) bound those of B A from inside.  rtol = 0 runs CG past the convergence of u (the
 * process is scale-free); the matrix then ends where r.z has fallen below 1e-200 of its
 * first value.  *contraction = 1 - lambda_min(T) (from below,
 * converging as the iterations grow), *lam_max = lambda_max(T) (may be NULL), *iters =
 * the Lanczos steps used (may be NULL).  Needs a context with one right-hand side, the
 * FP64 V-cycle and the standard CG beta (flexible = 0 or default).
 * Errors: NDMG_EINVAL, NDMG_EHIP, NDMG_EBREAKDOWN. */
int ndmg_contraction(ndmg_ctx* ctx, const double* d_b, double* d_u, double rtol, int maxit,
                     double* contraction, double* lam_max, int* iters);

/* Load vector b_e = (f, phi_e) (Sec. 2, the functional f_h) from f sampled at the
 * 2x2x2 Gauss-Legendre points of every element: d_f is [n^3][8][3] doubles, element
 * (c0, c1, c2) at row (c2 n + c1) n + c0, point q = q0 + 2 q1 + 4 q2 at local
 * coordinates (x_{q0}, x_{q1}, x_{q2}), x = (1 -+ 1/sqrt 3) / 2, components x, y, z.
 * d_b receives the padded layout.  For a batched context d_f holds one such array per
 * pair, in the pair order of the batch vectors, and d_b is a batch vector.
 * Errors: NDMG_EINVAL, NDMG_EHIP. */
int ndmg_assemble_rhs(ndmg_ctx* ctx, const double* d_f, double* d_b);

/* out = sum_r lam_r^T K u_r for nrhs vector pairs stored back to back (each of the
 * padded vector length of the context's single problem size), K = dA/dalpha the
 * curl-curl matrix of eq. (def bilinear form).  out is a host pointer.  Used for dL/dalpha = -sum_r lam_r^T K u_r.
 * Errors: NDMG_EINVAL, NDMG_EHIP. */
int ndmg_curlcurl_form(ndmg_ctx* ctx, const double* d_lam, const double* d_u, int nrhs,
                       double* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the curl-curl form of
 * ndmg_curlcurl_form without a context or workspace, for vectors of the padded layout
 * of an n^3 mesh of the cube (0, length)^3.  out (host) = sum_r lam_r^T K u_r over nrhs
 * vector pairs stored back to back.  Its partial sums live in a fixed 4 MiB device array
 * inside the library (one copy per GPU, kept until the process ends); meshes whose
 * (ceil((n+1)/64) (n+1)^2 partial sums plus a 256-byte result slot) exceed it are
 * rejected with NDMG_EINVAL before any device work (n <= 319).  The call allocates
 * nothing: no hipMalloc, no hipFree, no pinned host memory.  The work is enqueued on
 * `stream` (NULL = default stream) and the call waits for it once per right-hand side.
 * Calls that overlap on one GPU (several host threads, or a call on another stream
 * while one is running) share that array and race; callers serialise them.
 * Errors: NDMG_EINVAL, NDMG_EHIP. */
int ndmg_curlcurl_form_noalloc(int n, double length, const double* d_lam, const double* d_u, int nrhs,
                               double* out, void* stream);

/* Debug export of the FP64 local factors of a level (level as in ndmg_layout, >= 1) of
 * the first problem of a context with a single problem size (rebuilt on the host):
 * which = 0: A_T^{-1} (nI x nI, row-major), which = 1: the padded inverse Schur
 * complement of the vertex type `type` (0..26, per axis 0 low face, 1 inside, 2 high
 * face; 13 = interior), npad x npad row-major with zero rows/columns for slots that do
 * not exist for that type.  dims[0] receives the row count.  buf (host) must hold
 * dims[0]^2 doubles, or be NULL to query dims only.  Errors: NDMG_EINVAL. */
int ndmg_export_factor(const ndmg_ctx* ctx, int level, int which, int type, double* buf,
                       int* dims);

/* ---- single steps of one level (for tests and diagnostics) --------------------------
 * Vectors use the padded layout of the level(s) named (ndmg_layout), one per pair of
 * the context (a single problem size) back to back, in FP64.  level as in ndmg_layout.
 * In an FP32 context the input (and the old output of NDMG_OP_PROLONG) is rounded to
 * FP32 into level buffers of the context, the step runs in FP32 as inside the V-cycle,
 * and the result is widened to FP64 into out.
 *   NDMG_OP_APPLY     out = A_k in                                  (any level)
 *   NDMG_OP_SMOOTH    out = M_k^{-1} in, the smoother of the context (eq. Preconditioner
 *                     P or E) including its damping eta                 (level >= 1)
 *   NDMG_OP_RESTRICT  out (level k-1) = I_k^{k-1} in (level k), eq. (F2C)  (level >= 1)
 *   NDMG_OP_PROLONG   out (level k) += I_{k-1}^k in (level k-1)           (level >= 1)
 *   NDMG_OP_COARSE    out = A_0^{-1} in                               (level 0)
 *   NDMG_OP_PATCH     the patch products y_V = S_V^{-1} g|Gamma_V of the smoother alone,
 *                     on the condensed residual left in the context's level buffers by
 *                     the last smoothing step (for timing the kernel); in and out are
 *                     not read or written but must not be NULL           (level >= 1)
 * Errors: NDMG_EINVAL (bad level or op), NDMG_EHIP. */
#define NDMG_OP_APPLY 0
#define NDMG_OP_SMOOTH 1
#define NDMG_OP_RESTRICT 2
#define NDMG_OP_PROLONG 3
#define NDMG_OP_COARSE 4
#define NDMG_OP_PATCH 5
int ndmg_level_op(ndmg_ctx* ctx, int level, int op, const double* d_in, double* d_out);

/* ---- launch shapes: the autotuner's table ------------------------------------------
 * The plane-marching operator kernel (variant: waves per workgroup and ring depth; planes
 * per workgroup) and the vertex patch products (16-vertex groups per wave, for the
 * interior segment and for the segments on the box's faces and edges) take their launch
 * shapes from a process-wide table when it holds an entry for (size n, precision, mode,
 * class of pairs per launch: 1, 2-3, 4-15, 16-63, >= 64), else from a cost model.  The
 * table is measured on the device by paper_2205_05840_amd/tune.py.  A context keeps the
 * patch shapes of the table at its plan and setup; operator shapes are looked up per launch.
 *
 * ndmg_source_key: hash of the tuned kernels' sources, built into the library.
 * ndmg_tuning_load: replace the table by a file: a line "key <source key>", then lines
 *   "<stencil|patch> <n> <fp32|fp64> <mode> <pair class 0-4> <p0> <p1>" ('#' comments).
 *   A file keyed to other sources (or malformed) is refused with NDMG_EINVAL and the table
 *   is left as it was.
 * ndmg_tuning_set: add or replace one entry (a line of that format, no key needed).
 * ndmg_tuning_clear: empty the table (cost models everywhere).
 * ndmg_time_stencil: average duration in microseconds of `reps` launches of the operator
 *   kernel on an n^3 mesh with launch variant `variant` (0 .. count - 1 of the variants of
 *   that precision and mode) and kz planes per workgroup, forced for these launches only,
 *   on `count` caller vectors back to back (d_x, d_b for mode 1, d_y in the padded layout
 *   of the precision; d_part room for the partial sums of mode 2; d_alpha `count` device
 *   doubles), after 3 untimed launches, timed with HIP events on `stream`.  Launch r
 *   works on vector set r mod nrot (set r starts r count vectors after d_x, d_b, d_y), so
 *   that nrot sets larger than the last-level cache make every launch read HBM.
 * ndmg_stencil_shape: the shape a launch of the operator kernel takes now (the table's
 *   entry, or the cost model's choice).
 * Errors: NDMG_EINVAL (a variant that does not exist: the tuner's end of the list),
 * NDMG_EHIP. */
const char* ndmg_source_key(void);
int ndmg_tuning_load(const char* path);
int ndmg_tuning_set(const char* line);
int ndmg_tuning_clear(void);
int ndmg_time_stencil(int n, int precision, int mode, int count, int variant, int kz, const void* d_x,
                      const void* d_b, void* d_y, double* d_part, const double* d_alpha, int reps, int nrot,
                      void* stream, double* avg_us);
int ndmg_stencil_shape(int n, int precision, int mode, int count, int* variant, int* kz);

/* Release the context (host memory only; the workspace stays the caller's). */
int ndmg_destroy(ndmg_ctx* ctx);

/* Description of the last error on this thread ("" if none). */
const char* ndmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NDMG_H */
