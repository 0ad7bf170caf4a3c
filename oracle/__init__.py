"""CPU FP64 oracle for the hexahedral Nedelec V-cycle multigrid (Oh, arXiv 2205.05840).

This package is TEST INFRASTRUCTURE. It is a plain, slow, assembled-sparse-matrix
implementation of what the GPU library computes, written from the paper:

  * ``mesh``       level hierarchy (Sec. 3.1), compact interior-edge numbering,
                   subdomain index sets (Sec. 3.2)
  * ``element``    the 12x12 element mass and curl-curl matrices of the lowest-order
                   hexahedral Nedelec space (Sec. 2, eq. nedlec form / NDdof)
  * ``assemble``   the global A = alpha*K + M two independent ways (Kronecker form and
                   element-by-element), the nodal gradient G (de Rham check)
  * ``transfer``   natural injection I_{k-1}^k and its transpose (Sec. 3.1, eq. F2C)
  * ``exact``      exact discrete solves: sparse direct and a DST/DCT block solve
  * ``smoother``   vertex-based substructuring smoother, literal per-patch form and
                   factored form (Sec. 3.2.2, eq. Preconditioner P)
  * ``vcycle``     the symmetric V-cycle MG(k, g, z0, m) (Sec. 3.3, Fig. 1)
  * ``pcg``        textbook preconditioned CG around the V-cycle
  * ``rhs``        load vector b = (f, phi_e) from samples at the 2x2x2 Gauss points
  * ``contraction`` V-cycle contraction number ||E_k||_a (Sec. 4.2, eq. VCycleRecursion)
  * ``adjoint``    gradients of L = sum_k ||u_k - t_k||^2 w.r.t. b_k and alpha
  * ``coefficient`` alpha with jumps on a grid of boxes: cell-by-cell assembly (Sec. 6)
  * ``domain``     non-box domains: unions of boxes of the grid, the cube restricted (Sec. 6)
  * ``timestep``   implicit (average-acceleration Newmark) time stepping of Maxwell's
                   equations, each step the model problem (Sec. 1, eq. Maxwell timestep)

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg may
import it. It shares no code, headers, tables or helpers with the HIP library under
``paper_2205_05840_amd/``, and it imports nothing from there.

Functions whose result has no independent pin say "parity unpinned" in their
docstring. Every other function is pinned by a test under ``tests/`` against a
closed form, an invariant, a brute-force computation or a number printed in the
paper (Table 2).
"""
