"""Plain FP64 CPU oracle for hierarchical proximal Galerkin (hpG).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, table or
helper with the HIP library; the two meet only through the seeded input
generators in ``workloads/`` (which hold none of the method's arithmetic).

What it computes (Papadopoulos, "Hierarchical proximal Galerkin", arXiv
2412.13733):

* ``basis``    - Legendre P_n, the bubbles W_n of eq. (Wn), the hats, the
                 spectral-Galerkin Y_n and a Gauss-Legendre rule (Sec. 3).
* ``mesh``     - tensor-product meshes, the continuous space U_{h,p} and the
                 discontinuous space Psi_{h,p} with their DOF numbering (Sec. 3).
* ``hpmesh``   - the same with one degree per cell (obstacle), conforming by
                 the minimum rule on shared entities.
* ``assemble`` - the sparse matrices A, B, M_psi, the load vectors and the
                 nonlinear terms of eq. (pG) / eq. (pG:gradient) and their
                 Jacobian blocks D_psi, E_beta (Sec. 4.1-4.3).
* ``precond``  - the block preconditioner diag(alpha A, -S_hat) (Sec. 4.4-4.6)
                 and its block-Jacobi A-block on hp meshes.
* ``lvpp``     - the latent-variable proximal point loop with Newton and a
                 direct sparse LU of the full saddle matrix G of eq.
                 (pG-matrix) (Sec. 2, Sec. 4, remark on sparse LU in Sec. 4.4).

Every function is FP64 and deliberately unoptimised.  Where the paper is
silent the oracle takes the same documented reading as the GPU path
(quadrature rule, alpha schedule, stopping rules, line search); each reading
is named where it is used.

Parity status: all functions are pinned by ``tests/test_oracle_*.py``
(closed forms, brute-force QP at p=2, quadrature exactness, invariants),
except the gradient-constraint solve in 2-D/3-D, which is pinned only in 1-D
(closed form) and by residual/Jacobian consistency; its multi-dimensional
solutions are "parity unpinned".
"""
