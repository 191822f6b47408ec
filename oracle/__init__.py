"""CPU FP64 oracle for the two-phase TPFA Newton-Krylov-AMG hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code
with the GPU library: it reads the same seeded inputs (from
``paper_1611_00127_amd.inputs``) and nothing else.

Each function is a plain, slow, readable statement of what the paper (arXiv
1611.00127, Bui, Elman, Moulton) defines, or of the build's stated reading
where the paper is silent:

* ``tpfa``     Sec. 2 (TPFA fluxes, upwinding, harmonic permeability, backward
               Euler) -> residual F(u) and its exact Jacobian (Sec. 3).
* ``blocks``   Sec. 3.1 block structure (A_pp, A_ps, A_sp, A_ss), Sec. 3.2
               point ordering, Sec. 3.4 approximate Schur complement.
* ``amg``      classical AMG as chosen for the build: strength of connection,
               PMIS coarsening, direct interpolation, Galerkin product,
               l1-Jacobi V(1,1) cycle, dense coarsest solve.
* ``ilu``      block ILU(0), the first stage of the two-stage methods (Sec. 3.3).
* ``precond``  Algorithms 1-3 and Eqs. m_comb, m_add, m_bf.
* ``fgmres``   right-preconditioned flexible GMRES(m) with CGS2 and Givens.
* ``newton``   the Newton linearisation of Sec. 3.

Parity status: every function is pinned by the CPU tests (closed forms,
invariants, finite/complex-step differences, dense brute force), except
the full-solve iteration counts, which the paper's own tables cannot pin
(other AMG components, other data): "parity unpinned" for those counts.
"""
