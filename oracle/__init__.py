"""FP64 CPU oracle for BDDC-preconditioned GMRES on finite-element tangents.

TEST INFRASTRUCTURE ONLY. Nothing in the solver library imports, links or runs
this package; only the test-suite, the smoke check and the benchmark's CPU
baseline leg do. It is a plain, slow, obviously-correct restatement of the
method of Barnafi, Pavarino and Scacchi (arXiv 2208.06191), §3.2:

* ``fem``   - assembly of the unassembled element tangents into the global
               operator A = sum_i A^(i) and elimination of clamped DOFs.
* ``bddc``  - the non-overlapping decomposition, the primal (vertex / edge /
               face) constraints, counting-function weights, the constrained
               local (Neumann) and interior (Dirichlet) problems, the coarse
               basis Phi, the coarse matrix S_PiPi, the two- and three-level
               preconditioner M^-1_BDDC wrapped in the exact block
               factorisation of A^-1 (static condensation).
* ``gmres`` - right-preconditioned restarted GMRES with modified Gram-Schmidt
               and Givens rotations (the Krylov method the paper pairs with
               BDDC, §1 and §2 "Numerical approximation").

Everything is float64, built from numpy / scipy primitives (sparse products,
dense and sparse LU), with no blocking, fusion or reordering beyond what the
definitions state.
"""
