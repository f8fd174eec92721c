"""FP64 CPU oracle for the k-point AFQMC walker-batch step (test infrastructure).

This package is test infrastructure only.  It is imported by the tests, by the
smoke check of the repository entry module, and by the CPU-baseline leg of the
benchmark -- never by the GPU library or its Python binding, and it shares no
code with them.

Modules
-------
kpoint     -- the blocked k-point formulas (force bias, HS potential, Taylor
              propagation, Green's function, local energy and its adjoint),
              in the paper's order and notation, complex128 throughout.
supercell  -- brute force on the unfolded supercell: dense Cholesky operators,
              explicit 4-index integrals, the generic Green's function, energy,
              force bias and HS potential of the standard representation, and
              the generalized Fock matrix.  Tiny meshes only.
molecular  -- the standard-representation energy and force bias written with
              the half-rotated X, X-bar, T, T-bar intermediates; used for the
              Nk = 1 reduction.

Every function is pinned by tests against something other than itself
(closed forms, invariants, brute force, exact finite differences).  The phase
of the importance function (weights) is formula-only: parity unpinned beyond
the agreement of the blocked and supercell bookkeeping.
"""
