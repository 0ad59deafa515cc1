"""CPU FP64 oracle of the submatrix-method density matrix.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call or
link anything in this directory; only the tests, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP path: it takes plain numpy inputs (the block-column panel layout that
the seeded generators produce) and computes everything with numpy / LAPACK in
float64, step by step as the paper states the method.

Modules
  submatrix  -- index sets, submatrices, matrix sign by eigendecomposition,
                assembly of P, tr(PH), tr P, chemical-potential bisection,
                full-matrix projector (the exact reference).
  newton_schulz -- the plain dense Newton-Schulz sign iteration in float64
                (iteration counts and the convergence rule), and the scalar map.
  mlp        -- float64 forward / backward / Adam of the scaling network.
  overlap    -- a non-orthogonal basis: inverse square roots (Eq. 12 by its
                definition), P of Eq. 14 on every submatrix pair by the
                generalized symmetric eigendecomposition, tr(PH), tr(PS).
  fermi      -- the general f of Fig. 2 taken as the Fermi-Dirac occupation
                at inverse temperature beta: f(T_i) by eigendecomposition,
                the electron count and its mu-derivative, mu by bisection.
"""
