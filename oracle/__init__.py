"""FP64 CPU oracle for the particle-particle-ladder (PPL) response path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or call anything here.
The GPU library never imports it and shares no code with it: the packed-pair
indexing, the integrals, the right-hand side, the denominators, the DIIS
step and the gradients are all written out again here, plainly, from the
paper's definitions (and, where the paper is silent, the readings stated in
each module).

Modules:
  ppl       -- sigma = PPL(X), by definition, by a factored identity, by brute
               force, and entry by entry.
  response  -- model LR problem: RHS, denominators, Jacobi+DIIS solve, dense
               per-pair solve, sum-over-states solve, alpha.
  grads     -- vector-Jacobian products of sigma with respect to X and L.
  hhl       -- the hole-hole ladder over occupied-occupied Cholesky vectors
               (definition, factored identity, brute force, packed matrix).
  ring      -- the particle-hole (ring) term of the doubles-doubles Jacobian
               (definition, a route that never forms the integrals, matrix).
  chol      -- the pivoted Cholesky decomposition that produces the vectors.
  fns       -- perturbation-sensitive natural spinors (FNS++): MP2 and
               perturbed amplitudes, dressed diagonals, the averaged density,
               truncation by |occupation| and the semicanonical basis.

Every function is pinned by ``tests/test_oracle_*.py`` against brute force,
closed forms, invariants or finite differences.  Parity with the paper's
printed numbers is unpinned: the paper's molecular results need integrals
that are not available, and it prints no worked example of this path.
"""
from . import ppl, response, grads, hhl, ring, chol, fns  # noqa: F401
