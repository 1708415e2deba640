"""CPU oracle for the thread-safe multiphase lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product (the HIP library and
its Python binding) never calls it and has no CPU fallback.

Plain, slow, FP64 NumPy written from the paper (arXiv 2501.00846):
  * lattice.py   - D3Q27 velocities, weights and Hermite tensors (Sec. II.B).
  * scheme.py    - one whole-array time step in the order of Sec. II.D:
                   moments and forces -> pre-regularisation -> fused
                   stream/collide (push form, Eq. pushLB) -> interface
                   tracking by FTCS; plus the observables and diagnostics.
  * pointwise.py - a second, per-node implementation of the same step in pull
                   form (pure Python loops), used on tiny grids to check the
                   streaming/boundary indexing of scheme.py and at full sizes
                   on sampled nodes.

It shares no code with the HIP path.  Its only shared input is the seeded
generator module paper_2501_00846_amd.workloads (initial fields, no method
arithmetic).

Variants: the gradient closure of a2 (Eq. noneqts, readings G1-G4) and the
fourth-order phase-field stencils of the higher-order Allen-Cahn update
(future work at the end of Sec. II.A, readings H1-H3), both in scheme.py and
pointwise.py.

Readings of places where the paper is silent or garbled are listed in the
docstring of scheme.py; each function cites the section / equation it follows.
Parity status: every function here is pinned by tests under tests/ against
closed forms, invariants or brute force, except the normal-vector guard
epsilon where grad(phi) = 0 and the viscous-correction force beyond its
limits (uniform density, uniform flow), which are "parity unpinned".
"""
from . import lattice, scheme, pointwise  # noqa: F401
