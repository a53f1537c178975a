"""Plain FP64 CPU oracle for multigrid multilevel Monte Carlo trace estimation
with orthogonal projectors (Frommer, Jimenez-Merchan, Knechtli, Korzec,
Ramirez-Hidalgo, arXiv:2509.11424).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and
the benchmark's CPU-baseline leg may import it.  The GPU library never calls
it and shares no code with it: the two sides only share the seeded inputs of
``lattice_inputs``.

Everything here is written for a reader checking it against the paper: numpy
in complex128, no blocking or fusion beyond what a definition states.

Modules
  philox      counter-based Philox4x32-10 generator and Z4 probes (eq. z4)
  dirac       gamma matrices, clover term, Wilson-clover operator, dense D
  multigrid   aggregation, test vectors, block QR, P, P^H, Galerkin D_c
  solve       restarted GMRES and dense solves
  estimators  Hutchinson per-probe values for the plain, oblique (M_l) and
              orthogonal (O_l, F_l) decompositions, connected correlator
              G_rs(t), disconnected loops, variance estimator, MLMC N_l
  ptc         gauge-covariant parallel-transport convolution network
"""
