"""FP64 CPU oracle for the charge-conserving FEM-PIC cycle with the quasi-Helmholtz
field update (O'Connor, Crawford, Ramachandran, Luginsland, Shanker, arXiv 2103.06737).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call, link or run
anything in this package: only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it. It shares no code with the GPU library; both sides receive the
same seeded inputs from ``qh_inputs`` and compute independently.

Modules
  complex_   mesh complex K = {N, E, F, T} and its incidence matrices (Sec. II.C)
  whitney    barycentric geometry, Whitney forms W0..W3, Hodge and mixed matrices
             (Sec. II.C, the Hodge-matrix and [grad]/[curl]/[div] definitions)
  particles  gather, Boris push, tet walk, quantised path-integral deposit (Sec. II.A
             point particles, Sec. IV.B.1 path integral G^n); plain C in pic.c
  field      implicit field update: Crank-Nicolson (Newmark beta=1/4, gamma=1/2) on the
             semi-discrete system plus the Gauss-law solve for the non-solenoidal part
             (Sec. IV.B.1 eq. discreteGauss, Sec. IV.B.2 eq. reduceMEs)
  cotree     the literal tree/co-tree reduced system Z11..Z23 on tiny meshes (Sec. IV.B)
  learned    FP64 MLP forward/backward and flexible CG for the learned preconditioner
"""
