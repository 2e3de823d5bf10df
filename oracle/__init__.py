"""Plain, slow FP64 CPU oracle for the force-evaluation path.

TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product library
never does, and it shares no code, tables or constants with the HIP path.

Each function follows a passage of the paper (DIMOS, arXiv 2503.20541) or a
textbook definition the paper relies on, cited in its docstring. Floating
point is float64 throughout, except for the neighbour-list inclusion
predicate, which the method specifies here as an IEEE float32 expression
(round-to-nearest, no fused multiply-add) so that the GPU list can be checked
bit-exactly; numpy's float32 element-wise operations are correctly rounded
and never contracted.

Modules
  neighbors  - Verlet-list inclusion predicate, brute-force and tree-seeded lists
  nonbonded  - LJ (Eqs. 4-6) + real-space Ewald (Eq. 10), exclusion and self
               corrections (Eq. 12), energies, forces, virial
  bonded     - harmonic bonds and angles (Eqs. 1-2)
  bspline    - cardinal B-splines by recursion (Sec. II.A.2, PME paragraph)
  pme        - smooth particle-mesh Ewald in float64 with numpy.fft
  ewald      - alpha heuristic (Eq. 13), k_c root (Eq. 14), direct Ewald sum
  integrate  - velocity Verlet (Sec. II.D.1) in float64 and float32-emulated
  forcefield - sums the components for a synth.System-like object
  adjoint    - gradients of a velocity-Verlet trajectory loss (parameters,
               initial state, time step) by the reverse recursion, with a
               complex-safe force field for exact directional derivatives
"""
