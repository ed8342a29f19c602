"""Plain FP64 CPU oracle for the fast spectral Boltzmann collision operator
and the moment-realizability regime mask.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it, to check and to time the HIP
library.  It shares no code with the library; the seeded input generators in
``bz_inputs`` are the only code both sides use.

Modules
  spectral    the collision operator Q(f,f) of Sec. 4.4.1 in its fast spectral
              (Carleman, direction-quadrature) form, written with naive
              separable DFTs and a direct loop over directions; the
              conservative moment projection.
  maxwell2d   the same fast spectral operator for Maxwell molecules in two
              velocity dimensions (the 2d case of Sec. 4.4.1: constant
              Carleman kernel, equally spaced angles on the half circle) and
              its projection on the four invariants of two dimensions.
  directions  hemisphere quadrature rules (icosahedral axes, the paper's
              (theta, phi) product grid, equal-weight golden spiral).
  kinetic     macroscopic fields, the Maxwellian, the L1 distance of the
              kinetic-to-fluid criterion, and the penalised first-order IMEX
              update of the Boltzmann layer.
  mask        the realizability indicators of Sec. 3.2-3.3 / 4.5 and the
              regime update of Algorithm 1, in a fixed FP64 operation order.
"""
