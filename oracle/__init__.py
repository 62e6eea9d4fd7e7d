"""FP64 CPU oracle for the RI-HF hot path.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding)
never imports, links or calls anything here, and this package shares no code
with it: the only common module is ``synth`` (seeded inputs, no arithmetic of
the method).

Contents (plain numpy / scipy, FP64, no blocking or fusion beyond what the
definitions state):

* ``integrals`` - closed-form s-Gaussian one- and two-electron integrals and
  their nuclear derivatives (definitions in the paper's Notation section;
  Gaussian-product algebra from the textbook it cites).
* ``ri``        - screening, the RI fit path for J and K (eq. ri_eri, j_ri,
  k_ri), the B tensor under the L^{-1} convention (eq. biap) and a brute-force
  four-index RI tensor for small systems.
* ``scf``       - Roothaan closed-shell SCF with DIIS (Energy section).
* ``gradient``  - the analytic RI-HF gradient (eq. rihf_gradient) and a
  finite-difference gradient.

Parity status of each function is stated in its module header.
"""
