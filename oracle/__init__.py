"""Plain FP64 CPU oracle for the VMC force hot path (test infrastructure).

This package is test infrastructure, not product code: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP path (``paper_2511_05222_amd``);
both consume the seeded inputs of ``paper_2511_05222_amd.inputs`` and nothing
else.

Everything is numpy in float64 (complex128 where a derivative is taken by the
complex-step method).  Each function cites the passage of the paper it
follows; where the paper is silent the reading taken is stated.

Modules
  philox        counter-based RNG (Philox4x32-10) and the draws of a move
  gto           cartesian contracted GTOs: value, gradient, Laplacian
  wavefunction  Jastrow-Slater determinant, log|Psi|, local energy
  derivatives   SWCT warp, d/dR by complex step, d/dC by matrix calculus
  sampler       single-electron Metropolis (fresh-LU and Sherman-Morrison)
  estimators    energy, bare force and dE/dC estimators (shifted FP64 sums)
  zvector       Cholesky and conjugate-gradient solutions of H z = -b
  h2_closed_form  RHF energy of H2 in a minimal s basis (textbook integrals)
"""
