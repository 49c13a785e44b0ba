"""Plain FP64 CPU oracle for the FFT-CONV / NSPT hot path (test infrastructure).

This package is test infrastructure.  Only the test-suite, the smoke check of
the entry module and the CPU-baseline leg of the benchmark may import it; the
product path (the HIP library and its Python binding) never does, and the
oracle never imports the product path.  The two share no code: only the
seeded input generators of the top-level ``synth`` module serve both.

Contents (each function cites the passage of arXiv:2001.02835 it follows):

* ``series``  - the truncated star product by its definition (Section 2,
  eq. (5)), series dagger, series exponential, error metrics.
* ``fftconv`` - the five FFT-CONV steps (Section 2, Steps 1-5, eqs. (6)-(9))
  written with explicit DFT sums, used to pin the transform stage.
* ``tek``     - the TEK action (eq. (1)), twist tensor, and the dense
  (non-perturbative) staple and force of eq. (2).
* ``nspt``    - the perturbative staple/force tower (eq. (3)) and one
  Euler-Langevin step built from it.

Everything is complex128 / float64.  Speed is not a goal.
"""
