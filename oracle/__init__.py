"""FP64 CPU oracle for the Intermediate State Method (ISM) hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports it and shares no code with
it; the two meet only through the seeded inputs of the ``problems`` package.

Plain, slow, obviously-correct NumPy code in float64 / complex128:

* ``oracle.finite`` -- finite-dimensional problems (state transfer and gate
  synthesis): exact piecewise-constant exponential step map, forward and
  adjoint sweeps, the exact discrete gradient, the plain gradient method,
  and ISM with one gradient step per slice (Algorithm 1, Eq. (cible),
  Theorems 1 and 2, propagator assembling of Sec. 3).
* ``oracle.density`` -- density-matrix (Liouville-von Neumann) problems of the
  five-spin experiment of Sec. 4.A: conjugation step map, Hilbert-Schmidt inner
  product, exact gradient, plain method and ISM.
* ``oracle.gpe``    -- the 1-D Gross-Pitaevskii problem with Strang splitting
  (Eq. (OS)), its exact discrete adjoint and gradient, and the BEC variant of
  ISM (Sec. 4.C).

Every function with no external pin is listed as "parity unpinned" in its
module header; all functions here are pinned by tests in
``tests/test_oracle_*.py``.
"""
