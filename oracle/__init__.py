"""TEST INFRASTRUCTURE ONLY: the FP64 CPU oracle for the iterative Born solver.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product library never links or calls it.

* ``cbs_oracle.c``   -- plain C implementation of Algorithm 1 (own FFT,
  explicit staggered propagator matrix, adjoint, residual, gradient).
* ``core.py``        -- ctypes wrapper over the compiled oracle.
* ``analytic.py``    -- closed forms used to pin the oracle: homogeneous
  periodic solution, free-space Green's functions, penetrable-sphere series.
"""
