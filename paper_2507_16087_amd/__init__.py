"""MI355X (gfx950) iterative Born solver for the first-order acoustic
Helmholtz system with heterogeneous sound speed, density and absorption
(arXiv 2507.16087).

The solver lives in the HIP library ``libcbs.so`` behind the C ABI of
``include/cbs.h``; :mod:`.solver` is its Python binding, :mod:`.autograd`
wraps forward and adjoint solves as a ``torch.autograd.Function``,
:mod:`.serve` is the continuous-batching request loop and :mod:`.workloads`
draws the seeded synthetic inputs.
"""
