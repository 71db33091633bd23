"""Full-size parity against stored FP64 oracle references.

tests/golden/oracle_<workload>.npz is written by tests/golden/make_converged.py
from the oracle alone (Algorithm 1 from x = 0, FP64, on the workload's medium
and source): 20 000 seeded sample cells of every field, three whole pencils
through the source or focus, the norm and largest modulus of every field,
the iteration count and the stored state's scaled true residual.

* 128^3 random medium (1 MHz, lambda/6, point source at the centre): the
  oracle converged to a relative update of 1e-12 (scaled residual ~5e-12).
  - FP64 GPU iterate at the oracle's iteration count: <= 1e-10;
  - FP64 GPU solve stopped on its own scaled residual (1e-11): <= 1e-10;
  - refined FP32 at a scaled residual of 1e-7: <= 1e-5 (the accuracy gate of
    the refined path), and its error at the benchmark's residual of 1e-5 is
    printed beside it.
* 256^3 skull-like shell: the oracle cannot converge this case on the host in
  useful time (tens of thousands of iterations at seconds each), so the
  stored reference is a fixed iterate; the FP64 GPU iterate of the same count
  must equal it to 1e-10.  (The shell's refined-FP32 accuracy is checked
  against the FP64 GPU path in test_gpu_fullsize.py.)

Every comparison bounds the relative L2 error and the largest element-wise
error against the largest reference modulus, on the samples and the pencils,
and compares each field's whole-grid norm.
"""
import os

import numpy as np
import pytest

from paper_2507_16087_amd import workloads as W
from parity_util import close

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def cbs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_16087_amd import solver
    return solver


def _ref(name):
    path = os.path.join(GOLDEN, f"oracle_{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"no stored oracle reference for {name}")
    return dict(np.load(path, allow_pickle=False))


def _compare(p, u, ref, tol, what):
    """p: (n0, n1, n2) pressure, u: (3, n0, n1, n2) velocities (numpy)."""
    full = np.concatenate([np.asarray(u).reshape(3, -1), np.asarray(p).reshape(1, -1)])
    idx = ref["idx"]
    for f in range(4):
        close(full[f, idx], ref["samples"][f], tol, f"{what} field {f} samples")
    shape = np.asarray(p).shape
    xi = full.reshape((4,) + shape)
    i0, i1, i2 = (int(v) for v in ref["focus"])
    for name, sl in (("pencil0", (slice(None), i1, i2)), ("pencil1", (i0, slice(None), i2)),
                     ("pencil2", (i0, i1, slice(None)))):
        got = xi[(slice(None),) + sl]
        close(got, ref[name], tol, f"{what} {name}")
    nrm = np.sqrt(np.array([np.vdot(full[f], full[f]).real for f in range(4)]))
    want = np.sqrt(ref["norm2"])
    assert np.all(np.abs(nrm - want) <= tol * want), (what, nrm, want)


@pytest.fixture(scope="module")
def random128(cbs, report):
    ref = _ref("random128")
    assert bool(ref["converged"]) and float(ref["rel_residual"]) <= 1e-11
    report("random128: medium")
    pr = W.random3d(128)
    gm = cbs.Medium(pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, pml=pr.pml_cells)
    sp = pr.dense_source()
    # the planner's scalars are the oracle's
    a1, a2, lam1, lam2 = ref["scalars"]
    s = gm.scalars()
    for k, v in (("a1", a1), ("a2", a2), ("lam1", lam1.real), ("lam2", lam2.real)):
        assert abs(s[k] - v) <= 1e-12 * abs(v), k
    return pr, gm, sp, ref


def test_random128_fp64_iterate_at_oracle_count(cbs, random128, report):
    pr, gm, sp, ref = random128
    k = int(ref["iterations"])
    report(f"random128: FP64 {k} iterations")
    p, u, info = cbs.solve(gm, sp, tol=0.0, max_iter=k)
    assert info["iterations"] == k
    _compare(p, u, ref, 1e-10, f"fp64 iterate {k}")


def test_random128_fp64_converged_on_residual(cbs, random128, report):
    from paper_2507_16087_amd import _lib
    pr, gm, sp, ref = random128
    report("random128: FP64 to a scaled residual of 1e-11")
    p, u, info = cbs.solve(gm, sp, tol=1e-11, max_iter=100000, check_every=16,
                           stop_rule=_lib.CBS_STOP_RESIDUAL)
    assert info["converged"] and info["rel_residual"] <= 1e-11
    _compare(p, u, ref, 1e-10, "fp64 converged")


def test_random128_refined_accuracy(cbs, random128, report):
    pr, gm, sp, ref = random128
    report("random128: refined FP32 to 1e-7 and 1e-5")
    p, u, info = cbs.solve(gm, sp, tol=1e-7, prec="fp32_refined")
    assert info["converged"] and info["rel_residual"] <= 1e-7
    _compare(p, u, ref, 1e-5, "refined 1e-7")
    p5, u5, i5 = cbs.solve(gm, sp, tol=1e-5, prec="fp32_refined")
    full = np.concatenate([u5.reshape(3, -1), p5.reshape(1, -1)])[:, ref["idx"]]
    err = np.linalg.norm(full[3] - ref["samples"][3]) / np.linalg.norm(ref["samples"][3])
    print(f"random128 refined: residual {i5['rel_residual']:.2e} -> pressure error {err:.2e} "
          f"(samples); residual {info['rel_residual']:.2e} -> within 1e-5")


@pytest.mark.timeout(600)
def test_shell256_fp64_iterate_at_oracle_count(cbs, report):
    ref = _ref("shell256")
    k = int(ref["iterations"])
    report(f"shell256: medium, FP64 {k} iterations")
    pr = W.shell3d(256)
    gm = cbs.Medium(pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, pml=pr.pml_cells)
    p, u, info = cbs.solve(gm, pr.dense_source(), tol=0.0, max_iter=k)
    assert info["iterations"] == k
    _compare(p, u, ref, 1e-10, f"fp64 iterate {k}")
