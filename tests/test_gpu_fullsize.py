"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (autotuned plans of the same shapes).

* 128^3 random medium (1 MHz, lambda/6): FP64 iterates after 3 iterations
  against the oracle's, every cell, <= 1e-10.
* 256^3 skull-like shell (the benchmark workload): FP64 iterates after 2
  iterations against the oracle's on sampled cells and pencils, <= 1e-10;
  the refined-FP32 solution's scaled residual evaluated by the oracle's own
  operator equals the GPU-reported one; the refined solution at a scaled
  residual of 1e-7 is within 1e-5 of the FP64 GPU solution at 1e-8.  The
  FP64 GPU path stands in for a converged oracle here: the oracle's own
  256^3 solve would need some 40 000 iterations at seconds each on the host,
  so its contact at this size is iterate parity (here and, after 2600
  iterations, in test_gpu_oracle_refs.py) and the residual check.
"""
import numpy as np
import pytest

from paper_2507_16087_amd import workloads as W
from parity_util import maxrel, rel

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def cbs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_16087_amd import solver
    return solver


def _rel(a, b):
    """Error measure of the parity checks: the larger of the relative L2 error
    and the largest element-wise error over the largest reference modulus."""
    return max(rel(a, b), maxrel(a, b))


def test_random128_fp64_iterates(cbs, orc):
    pr = W.random3d(128)
    gm = cbs.Medium(pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, pml=pr.pml_cells)
    om = orc.OracleMedium(pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, pml=pr.pml_cells)
    sp = pr.dense_source()
    xi, _ = om.solve(om.source_hat(om.pressure_source(sp)), tol=0.0, max_iter=3)
    p, u, info = cbs.solve(gm, sp, tol=0.0, max_iter=3)
    assert info["iterations"] == 3
    assert _rel(p, xi[-1]) <= 1e-10 and _rel(u, xi[:-1]) <= 1e-10


@pytest.fixture(scope="module")
def shell(cbs, orc, report):
    report("shell3d 256^3: building workload, GPU medium and oracle medium")
    pr = W.shell3d(256)
    gm = cbs.Medium(pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, pml=pr.pml_cells)
    om = orc.OracleMedium(pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, pml=pr.pml_cells)
    return pr, gm, om


@pytest.mark.timeout(400)
def test_shell256_fp64_iterates_sampled(cbs, shell, report):
    pr, gm, om = shell
    report("shell3d 256^3: oracle 2 FP64 iterations")
    sp = pr.dense_source()
    so, sg = om.scalars(), gm.scalars()
    for k in ("a1", "a2", "lam1", "lam2"):
        assert abs(so[k] - sg[k]) <= 1e-12 * abs(so[k])
    shat = om.source_hat(om.pressure_source(sp))
    xi, _ = om.solve(shat, tol=0.0, max_iter=2)
    del shat
    p, u, info = cbs.solve(gm, sp, tol=0.0, max_iter=2)
    rng = np.random.default_rng(3)
    cells = rng.integers(0, pr.ncell, 20000)
    ref = xi[-1].ravel()[cells]
    assert _rel(p.ravel()[cells], ref) <= 1e-10
    for e in range(3):
        refu = xi[e].ravel()[cells]
        assert _rel(u[e].ravel()[cells], refu) <= 1e-10
    # whole pencils along each axis through the focus region
    for sl in [(slice(None), 128, 128), (150, slice(None), 128), (150, 128, slice(None))]:
        assert _rel(p[sl], xi[-1][sl]) <= 1e-10


@pytest.mark.timeout(900)
def test_shell256_refined_accuracy(cbs, shell, report):
    """The skull-like case is ill-conditioned: the error is ~40x the scaled
    residual, for FP64 and refined FP32 alike.  A 1e-5 error therefore needs a
    residual of ~1e-7; the refined path is solved to 1e-7 and compared with
    the FP64 solution at 1e-8 (error <= ~4e-7, 25x below the gate; FP64
    itself is iterate-pinned to the oracle)."""
    import torch
    from paper_2507_16087_amd import _lib
    pr, gm, om = shell
    sp = torch.from_numpy(pr.dense_source().ravel()).cuda()
    report("shell3d 256^3: refined FP32 solve to 1e-7")
    p32, u32, i32 = cbs.solve(gm, sp, tol=1e-7, prec="fp32_refined", max_iter=400000,
                              check_every=50)
    report(f"  {i32['iterations']} iterations; oracle residual of the result")
    assert i32["converged"] and i32["rel_residual"] <= 1e-7
    # the oracle's operator agrees with the GPU-reported residual
    xi = np.concatenate([u32.cpu().numpy(), p32.cpu().numpy()[None]])
    shat = om.source_hat(om.pressure_source(pr.dense_source()))
    r_orc = om.rel_residual(shat, xi)
    del shat, xi, u32
    assert abs(r_orc - i32["rel_residual"]) <= 1e-3 * i32["rel_residual"] + 1e-12
    report("shell3d 256^3: FP64 reference solve to 1e-8")
    ref, _, iref = cbs.solve(gm, sp, tol=1e-8, prec="fp64", max_iter=400000, check_every=200,
                             stop_rule=_lib.CBS_STOP_RESIDUAL, want_u=False)
    report(f"  {iref['iterations']} iterations")
    assert iref["converged"]
    e32 = (torch.linalg.norm(p32 - ref) / torch.linalg.norm(ref)).item()
    m32 = (torch.abs(p32 - ref).max() / torch.abs(ref).max()).item()
    print(f"256^3 shell at residual 1e-7: refined FP32 pressure error {e32:.2e} (max-abs {m32:.2e}, "
          f"{i32['iterations']} it) against FP64 at 1e-8 ({iref['iterations']} it)")
    assert e32 <= 1e-5 and m32 <= 1e-5, (e32, m32)
