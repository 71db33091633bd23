"""GPU parity on every axis length 2^a 3^b the plan table adds beyond the
powers of two and 6 * 2^k: FP64 iterates against the oracle's (eq. BornAlt,
Algorithm 1) with each new length in each pass role -- axis 0 (the pass that
carries the propagator of App. B.1), the strided axis 1, and the contiguous
last axis that carries the update -- forward and adjoint, and the refined
FP32 solve against the oracle's converged FP64 solution.  The plans of the
new lengths use radix-3 and radix-9 stages (cbs_plans.h)."""
import numpy as np
import pytest

from paper_2507_16087_amd import workloads as W
from parity_util import close

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

OMEGA = 2 * np.pi * 1e6
DX = 1500.0 / 1e6 / 6


@pytest.fixture(scope="module")
def cbs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_16087_amd import solver
    return solver


def _rot(t):
    return [t, t[1:] + t[:1], t[2:] + t[:2]]


# each triple in all three roles
SHAPES3 = (_rot((36, 72, 144)) + _rot((9, 27, 81)) + _rot((18, 54, 108)) + _rot((162, 216, 8)) +
           _rot((243, 12, 16)) + _rot((288, 6, 16)) + _rot((324, 4, 12)) + _rot((384, 6, 8)) +
           _rot((432, 4, 9)) + _rot((486, 4, 6)))
SHAPES2 = [(486, 18), (18, 486), (27, 384), (384, 27), (144, 81), (81, 144)]
NEW = {9, 18, 27, 36, 54, 72, 81, 108, 144, 162, 216, 243, 288, 324, 384, 432, 486}


def test_shape_lists_cover_every_new_length_in_every_role():
    for role in (0, 1, 2):
        assert {s[role] for s in SHAPES3} >= NEW, role


def _source(shape, seed):
    rng = np.random.default_rng(seed)
    F = len(shape) + 1
    s = np.zeros((F,) + shape, complex)
    flat = s.reshape(F, -1)
    idx = rng.choice(flat.shape[1], 3, replace=False)
    flat[-1, idx] = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    flat[0, idx[0]] = 0.2 - 0.1j
    return s


def _pair(orc, cbs, shape, seed):
    c, rho, alpha = W.small_random(shape, seed)
    pml = max(1, min(3, min(shape) // 4))
    om = orc.OracleMedium(shape, DX, OMEGA, c, rho, alpha, pml=pml)
    gm = cbs.Medium(shape, DX, OMEGA, c, rho, alpha, pml=pml)
    return om, gm


@pytest.mark.parametrize("shape", SHAPES3 + SHAPES2, ids=lambda s: "x".join(map(str, s)))
def test_fp64_iterates_new_lengths(orc, cbs, report, shape):
    report(f"sizes: fp64 iterates {shape}")
    om, gm = _pair(orc, cbs, shape, 21)
    s = _source(shape, 5)
    for adjoint in (False, True):
        xi, _ = om.solve(om.source_hat(s), tol=0.0, max_iter=12, adjoint=adjoint)
        p, u, info = cbs.solve(gm, s[-1], s[:-1], tol=0.0, max_iter=12, adjoint=adjoint)
        assert info["iterations"] == 12
        close(p, xi[-1], 1e-10, f"p adjoint={adjoint}")
        close(u, xi[:-1], 1e-10, f"u adjoint={adjoint}")


@pytest.mark.parametrize("shape", [(18, 36, 72), (81, 9, 27), (54, 108, 18), (384, 6, 8), (18, 486)],
                         ids=lambda s: "x".join(map(str, s)))
def test_refined_new_lengths(orc, cbs, report, shape):
    report(f"sizes: refined {shape}")
    om, gm = _pair(orc, cbs, shape, 22)
    s = _source(shape, 6)
    xs, info = om.solve(om.source_hat(s), tol=1e-12, max_iter=100000)
    assert info["converged"]
    p, u, ginfo = cbs.solve(gm, s[-1], s[:-1], tol=1e-7, prec="fp32_refined", inner_tol=1e-4)
    assert ginfo["converged"]
    close(p, xs[-1], 1e-5, "p")
    close(u, xs[:-1], 1e-5, "u")
