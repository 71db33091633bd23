"""The differentiable-solve workload at its full size, through
torch.autograd: 128^3 random medium (1 MHz, lambda/6), 8 single-cell shots
on the x = 20 face, 128 receivers on the x = 107 face, data from the medium
with a smooth bump (c up 3 %, rho down 3 %), J = sum_shots 1/2 |M p - d|^2.

* The refined-FP32 gradient against the FP64 gradient, each of dJ/dc,
  dJ/drho, dJ/dalpha: <= 1e-4 relative L2.  At this size the FP64 GPU path
  stands for the oracle: its iterates at 128^3 equal the oracle's to 1e-10
  and its autograd gradient equals the oracle's adjoint-state gradient to
  1e-8 on the scaled-down inversion (both tested elsewhere); the oracle's own
  128^3 solves would take hours per shot.
* Directional derivatives of J (FP64) against central differences of FP64
  solves along seeded smooth directions, taken in turn for c, rho and alpha:
  <= 1e-6.  The workload's sixteen seeded directions (5000 + k), taken for
  c, rho and alpha in turn (about 8 s each); CBS_FD_DIRECTIONS=n runs the
  first n.
"""
import os
import time

import numpy as np
import pytest

from paper_2507_16087_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

N = 128
DIRECTIONS = int(os.environ.get("CBS_FD_DIRECTIONS", "16"))


@pytest.fixture(scope="module")
def setup(report):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_16087_amd import solver
    from paper_2507_16087_amd.autograd import SolveSpec
    inv = W.inversion(N)
    pr = inv.model
    report(f"inversion {N}^3: {len(inv.shots)} shots, {inv.receivers.size} receivers; data solves")
    mt = solver.Medium(pr.shape, pr.dx, pr.omega, inv.true_c, inv.true_rho, pr.alpha,
                       pml=pr.pml_cells)
    data = []
    for sh in inv.shots:
        sp = np.zeros(pr.ncell, complex)
        sp[sh] = 1.0
        p, _, info = solver.solve(mt, sp, tol=1e-12, prec="fp64", want_u=False)
        assert info["converged"]
        data.append(p.ravel()[inv.receivers])
    del mt
    spec64 = SolveSpec(pr.shape, pr.dx, pr.omega, pr.pml_cells, "fp64", 1e-12)
    spec32 = SolveSpec(pr.shape, pr.dx, pr.omega, pr.pml_cells, "fp32_refined", 1e-8)
    return inv, data, spec64, spec32


def _misfit(inv, data, spec, c, rho, alpha):
    import torch
    from paper_2507_16087_amd.autograd import pressure
    pr = inv.model
    rec = torch.as_tensor(inv.receivers, device="cuda")
    J = 0.0
    for sh, d in zip(inv.shots, data):
        sp = torch.zeros(pr.ncell, dtype=torch.complex128, device="cuda")
        sp[int(sh[0])] = 1.0
        p = pressure(c, rho, alpha, sp, spec).reshape(-1)
        r = p[rec] - torch.as_tensor(d, device="cuda")
        J = J + 0.5 * (r.real ** 2 + r.imag ** 2).sum()
    return J


def _grads(inv, data, spec):
    import torch
    pr = inv.model
    m = [torch.tensor(a, device="cuda", requires_grad=True) for a in (pr.c, pr.rho, pr.alpha)]
    J = _misfit(inv, data, spec, *m)
    J.backward()
    return J.detach().item(), [t.grad.cpu().numpy() for t in m]


@pytest.fixture(scope="module")
def grads64(setup, report):
    inv, data, spec64, _ = setup
    t0 = time.perf_counter()
    J, g = _grads(inv, data, spec64)
    report(f"  FP64 J and gradient: {time.perf_counter() - t0:.1f} s (J = {J:.6e})")
    return J, g


@pytest.mark.timeout(900)
def test_refined_gradient_matches_fp64(setup, grads64, report):
    inv, data, _, spec32 = setup
    J64, g64 = grads64
    t0 = time.perf_counter()
    J32, g32 = _grads(inv, data, spec32)
    report(f"  refined FP32 J and gradient: {time.perf_counter() - t0:.1f} s")
    errs = [np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()) for a, b in zip(g32, g64)]
    print(f"128^3 inversion: refined vs FP64 gradient rel. L2 (c, rho, alpha) = "
          f"{errs[0]:.2e}, {errs[1]:.2e}, {errs[2]:.2e}; J rel. diff {abs(J32 - J64) / J64:.2e}")
    assert max(errs) <= 1e-4, errs


@pytest.mark.timeout(900)
@pytest.mark.parametrize("k", range(DIRECTIONS))
def test_directional_derivative_full_size(setup, grads64, report, k):
    """Relative perturbation m (1 + h v), v a smooth field with max |v| = 1.
    Error model of the central difference: O(h^2) truncation plus the misfit's
    own error (relative ~1e-12 from solves at a 1e-12 residual) divided by 2h.
    c and rho move the phase strongly, so h = 1e-5 (truncation ~1e-7
    relative); alpha changes J by only ~1e-3 J per unit, so h = 1e-3 keeps its
    difference above the misfit's round-off."""
    import torch
    inv, data, spec64, _ = setup
    pr = inv.model
    _, g = grads64
    which = k % 3
    base = [pr.c, pr.rho, pr.alpha]
    v = W.smooth_direction(pr.shape, 5000 + k) * base[which]
    ana = float((g[which] * v).sum())
    h = (1e-5, 1e-5, 1e-3)[which]
    vals = []
    for sgn in (1, -1):
        m = [torch.tensor(b, device="cuda") for b in base]
        m[which] = m[which] + sgn * h * torch.tensor(v, device="cuda")
        vals.append(float(_misfit(inv, data, spec64, *m)))
    fd = (vals[0] - vals[1]) / (2 * h)
    report(f"  direction {k} ({('c', 'rho', 'alpha')[which]}): analytic {ana:.9e}, "
           f"central difference {fd:.9e}, rel. diff {abs(fd - ana) / abs(ana):.1e}")
    assert abs(fd - ana) <= 1e-6 * abs(ana) + 1e-12 * abs(vals[0]) / h, (which, fd, ana)
