"""Misfit gradients through torch.autograd (adjoint solve + gradient kernel).

Setup shaped like the inversion workload, scaled down: shots on one face,
receivers on the opposite face, data from a medium with a smooth bump
(c up 3 %, rho down 3 %).  J = sum_shots 1/2 |M p - d|^2.
Checks: directional derivatives against central finite differences of FP64
solves, and the gradient against the FP64 oracle's adjoint-state gradient
(FP64 GPU to 1e-8, refined FP32 to 1e-4).
"""
import numpy as np
import pytest

from paper_2507_16087_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

N = 24
PML = 5


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    inv = W.inversion(N, shots_yz=(1, 2), receivers_yz=(4, 3), pml=PML)
    pr = inv.model
    from paper_2507_16087_amd import solver
    from paper_2507_16087_amd.autograd import SolveSpec
    # data from the bumped medium (FP64 GPU solves)
    mt = solver.Medium(pr.shape, pr.dx, pr.omega, inv.true_c, inv.true_rho, pr.alpha, pml=PML)
    data = []
    for sh in inv.shots:
        sp = np.zeros(pr.ncell, complex)
        sp[sh] = 1.0
        p, _, info = solver.solve(mt, sp, tol=1e-12, prec="fp64", want_u=False)
        assert info["converged"]
        data.append(p.ravel()[inv.receivers])
    spec64 = SolveSpec(pr.shape, pr.dx, pr.omega, PML, "fp64", 1e-12)
    spec32 = SolveSpec(pr.shape, pr.dx, pr.omega, PML, "fp32_refined", 1e-9)
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
    c = torch.tensor(pr.c, device="cuda", requires_grad=True)
    rho = torch.tensor(pr.rho, device="cuda", requires_grad=True)
    alpha = torch.tensor(pr.alpha, device="cuda", requires_grad=True)
    J = _misfit(inv, data, spec, c, rho, alpha)
    J.backward()
    return J.detach().item(), [t.grad.cpu().numpy() for t in (c, rho, alpha)]


def _oracle_grads(orc, inv, data):
    pr = inv.model
    om = orc.OracleMedium(pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, pml=PML)
    G = [np.zeros(pr.shape) for _ in range(3)]
    for sh, d in zip(inv.shots, data):
        sp = np.zeros(pr.ncell, complex)
        sp[sh] = 1.0
        s = om.pressure_source(sp.reshape(pr.shape))
        xi, info = om.solve(om.source_hat(s), tol=1e-13, max_iter=200000)
        assert info["converged"]
        g = np.zeros((4, pr.ncell), complex)
        g[3, inv.receivers] = xi[3].ravel()[inv.receivers] - d
        lam, info = om.solve(g.reshape((4,) + pr.shape), tol=1e-13, max_iter=200000, adjoint=True)
        assert info["converged"]
        for acc, part in zip(G, om.gradient(s, xi, lam)):
            acc += part
    return G


def test_gradient_matches_oracle(orc, setup):
    inv, data, spec64, spec32 = setup
    go = _oracle_grads(orc, inv, data)
    _, g64 = _grads(inv, data, spec64)
    _, g32 = _grads(inv, data, spec32)
    for a, b, c in zip(g64, g32, go):
        b_ = c.ravel()
        assert np.linalg.norm(a.ravel() - b_) <= 1e-8 * np.linalg.norm(b_)
        assert np.linalg.norm(b.ravel() - b_) <= 1e-4 * np.linalg.norm(b_)


@pytest.mark.parametrize("which", [0, 1, 2])
def test_directional_derivative_central_differences(setup, which):
    """Relative perturbations m (1 + h v) along smooth random directions v
    (so alpha stays non-negative)."""
    import torch
    inv, data, spec64, _ = setup
    pr = inv.model
    _, g = _grads(inv, data, spec64)
    base = [pr.c, pr.rho, pr.alpha]
    for seed in (5000, 5001):
        v = W.smooth_direction(pr.shape, seed) * base[which]
        ana = float((g[which] * v).sum())
        h = 2.5e-5      # O(h^2) truncation well below the 1e-6 gate; solves at 1e-12
        vals = []
        for sgn in (1, -1):
            m = [torch.tensor(b, device="cuda") for b in base]
            m[which] = m[which] + sgn * h * torch.tensor(v, device="cuda")
            vals.append(float(_misfit(inv, data, spec64, *m)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - ana) <= 1e-6 * abs(ana) + 1e-12 * abs(vals[0]), (which, fd, ana)
