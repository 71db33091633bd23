"""Pin of the oracle's adjoint-state misfit gradient (CPU only): directional
derivatives from the adjoint solve (Sec. 2.3, adjoint operator) against
central finite differences of the forward solve, for c, rho and alpha.

J(m) = 1/2 sum_shots |M p(m) - d|^2 with p the pressure row of A(m)^{-1} s_hat(m).
"""
import numpy as np
import pytest

from paper_2507_16087_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

OMEGA = 2 * np.pi * 1e6
DX = 1500.0 / 1e6 / 6
SHAPE = (28, 24)
PML = 5


def _setup():
    c, rho, alpha = W.small_random(SHAPE, 31, contrast=0.5)
    alpha = alpha + 2.0          # keep alpha - h v > 0 for every step below
    rng = np.random.default_rng(8)
    N = int(np.prod(SHAPE))
    shots = [np.ravel_multi_index((7, 8), SHAPE), np.ravel_multi_index((8, 15), SHAPE)]
    rec = np.array([np.ravel_multi_index((20, j), SHAPE) for j in (6, 9, 12, 15, 18)])
    d = [rng.standard_normal(rec.size) * 1e-9 + 1j * rng.standard_normal(rec.size) * 1e-9
         for _ in shots]
    return (c, rho, alpha), shots, rec, d, N


def _misfit(orc, media, shots, rec, d, grad=False):
    c, rho, alpha = media
    m = orc.OracleMedium(SHAPE, DX, OMEGA, c, rho, alpha, pml=PML)
    J = 0.0
    G = [np.zeros(SHAPE) for _ in range(3)]
    D = len(SHAPE)
    for s_idx, dk in zip(shots, d):
        sp = np.zeros(SHAPE, complex).ravel()
        sp[s_idx] = 1.0
        s = m.pressure_source(sp.reshape(SHAPE))
        xi, info = m.solve(m.source_hat(s), tol=1e-14, max_iter=100000)
        assert info["converged"]
        p = xi[D].ravel()
        r = p[rec] - dk
        J += 0.5 * np.vdot(r, r).real
        if grad:
            g = np.zeros((D + 1, int(np.prod(SHAPE))), complex)
            g[D, rec] = r
            lam, info = m.solve(g.reshape((D + 1,) + SHAPE), tol=1e-14, max_iter=100000,
                                adjoint=True)
            assert info["converged"]
            for acc, part in zip(G, m.gradient(s, xi, lam)):
                acc += part
    return J, G


@pytest.mark.parametrize("which", [0, 1, 2])
def test_gradient_matches_central_differences(orc, which):
    media, shots, rec, d, N = _setup()
    J0, G = _misfit(orc, media, shots, rec, d, grad=True)
    scale = [media[0], media[1], np.full(SHAPE, 10.0)][which]
    for seed in (5000, 5001):
        v = W.smooth_direction(SHAPE, seed, sigma=2.0) * scale
        ana = float((G[which] * v).sum())
        fd = []
        for h in (1e-3, 1e-4):
            mp = [a.copy() for a in media]
            mm = [a.copy() for a in media]
            mp[which] = mp[which] + h * v
            mm[which] = mm[which] - h * v
            Jp, _ = _misfit(orc, mp, shots, rec, d)
            Jm, _ = _misfit(orc, mm, shots, rec, d)
            fd.append((Jp - Jm) / (2 * h))
        # Taylor: central differences converge to the analytic derivative
        assert abs(fd[1] - ana) <= 1e-5 * abs(ana) + 1e-30, (which, fd, ana)
        assert abs(fd[1] - ana) <= abs(fd[0] - ana) + 1e-7 * abs(ana)   # solve-noise floor
