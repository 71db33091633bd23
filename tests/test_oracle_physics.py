"""Physics pins of the oracle (CPU only): its solutions against continuum
closed forms that do not come from the discretisation.

* 1-D: a single-cell source of strength 2c/dx radiates unit-amplitude waves
  (Sec. 2.3.1 source amplitude; App. A Green's function), also with absorption
  through the complex sound speed (eq. complex_sound_speed).
* 1-D: a speed-and-density step reflects and transmits with the impedance
  coefficients, with the interface half a cell to the right of the last cell
  of the first medium -- this fixes the direction of the staggered density
  average (App. B.1).
* 2-D / 3-D free-space Green's functions of the point source.
* Penetrable cylinder (2-D) and sphere (3-D, App. C) with contrast 1.5 in c
  and rho: error bounded and falling with resolution (staircasing).
"""
import numpy as np
import pytest

from oracle import analytic

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

F0 = 1e6
OMEGA = 2 * np.pi * F0
C0, RHO0 = 1500.0, 1000.0


def _solve_point(orc, shape, dx, c, rho, alpha, src, sp, pml, tol=1e-10):
    m = orc.OracleMedium(shape, dx, OMEGA, c, rho, alpha, pml=pml)
    s = np.zeros(shape, complex)
    s[tuple(src)] = sp
    xi, info = m.solve(m.source_hat(m.pressure_source(s)), tol=tol, max_iter=100000)
    assert info["converged"]
    return xi


@pytest.mark.parametrize("alpha", [0.0, 25.0])
def test_1d_unit_amplitude_point_source(orc, alpha):
    n, pml = 384, 48
    dx = C0 / F0 / 6
    xs = n // 2
    xi = _solve_point(orc, (n,), dx, np.full(n, C0), np.full(n, RHO0), np.full(n, alpha),
                      (xs,), 2 * C0 / dx, pml, tol=1e-12)
    x = (np.arange(n) - xs) * dx
    sel = (np.abs(x) > C0 / F0) & (np.arange(n) >= pml) & (np.arange(n) < n - pml)
    ccx = C0 / np.sqrt(1 - 2j * alpha * C0 / OMEGA)
    k = OMEGA / ccx
    ref = (2 * C0 / dx) * dx / (2 * ccx) * np.exp(-1j * k * np.abs(x))
    err = np.linalg.norm(xi[-1][sel] - ref[sel]) / np.linalg.norm(ref[sel])
    assert err < 2e-3, err
    if alpha == 0:
        assert np.abs(np.abs(xi[-1][sel]) - 1).max() < 5e-3


def test_1d_impedance_step_fixes_staggered_density(orc):
    n, pml = 512, 64
    dx = C0 / F0 / 8
    c2, rho2 = 2100.0, 1700.0
    j = 300                              # last cell of medium 1
    c = np.where(np.arange(n) <= j, C0, c2)
    rho = np.where(np.arange(n) <= j, RHO0, rho2)
    xs = j - 80
    xi = _solve_point(orc, (n,), dx, c, rho, np.zeros(n), (xs,), 2 * C0 / dx, pml, tol=1e-12)
    p = xi[-1]
    x = np.arange(n) * dx
    k1, k2 = OMEGA / C0, OMEGA / c2
    Z1, Z2 = RHO0 * C0, rho2 * c2
    R, T = (Z2 - Z1) / (Z2 + Z1), 2 * Z2 / (Z1 + Z2)
    idx = np.arange(n)
    sel = (idx >= pml) & (idx < n - pml) & (np.abs(idx - xs) * dx > C0 / F0)

    def model(xI):
        ph = np.exp(-1j * k1 * (xI - xs * dx))
        left = np.exp(-1j * k1 * np.abs(x - xs * dx)) + R * ph * np.exp(-1j * k1 * (xI - x))
        right = T * ph * np.exp(-1j * k2 * (x - xI))
        return np.where(x < xI, left, right)

    errs = {}
    for off in (-0.5, 0.5, 1.5):
        ref = model((j + off) * dx)
        keep = sel & (np.abs(x - (j + off) * dx) > 2 * dx)
        errs[off] = np.linalg.norm(p[keep] - ref[keep]) / np.linalg.norm(ref[keep])
    assert errs[0.5] < 2e-2, errs
    assert errs[0.5] < 0.2 * min(errs[-0.5], errs[1.5]), errs


def test_2d_point_source_greens_function(orc):
    n, pml = 128, 24
    dx = C0 / F0 / 6
    shape = (n, n)
    xi = _solve_point(orc, shape, dx, np.full(shape, C0), np.full(shape, RHO0),
                      np.zeros(shape), (n // 2, n // 2), 1.0, pml)
    I0, I1 = np.meshgrid(np.arange(n) - n // 2, np.arange(n) - n // 2, indexing="ij")
    r = np.hypot(I0, I1) * dx
    sel = (r > C0 / F0) & (np.maximum(np.abs(I0), np.abs(I1)) < n // 2 - pml)
    ref = analytic.greens_2d(r[sel], C0, OMEGA, dx * dx)
    err = np.linalg.norm(xi[-1][sel] - ref) / np.linalg.norm(ref)
    assert err < 5e-3, err


def test_3d_point_source_greens_function(orc):
    n, pml = 48, 12
    dx = C0 / F0 / 6
    shape = (n, n, n)
    xi = _solve_point(orc, shape, dx, np.full(shape, C0), np.full(shape, RHO0),
                      np.zeros(shape), (n // 2,) * 3, 1.0, pml, tol=1e-8)
    I = np.indices(shape) - n // 2
    r = np.sqrt((I ** 2).sum(0)) * dx
    sel = (r > C0 / F0) & (np.abs(I).max(0) < n // 2 - pml)
    ref = analytic.greens_3d(r[sel], C0, OMEGA, dx ** 3)
    err = np.linalg.norm(xi[-1][sel] - ref) / np.linalg.norm(ref)
    assert err < 3e-2, err


def _cylinder_error(orc, ppw, n):
    c1, rho1 = 1.5 * C0, 1.5 * RHO0
    lam = C0 / F0
    dx = lam / ppw
    shape = (n, n)
    ctr = np.array([n // 2, n // 2])
    R = 1.5 * lam
    I0, I1 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    inside = np.hypot(I0 - ctr[0], I1 - ctr[1]) * dx < R
    c = np.where(inside, c1, C0)
    rho = np.where(inside, rho1, RHO0)
    src = np.array([ctr[0] - int(round(3 * lam / dx)), ctr[1]])
    pml = 2 * ppw
    xi = _solve_point(orc, shape, dx, c, rho, np.zeros(shape), src, 1.0, pml, tol=1e-9)
    pos = np.stack([I0.ravel(), I1.ravel()], 1) * dx
    d = np.hypot(I0 - src[0], I1 - src[1]) * dx
    sel = (d > lam) & (np.minimum.reduce([I0, I1, n - 1 - I0, n - 1 - I1]) >= pml)
    ref = analytic.cylinder_series(pos[sel.ravel()], ctr * dx, src * dx, R, C0, RHO0, c1, rho1,
                                   OMEGA, mmax=60, sp_dx2=dx * dx)
    return np.linalg.norm(xi[-1][sel] - ref) / np.linalg.norm(ref)


@pytest.mark.slow
def test_2d_penetrable_cylinder_series(orc):
    e8 = _cylinder_error(orc, 8, 128)
    e12 = _cylinder_error(orc, 12, 192)
    assert e8 < 0.12 and e12 < 0.07, (e8, e12)
    assert e12 < 0.8 * e8, (e8, e12)


@pytest.mark.slow
def test_3d_penetrable_sphere_series(orc):
    """Fluid sphere, contrast 1.5 in c and rho (App. C), 64^3 at 8 points per
    wavelength, radius one wavelength, source two wavelengths from the centre;
    central slice outside one wavelength of the source and outside the layer."""
    c1, rho1 = 1.5 * C0, 1.5 * RHO0
    lam = C0 / F0
    ppw, n = 8, 64
    dx = lam / ppw
    shape = (n, n, n)
    ctr = np.array([n // 2] * 3)
    R = lam
    I = np.indices(shape)
    inside = np.sqrt(sum((I[d] - ctr[d]) ** 2 for d in range(3))) * dx < R
    c = np.where(inside, c1, C0)
    rho = np.where(inside, rho1, RHO0)
    src = np.array([ctr[0] - 2 * ppw, ctr[1], ctr[2]])
    xi = _solve_point(orc, shape, dx, c, rho, np.zeros(shape), src, 1.0, 16, tol=1e-7)
    sl = (slice(None), slice(None), ctr[2])
    I0, I1 = I[0][sl], I[1][sl]
    pos = np.stack([I0.ravel(), I1.ravel(), np.full(I0.size, ctr[2])], 1) * dx
    d = np.hypot(I0 - src[0], I1 - src[1]) * dx
    sel = (d > lam) & (np.minimum.reduce([I0, I1, n - 1 - I0, n - 1 - I1]) >= 16)
    ref = analytic.sphere_series(pos[sel.ravel()], ctr * dx, src * dx, R, C0, RHO0, c1, rho1,
                                 OMEGA, mmax=40, sp_dx3=dx ** 3)
    err = np.linalg.norm(xi[-1][sl][sel] - ref) / np.linalg.norm(ref)
    assert err < 6e-2, err
