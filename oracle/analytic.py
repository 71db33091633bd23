"""TEST INFRASTRUCTURE ONLY: closed-form references that pin the oracle.

Time convention: the first-order system of the paper carries +i omega with a
non-negative damping rate, so waves decay only for exp(+i omega t); outgoing
waves are exp(-i k r) and the radiating special functions are the Hankel
functions of the second kind.

* :func:`homogeneous_periodic` -- exact solution of the discrete staggered
  system in a uniform medium on the periodic grid (Schur complement per
  wavevector, derived from the Fourier form of the operator, App. B.1).
* :func:`greens_1d/2d/3d` -- free-space pressure of a single-cell pressure
  source of strength s_p (App. A: equivalent source -i omega s_p / c^2).
* :func:`sphere_series` -- penetrable fluid sphere in a point-source field
  (App. C, Anderson's expansion), with the incident coefficient taken at the
  source distance.
* :func:`cylinder_series` -- the 2-D analogue (penetrable circular cylinder in
  a line-source field), used for a fast heterogeneous-density pin.
"""
from __future__ import annotations

import numpy as np
from scipy import special as sp


def wavenumbers(shape, dx):
    return [2 * np.pi * np.fft.fftfreq(n, d=dx) for n in shape]


def homogeneous_periodic(shape, dx, omega, c, rho, alpha, s_u, s_p, gamma=0.0):
    """Solve the periodic staggered system for uniform c, rho, alpha, gamma.

    Rows:  D_u u_eta + F^-1[i k_eta S_eta p^]           = rho s_u_eta
           D_p p     + sum F^-1[i k_eta conj(S_eta) u^] = q s_p
    with D_u = rho (i w + gamma), D_p = (i w + gamma) q, q = (1 - 2i a c/w)/(rho c^2),
    S_eta = exp(i k_eta dx / 2).  Eliminating u per wavevector gives
    p^ = (shat_p^ - sum_eta i k_eta conj(S_eta) shat_u^/D_u) / (D_p + |k|^2 / D_u).
    """
    ndim = len(shape)
    q = (1 - 2j * alpha * c / omega) / (rho * c * c)
    Du = rho * (1j * omega + gamma)
    Dp = (1j * omega + gamma) * q
    ks = np.meshgrid(*wavenumbers(shape, dx), indexing="ij")
    axes = tuple(range(ndim))
    su_h = [np.fft.fftn(rho * s_u[e], axes=axes) for e in range(ndim)]
    sp_h = np.fft.fftn(q * s_p, axes=axes)
    S = [np.exp(1j * k * dx / 2) for k in ks]
    k2 = sum(k * k for k in ks)
    num = sp_h - sum(1j * ks[e] * np.conj(S[e]) * su_h[e] for e in range(ndim)) / Du
    ph = num / (Dp + k2 / Du)
    uh = [(su_h[e] - 1j * ks[e] * S[e] * ph) / Du for e in range(ndim)]
    out = np.stack([np.fft.ifftn(u, axes=axes) for u in uh] + [np.fft.ifftn(ph, axes=axes)])
    return out


def greens_1d(x, c, omega, sp_dx):
    """p(x) for s_p*dx concentrated at x=0: (s_p dx / 2c) exp(-i k |x|)."""
    k = omega / c
    return sp_dx / (2 * c) * np.exp(-1j * k * np.abs(x))


def greens_2d(r, c, omega, sp_dx2):
    """p(r) = (omega s_p dx^2 / 4 c^2) H0^(2)(k r)."""
    k = omega / c
    return omega * sp_dx2 / (4 * c * c) * sp.hankel2(0, k * r)


def greens_3d(r, c, omega, sp_dx3):
    """p(r) = (i omega s_p dx^3 / c^2) exp(-i k r) / (4 pi r)."""
    k = omega / c
    return 1j * omega * sp_dx3 / (c * c) * np.exp(-1j * k * r) / (4 * np.pi * r)


def _h2(m, x, derivative=False):
    return sp.spherical_jn(m, x, derivative) - 1j * sp.spherical_yn(m, x, derivative)


def sphere_series(points, centre, src, radius, c0, rho0, c1, rho1, omega, mmax=150,
                  sp_dx3=1.0):
    """Pressure at ``points`` (M x 3) for a unit-strength single-cell pressure
    source (s_p dx^3 = sp_dx3) at ``src`` near a fluid sphere.

    Incident field K h0(k0 |r - r_s|), K = k0^2 s_p dx^3 / (4 pi c0), expanded
    about the centre as sum (2m+1) h_m(k0 r_s) j_m(k0 r) P_m(cos theta) for
    r < r_s.  Scattered sum A_m P_m h_m(k0 r) outside; sum B_m P_m j_m(k1 r)
    inside.  A_m, B_m follow from continuity of pressure and of normal velocity
    (1/Z) dp/d(kr), Z = rho c, at r = R."""
    points = np.asarray(points, float)
    centre = np.asarray(centre, float)
    src = np.asarray(src, float)
    k0 = omega / c0
    k1 = omega / c1
    Z0, Z1 = rho0 * c0, rho1 * c1
    rs_vec = src - centre
    rs = np.linalg.norm(rs_vec)
    K = k0 * k0 * sp_dx3 / (4 * np.pi * c0)
    rel = points - centre
    r = np.linalg.norm(rel, axis=1)
    cos_t = np.where(r > 0, rel @ rs_vec / np.maximum(r, 1e-300) / rs, 1.0)
    out = np.zeros(len(points), np.complex128)
    ext = r > radius
    d = np.linalg.norm(points - src, axis=1)
    out[ext] = _h2(0, k0 * d[ext])
    R = radius
    for m in range(mmax + 1):
        Lm = _h2(m, k0 * rs)
        inc_p = (2 * m + 1) * Lm * sp.spherical_jn(m, k0 * R)
        inc_v = (2 * m + 1) * Lm * sp.spherical_jn(m, k0 * R, True) / Z0
        M = np.array([[_h2(m, k0 * R), -sp.spherical_jn(m, k1 * R)],
                      [_h2(m, k0 * R, True) / Z0, -sp.spherical_jn(m, k1 * R, True) / Z1]])
        A, B = np.linalg.solve(M, -np.array([inc_p, inc_v]))
        Pm = sp.eval_legendre(m, cos_t)
        out[ext] += A * Pm[ext] * _h2(m, k0 * r[ext])
        out[~ext] += B * Pm[~ext] * sp.spherical_jn(m, k1 * r[~ext])
    return K * out


def cylinder_series(points, centre, src, radius, c0, rho0, c1, rho1, omega, mmax=80,
                    sp_dx2=1.0):
    """2-D analogue of :func:`sphere_series` for a penetrable circular
    cylinder and a single-cell pressure source: incident field
    (omega s_p dx^2 / 4 c0^2) H0^(2)(k0 |r - r_s|), expanded with Graf's
    addition theorem as sum_m H_m(k0 r_s) J_m(k0 r) exp(i m (phi - phi_s))."""
    points = np.asarray(points, float)
    centre = np.asarray(centre, float)
    src = np.asarray(src, float)
    k0, k1 = omega / c0, omega / c1
    Z0, Z1 = rho0 * c0, rho1 * c1
    K = omega * sp_dx2 / (4 * c0 * c0)
    rel = points - centre
    r = np.hypot(rel[:, 0], rel[:, 1])
    phi = np.arctan2(rel[:, 1], rel[:, 0])
    sv = src - centre
    rs = np.hypot(*sv)
    phis = np.arctan2(sv[1], sv[0])
    ext = r > radius
    d = np.linalg.norm(points - src, axis=1)
    out = np.zeros(len(points), np.complex128)
    out[ext] = sp.hankel2(0, k0 * d[ext])
    R = radius
    for m in range(-mmax, mmax + 1):
        Lm = sp.hankel2(m, k0 * rs)
        inc_p = Lm * sp.jv(m, k0 * R)
        inc_v = Lm * sp.jvp(m, k0 * R) / Z0
        M = np.array([[sp.hankel2(m, k0 * R), -sp.jv(m, k1 * R)],
                      [sp.h2vp(m, k0 * R) / Z0, -sp.jvp(m, k1 * R) / Z1]])
        A, B = np.linalg.solve(M, -np.array([inc_p, inc_v]))
        e = np.exp(1j * m * (phi - phis))
        out[ext] += A * e[ext] * sp.hankel2(m, k0 * r[ext])
        out[~ext] += B * e[~ext] * sp.jv(m, k1 * r[~ext])
    return K * out
