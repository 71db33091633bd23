"""TEST INFRASTRUCTURE ONLY: ctypes wrapper over the compiled FP64 oracle.

Complex fields are numpy complex128 arrays of shape (ndim + 1, *grid) in the
order (u_0, .., u_{ndim-1}, p), where u_eta sits half a cell along axis eta.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liborc.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        L.orc_fft.argtypes = [C.c_int, i64p, dp, C.c_int]
        L.orc_mec.argtypes = [dp, C.c_int64, dp]
        L.orc_create.argtypes = [C.c_int, i64p, C.c_double, C.c_double, C.c_int, C.c_double,
                                 C.c_double, C.c_double, C.c_int, dp, dp, dp,
                                 C.POINTER(C.c_void_p)]
        L.orc_create.restype = C.c_int
        L.orc_create2.argtypes = [C.c_int, i64p, C.c_double, C.c_double, C.c_int, C.c_double,
                                  C.c_double, C.c_double, C.c_int, C.c_int, dp, dp, dp,
                                  C.POINTER(C.c_void_p)]
        L.orc_create2.restype = C.c_int
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_get_scalars.argtypes = [C.c_void_p, dp]
        L.orc_set_scalars.argtypes = [C.c_void_p, dp]
        L.orc_set_nu.argtypes = [C.c_void_p, C.c_double]
        L.orc_get_fields.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_apply_A.argtypes = [C.c_void_p, C.c_int, dp, dp]
        L.orc_propagator_at.argtypes = [C.c_void_p, C.c_int64, C.c_int, dp]
        L.orc_source_hat.argtypes = [C.c_void_p, dp, dp]
        L.orc_solve.argtypes = [C.c_void_p, C.c_int, dp, C.c_double, C.c_int64, dp, i64p,
                                dp, dp, dp]
        L.orc_solve.restype = C.c_int
        L.orc_rel_residual.argtypes = [C.c_void_p, C.c_int, dp, dp]
        L.orc_rel_residual.restype = C.c_double
        L.orc_gradient.argtypes = [C.c_void_p, dp, dp, dp, dp, dp, dp]
        _LIB = L
    return _LIB


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def fft(a: np.ndarray, sign: int = -1) -> np.ndarray:
    """Unnormalised DFT over all axes (sign -1 forward, +1 inverse)."""
    out = np.ascontiguousarray(a, dtype=np.complex128).copy()
    n = np.array(out.shape, dtype=np.int64)
    lib().orc_fft(out.ndim, n.ctypes.data_as(C.POINTER(C.c_int64)), _dp(out), sign)
    return out


def mec(points: np.ndarray):
    """Minimum enclosing circle of complex points -> (centre, radius)."""
    p = np.ascontiguousarray(np.asarray(points, dtype=np.complex128).ravel())
    res = np.zeros(3)
    lib().orc_mec(_dp(p), p.size, _dp(res))
    return complex(res[0], res[1]), float(res[2])


class OracleMedium:
    def __init__(self, shape, dx, omega, c, rho, alpha, pml=16, gmax=0.0,
                 beta=0.95, nu=0.9, shift_rule=0, collocated=False):
        self.shape = tuple(int(s) for s in shape)
        self.ndim = len(self.shape)
        self.ncell = int(np.prod(self.shape))
        self.F = self.ndim + 1
        self.dx, self.omega = float(dx), float(omega)
        self._c = np.ascontiguousarray(c, dtype=np.float64).reshape(self.shape)
        self._rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.shape)
        self._alpha = np.ascontiguousarray(alpha, dtype=np.float64).reshape(self.shape)
        n = np.array(self.shape, dtype=np.int64)
        h = C.c_void_p()
        rc = lib().orc_create2(self.ndim, n.ctypes.data_as(C.POINTER(C.c_int64)), self.dx,
                               self.omega, int(pml), float(gmax), float(beta), float(nu),
                               int(shift_rule), int(bool(collocated)), _dp(self._c), _dp(self._rho),
                               _dp(self._alpha), C.byref(h))
        if rc != 0:
            raise ValueError("oracle rejected the medium")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    # -- scalars ----------------------------------------------------------
    def scalars(self):
        o = np.zeros(8)
        lib().orc_get_scalars(self._h, _dp(o))
        return dict(a1=complex(o[0], o[1]), a2=complex(o[2], o[3]), lam1=o[4], lam2=o[5],
                    beta=o[6], nu=o[7])

    def set_scalars(self, a1, a2, lam1, lam2):
        s = np.array([a1.real, a1.imag, a2.real, a2.imag, lam1, lam2], dtype=np.float64)
        lib().orc_set_scalars(self._h, _dp(s))

    def set_nu(self, nu):
        lib().orc_set_nu(self._h, float(nu))

    def fields(self):
        q = np.zeros(self.shape, np.complex128)
        rb = np.zeros((self.ndim,) + self.shape)
        g = np.zeros(self.shape)
        gs = np.zeros((self.ndim,) + self.shape)
        lib().orc_get_fields(self._h, _dp(q), _dp(rb), _dp(g), _dp(gs))
        return dict(q=q, rhobar=rb, gamma=g, gamma_s=gs)

    # -- operators --------------------------------------------------------
    def _field(self, a):
        a = np.ascontiguousarray(a, dtype=np.complex128)
        assert a.size == self.F * self.ncell, (a.shape, self.F, self.shape)
        return a.reshape((self.F,) + self.shape)

    def apply_A(self, xi, adjoint=False):
        xi = self._field(xi)
        out = np.zeros_like(xi)
        lib().orc_apply_A(self._h, int(adjoint), _dp(xi), _dp(out))
        return out

    def propagator_at(self, flat_k, adjoint=False):
        out = np.zeros((self.F, self.F), np.complex128)
        lib().orc_propagator_at(self._h, int(flat_k), int(adjoint), _dp(out))
        return out

    def source_hat(self, s):
        s = self._field(s)
        out = np.zeros_like(s)
        lib().orc_source_hat(self._h, _dp(s), _dp(out))
        return out

    def pressure_source(self, sp):
        """Physical source array (F, *grid) with s_p on the pressure row."""
        s = np.zeros((self.F,) + self.shape, np.complex128)
        s[-1] = np.asarray(sp).reshape(self.shape)
        return s

    def solve(self, shat, tol=1e-10, max_iter=100000, adjoint=False, history=False,
              x0=None):
        """Algorithm 1 on A xi = shat.  Returns (xi, info dict)."""
        shat = self._field(shat)
        out = np.zeros_like(shat)
        it = C.c_int64(0)
        rel = C.c_double(0)
        hist = np.zeros(max(int(max_iter), 1)) if history else None
        x0p = None
        if x0 is not None:
            x0a = self._field(x0)
            x0p = _dp(x0a)
        st = lib().orc_solve(self._h, int(adjoint), _dp(shat), float(tol), int(max_iter),
                             _dp(out), C.byref(it), C.byref(rel),
                             _dp(hist) if hist is not None else None, x0p)
        info = dict(converged=(st == 0), iterations=it.value, rel_update=rel.value)
        if hist is not None:
            info["history"] = hist[: it.value]
        return out, info

    def rel_residual(self, shat, xi, adjoint=False):
        shat = self._field(shat)
        xi = self._field(xi)
        return lib().orc_rel_residual(self._h, int(adjoint), _dp(shat), _dp(xi))

    def scaled_state(self, xi):
        """x = C^{1/2} xi."""
        xi = self._field(xi)
        s = self.scalars()
        sc = np.array([np.sqrt(s["lam1"])] * self.ndim + [np.sqrt(s["lam2"])])
        return xi * sc.reshape((self.F,) + (1,) * self.ndim)

    def gradient(self, s, xi, lam):
        s = self._field(s)
        xi = self._field(xi)
        lam = self._field(lam)
        gc = np.zeros(self.shape)
        gr = np.zeros(self.shape)
        ga = np.zeros(self.shape)
        lib().orc_gradient(self._h, _dp(s), _dp(xi), _dp(lam), _dp(gc), _dp(gr), _dp(ga))
        return gc, gr, ga

    def assemble_dense(self, adjoint=False):
        """Dense matrix of A (or A^H) by applying it to unit vectors."""
        n = self.F * self.ncell
        M = np.zeros((n, n), np.complex128)
        e = np.zeros(n, np.complex128)
        for j in range(n):
            e[:] = 0
            e[j] = 1.0
            M[:, j] = self.apply_A(e, adjoint).ravel()
        return M
