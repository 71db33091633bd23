"""The host planner through cbs_plan_scalars, on the CPU (no GPU needed).

Its shifts a1, a2 (both shift rules) and scales lam1, lam2 must equal the
oracle's to 1e-12 on media whose diagonal values repeat or line up (a water
background puts most cells on one value; every cell outside the absorbing
layer has a purely imaginary velocity diagonal), at sizes where the planner
splits its scans over host threads, and in the degenerate cases: a medium
without a layer whose values all coincide (enclosing circle of radius 0, so
the scale floor of 1e-3 |a| applies), and a medium with two densities only.
"""
import ctypes as C

import numpy as np
import pytest

from paper_2507_16087_amd import _lib, solver
from paper_2507_16087_amd import workloads as W

DX, OMEGA = 2.5e-4, 2 * np.pi * 1e6


def _case(name):
    if name == "disc2d_256":
        pr = W.disc2d(256)
        return pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, 16
    if name == "shell3d_64":
        pr = W.shell3d(64)
        return pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, 8
    if name == "random3d_48":
        pr = W.random3d(48)
        return pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, 6
    if name == "water3d_48":
        s = (48, 48, 48)
        return s, DX, OMEGA, np.full(s, 1500.0), np.full(s, 1000.0), np.zeros(s), 6
    if name == "uniform_no_layer":
        s = (64, 64)
        return s, DX, OMEGA, np.full(s, 1500.0), np.full(s, 1000.0), np.full(s, 0.5), 0
    if name == "two_densities":
        s = (96, 96, 12)
        rho = np.where(np.arange(96)[:, None, None] < 40, 1000.0, 1800.0) * np.ones(s)
        return s, DX, OMEGA, np.full(s, 1500.0), rho, np.zeros(s), 0
    if name == "random1d_512":
        c, rho, alpha = W.small_random((512,), 11)
        return (512,), DX, OMEGA, c, rho, alpha, 40
    if name == "step1d_243":
        s = (243,)
        x = np.arange(243)
        return s, DX, OMEGA, np.where(x < 120, 1500.0, 2100.0), np.where(x < 120, 1000.0, 1700.0), \
            np.zeros(s), 20
    raise KeyError(name)


CASES = ["disc2d_256", "shell3d_64", "random3d_48", "water3d_48", "uniform_no_layer", "two_densities",
         "random1d_512", "step1d_243"]


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("rule", [0, 1])
def test_plan_scalars_match_oracle(orc, name, rule):
    shape, dx, omega, c, rho, alpha, pml = _case(name)
    got = solver.plan_scalars(shape, dx, omega, c, rho, alpha, pml=pml, shift_rule=rule)
    ref = orc.OracleMedium(shape, dx, omega, c, rho, alpha, pml=pml, shift_rule=rule).scalars()
    for k in ("a1", "a2"):
        assert abs(got[k] - ref[k]) <= 1e-12 * abs(ref[k]), (k, got[k], ref[k])
    for k in ("lam1", "lam2"):
        assert abs(got[k] - ref[k]) <= 1e-12 * ref[k], (k, got[k], ref[k])
    assert got["beta"] == 0.95 and got["nu"] == 0.9


def test_degenerate_medium_uses_the_scale_floor():
    """All values on one point: a equals it and lam = 1e-3 |a| / beta."""
    shape, dx, omega, c, rho, alpha, pml = _case("uniform_no_layer")
    got = solver.plan_scalars(shape, dx, omega, c, rho, alpha, pml=pml)
    d_u = complex(0.0, 1000.0 * omega)   # rho (i omega + gamma), gamma = 0
    assert abs(got["a1"] - d_u) <= 1e-15 * abs(d_u)
    assert abs(got["lam1"] - 1e-3 * abs(d_u) / 0.95) <= 1e-15 * got["lam1"]


def test_plan_scalars_rejects_bad_input():
    L = _lib.lib()
    shape = (16, 16)
    g = _lib.Grid()
    g.ndim, g.dx, g.omega, g.pml_cells = 2, DX, OMEGA, 2
    g.n[0], g.n[1], g.n[2] = 16, 16, 1
    c, rho, alpha = (np.full(shape, v) for v in (1500.0, 1000.0, 0.0))
    out = (C.c_double * 8)()
    ptrs = [C.c_void_p(a.ctypes.data) for a in (c, rho, alpha)]
    assert L.cbs_plan_scalars(C.byref(g), *ptrs, out) == _lib.CBS_OK
    assert L.cbs_plan_scalars(C.byref(g), *ptrs, None) == _lib.CBS_E_INVALID
    assert L.cbs_plan_scalars(C.byref(g), None, ptrs[1], ptrs[2], out) == _lib.CBS_E_INVALID
    bad = c.copy()
    bad[3, 4] = -1.0
    assert L.cbs_plan_scalars(C.byref(g), C.c_void_p(bad.ctypes.data), ptrs[1], ptrs[2], out) == \
        _lib.CBS_E_INVALID
    g.n[1] = 10                     # not a supported axis length
    assert L.cbs_plan_scalars(C.byref(g), *ptrs, out) == _lib.CBS_E_UNSUPPORTED
