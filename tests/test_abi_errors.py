"""Input validation of the C ABI, on the CPU: every rejected input returns its
status code before any device work (no GPU is touched)."""
import ctypes as C

import numpy as np
import pytest

from paper_2507_16087_amd import _lib as L


def _grid(n=(16, 16, 16), pml=4, ndim=3, beta=0.95, nu=0.9, rule=0, dx=1e-4, omega=6e6):
    g = L.Grid()
    g.ndim = ndim
    for d in range(3):
        g.n[d] = n[d] if d < len(n) else 1
    g.dx, g.omega, g.pml_cells, g.pml_gamma_max = dx, omega, pml, 0.0
    g.beta, g.nu, g.shift_rule = beta, nu, rule
    return g


def _create(g, c, rho, alpha):
    h = C.c_void_p()
    arrs = [np.ascontiguousarray(a, dtype=np.float64).ravel() for a in (c, rho, alpha)]
    st = L.lib().cbs_create_medium(C.byref(g), *[C.c_void_p(a.ctypes.data) for a in arrs],
                                   L.CBS_PTR_HOST, None, C.byref(h))
    return st, h


@pytest.mark.parametrize("bad", ["c0", "rho_neg", "alpha_neg", "nan", "inf"])
def test_invalid_medium_values(bad):
    shape = (16, 16, 16)
    c, rho, alpha = np.full(shape, 1500.0), np.full(shape, 1000.0), np.zeros(shape)
    if bad == "c0":
        c[3, 4, 5] = 0.0
    elif bad == "rho_neg":
        rho[1, 1, 1] = -1.0
    elif bad == "alpha_neg":
        alpha[2, 2, 2] = -1e-3
    elif bad == "nan":
        c[0, 0, 0] = np.nan
    else:
        alpha[0, 0, 0] = np.inf
    st, h = _create(_grid(), c, rho, alpha)
    assert st == L.CBS_E_INVALID and not h.value


@pytest.mark.parametrize("n,code", [((10, 16, 16), L.CBS_E_UNSUPPORTED), ((16, 7, 16), L.CBS_E_UNSUPPORTED),
                                    ((1024, 16, 16), L.CBS_E_UNSUPPORTED), ((768, 16, 16), L.CBS_E_UNSUPPORTED),
                                    ((16, 16, 2), L.CBS_E_UNSUPPORTED), ((16, 20, 16), L.CBS_E_UNSUPPORTED)])
def test_unsupported_sizes(n, code):
    shape = n
    ones = np.ones(shape)
    st, h = _create(_grid(n), ones * 1500, ones * 1000, ones * 0)
    assert st == code


SMOOTH = [a * b for a in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512) for b in (1, 3, 9, 27, 81, 243)
          if 4 <= a * b <= 512]


def test_every_smooth_length_is_accepted():
    """Every axis length 2^a 3^b in [4, 512] has a plan (the host planner runs
    its size checks without a device); 5, 7 and their multiples do not."""
    from paper_2507_16087_amd import solver
    assert len(SMOOTH) == 31
    for n in SMOOTH:
        shape = (n, 4)
        ones = np.ones(shape)
        s = solver.plan_scalars(shape, 1e-4, 6e6, ones * 1500, ones * 1000, ones * 0, pml=1)
        assert s["lam1"] > 0, n
    for n in SMOOTH:   # 1-D grids
        ones = np.ones(n)
        s = solver.plan_scalars((n,), 1e-4, 6e6, ones * 1500, ones * 1000, ones * 0, pml=1)
        assert s["lam1"] > 0, n
    for n in (5, 10, 14, 20, 40, 100, 1024):
        ones = np.ones((n, 4))
        with pytest.raises(Exception):
            solver.plan_scalars((n, 4), 1e-4, 6e6, ones * 1500, ones * 1000, ones * 0, pml=1)


@pytest.mark.parametrize("kw", [dict(pml=8), dict(pml=-1), dict(beta=-0.5), dict(nu=float("nan")),
                                dict(rule=3), dict(dx=0.0), dict(omega=-1.0)])
def test_invalid_grid(kw):
    shape = (16, 16, 16)
    ones = np.ones(shape)
    st, h = _create(_grid(**kw), ones * 1500, ones * 1000, ones * 0)
    assert st == L.CBS_E_INVALID


def test_invalid_dimension_and_null_pointers():
    ones = np.ones((16, 16))
    for nd in (0, 4):
        st, _ = _create(_grid((16, 16), ndim=nd), ones, ones, ones)
        assert st == L.CBS_E_UNSUPPORTED
    h = C.c_void_p()
    g = _grid()
    assert L.lib().cbs_create_medium(C.byref(g), None, None, None, 0, None, C.byref(h)) == L.CBS_E_INVALID
    assert L.lib().cbs_destroy_medium(None) == L.CBS_E_INVALID
    b = C.c_size_t()
    assert L.lib().cbs_workspace_bytes(None, 0, 1, C.byref(b)) == L.CBS_E_INVALID
    assert L.lib().cbs_pass_timing(None, 1) == L.CBS_E_INVALID
    assert L.lib().cbs_pass_timing_slots(None, 0x3F) == L.CBS_E_INVALID


def test_batch_workspace_size_query_on_cpu():
    b = C.c_size_t()
    g = _grid((32, 32, 32))
    assert L.lib().cbs_batch_workspace_bytes(C.byref(g), L.CBS_FP32_REFINED, 4, C.byref(b)) == L.CBS_OK
    per_cell = b.value / (4 * 32 ** 3)
    # per slot: x, w, y in complex128 and d, w, y in complex64 over 4 fields (288 B/cell) + small
    assert 288 <= per_cell < 320
    assert L.lib().cbs_batch_workspace_bytes(C.byref(g), 7, 4, C.byref(b)) == L.CBS_E_INVALID
    assert L.lib().cbs_batch_workspace_bytes(C.byref(g), 0, 0, C.byref(b)) == L.CBS_E_INVALID


@pytest.mark.parametrize("src,dst,nbytes,reps", [
    (0, 1 << 20, 64, 1),             # null source
    (1 << 20, 0, 64, 1),             # null destination
    ((1 << 20) + 8, 1 << 21, 64, 1),   # misaligned source
    (1 << 20, (1 << 21) + 4, 64, 1),   # misaligned destination
    (1 << 20, 1 << 21, 0, 1),        # no bytes
    (1 << 20, 1 << 21, 40, 1),       # not a multiple of 16
    (1 << 20, 1 << 21, 64, 0),       # no repetitions
    (1 << 20, (1 << 20) + 32, 64, 1),  # destination inside the source
    ((1 << 20) + 48, 1 << 20, 64, 1),  # source inside the destination
])
def test_stream_probe_rejects_bad_arguments(src, dst, nbytes, reps):
    """The pointers are never dereferenced: every case fails its checks first."""
    gbs = C.c_double(-1.0)
    st = L.lib().cbs_stream_probe(C.c_void_p(src), C.c_void_p(dst), nbytes, reps, C.byref(gbs), None)
    assert st == L.CBS_E_INVALID and gbs.value == -1.0
