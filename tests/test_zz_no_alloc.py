"""The allocation-free residual entry point (cbs_residual_noalloc) against
cbs_residual, through the C ABI: two calls in a row on one GPU, the second on
a smaller grid (its kernels reuse the file-scope device array the first call
left behind), each compared with cbs_residual on the same medium and fields
(rel residual to 1e-12, residual fields to 1e-12 relative, element-wise
bound included), with host and device pointers; a grid whose workspace
exceeds the array is refused with CBS_E_NOMEM before any device work."""
import ctypes as C

import numpy as np
import pytest

from paper_2507_16087_amd import workloads as W

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


def _fields(shape, seed):
    rng = np.random.default_rng(seed)
    F = len(shape) + 1

    def rc():
        return np.ascontiguousarray(rng.standard_normal((F,) + shape) + 1j * rng.standard_normal((F,) + shape))

    return rc(), rc()


def _vp(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return C.c_void_p(a.ctypes.data)


def _call(fn, gm, s, xi, adjoint, device, ws=None):
    import torch
    from paper_2507_16087_amd import _lib
    F, N = s.shape[0], int(np.prod(s.shape[1:]))
    D = F - 1
    if device:
        sp, su = (torch.from_numpy(s[-1].ravel()).cuda(), torch.from_numpy(s[:-1].ravel()).cuda())
        p, u = (torch.from_numpy(xi[-1].ravel()).cuda(), torch.from_numpy(xi[:-1].ravel()).cuda())
        rp = torch.empty(N, dtype=torch.complex128, device="cuda")
        ru = torch.empty(D * N, dtype=torch.complex128, device="cuda")
        kind = _lib.CBS_PTR_DEVICE
    else:
        sp, su = np.ascontiguousarray(s[-1].ravel()), np.ascontiguousarray(s[:-1].ravel())
        p, u = np.ascontiguousarray(xi[-1].ravel()), np.ascontiguousarray(xi[:-1].ravel())
        rp = np.empty(N, np.complex128)
        ru = np.empty(D * N, np.complex128)
        kind = _lib.CBS_PTR_HOST
    rel = C.c_double(-1.0)
    args = [gm.handle, _vp(sp), _vp(su), _vp(p), _vp(u), int(adjoint), _lib.CBS_RHS_PHYSICAL, kind,
            C.byref(rel), _vp(rp), _vp(ru)]
    if fn == "cbs_residual":
        args += [_vp(ws), ws.numel(), None]
    else:
        args += [None]
    st = getattr(_lib.lib(), fn)(*args)
    torch.cuda.synchronize()
    assert st == _lib.CBS_OK, (fn, _lib.STATUS_NAMES.get(st, st))
    if device:
        rp, ru = rp.cpu().numpy(), ru.cpu().numpy()
    return rel.value, rp, ru


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _maxrel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("device", [False, True])
def test_noalloc_residual_matches_cbs_residual_twice(cbs, device):
    import torch
    for k, (shape, adjoint) in enumerate([((48, 32, 36), False), ((24, 16, 18), True)]):
        c, rho, alpha = W.small_random(shape, 40 + k)
        gm = cbs.Medium(shape, DX, OMEGA, c, rho, alpha, pml=2)
        ws = torch.empty(gm.workspace_bytes("fp64"), dtype=torch.uint8, device="cuda")
        s, xi = _fields(shape, 50 + k)
        ref = _call("cbs_residual", gm, s, xi, adjoint, device, ws)
        got = _call("cbs_residual_noalloc", gm, s, xi, adjoint, device)
        assert abs(got[0] - ref[0]) <= 1e-12 * ref[0], (shape, got[0], ref[0])
        for a, b in zip(got[1:], ref[1:]):
            assert _rel(a, b) <= 1e-12 and _maxrel(a, b) <= 1e-12, shape


def test_noalloc_refuses_a_grid_beyond_its_array(cbs):
    from paper_2507_16087_amd import _lib
    shape = (96, 96, 96)
    c, rho, alpha = W.small_random(shape, 3)
    gm = cbs.Medium(shape, DX, OMEGA, c, rho, alpha, pml=2)
    assert gm.workspace_bytes("fp64") > _lib.CBS_NOALLOC_SCRATCH_BYTES
    s, xi = _fields((8,), 1)            # never read: the size check comes first
    rel = C.c_double(-1.0)
    st = _lib.lib().cbs_residual_noalloc(gm.handle, _vp(s), None, _vp(xi), None, 0, _lib.CBS_RHS_PHYSICAL,
                                         _lib.CBS_PTR_HOST, C.byref(rel), None, None, None)
    assert st == _lib.CBS_E_NOMEM and rel.value == -1.0
