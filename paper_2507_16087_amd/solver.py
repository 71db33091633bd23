"""Python binding of the gfx950 solver: argument marshalling over the C ABI.

Every step of the solve runs in the HIP library; this module only converts
arrays to pointers and allocates caller-owned device memory (workspaces,
outputs) through torch's allocator.  Host inputs may be numpy arrays
(pointer kind HOST); device inputs are torch CUDA tensors (kind DEVICE).
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _lib as L

PREC = {"fp64": L.CBS_FP64, "fp32_refined": L.CBS_FP32_REFINED}


def _torch():
    import torch
    return torch


def _is_tensor(a) -> bool:
    try:
        import torch
    except ImportError:
        return False
    return isinstance(a, torch.Tensor)


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(a):
    if a is None:
        return None
    if _is_tensor(a):
        return C.c_void_p(a.data_ptr())
    return C.c_void_p(a.ctypes.data)


def _host_c128(a, count):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if a.size != count:
        raise ValueError(f"expected {count} complex values, got {a.size}")
    return a


def _dev_c128(a, count):
    if a is None:
        return None
    torch = _torch()
    if a.dtype != torch.complex128 or not a.is_contiguous() or not a.is_cuda:
        raise ValueError("device arrays must be contiguous complex128 CUDA tensors")
    if a.numel() != count:
        raise ValueError(f"expected {count} complex values, got {a.numel()}")
    return a


def _grid(shape, dx, omega, pml, gamma_max, beta, nu, shift_rule, collocated):
    g = L.Grid()
    g.ndim = len(shape)
    for d in range(3):
        g.n[d] = shape[d] if d < len(shape) else 1
    g.dx, g.omega, g.pml_cells, g.pml_gamma_max = float(dx), float(omega), int(pml), float(gamma_max)
    g.beta, g.nu, g.shift_rule = float(beta), float(nu), int(shift_rule)
    g.collocated = int(bool(collocated))
    return g


def plan_scalars(shape: Sequence[int], dx: float, omega: float, c, rho, alpha, pml: int = 16,
                 gamma_max: float = 0.0, beta: float = 0.95, nu: float = 0.9, shift_rule: int = 0,
                 collocated: bool = False) -> dict:
    """The split scalars (shifts a1, a2, scales lam1, lam2, beta, nu) a medium
    of these arguments would use, computed on the host alone (no GPU)."""
    shape = tuple(int(s) for s in shape)
    g = _grid(shape, dx, omega, pml, gamma_max, beta, nu, shift_rule, collocated)
    n = int(np.prod(shape))
    arrs = [np.ascontiguousarray(a, dtype=np.float64).ravel() for a in (c, rho, alpha)]
    if any(a.size != n for a in arrs):
        raise ValueError("medium arrays must have prod(shape) cells")
    o = (C.c_double * 8)()
    L.check(L.lib().cbs_plan_scalars(C.byref(g), *[_ptr(a) for a in arrs], o), "cbs_plan_scalars")
    return dict(a1=complex(o[0], o[1]), a2=complex(o[2], o[3]), lam1=o[4], lam2=o[5], beta=o[6], nu=o[7])


class Medium:
    """A medium (c, rho, alpha on the grid) planned for the solver."""

    def __init__(self, shape: Sequence[int], dx: float, omega: float, c, rho, alpha,
                 pml: int = 16, gamma_max: float = 0.0, beta: float = 0.95, nu: float = 0.9,
                 shift_rule: int = 0, collocated: bool = False, stream=None):
        self.shape = tuple(int(s) for s in shape)
        self.ndim = len(self.shape)
        self.ncell = int(np.prod(self.shape))
        self.F = self.ndim + 1
        self.dx, self.omega = float(dx), float(omega)
        g = _grid(self.shape, dx, omega, pml, gamma_max, beta, nu, shift_rule, collocated)
        self.grid = g
        if _is_tensor(c):
            arrs = [t.contiguous().to(_torch().float64) for t in (c, rho, alpha)]
            kind = L.CBS_PTR_DEVICE
            sp = _stream_ptr(stream)
        else:
            arrs = [np.ascontiguousarray(a, dtype=np.float64).ravel() for a in (c, rho, alpha)]
            kind = L.CBS_PTR_HOST
            sp = _stream_ptr(stream) if _torch().cuda.is_available() else None
        for a in arrs:
            if (a.numel() if _is_tensor(a) else a.size) != self.ncell:
                raise ValueError("medium arrays must have prod(shape) cells")
        h = C.c_void_p()
        L.check(L.lib().cbs_create_medium(C.byref(g), *[_ptr(a) for a in arrs], kind, sp,
                                          C.byref(h)), "cbs_create_medium")
        self._h = h
        # held here so that the handle can be released during interpreter
        # shutdown, when module globals may already be gone
        self._destroy = L.lib().cbs_destroy_medium

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def scalars(self) -> dict:
        o = (C.c_double * 8)()
        L.check(L.lib().cbs_medium_scalars(self._h, o), "cbs_medium_scalars")
        return dict(a1=complex(o[0], o[1]), a2=complex(o[2], o[3]), lam1=o[4], lam2=o[5],
                    beta=o[6], nu=o[7])

    def set_scalars(self, a1, a2, lam1, lam2):
        v = (C.c_double * 6)(a1.real, a1.imag, a2.real, a2.imag, lam1, lam2)
        L.check(L.lib().cbs_set_scalars(self._h, v), "cbs_set_scalars")

    def pass_config(self, prec="fp64") -> list:
        """Pass plans of one iteration at this precision, in launch order (tuned
        by the first solve): kind, axis length, columns per work-group, wide
        radix split, variant, and the number of last-axis column blocks the
        middle passes run in."""
        cfg = (C.c_int32 * 20)()
        L.check(L.lib().cbs_pass_config(self._h, PREC[prec], cfg), "cbs_pass_config")
        return [dict(kind=cfg[4 * i], n=cfg[4 * i + 1], cols=cfg[4 * i + 2],
                     wide=cfg[4 * i + 3] & 1, variant=(cfg[4 * i + 3] >> 1) & 15,
                     blocks=cfg[4 * i + 3] >> 5)
                for i in range(5) if cfg[4 * i] >= 0]

    def workspace_bytes(self, prec="fp64", batch=1) -> int:
        b = C.c_size_t()
        L.check(L.lib().cbs_workspace_bytes(self._h, PREC[prec], int(batch), C.byref(b)),
                "cbs_workspace_bytes")
        return b.value

    def workspace(self, prec="fp64"):
        torch = _torch()
        return torch.empty(self.workspace_bytes(prec), dtype=torch.uint8, device="cuda")


def _opts(tol, max_iter, prec, check_every, inner_tol, rhs_kind, ptr_kind, stop_rule, max_outer,
          max_inner=0):
    o = L.SolveOpts()
    o.max_inner = int(max_inner)
    o.tol, o.max_iter, o.prec = float(tol), int(max_iter), PREC[prec]
    o.check_every, o.inner_tol = int(check_every), float(inner_tol)
    o.rhs_kind, o.ptr_kind, o.stop_rule, o.max_outer = int(rhs_kind), int(ptr_kind), int(stop_rule), int(max_outer)
    return o


def solve(m: Medium, s_p, s_u=None, *, tol=1e-8, max_iter=100000, prec="fp64", check_every=32,
          inner_tol=0.0, equation_rhs=False, stop_rule=L.CBS_STOP_UPDATE, max_outer=0,
          max_inner=0, adjoint=False, want_u=True, workspace=None, stream=None, raise_on_cap=False):
    """Solve A xi = s_hat (or A^H xi = s_hat).  Returns (p, u, info).

    numpy inputs give numpy outputs (host pointers); CUDA tensors give CUDA
    tensors (device pointers, no host copies)."""
    device = _is_tensor(s_p)
    N = m.ncell
    if device:
        torch = _torch()
        sp = _dev_c128(s_p.reshape(-1), N)
        su = _dev_c128(s_u.reshape(-1), m.ndim * N) if s_u is not None else None
        p = torch.empty(N, dtype=torch.complex128, device=sp.device)
        u = torch.empty(m.ndim * N, dtype=torch.complex128, device=sp.device) if want_u else None
        kind = L.CBS_PTR_DEVICE
    else:
        sp = _host_c128(s_p, N)
        su = _host_c128(s_u, m.ndim * N)
        p = np.empty(N, np.complex128)
        u = np.empty(m.ndim * N, np.complex128) if want_u else None
        kind = L.CBS_PTR_HOST
    ws = workspace if workspace is not None else m.workspace(prec)
    o = _opts(tol, max_iter, prec, check_every, inner_tol,
              L.CBS_RHS_EQUATION if equation_rhs else L.CBS_RHS_PHYSICAL, kind, stop_rule, max_outer,
              max_inner)
    info = L.SolveInfo()
    fn = L.lib().cbs_solve_adjoint if adjoint else L.lib().cbs_solve
    st = fn(m.handle, _ptr(sp), _ptr(su), C.byref(o), _ptr(p), _ptr(u), C.c_void_p(ws.data_ptr()),
            ws.numel(), C.byref(info), _stream_ptr(stream))
    allow = (L.CBS_OK,) if raise_on_cap else (L.CBS_OK, L.CBS_NOT_CONVERGED)
    L.check(st, "cbs_solve_adjoint" if adjoint else "cbs_solve", allow)
    d = info.as_dict()
    d["converged"] = st == L.CBS_OK
    p = p.reshape(m.shape)
    if u is not None:
        u = u.reshape((m.ndim,) + m.shape)
    return p, u, d


def solve_split(m: Medium, parts: int, s_p, s_u=None, *, tol=1e-8, max_iter=100000, prec="fp64",
                check_every=32, inner_tol=0.0, stop_rule=L.CBS_STOP_UPDATE, max_outer=0, max_inner=0,
                want_u=True, stream=None):
    """The solve of :func:`solve` split into `parts` axis-0 slabs the way
    that many GPUs would run it (cbs_solve_split), on the current device.
    Returns (p, u, info) like :func:`solve`."""
    torch = _torch()
    device = _is_tensor(s_p)
    N = m.ncell
    if device:
        sp = _dev_c128(s_p.reshape(-1), N)
        su = _dev_c128(s_u.reshape(-1), m.ndim * N) if s_u is not None else None
        p = torch.empty(N, dtype=torch.complex128, device=sp.device)
        u = torch.empty(m.ndim * N, dtype=torch.complex128, device=sp.device) if want_u else None
        kind = L.CBS_PTR_DEVICE
    else:
        sp = _host_c128(s_p, N)
        su = _host_c128(s_u, m.ndim * N)
        p = np.empty(N, np.complex128)
        u = np.empty(m.ndim * N, np.complex128) if want_u else None
        kind = L.CBS_PTR_HOST
    nb = C.c_size_t()
    L.check(L.lib().cbs_split_workspace_bytes(m.handle, PREC[prec], int(parts), C.byref(nb)),
            "cbs_split_workspace_bytes")
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    o = _opts(tol, max_iter, prec, check_every, inner_tol, L.CBS_RHS_PHYSICAL, kind, stop_rule, max_outer,
              max_inner)
    info = L.SolveInfo()
    st = L.lib().cbs_solve_split(m.handle, int(parts), _ptr(sp), _ptr(su), C.byref(o), _ptr(p), _ptr(u),
                                 C.c_void_p(ws.data_ptr()), ws.numel(), C.byref(info), _stream_ptr(stream))
    L.check(st, "cbs_solve_split", (L.CBS_OK, L.CBS_NOT_CONVERGED))
    d = info.as_dict()
    d["converged"] = st == L.CBS_OK
    p = p.reshape(m.shape)
    if u is not None:
        u = u.reshape((m.ndim,) + m.shape)
    return p, u, d


def residual(m: Medium, s_p, s_u, p, u=None, *, adjoint=False, equation_rhs=False,
             want_fields=False, workspace=None, stream=None):
    """Scaled FP64 residual |y - (L+V) x| / |y|; optionally the physical
    residual fields (r_p, r_u)."""
    device = _is_tensor(p)
    N = m.ncell
    if device:
        torch = _torch()
        args = [_dev_c128(s_p.reshape(-1), N),
                _dev_c128(s_u.reshape(-1), m.ndim * N) if s_u is not None else None,
                _dev_c128(p.reshape(-1), N),
                _dev_c128(u.reshape(-1), m.ndim * N) if u is not None else None]
        rp = torch.empty(N, dtype=torch.complex128, device=p.device) if want_fields else None
        ru = torch.empty(m.ndim * N, dtype=torch.complex128, device=p.device) if want_fields else None
        kind = L.CBS_PTR_DEVICE
    else:
        args = [_host_c128(s_p, N), _host_c128(s_u, m.ndim * N), _host_c128(p, N),
                _host_c128(u, m.ndim * N)]
        rp = np.empty(N, np.complex128) if want_fields else None
        ru = np.empty(m.ndim * N, np.complex128) if want_fields else None
        kind = L.CBS_PTR_HOST
    ws = workspace if workspace is not None else m.workspace("fp64")
    rel = C.c_double()
    L.check(L.lib().cbs_residual(m.handle, *[_ptr(a) for a in args], int(adjoint),
                                 L.CBS_RHS_EQUATION if equation_rhs else L.CBS_RHS_PHYSICAL, kind,
                                 C.byref(rel), _ptr(rp), _ptr(ru), C.c_void_p(ws.data_ptr()),
                                 ws.numel(), _stream_ptr(stream)), "cbs_residual")
    if want_fields:
        return rel.value, rp.reshape(m.shape), ru.reshape((m.ndim,) + m.shape)
    return rel.value


def gradient(m: Medium, s_p, s_u, p, u, lp, lu, stream=None):
    """Adjoint-state misfit gradient (dJ/dc, dJ/drho, dJ/dalpha)."""
    device = _is_tensor(p)
    N = m.ncell
    if device:
        torch = _torch()
        args = [_dev_c128(s_p.reshape(-1), N),
                _dev_c128(s_u.reshape(-1), m.ndim * N) if s_u is not None else None,
                _dev_c128(p.reshape(-1), N),
                _dev_c128(u.reshape(-1), m.ndim * N) if u is not None else None,
                _dev_c128(lp.reshape(-1), N),
                _dev_c128(lu.reshape(-1), m.ndim * N) if lu is not None else None]
        outs = [torch.empty(N, dtype=torch.float64, device=p.device) for _ in range(3)]
        kind = L.CBS_PTR_DEVICE
    else:
        args = [_host_c128(s_p, N), _host_c128(s_u, m.ndim * N), _host_c128(p, N),
                _host_c128(u, m.ndim * N), _host_c128(lp, N), _host_c128(lu, m.ndim * N)]
        outs = [np.empty(N) for _ in range(3)]
        kind = L.CBS_PTR_HOST
    L.check(L.lib().cbs_gradient(m.handle, *[_ptr(a) for a in args], kind,
                                 *[_ptr(o) for o in outs], _stream_ptr(stream) if device else None),
            "cbs_gradient")
    return tuple(o.reshape(m.shape) for o in outs)


class Batch:
    """Same-shape slots advanced together (continuous batching).

    Owns a device workspace (torch allocation) sized for ``max_slots`` solves
    and a HIP stream; every call must come from one thread at a time."""

    def __init__(self, shape, dx_ref, prec="fp32_refined", max_slots=4, stream=None):
        torch = _torch()
        self.shape = tuple(int(s) for s in shape)
        self.ndim = len(self.shape)
        self.ncell = int(np.prod(self.shape))
        self.prec = prec
        self.max_slots = int(max_slots)
        g = L.Grid()
        g.ndim = self.ndim
        for d in range(3):
            g.n[d] = self.shape[d] if d < self.ndim else 1
        g.dx, g.omega = float(dx_ref), 1.0
        self.grid = g
        b = C.c_size_t()
        L.check(L.lib().cbs_batch_workspace_bytes(C.byref(g), PREC[prec], self.max_slots, C.byref(b)),
                "cbs_batch_workspace_bytes")
        self.workspace_bytes = b.value
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device="cuda")
        h = C.c_void_p()
        L.check(L.lib().cbs_batch_create(C.byref(g), PREC[prec], self.max_slots,
                                         C.c_void_p(self.ws.data_ptr()), self.workspace_bytes,
                                         C.c_void_p(self.stream.cuda_stream), C.byref(h)),
                "cbs_batch_create")
        self._h = h
        self._destroy = L.lib().cbs_batch_destroy
        self.media = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._destroy(h)
            self._h = None

    def submit(self, m: Medium, s_p, s_u=None, *, tol=1e-5, max_iter=200000, inner_tol=0.0,
               max_outer=0, max_inner=0) -> int:
        """Start a solve in a free slot; returns the slot index or -1 if full."""
        device = _is_tensor(s_p)
        N = m.ncell
        sp = _dev_c128(s_p.reshape(-1), N) if device else _host_c128(s_p, N)
        su = None
        if s_u is not None:
            su = _dev_c128(s_u.reshape(-1), m.ndim * N) if device else _host_c128(s_u, m.ndim * N)
        o = _opts(tol, max_iter, self.prec, 0, inner_tol, L.CBS_RHS_PHYSICAL,
                  L.CBS_PTR_DEVICE if device else L.CBS_PTR_HOST, L.CBS_STOP_UPDATE, max_outer,
                  max_inner)
        slot = C.c_int32(-1)
        st = L.lib().cbs_batch_submit(self._h, m.handle, _ptr(sp), _ptr(su), C.byref(o), C.byref(slot))
        if st == L.CBS_E_NOMEM:
            return -1
        L.check(st, "cbs_batch_submit")
        self.media[slot.value] = m      # keep the medium alive while its slot runs
        return slot.value

    def step(self, iterations=32):
        """Advance every active slot; returns the list of finished slots."""
        mask = (C.c_uint8 * self.max_slots)()
        L.check(L.lib().cbs_batch_step(self._h, int(iterations), mask), "cbs_batch_step")
        return [i for i in range(self.max_slots) if mask[i]]

    def retire(self, slot, want_u=False, device=False):
        """Copy a finished slot's (p, u) out and free the slot."""
        torch = _torch()
        N = self.ncell
        if device:
            p = torch.empty(N, dtype=torch.complex128, device="cuda")
            u = torch.empty(self.ndim * N, dtype=torch.complex128, device="cuda") if want_u else None
            kind = L.CBS_PTR_DEVICE
        else:
            p = np.empty(N, np.complex128)
            u = np.empty(self.ndim * N, np.complex128) if want_u else None
            kind = L.CBS_PTR_HOST
        info = L.SolveInfo()
        st = L.lib().cbs_batch_retire(self._h, int(slot), _ptr(p), _ptr(u), kind, C.byref(info))
        if st in (L.CBS_OK, L.CBS_NOT_CONVERGED, L.CBS_E_DIVERGED):   # the slot is free again
            self.media.pop(int(slot), None)
        L.check(st, "cbs_batch_retire", (L.CBS_OK, L.CBS_NOT_CONVERGED))
        d = info.as_dict()
        d["converged"] = st == L.CBS_OK
        p = p.reshape(self.shape)
        if u is not None:
            u = u.reshape((self.ndim,) + self.shape)
        return p, u, d
