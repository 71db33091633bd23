"""Continuous-batching request loop for the iterative Born solver.

Requests (a grid, a frequency, a medium and a source) arrive over time.  Each
is admitted when its HBM footprint fits the budget and a slot of its grid
shape is free (:class:`Admission`: requests of one shape keep their arrival
order, but a shape whose pool is full or whose request does not fit yet does
not hold back requests of other shapes; a request that could never fit the
budget is closed with an error; idle pools of other shapes give their
workspace back when memory is short; and a request blocked on memory longer
than ``max_wait_s`` stops later requests from taking memory until it is
admitted).  Admitted requests are planned (medium setup, on a host thread
pool) and submitted as slots of a per-shape :class:`solver.Batch`.  Every
shape pool runs on its own HIP stream and host thread, advancing all of its
active slots together (one kernel launch per pass covers every slot) a fixed
number of iterations per step, retiring finished slots and taking new ones
between steps.  Pools of different shapes therefore overlap on the device,
and a request that arrives while others run joins the next step of its pool.

A slot's result depends only on its own request: same kernels and plans as
a single solve, no data shared between slots, deterministic reductions.

Latency is measured from a request's arrival to its result being on the host.
"""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import queue
import threading
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import solver

MEDIUM_BYTES_PER_CELL = 8 * 3 + 16 + 4 * 3 + 8 + 8 * 3   # rhobar, q (FP64, FP32), c, rho, alpha


@dataclasses.dataclass
class _PoolState:
    reserved: int = 0       # admitted requests of this shape not finished yet
    ws_bytes: int = 0       # the pool's batch workspace


class Admission:
    """Admission by HBM footprint, without a device (the server drives it).

    State: the byte budget, the bytes in use (media of admitted requests plus
    the workspace of every open pool) and, per shape, the requests admitted
    and not yet finished.  :meth:`select` walks the pending requests in
    arrival order and decides, for each, one of:

    * admit -- its pool has a free slot and its footprint (medium, plus the
      pool's workspace if the pool is not open yet) fits the free budget,
      after closing idle pools of other shapes (oldest first) if needed;
    * fail -- its footprint exceeds the whole budget, so it could never run;
    * wait -- otherwise.  Later requests of the same shape wait too (one
      FIFO per shape); other shapes are still considered, unless this request
      has waited on memory for more than ``max_wait_s``, in which case the
      walk stops so that it is the next to get memory.
    """

    def __init__(self, budget: int, slots_per_pool: int, max_wait_s: float,
                 medium_bytes: Callable[[tuple], int], pool_bytes: Callable[[tuple], int]):
        self.budget, self.slots, self.max_wait = int(budget), int(slots_per_pool), float(max_wait_s)
        self.medium_bytes, self.pool_bytes = medium_bytes, pool_bytes
        self.used = 0
        self.pools: Dict[tuple, _PoolState] = {}     # open pools, oldest first
        self.memory_waits = 0                        # requests that waited on memory at least once
        self._waited: set = set()
        self.evictions = 0

    def select(self, pending, now: float):
        """pending: objects with .shape, .arrival, .rid in arrival order.
        Returns (admitted, failed, evicted shapes); the state is updated for
        the admitted requests and the closed pools."""
        admitted, failed, evicted = [], [], []
        blocked = set()
        for req in pending:
            shape = req.shape
            if shape in blocked:
                continue
            med, ws = self.medium_bytes(shape), self.pool_bytes(shape)
            if med + ws > self.budget:
                failed.append(req)
                continue
            pool = self.pools.get(shape)
            if pool is not None and pool.reserved >= self.slots:
                blocked.add(shape)
                continue
            need = med + (0 if pool is not None else ws)
            if self.used + need > self.budget:
                for other, st in list(self.pools.items()):
                    if self.used + need <= self.budget:
                        break
                    if other != shape and st.reserved == 0:
                        self.used -= st.ws_bytes
                        del self.pools[other]
                        evicted.append(other)
                        self.evictions += 1
            if self.used + need > self.budget:
                blocked.add(shape)
                if req.rid not in self._waited:
                    self._waited.add(req.rid)
                    self.memory_waits += 1
                if now - req.arrival > self.max_wait:
                    break
                continue
            if pool is None:
                pool = self.pools[shape] = _PoolState(ws_bytes=ws)
            pool.reserved += 1
            self.used += need
            admitted.append(req)
        return admitted, failed, evicted

    def release(self, shape) -> None:
        """A request of this shape finished (or failed after admission)."""
        self.pools[shape].reserved -= 1
        self.used -= self.medium_bytes(shape)


@dataclasses.dataclass
class Result:
    rid: int
    shape: tuple
    arrival: float
    admitted: float = 0.0
    submitted: float = 0.0
    done: float = 0.0
    iterations: int = 0
    outer: int = 0
    rel_residual: float = -1.0
    converged: bool = False
    error: Optional[str] = None     # set when planning or the solve failed
    p: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class _Pool:
    def __init__(self, server: "Server", shape, dx):
        self.server = server
        self.shape = shape
        self.batch = solver.Batch(shape, dx, prec=server.prec, max_slots=server.slots_per_pool)
        self.inbox: "queue.Queue" = queue.Queue()
        self.reserved = 0          # slots promised to admitted requests (planning or running)
        self.slot_rid: Dict[int, int] = {}
        self.thread = threading.Thread(target=self._loop, daemon=True)
        self.stop = False
        self.thread.start()

    def _loop(self):
        import torch
        torch.cuda.set_device(0)
        while True:
            try:
                item = self.inbox.get(timeout=0.002 if self.slot_rid else 0.05)
            except queue.Empty:
                item = None
            while item is not None:
                rid, medium, sp = item
                try:
                    slot = self.batch.submit(medium, sp, tol=self.server.tol,
                                             inner_tol=self.server.inner_tol)
                except solver.L.CbsError as e:
                    self.server._fail(rid, self, f"submit: {e}")
                    slot = None
                if slot is not None:
                    assert slot >= 0, "admission promised a free slot"
                    self.slot_rid[slot] = rid
                    self.server._mark(rid, "submitted")
                try:
                    item = self.inbox.get_nowait()
                except queue.Empty:
                    item = None
            if not self.slot_rid:
                if self.stop:
                    return
                continue
            for slot in self.batch.step(self.server.step_iters):
                rid = self.slot_rid.pop(slot)
                try:
                    p, _, info = self.batch.retire(slot)
                except solver.L.CbsError as e:    # e.g. a diverged solve
                    self.server._fail(rid, self, f"solve: {e}")
                    continue
                self.server._finish(rid, self, p, info)


class Server:
    """Serve a stream of solve requests with continuous batching."""

    def __init__(self, prec="fp32_refined", tol=1e-5, inner_tol=0.0, slots_per_pool=4,
                 step_iters=32, hbm_budget: Optional[int] = None, plan_workers=4,
                 keep_fields=False, max_wait_s: float = 5.0):
        import torch
        self.prec, self.tol, self.inner_tol = prec, tol, inner_tol
        self.slots_per_pool, self.step_iters = slots_per_pool, step_iters
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.8 * free)
        self.budget = hbm_budget
        self._ws_bytes: Dict[tuple, int] = {}
        self.adm = Admission(hbm_budget, slots_per_pool, max_wait_s, self._medium_bytes,
                             self._pool_bytes)
        self.keep_fields = keep_fields
        self.pools: Dict[tuple, _Pool] = {}
        self.results: Dict[int, Result] = {}
        self.lock = threading.Lock()
        self.cv = threading.Condition(self.lock)
        self.planner = cf.ThreadPoolExecutor(max_workers=plan_workers)
        self.timeline: List[tuple] = []   # (time, active solves)
        self.active = 0

    @property
    def used(self) -> int:
        return self.adm.used

    # -- accounting -------------------------------------------------------
    def _mark(self, rid, what):
        with self.lock:
            setattr(self.results[rid], what, time.perf_counter())

    def _finish(self, rid, pool, p, info, error=None):
        with self.cv:
            r = self.results[rid]
            r.done = time.perf_counter()
            if error is None:
                r.iterations, r.outer = info["iterations"], info["outer"]
                r.rel_residual, r.converged = info["rel_residual"], info["converged"]
            r.error = error
            if self.keep_fields:
                r.p = p
            self.adm.release(pool.shape)
            self.active -= 1
            self.timeline.append((r.done, self.active))
            self.cv.notify_all()

    def _fail(self, rid, pool, error: str):
        """Close a request that could not be planned or solved; its slot
        reservation and HBM share are released like a finished one's."""
        self._finish(rid, pool, None, None, error=error)

    @staticmethod
    def _medium_bytes(shape):
        return int(np.prod(shape)) * MEDIUM_BYTES_PER_CELL

    def _pool_bytes(self, shape) -> int:
        """Workspace of a pool of this shape (slots_per_pool solves)."""
        shape = tuple(shape)
        if shape not in self._ws_bytes:
            import ctypes as C
            g = solver.L.Grid()
            g.ndim = len(shape)
            for d in range(3):
                g.n[d] = shape[d] if d < len(shape) else 1
            g.dx, g.omega = 1.0, 1.0
            nb = C.c_size_t()
            solver.L.check(solver.L.lib().cbs_batch_workspace_bytes(
                C.byref(g), solver.PREC[self.prec], self.slots_per_pool, C.byref(nb)),
                "cbs_batch_workspace_bytes")
            self._ws_bytes[shape] = nb.value
        return self._ws_bytes[shape]

    def footprint(self, shape, new_pool: bool) -> int:
        """HBM bytes admitting one request of this shape needs now."""
        return self._medium_bytes(shape) + (self._pool_bytes(shape) if new_pool else 0)

    # -- admission --------------------------------------------------------
    def _start(self, req):
        """Open the request's pool if needed and plan its medium."""
        pr = req.problem
        pool = self.pools.get(pr.shape)
        if pool is None:
            pool = _Pool(self, pr.shape, pr.dx)
            self.pools[pr.shape] = pool
        self.active += 1
        now = time.perf_counter()
        self.timeline.append((now, self.active))
        self.results[req.rid].admitted = now

        def plan():
            try:
                m = solver.Medium(pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, pml=pr.pml_cells)
            except (solver.L.CbsError, ValueError) as e:
                self._fail(req.rid, pool, f"plan: {e}")
                return
            pool.inbox.put((req.rid, m, pr.dense_source().ravel()))

        self.planner.submit(plan)

    def _close_pool(self, shape):
        """Stop an idle pool's thread and drop its batch (workspace)."""
        pool = self.pools.pop(shape)
        pool.stop = True
        pool.thread.join()
        del pool.batch

    def run(self, requests, time_scale: float = 1.0) -> dict:
        """Replay `requests` (arrival_s relative to start, divided by
        time_scale) and return per-request results and latency statistics."""
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        t0 = time.perf_counter()
        pending: List[_Pending] = []
        i = 0
        for r in reqs:
            self.results[r.rid] = Result(r.rid, r.problem.shape, t0 + r.arrival_s / time_scale)
        while True:
            now = time.perf_counter()
            while i < len(reqs) and t0 + reqs[i].arrival_s / time_scale <= now:
                rq = reqs[i]
                pending.append(_Pending(rq.rid, rq.problem.shape, self.results[rq.rid].arrival, rq))
                i += 1
            if pending:
                with self.lock:
                    admitted, failed, evicted = self.adm.select(pending, now)
                for shape in evicted:
                    self._close_pool(shape)
                with self.cv:
                    for pq in admitted:
                        self._start(pq.req)
                    for pq in failed:
                        r = self.results[pq.rid]
                        r.done = time.perf_counter()
                        r.error = "footprint exceeds the HBM budget"
                    self.cv.notify_all()
                gone = {id(pq) for pq in admitted + failed}
                pending = [pq for pq in pending if id(pq) not in gone]
            with self.cv:
                if i == len(reqs) and not pending and all(r.done > 0 for r in self.results.values()):
                    break
                self.cv.wait(timeout=0.002)
            dead = [p for p in self.pools.values() if not p.thread.is_alive()]
            if dead:
                raise RuntimeError(f"serving thread of pool {dead[0].shape} ended unexpectedly")
        for p in self.pools.values():
            p.stop = True
        for p in self.pools.values():
            p.thread.join()
        self.planner.shutdown(wait=True)
        res = [self.results[r.rid] for r in reqs]
        lat = np.array([r.latency for r in res]) * 1e3
        span = max(r.done for r in res) - t0
        by_size = {}
        for shape in sorted({r.shape for r in res}):
            ls = np.array([r.latency for r in res if r.shape == shape]) * 1e3
            by_size["x".join(map(str, shape))] = dict(
                count=int(ls.size), p50_ms=float(np.percentile(ls, 50)),
                p99_ms=float(np.percentile(ls, 99)))
        return dict(results=res, p50_ms=float(np.percentile(lat, 50)),
                    p99_ms=float(np.percentile(lat, 99)), solves_per_s=len(res) / span,
                    wall_s=span, max_concurrency=max((a for _, a in self.timeline), default=0),
                    converged=sum(r.converged for r in res),
                    failed=sum(r.error is not None for r in res),
                    by_size=by_size, budget_bytes=self.budget,
                    memory_waits=self.adm.memory_waits, pool_evictions=self.adm.evictions)


@dataclasses.dataclass
class _Pending:
    rid: int
    shape: tuple
    arrival: float
    req: object
