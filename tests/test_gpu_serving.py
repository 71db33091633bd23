"""Continuous batching: a slot's result is the same alone and in a mix.

Batched slots run the single-solve driver's kernels and plans, each slot on
its own data with deterministic reductions, so the design target is bitwise
equality; the gate is 1e-12 relative.  A small mixed-size request stream
through the server is also checked against the FP64 oracle.
"""
import numpy as np
import pytest

from paper_2507_16087_amd import workloads as W
from parity_util import maxrel, rel

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def cbs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_16087_amd import solver
    return solver


def _prob(n, f, seed, pml=6):
    rng = np.random.default_rng(seed)
    src = tuple(int(v) for v in rng.integers(pml, n - pml, 3))
    pr = W.random3d(n, f, seed=seed, src=src)
    pr.pml_cells = pml
    return pr


def _medium(cbs, pr):
    return cbs.Medium(pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, pml=pr.pml_cells)


def _rel(a, b):
    """Error measure of the parity checks: the larger of the relative L2 error
    and the largest element-wise error over the largest reference modulus."""
    return max(rel(a, b), maxrel(a, b))


@pytest.mark.parametrize("prec", ["fp32_refined", "fp64"])
def test_slot_in_mix_equals_single_solve(cbs, prec):
    probs = [_prob(32, f, 100 + i) for i, f in enumerate([1e6, 6e5, 8e5])]
    tol = 1e-6 if prec == "fp32_refined" else 1e-8
    alone = []
    for pr in probs:
        m = _medium(cbs, pr)
        p, _, info = cbs.solve(m, pr.dense_source(), tol=tol, prec=prec, want_u=False)
        assert info["converged"]
        alone.append((p, info))
    b = cbs.Batch(probs[0].shape, probs[0].dx, prec=prec, max_slots=4)
    media = [_medium(cbs, pr) for pr in probs]
    slots = {b.submit(m, pr.dense_source(), tol=tol): k for k, (m, pr) in enumerate(zip(media, probs))}
    out = {}
    # stagger: retire as they finish, keep stepping
    while len(out) < len(probs):
        for s in b.step(16):
            out[slots[s]] = b.retire(s)
    for k, (p, info) in enumerate(alone):
        pb, _, ib = out[k]
        assert ib["iterations"] == info["iterations"]
        assert ib["outer"] == info["outer"]
        assert _rel(pb, p) <= 1e-12


def test_server_stream_alone_vs_mix_and_oracle(cbs, orc):
    from paper_2507_16087_amd.serve import Server
    sizes = [24, 32, 24, 48, 32, 24, 48, 32]
    reqs = []
    t = 0.0
    rng = np.random.default_rng(7)
    for i, n in enumerate(sizes):
        t += float(rng.exponential(0.02))
        pr = _prob(n, float(rng.uniform(4e5, 1e6)), 200 + i)
        reqs.append(W.Request(i, t, pr))
    srv = Server(tol=1e-6, slots_per_pool=3, step_iters=16, keep_fields=True)
    out = srv.run(reqs)
    assert out["converged"] == len(reqs)
    assert out["max_concurrency"] >= 2
    assert out["p99_ms"] >= out["p50_ms"] > 0
    mixed = {r.rid: r for r in out["results"]}
    # each request again, alone in its own server
    for req in reqs[:5]:
        solo = Server(tol=1e-6, slots_per_pool=1, step_iters=16, keep_fields=True).run([req])
        r = solo["results"][0]
        assert r.iterations == mixed[req.rid].iterations
        assert _rel(r.p, mixed[req.rid].p) <= 1e-12
    # one small request against the oracle
    pr = reqs[0].problem
    om = orc.OracleMedium(pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, pml=pr.pml_cells)
    xi, info = om.solve(om.source_hat(om.pressure_source(pr.dense_source())), tol=1e-11,
                        max_iter=200000)
    assert info["converged"]
    assert _rel(mixed[0].p, xi[-1]) <= 1e-5


def test_batch_rejects_wrong_shape_and_full(cbs):
    pr = _prob(24, 1e6, 1)
    other = _prob(32, 1e6, 2)
    b = cbs.Batch(pr.shape, pr.dx, prec="fp64", max_slots=1)
    from paper_2507_16087_amd import _lib
    with pytest.raises(_lib.CbsError):
        b.submit(_medium(cbs, other), other.dense_source())
    m = _medium(cbs, pr)
    assert b.submit(m, pr.dense_source(), tol=1e-8) == 0
    assert b.submit(m, pr.dense_source(), tol=1e-8) == -1     # full
    while not b.step(32):
        pass
    p, _, info = b.retire(0)
    assert info["converged"]


def test_concurrent_solves_on_one_medium(cbs):
    """The ABI lets several threads solve on one medium with their own
    workspaces and streams; the first solves tune the plans once.  Four
    threads, fresh medium, must each reproduce the serial result."""
    import threading
    import torch
    pr = _prob(32, 1e6, 77)
    sp = torch.from_numpy(pr.dense_source().ravel()).cuda()
    m = _medium(cbs, pr)
    out = [None] * 4
    err = []

    def work(i):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                p, _, info = cbs.solve(m, sp, tol=1e-7, prec="fp32_refined", want_u=False, stream=st)
            st.synchronize()
            out[i] = (p.cpu().numpy(), info["iterations"])
        except Exception as e:   # pragma: no cover - reported below
            err.append(repr(e))

    th = [threading.Thread(target=work, args=(i,)) for i in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not err, err
    ref, _, iref = cbs.solve(m, sp, tol=1e-7, prec="fp32_refined", want_u=False)
    for p, it in out:
        assert it == iref["iterations"]
        assert _rel(p, ref.cpu().numpy()) <= 1e-12


def test_small_request_passes_a_blocked_large_one(cbs):
    """One slot per pool: a second 96^3 request waits for the first one's slot,
    but a 24^3 request arriving after it is admitted at once (its pool has a
    free slot and it fits the budget) and finishes before either 96^3 one."""
    from paper_2507_16087_amd.serve import Server
    big0, big1 = _prob(96, 1e6, 301), _prob(96, 1e6, 302)
    small = _prob(24, 1e6, 303)
    reqs = [W.Request(0, 0.0, big0), W.Request(1, 0.001, big1), W.Request(2, 0.002, small)]
    out = Server(tol=1e-6, slots_per_pool=1, step_iters=16).run(reqs)
    assert out["converged"] == 3
    r = {x.rid: x for x in out["results"]}
    assert r[2].admitted < r[1].admitted
    assert r[2].done < r[0].done and r[2].done < r[1].done
    assert out["by_size"]["24x24x24"]["count"] == 1


def test_request_larger_than_the_budget_is_closed(cbs):
    """A budget that holds one 24^3 pool and medium but not a 48^3 one: the
    48^3 request is closed with an error at once and the others complete."""
    from paper_2507_16087_amd.serve import Server
    probe = Server(tol=1e-6, slots_per_pool=2)
    budget = probe.footprint((24, 24, 24), True) + 2 * Server._medium_bytes((24, 24, 24))
    assert probe.footprint((48, 48, 48), True) > budget
    reqs = [W.Request(0, 0.0, _prob(24, 1e6, 311)), W.Request(1, 0.0, _prob(48, 1e6, 312)),
            W.Request(2, 0.0, _prob(24, 1e6, 313))]
    out = Server(tol=1e-6, slots_per_pool=2, hbm_budget=budget).run(reqs)
    assert out["converged"] == 2 and out["failed"] == 1
    assert "budget" in out["results"][1].error
