"""Failure handling forced from the host; every kernel still exits normally.

* divergence: a scale below the scattering potential (beta = 4, so |V| = 4)
  or an over-relaxed step makes the iterate grow; the solver reports
  CBS_E_DIVERGED and leaves the outputs untouched;
* iteration cap: CBS_NOT_CONVERGED with the last iterate returned;
* undersized workspace: CBS_E_NOMEM before any device work;
* admission: a server whose HBM budget admits one request at a time still
  completes every request (queued, not failed).
"""
import numpy as np
import pytest

from paper_2507_16087_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def cbs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_16087_amd import solver
    return solver


def _prob(n=24):
    pr = W.random3d(n, 1e6, seed=31, src=(n // 2,) * 3)
    pr.pml_cells = 5
    return pr


@pytest.mark.parametrize("prec,kw", [("fp64", dict(beta=4.0)), ("fp32_refined", dict(beta=4.0)),
                                     ("fp64", dict(nu=3.0))])
def test_divergence_detected(cbs, prec, kw):
    from paper_2507_16087_amd import _lib
    pr = _prob()
    m = cbs.Medium(pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, pml=pr.pml_cells, **kw)
    with pytest.raises(_lib.CbsError) as e:
        cbs.solve(m, pr.dense_source(), tol=1e-8, prec=prec, max_iter=20000)
    assert e.value.status == _lib.CBS_E_DIVERGED


def test_iteration_cap_returns_last_iterate(cbs, orc):
    pr = _prob()
    m = cbs.Medium(pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, pml=pr.pml_cells)
    p, u, info = cbs.solve(m, pr.dense_source(), tol=1e-14, max_iter=9, check_every=4)
    assert not info["converged"] and info["iterations"] == 9 and info["status"] == 1
    om = orc.OracleMedium(pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, pml=pr.pml_cells)
    xi, _ = om.solve(om.source_hat(om.pressure_source(pr.dense_source())), tol=0.0, max_iter=9)
    assert np.linalg.norm(p - xi[-1]) <= 1e-10 * np.linalg.norm(xi[-1])


def test_small_workspace_rejected(cbs):
    import torch
    from paper_2507_16087_amd import _lib
    pr = _prob()
    m = cbs.Medium(pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, pml=pr.pml_cells)
    ws = torch.empty(m.workspace_bytes("fp64") - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(_lib.CbsError) as e:
        cbs.solve(m, pr.dense_source(), workspace=ws)
    assert e.value.status == _lib.CBS_E_NOMEM


def test_admission_queues_when_budget_is_tight(cbs):
    from paper_2507_16087_amd.serve import Server
    reqs = []
    for i in range(4):
        pr = _prob(24)
        pr.name = f"r{i}"
        reqs.append(W.Request(i, 0.0, pr))
    probe = Server(tol=1e-6, slots_per_pool=2)
    one = probe.footprint((24, 24, 24), True)          # pool workspace + one medium
    half_medium = Server._medium_bytes((24, 24, 24)) // 2
    srv = Server(tol=1e-6, slots_per_pool=2, hbm_budget=one + half_medium)
    out = srv.run(reqs)
    assert out["converged"] == 4
    assert out["max_concurrency"] == 1


def test_invalid_arguments_on_a_medium(cbs):
    """Argument checks that need a live medium: unknown precision, an empty
    batch, a non-positive scale; each returns CBS_E_INVALID and changes
    nothing."""
    import ctypes as C
    from paper_2507_16087_amd import _lib
    pr = _prob(8)
    m = cbs.Medium(pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, pml=2)
    L = _lib.lib()
    cfg = (C.c_int32 * 20)()
    nb = C.c_size_t(0)
    assert L.cbs_pass_config(m._h, 7, cfg) == _lib.CBS_E_INVALID
    assert L.cbs_workspace_bytes(m._h, 7, 1, C.byref(nb)) == _lib.CBS_E_INVALID
    assert L.cbs_workspace_bytes(m._h, 0, 0, C.byref(nb)) == _lib.CBS_E_INVALID
    before = m.scalars()
    a1, a2 = before["a1"], before["a2"]
    bad = (C.c_double * 6)(a1.real, a1.imag, a2.real, a2.imag, -1.0, before["lam2"])
    assert L.cbs_set_scalars(m._h, bad) == _lib.CBS_E_INVALID
    assert m.scalars() == before


def test_server_reports_a_request_it_cannot_plan(cbs):
    """A request whose medium is rejected (a negative sound speed) is closed
    with an error; the requests around it still complete and the run ends."""
    from paper_2507_16087_amd.serve import Server
    reqs = []
    for i in range(3):
        pr = _prob(24)
        if i == 1:
            pr.c = np.array(pr.c, copy=True)
            pr.c.flat[0] = -1.0
        reqs.append(W.Request(i, 0.0, pr))
    out = Server(tol=1e-6, slots_per_pool=2).run(reqs)
    assert out["converged"] == 2 and out["failed"] == 1
    bad = out["results"][1]
    assert bad.error is not None and "plan" in bad.error and not bad.converged
