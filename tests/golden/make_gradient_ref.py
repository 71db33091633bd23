"""Write the FP64 oracle's misfit gradient for one shot of the 128^3 inversion
workload.

TEST INFRASTRUCTURE ONLY.  This script calls the CPU oracle (``oracle/``) and
the seeded input generators, nothing else.  For the first shot of the
inversion workload (a unit point source on the x = 20 face, 128 receivers on
the x = 107 face):

1. data d: the oracle's pressure at the receivers for the medium with the
   smooth bump (c up 3 %, rho down 3 %), Algorithm 1 to a relative update of
   1e-12;
2. the forward solution xi on the model medium, to 1e-12;
3. the adjoint solution lambda of A^H lambda = g with g_p = M^T (M p - d) at
   the receivers (Sec. 2.3 adjoint operator), to 1e-12;
4. the adjoint-state gradient of J = 1/2 |M p - d|^2 with respect to c, rho
   and alpha (the oracle's gradient formula).

Stored (tests/golden/oracle_gradient128.npz): the data d, J, the three
gradients at 20 000 seeded cells (the same draw as the solution references)
and their whole-grid norms, and each solve's iteration count and relative
update.  ``OMP_NUM_THREADS`` sets the oracle's thread count.

Usage:  python tests/golden/make_gradient_ref.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

from oracle import core as orc                      # noqa: E402
from paper_2507_16087_amd import workloads as W     # noqa: E402
from make_converged import sample_cells              # noqa: E402

TOL = 1e-12


def solve(m, rhs, adjoint=False, what=""):
    t0 = time.time()
    xi, info = m.solve(rhs, tol=TOL, max_iter=100000, adjoint=adjoint)
    print(f"{what}: {info['iterations']} iterations, rel update {info['rel_update']:.3e}, "
          f"{time.time() - t0:.0f} s", flush=True)
    assert info["converged"], info
    return xi, info


def main() -> None:
    inv = W.inversion(128)
    pr = inv.model
    shot = inv.shots[0]
    rec = inv.receivers
    sp = np.zeros(pr.ncell, complex)
    sp[shot] = 1.0
    sp = sp.reshape(pr.shape)

    mt = orc.OracleMedium(pr.shape, pr.dx, pr.omega, inv.true_c, inv.true_rho, pr.alpha,
                          pml=pr.pml_cells)
    xt, it_d = solve(mt, mt.source_hat(mt.pressure_source(sp)), what="data (bumped medium)")
    d = xt[3].ravel()[rec].copy()
    del mt, xt

    m = orc.OracleMedium(pr.shape, pr.dx, pr.omega, pr.c, pr.rho, pr.alpha, pml=pr.pml_cells)
    s = m.pressure_source(sp)
    xi, it_f = solve(m, m.source_hat(s), what="forward (model medium)")
    res = xi[3].ravel()[rec] - d
    J = 0.5 * float(np.vdot(res, res).real)
    g = np.zeros((4, pr.ncell), complex)
    g[3, rec] = res
    lam, it_a = solve(m, g.reshape((4,) + pr.shape), adjoint=True, what="adjoint")
    gc, grho, galpha = m.gradient(s, xi, lam)
    idx = sample_cells(pr.shape)
    grads = [gc.ravel(), grho.ravel(), galpha.ravel()]
    out = os.path.join(HERE, "oracle_gradient128.npz")
    np.savez_compressed(
        out, shot=np.array(shot), receivers=rec, d=d, J=J, idx=idx,
        samples=np.stack([gr[idx] for gr in grads]),
        norm2=np.array([float(np.dot(gr, gr)) for gr in grads]),
        iterations=np.array([it_d["iterations"], it_f["iterations"], it_a["iterations"]]),
        rel_update=np.array([it_d["rel_update"], it_f["rel_update"], it_a["rel_update"]]),
        tol=TOL)
    print(f"wrote {out}: J = {J:.6e}", flush=True)


if __name__ == "__main__":
    main()
