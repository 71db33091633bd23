"""Write FP64 oracle references (converged, or a fixed iterate) for the
full-size workloads.

TEST INFRASTRUCTURE ONLY.  This script calls the CPU oracle (``oracle/``) and
the seeded input generators, nothing else.  It runs Algorithm 1 from x = 0 on
the workload's medium and source until the relative update falls to the
target (or a wall-clock budget ends), in chunks that resume from the scaled
state of the previous chunk, and stores what the GPU tests compare against:

* ``idx``: 20 000 seeded random cells (flat indices), ``samples``: every
  field (u_0, u_1, u_2, p) at those cells;
* three pencils through the source (or focus) cell along each axis, all
  fields, ``pencil{0,1,2}``;
* ``norm2``: the squared L2 norm of each whole field, and ``fabs_max``: the
  largest modulus of each field;
* the iteration count (a run capped by --max-iters or the budget stores
  that iterate, not a converged one), the last relative update and the scaled true
  residual |y - (L+V) x| / |y| of the stored state, evaluated by the oracle's
  own operator.

Usage:  python tests/golden/make_converged.py random128 [--tol 1e-10]
                                               [--budget-hours H] [--chunk K]
                                               [--max-iters K] [--ckpt-dir DIR]
        python tests/golden/make_converged.py shell256 ...

With ``--ckpt-dir DIR`` the scaled state is checkpointed in DIR after every
chunk, so a killed run resumes where it stopped (without it, nothing is saved
between chunks).  ``OMP_NUM_THREADS`` sets the oracle's
thread count.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import core as orc                      # noqa: E402
from paper_2507_16087_amd import workloads as W     # noqa: E402

NSAMPLE = 20000
SAMPLE_SEED = 77


def problem(name: str):
    if name == "random128":
        return W.random3d(128), (64, 64, 64)
    if name == "shell256":
        # the focus of the bowl: (76, 64, 64) mm at 0.5 mm cells
        return W.shell3d(256), (152, 128, 128)
    raise SystemExit(f"unknown workload {name}")


def sample_cells(shape) -> np.ndarray:
    rng = np.random.default_rng(SAMPLE_SEED)
    return np.sort(rng.choice(int(np.prod(shape)), size=NSAMPLE, replace=False)).astype(np.int64)


def extract(xi: np.ndarray, shape, idx, focus):
    F = xi.shape[0]
    flat = xi.reshape(F, -1)
    out = dict(samples=flat[:, idx].copy())
    i0, i1, i2 = focus
    out["pencil0"] = xi[:, :, i1, i2].copy()
    out["pencil1"] = xi[:, i0, :, i2].copy()
    out["pencil2"] = xi[:, i0, i1, :].copy()
    out["norm2"] = np.array([np.vdot(flat[f], flat[f]).real for f in range(F)])
    out["fabs_max"] = np.array([np.abs(flat[f]).max() for f in range(F)])
    return out


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["random128", "shell256"])
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--chunk", type=int, default=200)
    ap.add_argument("--budget-hours", type=float, default=1e9)
    ap.add_argument("--max-iters", type=int, default=0,
                    help="stop after this many iterations in all (0: no cap)")
    ap.add_argument("--ckpt-dir", default=None,
                    help="directory for the resumable checkpoint (default: none)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()

    prob, focus = problem(a.workload)
    shape = prob.shape
    out_path = a.out or os.path.join(HERE, f"oracle_{a.workload}.npz")
    ck_state = ck_meta = None
    if a.ckpt_dir:
        os.makedirs(a.ckpt_dir, exist_ok=True)
        ck_state = os.path.join(a.ckpt_dir, f"{a.workload}_x.npy")
        ck_meta = os.path.join(a.ckpt_dir, f"{a.workload}_meta.json")

    m = orc.OracleMedium(shape, prob.dx, prob.omega, prob.c, prob.rho, prob.alpha,
                         pml=prob.pml_cells)
    shat = m.source_hat(m.pressure_source(prob.dense_source()))
    sc = m.scalars()
    lam = np.array([sc["lam1"]] * 3 + [sc["lam2"]])
    root = np.sqrt(lam).reshape(4, 1, 1, 1)

    iters, rel, x0 = 0, float("inf"), None
    if ck_state and os.path.exists(ck_state) and os.path.exists(ck_meta):
        meta = json.load(open(ck_meta))
        iters, rel = int(meta["iterations"]), float(meta["rel_update"])
        x0 = np.load(ck_state)
        print(f"resuming {a.workload} at iteration {iters} (rel update {rel:.3e})", flush=True)

    t_end = time.time() + a.budget_hours * 3600.0
    xi = None if x0 is None else x0 / root
    while rel > a.tol and time.time() < t_end and (a.max_iters <= 0 or iters < a.max_iters):
        t0 = time.time()
        chunk = a.chunk if a.max_iters <= 0 else min(a.chunk, a.max_iters - iters)
        xi, info = m.solve(shat, tol=a.tol, max_iter=chunk, x0=x0)
        iters += info["iterations"]
        rel = info["rel_update"]
        x0 = xi * root                                  # scaled state x = C^{1/2} xi
        if ck_state:
            np.save(ck_state + ".tmp.npy", x0)
            os.replace(ck_state + ".tmp.npy", ck_state)
            with open(ck_meta + ".tmp", "w") as f:
                json.dump(dict(iterations=iters, rel_update=rel), f)
            os.replace(ck_meta + ".tmp", ck_meta)
        print(f"{a.workload}: {iters} iterations, rel update {rel:.3e}, "
              f"{(time.time() - t0) / max(info['iterations'], 1):.2f} s/iteration", flush=True)
        if info["converged"]:
            break

    res = m.rel_residual(shat, xi)
    idx = sample_cells(shape)
    data = extract(xi, shape, idx, focus)
    np.savez_compressed(out_path, idx=idx, focus=np.array(focus), iterations=iters,
                        rel_update=rel, rel_residual=res, tol=a.tol, converged=bool(rel <= a.tol),
                        scalars=np.array([sc["a1"], sc["a2"], sc["lam1"], sc["lam2"]]),
                        workload=a.workload, **data)
    print(f"wrote {out_path}: {iters} iterations, rel update {rel:.3e}, "
          f"scaled residual {res:.3e}", flush=True)


if __name__ == "__main__":
    main()
