"""Tuned pass sets kept across processes in the file CBS_TUNE_FILE names.

* A shape no other test tunes: its first solve tunes and appends one line
  whose pass set is the one the medium reports.
* Another fresh shape with a line written by hand (a different propagator
  layout, and two column blocks where they fit): the solve takes that set
  as it stands, and its FP64 iterates still equal the oracle's.
* A line that does not fit its shape is ignored, and the solve tunes.
"""
import numpy as np
import pytest

from paper_2507_16087_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

DX, OMEGA = 2.5e-4, 2 * np.pi * 1e6
PINS = ("CBS_PROP_VARIANT", "CBS_LAST_VARIANT", "CBS_STRIDED_VARIANT", "CBS_COLUMN_BLOCKS", "CBS_AUTOTUNE")
AXIS = {0: 2, 1: 2, 2: 1, 3: 1, 4: 0}     # axis of each pass kind on a 3-D grid


@pytest.fixture
def cbs(monkeypatch, tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    for k in PINS:
        monkeypatch.delenv(k, raising=False)
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("CBS_TUNE_FILE", str(path))
    from paper_2507_16087_amd import solver
    return solver, path


def _prefix(shape):
    return f"cbs-tune-v1 gfx950 3 {shape[0]} {shape[1]} {shape[2]} 1 -1 -1 -1 -1 "


def _line(shape, plans, blocks):
    parts = [_prefix(shape) + f"{len(plans)} {blocks}"]
    for p in plans:
        parts.append(f"{p['kind']} {AXIS[p['kind']]} {p['n']} {p['cols']} {p['wide']} {p['variant']}")
    return " ".join(parts) + "\n"


def _solve_pair(orc, cbs, shape, seed):
    c, rho, alpha = W.small_random(shape, seed)
    om = orc.OracleMedium(shape, DX, OMEGA, c, rho, alpha, pml=2)
    gm = cbs.Medium(shape, DX, OMEGA, c, rho, alpha, pml=2)
    return om, gm


def _check_iterates(om, gm, cbs, shape):
    s = np.zeros((4,) + shape, complex)
    s.reshape(4, -1)[-1, [5, 300]] = [1.0, 0.5j]
    xi, _ = om.solve(om.source_hat(s), tol=0.0, max_iter=12)
    p, u, _ = cbs.solve(gm, s[-1], s[:-1], tol=0.0, max_iter=12)
    rel = lambda a, b: np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))
    assert rel(p, xi[-1]) <= 1e-10 and rel(u, xi[:-1]) <= 1e-10


def test_first_solve_appends_its_line(orc, cbs):
    solver, path = cbs
    shape = (24, 16, 32)
    om, gm = _solve_pair(orc, solver, shape, 41)
    _check_iterates(om, gm, solver, shape)
    lines = [ln for ln in path.read_text().splitlines() if ln.startswith(_prefix(shape))]
    assert len(lines) == 1
    plans = gm.pass_config("fp64")
    assert lines[0] + "\n" == _line(shape, plans, plans[1]["blocks"])


def test_line_written_by_hand_is_used(orc, cbs):
    solver, path = cbs
    shape = (32, 24, 16)
    om, gm = _solve_pair(orc, solver, shape, 42)
    plans = gm.pass_config("fp64")            # untuned defaults before the first solve
    prop = next(p for p in plans if p["kind"] == 4)
    prop["variant"] = 5 if prop["variant"] != 5 else 2
    lw = shape[-1] // 2
    blocks = 2 if all(lw % p["cols"] == 0 for p in plans if p["kind"] in (2, 3, 4)) else 1
    path.write_text(_line(shape, plans, blocks))
    _check_iterates(om, gm, solver, shape)
    got = gm.pass_config("fp64")
    want = [dict(p, blocks=(blocks if p["kind"] in (2, 3, 4) else 1)) for p in plans]
    assert got == want
    assert len(path.read_text().splitlines()) == 1     # nothing appended: no tuning ran


def test_line_that_does_not_fit_is_ignored(orc, cbs):
    solver, path = cbs
    shape = (16, 32, 24)
    om, gm = _solve_pair(orc, solver, shape, 43)
    plans = gm.pass_config("fp64")
    bad = [dict(p) for p in plans]
    bad[0]["cols"] = 3                         # not a power of two
    path.write_text(_line(shape, bad, 1))
    _check_iterates(om, gm, solver, shape)
    assert gm.pass_config("fp64")[0]["cols"] != 3
    assert len(path.read_text().splitlines()) == 2     # the tuned line was appended
