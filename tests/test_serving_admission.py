"""Admission policy of the request server (CPU only: the policy needs no
device).  Sizes are abstract byte counts: a medium costs ``med[shape]`` and
a shape's pool workspace ``ws[shape]``."""
import dataclasses

from paper_2507_16087_amd.serve import Admission

MED = {"S": 1, "M": 4, "L": 20}
WS = {"S": 10, "M": 30, "L": 100}


@dataclasses.dataclass
class Req:
    rid: int
    shape: str
    arrival: float


def _adm(budget, slots=2, max_wait=5.0):
    return Admission(budget, slots, max_wait, MED.__getitem__, WS.__getitem__)


def test_full_pool_does_not_block_other_shapes():
    a = _adm(1000, slots=1)
    pend = [Req(0, "L", 0.0), Req(1, "L", 0.1), Req(2, "S", 0.2)]
    adm, fail, ev = a.select(pend, 0.3)
    assert [r.rid for r in adm] == [0, 2] and not fail and not ev
    # request 1 waits for its pool's slot; a later M is still admitted
    adm, _, _ = a.select([pend[1], Req(3, "M", 0.4)], 0.5)
    assert [r.rid for r in adm] == [3]
    a.release("L")
    adm, _, _ = a.select([pend[1]], 0.6)
    assert [r.rid for r in adm] == [1]


def test_same_shape_keeps_arrival_order():
    a = _adm(1000, slots=1)
    adm, _, _ = a.select([Req(0, "M", 0.0), Req(1, "M", 0.1), Req(2, "M", 0.2)], 0.3)
    assert [r.rid for r in adm] == [0]
    a.release("M")
    adm, _, _ = a.select([Req(2, "M", 0.2), Req(1, "M", 0.1)][::-1], 0.4)
    assert [r.rid for r in adm] == [1]


def test_request_that_can_never_fit_fails():
    a = _adm(110)                      # L needs 20 + 100 > 110 even alone
    adm, fail, _ = a.select([Req(0, "L", 0.0), Req(1, "S", 0.0)], 0.1)
    assert [r.rid for r in fail] == [0] and [r.rid for r in adm] == [1]
    assert a.used == MED["S"] + WS["S"]


def test_memory_blocked_shape_does_not_block_smaller_ones():
    a = _adm(135, slots=4)             # L pool + one L medium = 120
    adm, _, _ = a.select([Req(0, "L", 0.0)], 0.0)
    assert [r.rid for r in adm] == [0] and a.used == 120
    # a second L needs 20 more (140 > 135) and waits; S (pool 10 + medium 1) fits
    adm, _, _ = a.select([Req(1, "L", 0.1), Req(2, "S", 0.2)], 0.3)
    assert [r.rid for r in adm] == [2] and a.memory_waits == 1


def test_idle_pool_gives_back_its_workspace():
    a = _adm(125, slots=2)
    adm, _, _ = a.select([Req(0, "M", 0.0)], 0.0)      # M pool: 34
    assert adm and a.used == 34
    a.release("M")                                    # M pool idle, workspace 30 still held
    assert a.used == 30
    adm, fail, ev = a.select([Req(1, "L", 1.0)], 1.0)   # L needs 120: close the idle M pool
    assert [r.rid for r in adm] == [1] and ev == ["M"] and a.evictions == 1
    assert a.used == 120 and "M" not in a.pools


def test_busy_pool_is_not_evicted():
    a = _adm(125, slots=2)
    a.select([Req(0, "M", 0.0)], 0.0)
    adm, fail, ev = a.select([Req(1, "L", 1.0)], 1.0)
    assert not adm and not fail and not ev


def test_long_wait_on_memory_stops_later_admissions():
    a = _adm(139, slots=4, max_wait=2.0)
    a.select([Req(0, "L", 0.0)], 0.0)                  # used 120
    late = Req(1, "L", 0.5)                           # needs 20 more: 140 > 139, waits
    small = Req(2, "S", 0.6)                          # needs 11: 131 <= 139
    adm, _, _ = a.select([late, small], 1.0)          # late has waited 0.5 s only
    assert [r.rid for r in adm] == [2]
    a.release("S")                                    # used 130 (S pool stays open)
    small2 = Req(3, "S", 3.0)                         # needs 1: would fit
    adm, _, _ = a.select([late, small2], 3.0)         # late has waited 2.5 s > 2 s: S waits
    assert not adm
    a.release("L")                                    # used 110: late fits, then S
    adm, _, _ = a.select([late, small2], 3.1)
    assert [r.rid for r in adm] == [1, 3]


def test_release_returns_medium_bytes():
    a = _adm(1000, slots=3)
    a.select([Req(0, "S", 0.0), Req(1, "S", 0.0), Req(2, "M", 0.0)], 0.0)
    assert a.used == 2 * MED["S"] + WS["S"] + MED["M"] + WS["M"]
    for s in ("S", "S", "M"):
        a.release(s)
    assert a.used == WS["S"] + WS["M"]
    assert a.pools["S"].reserved == 0 and a.pools["M"].reserved == 0
