"""Pins of the oracle's absorbing-layer profile and median shift (CPU only).

The paper fixes neither: it says only that the absorbing rate gamma enforces
an absorbing layer and is generated algorithmically, evaluated at the
staggered points on the staggered grid (Sec. 2.1, App. B.1), and Algorithm 1's
preprocessing names the median as one choice of the complex shifts.  The
readings taken:

* layer: gamma(x) = gmax * sum_eta r_eta(x_eta)^2, where r is the distance of
  the position (cell index; staggered points at index + 1/2) from the
  interior interval [L, N-1-L] measured around the periodic grid, divided by
  L + 1/2; gmax = omega unless given; no layer for L = 0.  The velocity row
  eta takes the same formula with x_eta + 1/2 on its own axis (cell centres on
  the collocated grid).
* median shift: a1 = median(Re D_u) + i median(Im D_u) over the values of all
  ndim velocity planes, a2 likewise over D_p; an even count takes the mean of
  the two middle values.

The layer is pinned against hand-worked tables of the distance and against a
NumPy statement that measures the periodic distance differently (minimum over
the three periodic images of the interval); the median against numpy.median
of the diagonal values built from c, rho, alpha in NumPy.
"""
import numpy as np
import pytest

from paper_2507_16087_amd import workloads as W

OMEGA = 2 * np.pi * 1e6
DX = 0.25e-3

# Distance to the interior, in cells, worked out by hand for two small axes.
# N = 10, L = 3: interior [3, 6]; the seam lies between cells 9 and 0, whose
# midpoint 9.5 is 3.5 cells from both ends of the interior.
HAND_10_3 = dict(centre=[3, 2, 1, 0, 0, 0, 0, 1, 2, 3],
                 stag=[2.5, 1.5, 0.5, 0, 0, 0, 0.5, 1.5, 2.5, 3.5])
# N = 9, L = 2 (odd length): interior [2, 6].  Cell 8 is 2 cells from the
# interior's upper end and 3 (through the seam) from its lower end.
HAND_9_2 = dict(centre=[2, 1, 0, 0, 0, 0, 0, 1, 2],
                stag=[1.5, 0.5, 0, 0, 0, 0, 0.5, 1.5, 2.5])


def _uniform(shape):
    one = np.ones(shape)
    return 1500.0 * one, 1000.0 * one, np.zeros(shape)


def _r_images(t, n, L):
    """Distance of positions t from [L, n-1-L] on a ring of length n, as the
    smallest distance to any of the interval's three nearest periodic copies,
    over L + 1/2."""
    if L == 0:
        return np.zeros_like(t, dtype=float)
    t = np.asarray(t, dtype=float)
    best = np.full(t.shape, np.inf)
    for m in (-1, 0, 1):
        lo, hi = L + m * n, n - 1 - L + m * n
        d = np.maximum(0.0, np.maximum(lo - t, t - hi))
        best = np.minimum(best, d)
    return best / (L + 0.5)


@pytest.mark.parametrize("n,L,hand", [(10, 3, HAND_10_3), (9, 2, HAND_9_2)])
def test_layer_profile_hand_tables_1d(orc, n, L, hand):
    c, rho, alpha = _uniform((n,))
    gmax = 1.7e6
    m = orc.OracleMedium((n,), DX, OMEGA, c, rho, alpha, pml=L, gmax=gmax)
    f = m.fields()
    rc = np.array(hand["centre"], float) / (L + 0.5)
    rs = np.array(hand["stag"], float) / (L + 0.5)
    np.testing.assert_allclose(f["gamma"], gmax * rc ** 2, rtol=1e-15, atol=0)
    np.testing.assert_allclose(f["gamma_s"][0], gmax * rs ** 2, rtol=1e-15, atol=0)
    # the staggered point on the seam carries the full rate, r = 1
    assert f["gamma_s"][0][-1] == pytest.approx(gmax, rel=1e-15)
    # the second statement of the reading agrees with the hand tables
    np.testing.assert_allclose(_r_images(np.arange(n), n, L), rc, rtol=0, atol=1e-15)
    np.testing.assert_allclose(_r_images(np.arange(n) + 0.5, n, L), rs, rtol=0, atol=1e-15)


@pytest.mark.parametrize("shape,L,gmax,colloc", [
    ((12, 9), 3, 0.0, False),          # odd axis, default gmax = omega
    ((7, 10, 8), 2, 2.5e6, False),     # odd axis in 3-D
    ((8, 6, 10), 0, 0.0, False),       # no layer
    ((9, 12), 4, 0.0, True),           # collocated: every field at the centres
    ((16,), 7, 0.0, False),            # layer of almost half the axis
])
def test_layer_profile_matches_reading(orc, shape, L, gmax, colloc):
    c, rho, alpha = W.small_random(shape, 11)
    m = orc.OracleMedium(shape, DX, OMEGA, c, rho, alpha, pml=L, gmax=gmax,
                         collocated=colloc)
    f = m.fields()
    g = gmax if gmax > 0 else OMEGA
    D = len(shape)
    idx = np.meshgrid(*[np.arange(n, dtype=float) for n in shape], indexing="ij")

    def gamma_at(shift_axis):
        tot = np.zeros(shape)
        for d in range(D):
            t = idx[d] + (0.5 if d == shift_axis else 0.0)
            tot += _r_images(t, shape[d], L) ** 2
        return g * tot

    np.testing.assert_allclose(f["gamma"], gamma_at(None), rtol=1e-14, atol=0)
    for e in range(D):
        want = gamma_at(None if colloc else e)
        np.testing.assert_allclose(f["gamma_s"][e], want, rtol=1e-14, atol=0)
    if L > 0:
        # r stays in [0, 1]; the staggered point on the seam of its own axis
        # has r = 1 there, so its rate is at least gmax
        assert f["gamma"].max() <= D * g * (1 + 1e-15)
        if not colloc:
            seam = tuple([0] * (D - 1) + [shape[-1] - 1])
            assert f["gamma_s"][D - 1][seam] >= g * (1 - 1e-15)
    else:
        assert not f["gamma"].any() and not f["gamma_s"].any()


def _diagonals(shape, c, rho, alpha, gam, gams):
    """D_u (ndim planes) and D_p from c, rho, alpha and the layer rates."""
    D = len(shape)
    q = (1 - 2j * alpha * c / OMEGA) / (rho * c ** 2)
    Du = np.stack([0.5 * (rho + np.roll(rho, -1, axis=e)) * (1j * OMEGA + gams[e])
                   for e in range(D)])
    Dp = (1j * OMEGA + gam) * q
    return Du, Dp


@pytest.mark.parametrize("shape,L", [
    ((9,), 2),          # D_u 9 values, D_p 9: odd counts
    ((5, 7), 1),        # D_u 70 (even), D_p 35 (odd)
    ((6, 8), 2),        # even counts
    ((4, 6, 5), 1),     # 3-D, D_u 360, D_p 120
])
@pytest.mark.parametrize("medium", ["random", "two_values"])
def test_median_shift_is_componentwise_median(orc, shape, L, medium):
    if medium == "random":
        c, rho, alpha = W.small_random(shape, 5)
    else:
        # repeated values: two materials, so the median sits on ties
        c, rho, alpha = _uniform(shape)
        half = np.zeros(shape, bool)
        half[: shape[0] // 2] = True
        c[half], rho[half] = 1800.0, 1500.0
    m = orc.OracleMedium(shape, DX, OMEGA, c, rho, alpha, pml=L, shift_rule=1)
    f = m.fields()
    Du, Dp = _diagonals(shape, c, rho, alpha, f["gamma"], f["gamma_s"])
    a1 = np.median(Du.real) + 1j * np.median(Du.imag)
    a2 = np.median(Dp.real) + 1j * np.median(Dp.imag)
    s = m.scalars()
    assert abs(s["a1"] - a1) <= 1e-14 * abs(a1)
    assert abs(s["a2"] - a2) <= 1e-14 * abs(a2)
    # the scales make max |V| = beta on each block (the layer and the
    # heterogeneity keep the radii well above the 1e-3 |a| floor here)
    assert np.abs(Du - s["a1"]).max() / s["lam1"] == pytest.approx(s["beta"], rel=1e-13)
    assert np.abs(Dp - s["a2"]).max() / s["lam2"] == pytest.approx(s["beta"], rel=1e-13)


def test_median_of_even_count_is_mean_of_middle_pair(orc):
    """A 1-D axis of 4 cells without a layer: D_p takes exactly the values of
    the cells, so the median of an even count is visible directly."""
    shape = (4,)
    c = np.array([1500.0, 1600.0, 1700.0, 1900.0])
    rho = np.full(shape, 1000.0)
    alpha = np.zeros(shape)
    m = orc.OracleMedium(shape, DX, OMEGA, c, rho, alpha, pml=0, shift_rule=1)
    dp = 1j * OMEGA / (rho * c ** 2)          # purely imaginary, no absorption
    srt = np.sort(dp.imag)
    want = 1j * 0.5 * (srt[1] + srt[2])
    assert abs(m.scalars()["a2"] - want) <= 1e-15 * abs(want)
