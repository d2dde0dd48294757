"""The curve-inclusion inputs (geometry only): the inscribed polygon of a
circle and the open square of the inclusion workload, checked against
their construction."""
import math

import numpy as np
import pytest

import hb_inputs


@pytest.fixture(scope="module")
def bump256():
    # the inclusion workload's grid, medium and frequency (that of
    # hb_inputs.configs.c4) with a minimal table, which the curves do not use
    return hb_inputs.configs.bump_problem(256, 2 * math.pi * 256 / 8, nbox=1, nI=2)


@pytest.mark.parametrize("ns", [3, 8, 257])
def test_circle_is_the_inscribed_polygon(bump256, ns):
    c, r = np.array([0.45, 0.55]), 0.2
    cv = hb_inputs.circle(bump256, c, r, ns)
    assert cv.Ns == ns
    # equal chords of the circle: length 2 r sin(pi/ns), midpoints at
    # distance r cos(pi/ns) from the centre, one per arc of 2 pi / ns
    assert np.allclose(cv.w, 2 * r * math.sin(math.pi / ns))
    d = cv.centres - c
    assert np.allclose(np.hypot(d[:, 0], d[:, 1]), r * math.cos(math.pi / ns))
    ang = np.sort(np.mod(np.arctan2(d[:, 1], d[:, 0]), 2 * math.pi))
    assert np.allclose(np.diff(ang), 2 * math.pi / ns)
    # the perimeter tends to 2 pi r from below
    assert cv.w.sum() < 2 * math.pi * r
    assert np.allclose(cv.slowness, bump256.meta["medium"].slowness(cv.centres))


def test_open_square_of_the_inclusion_workload(bump256):
    side, ppw = 0.8, 20
    cv = hb_inputs.open_square(bump256, (0.5, 0.5), side, ppw)
    wmax = 2 * math.pi / (bump256.omega * bump256.slowness.max() * ppw)
    k = math.ceil(side / wmax)
    assert cv.Ns == 3 * k == 1998                 # the count the workload is quoted with
    assert np.all(cv.w <= wmax * (1 + 1e-12))
    assert math.isclose(cv.w.sum(), 3 * side)
    x, y = cv.centres[:, 0], cv.centres[:, 1]
    lo, hi = 0.5 - side / 2, 0.5 + side / 2
    left, bottom, right = np.isclose(x, lo), np.isclose(y, lo), np.isclose(x, hi)
    assert np.all(left | bottom | right)
    assert left.sum() == bottom.sum() == right.sum() == k
    assert not np.any(np.isclose(y, hi))          # the top side is open
    # each side split evenly: centres at the midpoints of k equal pieces
    t = (np.arange(k) + 0.5) / k
    assert np.allclose(np.sort(y[left]), lo + t * side)
    assert np.allclose(np.sort(x[bottom]), lo + t * side)
    assert np.allclose(np.sort(y[right]), lo + t * side)
