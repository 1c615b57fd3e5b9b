"""Pins of the oracle's window filters (max filtering, Sec. 2.3; median
filtering, Sec. 1) against routines that share nothing with it: scipy's rank
filters with periodic wrap, a NumPy brute force over rolled copies, and
special cases (duality, signed zeros, NaN confinement, spike removal)."""
import numpy as np
import pytest
from scipy import ndimage

import oracle as O
from paper_2406_08923_amd import inputs


def star_mask(ndim, r):
    m = np.zeros((2 * r + 1,) * ndim)
    for a in range(ndim):
        for k in range(2 * r + 1):
            idx = [r] * ndim
            idx[a] = k
            m[tuple(idx)] = 1.0
    return m


def box_mask(ndim, r):
    return np.ones((2 * r + 1,) * ndim)


def custom_mask(ndim, r, seed):
    rng = np.random.default_rng(seed)
    m = (rng.uniform(size=(2 * r + 1,) * ndim) < 0.5).astype(float)
    m[(r,) * ndim] = 1.0
    if int(m.sum()) % 2 == 0:  # odd count: scipy's median is the middle one
        flat = m.reshape(-1)
        flat[np.flatnonzero(flat == 0)[0]] = 1.0
    return m


def brute(f, r, mask, reduce):
    """Interior filter by stacking periodic shifts: out[p] = reduce over s in
    window of f[p + s] (np.roll by -s brings f[p + s] to p)."""
    nd = f.ndim
    offs = [np.array(k) - r for k in np.argwhere(mask != 0)]  # [sz, sy, sx] order
    stack = np.stack([np.roll(f, tuple(-o), axis=tuple(range(nd))) for o in offs])
    return reduce(stack)


CASES = [((40,), 3), ((17, 23), 2), ((9, 8, 11), 1), ((12, 7, 6), 2)]


@pytest.mark.parametrize("n,r", CASES)
@pytest.mark.parametrize("shape", ["box", "star", "custom"])
def test_filters_match_scipy_rank_filters_with_wrap(n, r, shape):
    nd = len(n)
    f = inputs.uniform_field(n, 3)
    mask = {"box": box_mask(nd, r), "star": star_mask(nd, r),
            "custom": custom_mask(nd, r, 4)}[shape]
    pad = O.pad_periodic(f, r)
    fp = mask.astype(bool)
    cases = [(O.FILTER_MAX, ndimage.maximum_filter(f, footprint=fp, mode="wrap")),
             (O.FILTER_MIN, ndimage.minimum_filter(f, footprint=fp, mode="wrap"))]
    # scipy's one-dimensional rank-filter path does not honour holes in the
    # footprint (it disagrees with every rank of the brute force below), so
    # 1-D masks with holes are pinned by the brute force only
    if not (nd == 1 and shape == "custom"):
        cases.append((O.FILTER_MEDIAN, ndimage.median_filter(f, footprint=fp, mode="wrap")))
    for op, ref in cases:
        got = O.interior(O.filter(pad, r, mask, op), r)
        assert np.array_equal(got, ref), (op, shape)


@pytest.mark.parametrize("n,r", CASES)
def test_filters_match_brute_force_over_shifts(n, r):
    nd = len(n)
    f = inputs.uniform_field(n, 5)
    mask = custom_mask(nd, r, 9)
    m = int(mask.sum())
    pad = O.pad_periodic(f, r)
    assert np.array_equal(O.interior(O.filter(pad, r, mask, O.FILTER_MAX), r),
                          brute(f, r, mask, lambda s: s.max(axis=0)))
    assert np.array_equal(O.interior(O.filter(pad, r, mask, O.FILTER_MIN), r),
                          brute(f, r, mask, lambda s: s.min(axis=0)))
    assert np.array_equal(O.interior(O.filter(pad, r, mask, O.FILTER_MEDIAN), r),
                          brute(f, r, mask, lambda s: np.sort(s, axis=0)[(m - 1) // 2]))


def test_even_window_takes_the_lower_median():
    f = inputs.uniform_field((30, 20), 6)
    mask = np.zeros((3, 3))
    mask[1, 0] = mask[1, 1] = mask[1, 2] = mask[0, 1] = 1.0  # four cells
    got = O.interior(O.filter(O.pad_periodic(f, 1), 1, mask, O.FILTER_MEDIAN), 1)
    assert np.array_equal(got, brute(f, 1, mask, lambda s: np.sort(s, axis=0)[1]))


def test_max_min_duality_and_asymmetric_orientation():
    f = inputs.uniform_field((21, 13, 9), 7)
    r = 2
    mask = np.zeros((5, 5, 5))
    mask[2, 2, 2] = mask[2, 2, 4] = mask[4, 1, 2] = 1.0  # offsets (0,0,0) (+2,0,0) (0,-1,+2)
    mx = O.interior(O.filter(O.pad_periodic(f, r), r, mask, O.FILTER_MAX), r)
    mn = O.interior(O.filter(O.pad_periodic(-f, r), r, mask, O.FILTER_MIN), r)
    assert np.array_equal(mx, -mn)
    # orientation: out[z, y, x] = max(f[z, y, x], f[z, y, x + 2], f[z + 2, y - 1, x])
    want = np.maximum(np.maximum(f, np.roll(f, -2, axis=2)), np.roll(np.roll(f, -2, axis=0), 1, axis=1))
    assert np.array_equal(mx, want)


def test_signed_zeros_are_ordered():
    f = np.array([-0.0, 0.0, -0.0, -0.0, 0.0, -1.0, -0.0, 2.0])
    pad = O.pad_periodic(f, 1)
    mx = O.interior(O.filter(pad, 1, np.ones(3), O.FILTER_MAX), 1)
    mn = O.interior(O.filter(pad, 1, np.ones(3), O.FILTER_MIN), 1)
    # windows (periodic): [2,-0,0] [-0,0,-0] [0,-0,-0] [-0,-0,0] [-0,0,-1] [0,-1,-0] [-1,-0,2] [-0,2,-0]
    assert np.array_equal(np.signbit(mx), [False, False, False, False, False, False, False, False])
    assert list(mx) == [2.0, 0.0, 0.0, 0.0, 0.0, 0.0, 2.0, 2.0]
    assert np.array_equal(np.signbit(mn), [True, True, True, True, True, True, True, True])
    med = O.interior(O.filter(pad, 1, np.ones(3), O.FILTER_MEDIAN), 1)
    # sorted windows with -0 < +0: [-0,0,2] [-0,-0,0] [-0,-0,0] [-0,-0,0] [-1,-0,0] [-1,-0,0] [-1,-0,2] [-0,-0,2]
    assert list(med) == [0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0]
    assert list(np.signbit(med)) == [False, True, True, True, True, True, True, True]


def test_nan_stays_inside_its_windows():
    f = inputs.uniform_field((10, 9, 8), 8)
    f[4, 3, 2] = np.nan  # z, y, x
    r = 1
    for op in (O.FILTER_MAX, O.FILTER_MIN, O.FILTER_MEDIAN):
        got = O.interior(O.filter(O.pad_periodic(f, r), r, star_mask(3, r), op), r)
        nan = np.isnan(got)
        want = np.zeros_like(nan)
        for dz, dy, dx in [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]:
            want[(4 + dz) % 8, (3 + dy) % 9, (2 + dx) % 10] = True
        assert np.array_equal(nan, want), op


def test_median_removes_an_isolated_spike_and_keeps_constants():
    f = np.full((7, 8, 9), 0.25)
    f[3, 4, 5] = 100.0
    got = O.interior(O.filter(O.pad_periodic(f, 1), 1, box_mask(3, 1), O.FILTER_MEDIAN), 1)
    assert np.all(got == 0.25)
    mx = O.interior(O.filter(O.pad_periodic(f, 1), 1, box_mask(3, 1), O.FILTER_MAX), 1)
    assert int((mx == 100.0).sum()) == 27


def test_filter_at_matches_full_field():
    f = inputs.uniform_field((16, 12, 10), 2)
    pad = O.pad_periodic(f, 2)
    mask = custom_mask(3, 2, 1)
    full = O.filter(pad, 2, mask, O.FILTER_MEDIAN)
    pts = np.array([[0, 0, 0], [15, 11, 9], [3, 7, 2], [8, 0, 9]])
    got = O.filter_at(pad, 2, mask, O.FILTER_MEDIAN, pts)
    assert np.array_equal(got, full[pts[:, 2] + 2, pts[:, 1] + 2, pts[:, 0] + 2])
    with pytest.raises(ValueError):
        O.filter(pad, 2, mask, 7)
