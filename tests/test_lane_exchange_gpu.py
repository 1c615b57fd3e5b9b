"""GPU parity of the lane-exchange kernels (x neighbours moved across the
wave's lanes, no LDS): the one-iteration 3-D star march and the 3-D box
max/min filter.

Both evaluate exactly what the LDS marches evaluate (the star sums the same
taps in the same order; a filter picks one window element), so each case is
checked bitwise against the LDS march and, through the shared helpers, against
the FP64 oracle (1e-12 normwise for FP64, the per-point rounding bound for
FP32/BF16, bitwise for filters).
"""
import numpy as np
import pytest

import oracle as O
import test_linear_gpu as L
from closed_forms import diffusion_star_exact

torch = pytest.importorskip("torch")
import paper_2406_08923_amd as S  # noqa: E402

pytestmark = pytest.mark.gpu

DPP = 1 << 17           # lane-exchange bit of the STAR3D flag word
XCD, YFIRST = 1, 4
PF3 = 3 << 4            # three planes in flight
LDS_ONE = (4, 2, 8, 0x221)  # one-iteration LDS march

STAR_TILES = [(4, 2, 8, DPP | XCD), (8, 4, 5, DPP | XCD | YFIRST), (4, 4, 64, DPP),
              (8, 2, 13, DPP | XCD), (8, 2, 16, DPP | XCD | PF3), (4, 4, 7, DPP | PF3)]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("tile", STAR_TILES)
@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("dtype", L.DTYPES)
def test_star_lane_exchange_matches_oracle_and_lds_march(dtype, r, tile):
    # 70 columns: two tile columns of 64 - 2r outputs, the second ragged;
    # ragged rows and z chunks; asymmetric taps catch a swapped shift
    dims = (70, 37, 29)
    g = L.rand_star(r, 30 + r) * (0.3 if r > 2 else 1.0)
    plan = L.run_case(dims, r, g, dtype, S.STAR3D, tile=tile)
    assert plan.variant == S.STAR3D and plan.tile[3] & DPP
    for iters in (1, 3):
        got, _, _ = L.run_star_iters(dims, r, g, dtype, tile, iters)
        ref, _, _ = L.run_star_iters(dims, r, g, dtype, LDS_ONE, iters)
        assert np.array_equal(got, ref), (tile, iters)


@pytest.mark.parametrize("dims,r", [((3, 3, 3), 3), ((5, 4, 7), 3), ((58, 9, 4), 3),
                                    ((59, 9, 4), 3), ((1, 1, 1), 1), ((130, 2, 3), 1)])
def test_star_lane_exchange_tiny_and_edge_grids(dims, r):
    # n < 2r (images on both sides), exactly one tile column (58 = 64 - 2r)
    # and one past it, single columns
    g = L.rand_star(r, 2)
    for tile in ((4, 2, 2, DPP | XCD), (8, 4, 3, DPP), (4, 2, 5, DPP | PF3)):
        L.run_case(dims, r, g, S.F64, S.STAR3D, tile=tile)
        got, _, _ = L.run_star_iters(dims, r, g, S.F64, tile, 2)
        ref, _, _ = L.run_star_iters(dims, r, g, S.F64, LDS_ONE, 2)
        assert np.array_equal(got, ref), (dims, tile)


def test_star_lane_exchange_chained_diffusion():
    g = diffusion_star_exact(3, 3, 0.2)
    L.run_case((40, 33, 21), 3, g, S.F64, S.STAR3D, tile=(4, 4, 16, DPP | XCD), iters=7)


def test_star_lane_exchange_user_halo():
    # non-periodic: the caller's halo is read, only the interior written
    dims, r = (45, 26, 17), 3
    g = L.rand_star(3, 4)
    rng = np.random.default_rng(12)
    a_host = rng.uniform(-1, 1, O.padded_shape(dims, r))
    plan = S.LinearPlan(dims, r, g, bc=S.USER_HALO, variant=S.STAR3D, tile=(8, 2, 8, DPP | XCD))
    b = plan.empty(fill=123.0)
    plan.apply(L.dev(a_host, S.F64), b, 1)
    got = L.host(b)
    L.assert_close(O.interior(got, r), O.interior(O.xcorr(a_host, r, g), r), S.F64)
    mask = np.ones(got.shape, bool)
    O.interior(mask, r)[...] = False
    assert np.all(got[mask] == 123.0)


def test_star_lane_exchange_pitched_layout():
    # interior rows starting on a 128-byte boundary, rows longer than needed
    dims, r = (70, 21, 19), 3
    g = L.rand_star(3, 8)
    got, _, inner = L.run_star_iters(dims, r, g, S.F64, (8, 2, 8, DPP | XCD), 3,
                                     layout=(96, 16))
    ref, _, _ = L.run_star_iters(dims, r, g, S.F64, LDS_ONE, 3, layout=(96, 16))
    assert np.array_equal(got, ref)


def test_star_lane_exchange_validation():
    g = diffusion_star_exact(3, 3, 0.1)
    with pytest.raises(S.StencilError):  # one iteration per launch only
        S.LinearPlan((64, 64, 64), 3, g, variant=S.STAR3D, tile=(4, 2, 8, DPP | 0x2000))
    with pytest.raises(S.StencilError):  # not with the cached march
        S.LinearPlan((64, 64, 64), 3, g, variant=S.STAR3D, tile=(4, 2, 8, DPP | 0x8))
    p = S.LinearPlan((64, 64, 64), 3, g, variant=S.STAR3D, tile=(4, 3, 8, DPP))
    a, b = p.empty(0.0), p.empty(0.0)
    with pytest.raises(S.StencilError):  # (4, 3) is not a built shape
        p.apply(a, b, 1)
    p = S.LinearPlan((64, 64, 64), 1, np.ones((3, 3, 3)), op=S.OP_MAX, variant=S.STAR3D,
                     tile=(4, 4, 8, DPP | (4 << 4)))
    a, b = p.empty(0.0), p.empty(0.0)
    with pytest.raises(S.StencilError):  # prefetch depth 4 is not built
        p.apply(a, b, 1)


@pytest.mark.parametrize("op", [S.OP_MAX, S.OP_MIN])
@pytest.mark.parametrize("r", [1, 2, 3])
@pytest.mark.parametrize("tile", [(4, 2, 16, DPP | XCD), (8, 4, 5, DPP), (4, 4, 64, DPP | XCD),
                                  (8, 2, 7, DPP | XCD | PF3), (4, 2, 32, DPP | PF3)])
@pytest.mark.parametrize("dtype", L.DTYPES)
def test_box_filter_lane_exchange_bit_exact(dtype, op, r, tile):
    dims = (70, 33, 21)
    mask = np.ones((2 * r + 1,) * 3)
    got, ref, plan, res = L.run_filter(dims, r, mask, op, dtype, variant=S.STAR3D, tile=tile)
    assert plan.variant == S.STAR3D and plan.tile[3] & DPP
    assert L.same_bits(got, ref)
    assert np.array_equal(res, O.fill_periodic(res.copy(), r))
    lds, _, _, _ = L.run_filter(dims, r, mask, op, dtype, variant=S.STAR3D, tile=(4, 0, 16, 0))
    assert L.same_bits(got, lds)


@pytest.mark.parametrize("op", [S.OP_MAX, S.OP_MIN])
def test_box_filter_lane_exchange_signed_zeros_nan_user_halo(op):
    dims, r = (40, 20, 12), 1
    rng = np.random.default_rng(5)
    inner = rng.choice(np.array([-0.0, 0.0, -1.0, 1.0]), size=dims[::-1])
    inner[5, 7, 9] = np.nan
    got, ref, _, _ = L.run_filter(dims, r, np.ones((3, 3, 3)), op, S.F64, variant=S.STAR3D,
                                  tile=(4, 2, 8, DPP | XCD), inner=inner)
    assert L.same_bits(got, ref)
    assert int(np.isnan(got).sum()) == 27
    a_host = np.random.default_rng(13).uniform(-1, 1, O.padded_shape((45, 26, 17), 2))
    mask = np.ones((5, 5, 5))
    plan = S.LinearPlan((45, 26, 17), 2, mask, bc=S.USER_HALO, variant=S.STAR3D,
                        tile=(8, 2, 8, DPP | XCD), op=op)
    b = plan.empty(fill=123.0)
    plan.apply(L.dev(a_host, S.F64), b, 1)
    out = L.host(b)
    code = O.FILTER_MAX if op == S.OP_MAX else O.FILTER_MIN
    want = O.filter(a_host, 2, mask, code)
    assert np.array_equal(O.interior(out, 2), O.interior(want, 2))


# ---------------------------------------------------------------------------
# dense radius-1 box (BOX3D): z march with a ring of partial sums, x taps by
# lane exchange; not bitwise any other kernel (its own summation order), so
# checked against the oracle only
# ---------------------------------------------------------------------------

def rand_box(seed, r_pad=1):
    rng = np.random.default_rng(seed)
    k = 2 * r_pad + 1
    g = np.zeros((k, k, k))
    g[r_pad - 1:r_pad + 2, r_pad - 1:r_pad + 2, r_pad - 1:r_pad + 2] = rng.uniform(0.2, 1.0, (3, 3, 3)) * \
        rng.choice([-1.0, 1.0], (3, 3, 3))
    return g


BOX_TILES = [None, (4, 2, 16, XCD), (8, 1, 5, 0), (4, 1, 64, XCD | PF3), (8, 2, 7, XCD | PF3)]


@pytest.mark.parametrize("tile", BOX_TILES)
@pytest.mark.parametrize("dtype", L.DTYPES)
def test_dense_box_matches_oracle(dtype, tile):
    dims = (70, 37, 29)  # two tile columns of 62, ragged rows and z chunks
    g = rand_box(40) * 0.1
    plan = L.run_case(dims, 1, g, dtype, S.BOX3D if tile else S.VARIANT_AUTO, tile=tile)
    assert plan.variant == S.BOX3D


def test_dense_box_chained_and_wider_padding():
    L.run_case((45, 26, 17), 1, rand_box(41) * 0.05, S.F64, S.BOX3D, tile=(4, 2, 8, XCD), iters=5)
    # radius-1 taps in radius-2 padding
    plan = L.run_case((40, 20, 12), 2, rand_box(42, r_pad=2) * 0.1, S.F64, S.VARIANT_AUTO)
    assert plan.variant == S.BOX3D


@pytest.mark.parametrize("dims", [(3, 3, 3), (1, 1, 1), (62, 5, 4), (63, 5, 4), (2, 70, 9)])
def test_dense_box_tiny_and_edge_grids(dims):
    for tile in ((4, 1, 2, XCD), (8, 2, 3, PF3)):
        L.run_case(dims, 1, rand_box(43), S.F64, S.BOX3D, tile=tile)


def test_dense_box_user_halo_and_choice():
    dims = (45, 26, 17)
    g = rand_box(44)
    rng = np.random.default_rng(14)
    a_host = rng.uniform(-1, 1, O.padded_shape(dims, 1))
    plan = S.LinearPlan(dims, 1, g, bc=S.USER_HALO)
    assert plan.variant == S.BOX3D
    b = plan.empty(fill=123.0)
    plan.apply(L.dev(a_host, S.F64), b, 1)
    got = L.host(b)
    L.assert_close(O.interior(got, 1), O.interior(O.xcorr(a_host, 1, g), 1), S.F64)
    mask = np.ones(got.shape, bool)
    O.interior(mask, 1)[...] = False
    assert np.all(got[mask] == 123.0)
    g2 = g.copy()
    g2[0, 0, 0] = 0.0  # not every tap: the gather kernel
    assert S.LinearPlan(dims, 1, g2).variant == S.GENERIC
    with pytest.raises(S.StencilError):
        S.LinearPlan(dims, 1, g2, variant=S.BOX3D)
    with pytest.raises(S.StencilError):
        S.LinearPlan(dims, 1, diffusion_star_exact(3, 1, 0.1), variant=S.BOX3D)
