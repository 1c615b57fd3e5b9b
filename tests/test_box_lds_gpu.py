"""GPU parity of the dense 3-D box kernel for radius 2..4 (Eq. 3 with every
tap of the (2R+1)^3 box nonzero; the LDS march of `box3d_lds.hpp`).

Each case runs through the C-ABI plan and is compared, through the shared
helpers, with the FP64 oracle: 1e-12 normwise for FP64, the per-point rounding
bound for FP32/BF16, and the output halo bitwise equal to the periodic image
of the interior. Grids span several 64-column tiles, ragged row blocks and
ragged z chunks.
"""
import numpy as np
import pytest

import oracle as O
import test_linear_gpu as L

torch = pytest.importorskip("torch")
import paper_2406_08923_amd as S  # noqa: E402

pytestmark = pytest.mark.gpu

XCD = 1


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dense_box(R, seed, r_pad=None):
    """All (2R+1)^3 taps nonzero (random sign and size), centred in a
    (2 r_pad + 1)^3 tensor; scaled so that the sum of |taps| is 1."""
    r_pad = R if r_pad is None else r_pad
    rng = np.random.default_rng(seed)
    k, K = 2 * r_pad + 1, 2 * R + 1
    taps = rng.uniform(0.2, 1.0, (K, K, K)) * rng.choice([-1.0, 1.0], (K, K, K))
    g = np.zeros((k, k, k))
    s = slice(r_pad - R, r_pad + R + 1)
    g[s, s, s] = taps / np.abs(taps).sum()
    return g


# (waves, outputs per lane, z planes per workgroup, flags)
TILES = [None, (4, 4, 16, XCD), (4, 8, 5, 0), (4, 4, 7, 0), (4, 8, 64, XCD)]


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("R", [2, 3, 4])
@pytest.mark.parametrize("dtype", L.DTYPES)
def test_dense_box_radius_2_to_4_matches_oracle(dtype, R, tile):
    dims = (130, 37, 29)  # three tile columns of 64, ragged rows and z chunks
    plan = L.run_case(dims, R, dense_box(R, 50 + R), dtype,
                      S.BOX3D if tile else S.VARIANT_AUTO, tile=tile)
    assert plan.variant == S.BOX3D
    if tile is None:  # small grid: the shallowest default z chunk
        assert plan.tile == (4, 8 if dtype != S.F64 and R == 4 else 4, 32, XCD)


@pytest.mark.parametrize("tile", [(4, 4, 16, XCD), (4, 8, 5, 0), (4, 4, 128, XCD), (8, 8, 7, XCD),
                                  (8, 4, 128, 0)])
@pytest.mark.parametrize("dtype", L.DTYPES)
def test_dense_27_point_box_on_the_lds_march_matches_oracle(dtype, tile):
    # radius 1 with 4 or 8 outputs per lane: the LDS march (outputs stored as
    # whole rows through LDS); 1 or 2 rows per lane keep the lane-exchange march
    plan = L.run_case((130, 37, 29), 1, dense_box(1, 49), dtype, S.BOX3D, tile=tile)
    assert plan.tile == tile
    for dims in ((1, 1, 1), (64, 3, 2), (65, 33, 7)):
        L.run_case(dims, 1, dense_box(1, 48), S.F64, S.BOX3D, tile=tile)


@pytest.mark.parametrize("R", [2, 3, 4])
def test_dense_box_radius_2_to_4_tiny_and_edge_grids(R):
    for dims in ((R, R, R), (64, R, R + 1), (65, 2 * R + 1, R), (R, 70, 9), (63, 33, 2 * R)):
        for tile in ((4, 4, 2, XCD), (4, 8, 3, 0)):
            L.run_case(dims, R, dense_box(R, 60 + R), S.F64, S.BOX3D, tile=tile)


def test_dense_box_radius_2_to_4_chained_and_wider_padding():
    # five chained iterations (the halo refreshed between them)
    L.run_case((45, 26, 17), 2, dense_box(2, 61), S.F64, S.BOX3D, tile=(4, 8, 8, XCD), iters=5)
    L.run_case((40, 20, 12), 3, dense_box(3, 62), S.F64, S.VARIANT_AUTO, iters=3)
    # radius-2 and radius-3 taps in radius-4 padding (the rows carry 2 * 4 halo cells)
    for R in (2, 3):
        plan = L.run_case((70, 21, 13), 4, dense_box(R, 63, r_pad=4), S.F64, S.VARIANT_AUTO)
        assert plan.variant == S.BOX3D


@pytest.mark.parametrize("R", [2, 3])
def test_dense_box_radius_2_to_4_user_halo_and_choice(R):
    dims = (70, 26, 17)
    g = dense_box(R, 70 + R)
    rng = np.random.default_rng(15)
    a_host = rng.uniform(-1, 1, O.padded_shape(dims, R))
    plan = S.LinearPlan(dims, R, g, bc=S.USER_HALO)
    assert plan.variant == S.BOX3D
    b = plan.empty(fill=123.0)
    plan.apply(L.dev(a_host, S.F64), b, 1)
    got = L.host(b)
    L.assert_close(O.interior(got, R), O.interior(O.xcorr(a_host, R, g), R), S.F64)
    mask = np.ones(got.shape, bool)
    O.interior(mask, R)[...] = False
    assert np.all(got[mask] == 123.0)  # user halo: the halo is the caller's
    g2 = g.copy()
    g2[R, R, 0] = 0.0  # one tap missing: the gather kernel
    assert S.LinearPlan(dims, R, g2).variant == S.GENERIC
    with pytest.raises(S.StencilError):
        S.LinearPlan(dims, R, g2, variant=S.BOX3D)
    with pytest.raises(S.StencilError):  # 8 waves: 2-D and 27-point boxes only
        S.LinearPlan(dims, R, g, variant=S.BOX3D, tile=(8, 4, 16, XCD))
    with pytest.raises(S.StencilError):
        S.LinearPlan(dims, R, g, variant=S.BOX3D, tile=(4, 2, 16, XCD))


def test_dense_box_radius_2_to_4_default_shape_at_512():
    # deepest z chunk that keeps 512 workgroups: 128 planes in FP64 at 512^3,
    # 64 in FP32 below radius 4 (a plan only: no launch)
    for R, dtype, want in ((2, S.F64, (4, 4, 128, XCD)), (3, S.F32, (4, 4, 64, XCD)),
                           (4, S.F32, (4, 8, 128, XCD)), (3, S.F64, (4, 4, 128, XCD))):
        assert S.LinearPlan((512, 512, 512), R, dense_box(R, 3), dtype=dtype).tile == want
    assert S.LinearPlan((256, 256, 256), 3, dense_box(3, 3)).tile == (4, 4, 32, XCD)
    # the 27-point box: eight outputs per lane in FP64, four in FP32
    assert S.LinearPlan((512, 512, 512), 1, dense_box(1, 3)).tile == (8, 8, 128, XCD)
    assert S.LinearPlan((512, 512, 512), 1, dense_box(1, 3), dtype=S.F32).tile == (4, 4, 128, XCD)


@pytest.mark.parametrize("R", [5, 6, 7, 8])
@pytest.mark.parametrize("dtype", [S.F64, S.F32])
def test_dense_box_radius_5_to_8_matches_oracle(dtype, R):
    # rings of 11 .. 17 partial sums, four outputs per lane; several z chunks
    dims = (70, 21, 19)
    for tile in (None, (4, 4, 7, 0)):
        plan = L.run_case(dims, R, dense_box(R, 80 + R), dtype,
                          S.BOX3D if tile else S.VARIANT_AUTO, tile=tile)
        assert plan.variant == S.BOX3D
    with pytest.raises(S.StencilError):  # eight outputs per lane are not built here
        S.LinearPlan(dims, R, dense_box(R, 80 + R), variant=S.BOX3D, tile=(4, 8, 16, XCD))


def test_dense_box_radius_2_to_4_autotune_candidates_match_the_oracle():
    # every candidate the plan-time search may pick gives oracle results: run
    # the search, then each built shape explicitly
    dims = (96, 40, 40)
    g = dense_box(3, 90)
    plan = L.run_case(dims, 3, g, S.F64, S.VARIANT_AUTO, autotune=True)
    assert plan.variant in (S.BOX3D, S.GENERIC)
    for e in (4, 8):
        for lz in (32, 64, 128):
            L.run_case(dims, 3, g, S.F64, S.BOX3D, tile=(4, e, lz, XCD))


# ---------------------------------------------------------------------------
# dense 2-D boxes (radius 1..4): the same LDS march over one plane
# ---------------------------------------------------------------------------

def dense_box2(R, seed, r_pad=None):
    r_pad = R if r_pad is None else r_pad
    rng = np.random.default_rng(seed)
    k, K = 2 * r_pad + 1, 2 * R + 1
    taps = rng.uniform(0.2, 1.0, (K, K)) * rng.choice([-1.0, 1.0], (K, K))
    g = np.zeros((k, k))
    s = slice(r_pad - R, r_pad + R + 1)
    g[s, s] = taps / np.abs(taps).sum()
    return g


@pytest.mark.parametrize("tile", [None, (4, 4, 1, XCD), (4, 8, 1, 0), (4, 4, 3, XCD), (4, 8, 16, 0),
                                  (8, 8, 2, XCD)])
@pytest.mark.parametrize("R", [1, 2, 3, 4, 6, 8])
@pytest.mark.parametrize("dtype", L.DTYPES)
def test_dense_2d_box_matches_oracle(dtype, R, tile):
    # three tile columns of 64, ragged row blocks; a workgroup walks 1, 3 or
    # 16 blocks of rows (more than the grid holds in the last case)
    dims = (130, 77)
    plan = L.run_case(dims, R, dense_box2(R, 20 + R), dtype,
                      S.BOX3D if tile else S.VARIANT_AUTO, tile=tile)
    assert plan.variant == S.BOX3D
    if tile is None:
        assert plan.tile == (8, 4, 1, XCD)


@pytest.mark.parametrize("R", [1, 2, 3, 4])
def test_dense_2d_box_tiny_edge_chained_and_wider_padding(R):
    for dims in ((R, R), (64, R), (65, 2 * R + 1), (R, 70), (200, 33)):
        for tile in ((4, 4, 1, XCD), (4, 8, 2, 0), (4, 4, 5, XCD), (8, 4, 1, XCD), (8, 8, 3, 0)):
            L.run_case(dims, R, dense_box2(R, 30 + R), S.F64, S.BOX3D, tile=tile)
    L.run_case((70, 45), R, dense_box2(R, 31 + R), S.F64, S.VARIANT_AUTO, iters=3)
    plan = L.run_case((66, 40), 6, dense_box2(R, 32 + R, r_pad=6), S.F64, S.VARIANT_AUTO)
    assert plan.variant == S.BOX3D


def test_dense_2d_box_user_halo_and_choice():
    dims, R = (90, 41), 3
    g = dense_box2(R, 40)
    rng = np.random.default_rng(16)
    a_host = rng.uniform(-1, 1, O.padded_shape(dims, R))
    plan = S.LinearPlan(dims, R, g, bc=S.USER_HALO)
    assert plan.variant == S.BOX3D
    b = plan.empty(fill=123.0)
    plan.apply(L.dev(a_host, S.F64), b, 1)
    got = L.host(b)
    L.assert_close(O.interior(got, R), O.interior(O.xcorr(a_host, R, g), R), S.F64)
    mask = np.ones(got.shape, bool)
    O.interior(mask, R)[...] = False
    assert np.all(got[mask] == 123.0)
    g2 = g.copy()
    g2[0, R] = 0.0  # a star-free box with one tap missing: the gather kernel
    assert S.LinearPlan(dims, R, g2).variant == S.GENERIC
    assert S.LinearPlan(dims, 8, dense_box2(8, 41)).variant == S.BOX3D
    # default: one block of 32 rows per workgroup
    assert S.LinearPlan((16384, 16384), 2, dense_box2(2, 42)).tile == (8, 4, 1, XCD)
    # 2-D arrays of 4 GiB or more stay on the gather kernel
    big = S.LinearPlan((1 << 15, 1 << 14), 2, dense_box2(2, 43))
    assert big.variant == S.GENERIC
    with pytest.raises(S.StencilError):
        S.LinearPlan((1 << 15, 1 << 14), 2, dense_box2(2, 43), variant=S.BOX3D)
