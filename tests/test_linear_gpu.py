"""GPU parity of the linear path (halo, cross-correlation variants, copy)
against the CPU oracle, through the C ABI.

FP64 bar: normwise max relative error <= 1e-12 per output. FP32 / BF16 bar:
the rounding bound of the arithmetic, per point,
    |gpu - oracle| <= 2 (ntaps + 1) u32 sum_s |g_s| |f_{p+s}| + u_out |oracle|,
with u32 = 2^-24 (FP32 accumulation), u_out = 2^-24 (FP32) or 2^-8 (BF16
result rounding); inputs are exactly representable in the storage type.
"""
import math

import numpy as np
import pytest

import oracle as O
from closed_forms import diffusion_star_exact, laplacian_symbol_grid
from paper_2406_08923_amd import inputs

torch = pytest.importorskip("torch")
import paper_2406_08923_amd as S  # noqa: E402
from paper_2406_08923_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def to_storage_values(a, dtype):
    if dtype == S.F32:
        return a.astype(np.float32).astype(np.float64)
    if dtype == S.BF16:
        return inputs.to_bf16_values(a)
    return a


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda").to(S.torch_dtype(dtype))


def host(t):
    return t.to(torch.float64).cpu().numpy()


def u_out(dtype):
    return {S.F64: 2.0 ** -53, S.F32: 2.0 ** -24, S.BF16: 2.0 ** -8}[dtype]


def assert_close(gpu, ref, dtype, absconv=None, ntaps=1, what=""):
    if dtype == S.F64:
        err = np.max(np.abs(gpu - ref)) / max(np.max(np.abs(ref)), 1e-300)
        assert err <= 1e-12, "%s: normwise rel err %.3e" % (what, err)
    else:
        bound = 2 * (ntaps + 1) * 2.0 ** -24 * absconv + u_out(dtype) * np.abs(ref)
        bad = np.abs(gpu - ref) > bound
        assert not bad.any(), "%s: %d points over the bound, worst %.3e" % (
            what, int(bad.sum()), float(np.max(np.abs(gpu - ref) - bound)))


def oracle_apply(inner, r, g, iters, bc=S.PERIODIC, padded_in=None):
    if bc == S.PERIODIC:
        return O.xcorr_periodic_iterate(O.pad_periodic(inner, r), r, g, iters)
    return O.xcorr(padded_in, r, g)


def run_case(dims, r, g, dtype, variant, tile=None, iters=1, seed=1, autotune=False):
    inner = to_storage_values(inputs.uniform_field(dims, seed), dtype)
    plan = S.LinearPlan(dims, r, g, dtype=dtype, variant=variant, tile=tile, autotune=autotune)
    a_host = np.full(O.padded_shape(dims, r), 7.0)  # halo garbage: the library fills it
    O.interior(a_host, r)[...] = inner
    a = dev(a_host, dtype)
    b = plan.empty(fill=-3.0)
    res = host(plan.apply(a, b, iters))
    torch.cuda.synchronize()
    ref = oracle_apply(inner, r, g, iters)
    ntaps = int(np.count_nonzero(g))
    absconv = None
    if dtype != S.F64:
        assert iters == 1
        absconv = O.xcorr(np.abs(O.pad_periodic(inner, r)), r, np.abs(g))
    what = "%s r=%d var=%d tile=%s" % (dims, r, variant, tile)
    assert_close(O.interior(res, r), O.interior(ref, r), dtype,
                 None if absconv is None else O.interior(absconv, r), ntaps, what=what)
    # the halo written by the library is the exact periodic image of its interior
    assert np.array_equal(res, O.fill_periodic(res.copy(), r)), what + ": halo"
    return plan


# ---------------------------------------------------------------------------
# periodic halo and copy: exact
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dims,r", [((1000,), 1), ((77,), 8), ((40, 33), 3), ((5, 4), 3),
                                    ((37, 29, 23), 3), ((6, 5, 4), 4), ((64, 64, 64), 1)])
@pytest.mark.parametrize("dtype", [S.F64, S.F32, S.BF16])
def test_halo_periodic_exact(dims, r, dtype):
    inner = to_storage_values(inputs.uniform_field(dims, 3), dtype)
    pad = np.full(O.padded_shape(dims, r), np.nan)
    O.interior(pad, r)[...] = inner
    t = dev(pad, dtype)
    S.halo_periodic(t, dims, r, dtype)
    got = host(t)
    ref = O.fill_periodic(pad.copy(), r)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("nbytes", [16, 4096 + 16, 1 << 24])
def test_copy_exact(nbytes):
    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    S.copy(src, dst)
    assert torch.equal(src, dst)


# ---------------------------------------------------------------------------
# cross-correlation, small grids spanning several tiles with ragged tails
# ---------------------------------------------------------------------------

DTYPES = [S.F64, S.F32, S.BF16]


def rand_star(r, seed):
    rng = np.random.default_rng(seed)
    g = np.zeros((2 * r + 1,) * 3)
    for a in range(3):
        for m in range(-r, r + 1):
            idx = [r, r, r]
            idx[a] = r + m
            g[tuple(idx)] = rng.uniform(-1, 1)
    return g


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("tile", [(8, 2, 64, 0x120), (4, 4, 64, 0x125), (8, 4, 8, 0x121),
                                  (16, 2, 13, 0x120), (4, 2, 5, 0x225), (4, 4, 64, 0x222),
                                  (8, 2, 7, 0x227), (2, 2, 1, 0x421), (2, 4, 9, 0x424),
                                  (4, 2, 6, 0x423), (1, 4, 11, 0x825), (2, 2, 64, 0x821),
                                  (4, 1, 64, 0x8), (4, 4, 13, 0x9), (2, 4, 7, 0xd),
                                  (8, 2, 5, 0x9), (4, 2, 64, 0xa)])
def test_star3d_tiles_diffusion(dtype, tile):
    g = diffusion_star_exact(3, 3, 0.0815)
    run_case((70, 37, 29), 3, g, dtype, S.STAR3D, tile=tile)


@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("dtype", [S.F64, S.F32])
def test_star3d_asymmetric_random_taps(r, dtype):
    # asymmetric coefficients: a swapped side or axis would show
    run_case((67, 21, 19), r, rand_star(r, 10 + r), dtype, S.STAR3D, tile=(4, 4, 8, 0x121))
    run_case((67, 21, 19), r, rand_star(r, 10 + r), dtype, S.STAR3D, tile=(16, 2, 5, 0x120))
    run_case((67, 21, 19), r, rand_star(r, 10 + r), dtype, S.STAR3D, tile=(2, 4, 6, 0x425))
    run_case((67, 21, 19), r, rand_star(r, 10 + r), dtype, S.STAR3D, tile=(4, 2, 6, 0x9))
    run_case((67, 21, 19), r, rand_star(r, 10 + r), dtype, S.STAR3D, tile=(2, 2, 9, 0x821))


def test_star3d_tap_radius_below_padding():
    # radius-4 padding, radius-2 taps: the plan runs a radius-2 kernel
    g = np.zeros((9, 9, 9))
    g[2:7, 2:7, 2:7] = rand_star(2, 5)
    p = run_case((40, 20, 12), 4, g, S.F64, S.STAR3D, tile=(4, 2, 8, 0x221))
    assert p.variant == S.STAR3D


@pytest.mark.parametrize("dims,r", [((3, 3, 3), 3), ((5, 4, 7), 3), ((4, 5, 6), 4), ((1, 1, 1), 1)])
def test_star3d_tiny_periodic_grids(dims, r):
    # n < 2r: a point has periodic images on both sides
    run_case(dims, r, rand_star(r, 2), S.F64, S.STAR3D, tile=(4, 2, 2, 0x221))
    run_case(dims, r, rand_star(r, 2), S.F64, S.STAR3D, tile=(8, 2, 3, 0x120))
    run_case(dims, r, rand_star(r, 2), S.F64, S.STAR3D, tile=(2, 4, 2, 0x9))
    run_case(dims, r, rand_star(r, 2), S.F64, S.GENERIC)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("dims,r", [((1000,), 1), ((1000,), 3), ((333,), 8), ((50, 37), 2),
                                    ((23, 17, 11), 2), ((30, 20, 10), 3)])
def test_generic_dense(dtype, dims, r):
    g = np.random.default_rng(7).uniform(-1, 1, (2 * r + 1,) * len(dims))
    run_case(dims, r, g, dtype, S.GENERIC)


@pytest.mark.parametrize("e", [1, 2, 4, 8])
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,r", [(5000, 1), (777, 4), (3, 3)])
def test_line1d(e, dtype, n, r):
    g = np.random.default_rng(8).uniform(-1, 1, 2 * r + 1)
    run_case((n,), r, g, dtype, S.LINE1D, tile=(e,))


def test_sparse_box_is_not_a_star():
    g = np.zeros((3, 3, 3))
    g[1, 1, 1] = 1.0
    g[0, 0, 1] = 0.5  # an off-axis tap
    with pytest.raises(S.StencilError):
        S.LinearPlan((8, 8, 8), 1, g, variant=S.STAR3D)
    run_case((19, 13, 11), 1, g, S.F64, S.VARIANT_AUTO)


def test_r0_copy_stencil():
    run_case((33, 17, 9), 0, np.array([[[2.0]]]), S.F64, S.GENERIC)


@pytest.mark.parametrize("variant,tile", [(S.STAR3D, (4, 4, 16, 0x125)), (S.GENERIC, None)])
@pytest.mark.parametrize("iters", [6, 7])
def test_chained_iterations_ping_pong(variant, tile, iters):
    g = diffusion_star_exact(3, 3, 0.2)
    run_case((40, 33, 21), 3, g, S.F64, variant, tile=tile, iters=iters)


@pytest.mark.parametrize("variant", [S.STAR3D, S.GENERIC])
def test_user_halo_reads_caller_halo_and_writes_interior_only(variant):
    dims, r = (45, 26, 17), 3
    g = rand_star(3, 4)
    rng = np.random.default_rng(12)
    a_host = rng.uniform(-1, 1, O.padded_shape(dims, r))  # non-periodic halo
    plan = S.LinearPlan(dims, r, g, bc=S.USER_HALO, variant=variant,
                        tile=(4, 2, 8, 0x221) if variant == S.STAR3D else None)
    a = dev(a_host, S.F64)
    b = plan.empty(fill=123.0)
    plan.apply(a, b, 1)
    got = host(b)
    ref = O.xcorr(a_host, r, g)
    assert_close(O.interior(got, r), O.interior(ref, r), S.F64)
    mask = np.ones(got.shape, bool)
    O.interior(mask, r)[...] = False
    assert np.all(got[mask] == 123.0)
    assert np.array_equal(host(a), a_host)  # input untouched
    with pytest.raises(S.StencilError):
        plan.apply(a, b, 2)


def test_autotuned_plan_matches_oracle():
    g = diffusion_star_exact(3, 3, 0.0815)
    p = run_case((96, 48, 40), 3, g, S.F64, S.VARIANT_AUTO, autotune=True)
    assert p.variant in (S.STAR3D, S.GENERIC)


def test_apply_validation_on_device():
    plan = S.LinearPlan((16, 16, 16), 1, np.ones((3, 3, 3)))
    a = plan.empty(0.0)
    with pytest.raises(S.StencilError):
        S.check(S.lib().stencil_apply(plan._h, S.ptr(a), S.ptr(a), 1, None))  # aliasing
    assert plan.apply(a, plan.empty(0.0), 0) is a  # iters = 0 is a no-op


# ---------------------------------------------------------------------------
# full sizes of the benchmark workloads
# ---------------------------------------------------------------------------

# ---------------------------------------------------------------------------
# two chained iterations per launch (3-D star, periodic)
# ---------------------------------------------------------------------------

T2_TILES = [(8, 2, 32, 0x2101), (16, 1, 64, 0x2101), (16, 2, 16, 0x2101), (12, 2, 8, 0x2105),
            (8, 2, 32, 0x2201), (8, 4, 16, 0x2101), (12, 2, 64, 0x2101), (8, 2, 32, 0x2105),
            # pair-layout LDS planes (bit 16)
            (12, 2, 64, 0x12101), (8, 2, 32, 0x12101), (12, 2, 8, 0x12105)]
ONE_TILE = (4, 2, 8, 0x221)


def run_star_iters(dims, r, g, dtype, tile, iters, seed=3, layout=(0, 0)):
    inner = to_storage_values(inputs.uniform_field(dims, seed), dtype)
    plan = S.LinearPlan(dims, r, g, dtype=dtype, variant=S.STAR3D, tile=tile,
                        row_pitch=layout[0], x_offset=layout[1])
    a = plan.empty(fill=5.0)
    pad = np.full(O.padded_shape(dims, r), 7.0)  # halo garbage: the library ignores it
    O.interior(pad, r)[...] = inner
    plan.padded(a).copy_(dev(pad, dtype))
    b = plan.empty(fill=-3.0)
    res = plan.apply(a, b, iters)
    return host(plan.padded(res)), plan, inner


@pytest.mark.parametrize("tile", T2_TILES)
@pytest.mark.parametrize("dtype", DTYPES)
def test_star_two_iterations_bitwise_equal_to_one_iteration_launches(tile, dtype):
    dims, r = (70, 45, 37), 3
    g = diffusion_star_exact(3, 3, 0.0815)
    for iters in (2, 5, 6):
        got, plan, inner = run_star_iters(dims, r, g, dtype, tile, iters)
        assert (plan.tile[3] >> 12) & 15 == 2
        ref, _, _ = run_star_iters(dims, r, g, dtype, ONE_TILE, iters)
        assert np.array_equal(got, ref), (tile, iters)
        if dtype == S.F64:
            want = oracle_apply(inner, r, g, iters)
            assert_close(O.interior(got, r), O.interior(want, r), S.F64, what=str((tile, iters)))
            assert np.array_equal(got, O.fill_periodic(got.copy(), r))


@pytest.mark.parametrize("r", [1, 2, 4])
@pytest.mark.parametrize("tile", [(16, 2, 16, 0x2101), (12, 2, 16, 0x2101), (8, 2, 16, 0x2101),
                                  (8, 2, 16, 0x2201)])
def test_star_two_iterations_other_radii_random_taps(r, tile):
    # 1024-lane (shifting-window march; 64 x 16 and 128 x 8 lanes) and
    # 768/512-lane (register rings for r <= 3) workgroups
    dims = (66, 29, 31)
    g = rand_star(r, 21) * 0.15
    got, _, inner = run_star_iters(dims, r, g, S.F64, tile, 4)
    ref, _, _ = run_star_iters(dims, r, g, S.F64, (4, 2, 8, 0x221), 4)
    assert np.array_equal(got, ref)
    want = oracle_apply(inner, r, g, 4)
    assert_close(O.interior(got, r), O.interior(want, r), S.F64)


@pytest.mark.parametrize("dtype", [S.F32, S.BF16])
def test_star_two_iterations_radius_4_four_rows(dtype):
    # radius 4, four rows per lane (the shifting-window march, whose BF16
    # instance spills registers): bitwise equal to one-iteration launches
    dims, r = (66, 29, 31), 4
    g = rand_star(r, 23) * 0.15
    for iters in (2, 4, 5):
        got, plan, inner = run_star_iters(dims, r, g, dtype, (8, 4, 16, 0x2101), iters)
        assert (plan.tile[3] >> 12) & 15 == 2
        ref, _, _ = run_star_iters(dims, r, g, dtype, (4, 2, 8, 0x221), iters)
        assert np.array_equal(got, ref), iters


@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("tile", [(12, 2, 16, 0x12101), (8, 2, 16, 0x12105)])
@pytest.mark.parametrize("dtype", DTYPES)
def test_star_two_iterations_pair_layout_radii_random_taps(r, tile, dtype):
    # pair-layout LDS planes: every radius the layout takes, asymmetric taps,
    # a grid that is not a multiple of the tile in any axis
    dims = (66, 29, 31)
    g = rand_star(r, 23) * 0.15
    got, plan, inner = run_star_iters(dims, r, g, dtype, tile, 4)
    assert plan.tile[3] & (1 << 16)
    ref, _, _ = run_star_iters(dims, r, g, dtype, (4, 2, 8, 0x221), 4)
    assert np.array_equal(got, ref)
    if dtype == S.F64:
        want = oracle_apply(inner, r, g, 4)
        assert_close(O.interior(got, r), O.interior(want, r), S.F64)


QUAD_TILES = [(8, 4, 32, 0x12101), (8, 4, 8, 0x12105), (8, 4, 64, 0x12100)]


@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("tile", QUAD_TILES)
@pytest.mark.parametrize("dtype", [S.F32, S.BF16])
def test_star_two_iterations_quad_layout_radii_random_taps(r, tile, dtype):
    # quad-layout LDS planes (4-byte arithmetic, four rows per lane): every
    # radius, asymmetric taps, a grid that is not a multiple of the tile (64
    # lanes less 2r halo columns, 32 rows less 2r) in any axis
    dims = (66, 29, 31)
    g = rand_star(r, 23) * 0.15
    for iters in (4, 5):  # two-iteration launches only / plus one single
        got, plan, inner = run_star_iters(dims, r, g, dtype, tile, iters)
        assert plan.tile[3] & (1 << 16) and plan.tile[1] == 4
        ref, _, _ = run_star_iters(dims, r, g, dtype, (4, 2, 8, 0x221), iters)
        assert np.array_equal(got, ref), (tile, iters)


@pytest.mark.parametrize("dims,r", [((3, 3, 3), 3), ((5, 4, 7), 4), ((1, 1, 1), 1),
                                    ((130, 7, 5), 2), ((56, 24, 9), 4), ((57, 25, 9), 4)])
def test_star_two_iterations_quad_layout_tiny_and_edge_grids(dims, r):
    # n < 2r, single cells, and exactly one tile (56 = 64 - 2r columns,
    # 24 = 32 - 2r rows) and one past it
    g = rand_star(r, 8) * 0.2
    for iters in (2, 3):
        got, _, _ = run_star_iters(dims, r, g, S.F32, (8, 4, 16, 0x12101), iters)
        ref, _, _ = run_star_iters(dims, r, g, S.F32, (4, 2, 8, 0x221), iters)
        assert np.array_equal(got, ref), (dims, iters)
        assert np.array_equal(got, O.fill_periodic(got.copy(), r))


def test_star_two_iterations_quad_layout_pitched_and_rejects():
    dims, r = (70, 45, 37), 3
    g = diffusion_star_exact(3, 3, 0.0815)
    got, _, _ = run_star_iters(dims, r, g, S.F32, (8, 4, 16, 0x12101), 6, layout=(128, 32))
    ref, _, _ = run_star_iters(dims, r, g, S.F32, ONE_TILE, 6)
    assert np.array_equal(got, ref)
    # FP64 (pairs only), several waves along x, one iteration per launch
    for dtype, tile in ((S.F64, (8, 4, 16, 0x12101)), (S.F32, (4, 4, 16, 0x12201)),
                        (S.F32, (8, 4, 16, 0x11101))):
        with pytest.raises(S.StencilError):
            S.LinearPlan((32, 32, 32), 3, g, dtype=dtype, variant=S.STAR3D, tile=tile)


@pytest.mark.parametrize("dims,r", [((3, 3, 3), 3), ((5, 4, 7), 3), ((1, 1, 1), 1),
                                    ((130, 7, 5), 2)])
@pytest.mark.parametrize("tile", [(8, 2, 32, 0x2101), (12, 2, 64, 0x2101), (12, 2, 64, 0x12101)])
def test_star_two_iterations_tiny_and_thin_grids(dims, r, tile):
    g = rand_star(r, 8) * 0.2
    for iters in (4, 5):  # two-iteration launches only / plus one single
        got, _, inner = run_star_iters(dims, r, g, S.F64, tile, iters)
        want = oracle_apply(inner, r, g, iters)
        assert_close(O.interior(got, r), O.interior(want, r), S.F64)
        assert np.array_equal(got, O.fill_periodic(got.copy(), r))


@pytest.mark.parametrize("dtype,tile", [(S.F32, (8, 2, 32, 0x2101)), (S.F64, (12, 2, 16, 0x12101)),
                                        (S.BF16, (8, 2, 16, 0x12105))])
def test_star_two_iterations_pitched_layout(dtype, tile):
    # rows of 128 elements with the interior at column 32, in the row and the
    # pair LDS layouts
    dims, r = (70, 45, 37), 3
    g = diffusion_star_exact(3, 3, 0.0815)
    got, _, inner = run_star_iters(dims, r, g, dtype, tile, 6, layout=(128, 32))
    ref, _, _ = run_star_iters(dims, r, g, dtype, ONE_TILE, 6)
    assert np.array_equal(got, ref)


def test_star_plan_without_tile_keeps_the_default_shape():
    g = diffusion_star_exact(3, 3, 0.1)
    p = S.LinearPlan((40, 40, 40), 3, g, variant=S.STAR3D)
    assert p.variant == S.STAR3D and p.tile[0] > 0


def test_star_two_iterations_needs_periodic_lds_variant():
    g = diffusion_star_exact(3, 3, 0.1)
    for bc, tile in ((S.USER_HALO, (8, 2, 32, 0x2101)), (S.PERIODIC, (4, 2, 32, 0x2109)),
                     (S.PERIODIC, (8, 2, 32, 0x3101))):
        with pytest.raises(S.StencilError):
            S.LinearPlan((32, 32, 32), 3, g, bc=bc, variant=S.STAR3D, tile=tile)


def test_star_pair_layout_rejects_other_shapes():
    g3 = diffusion_star_exact(3, 3, 0.1)
    # one iteration per launch, four rows per lane, 1024 lanes
    for tile in ((8, 2, 32, 0x10101), (8, 4, 16, 0x12101), (16, 2, 16, 0x12101),
                 (8, 2, 32, 0x12201)):
        with pytest.raises(S.StencilError):
            S.LinearPlan((32, 32, 32), 3, g3, variant=S.STAR3D, tile=tile)
    # radius 5 (padding 5): beyond the star kernels
    g5 = rand_star(5, 5) * 0.1
    with pytest.raises(S.StencilError):
        S.LinearPlan((32, 32, 32), 5, g5, variant=S.STAR3D, tile=(8, 2, 32, 0x12101))


# ---------------------------------------------------------------------------
# pitched layout: interior at column x_offset of rows of row_pitch elements
# ---------------------------------------------------------------------------

def run_pitched(dims, r, g, dtype, variant, row_pitch, x_offset, tile=None, iters=1, seed=5,
                bc=S.PERIODIC):
    inner = to_storage_values(inputs.uniform_field(dims, seed), dtype)
    plan = S.LinearPlan(dims, r, g, dtype=dtype, variant=variant, tile=tile, bc=bc,
                        row_pitch=row_pitch, x_offset=x_offset)
    store = np.full(plan.storage_shape, 11.0)  # cells outside the padded rows
    pad = np.full(O.padded_shape(dims, r), 7.0)
    O.interior(pad, r)[...] = inner
    if bc == S.USER_HALO:
        pad = O.pad_periodic(inner, r)
    lo = plan.x_offset - r
    store[..., lo:lo + dims[0] + 2 * r] = pad
    a = dev(store, dtype)
    b = plan.empty(fill=-3.0)
    res_t = plan.apply(a, b, iters)
    full = host(res_t)
    res = host(plan.padded(res_t))
    torch.cuda.synchronize()
    ref = oracle_apply(inner, r, g, iters)
    ntaps = int(np.count_nonzero(g))
    absconv = None
    if dtype != S.F64:
        assert iters == 1
        absconv = O.interior(O.xcorr(np.abs(O.pad_periodic(inner, r)), r, np.abs(g)), r)
    what = "%s r=%d pitch=%d ox=%d" % (dims, r, row_pitch, x_offset)
    assert_close(O.interior(res, r), O.interior(ref, r), dtype, absconv, ntaps, what=what)
    if bc == S.PERIODIC:
        assert np.array_equal(res, O.fill_periodic(res.copy(), r)), what + ": halo"
    # columns outside [x_offset - r, x_offset + nx + r) are never touched
    outside = np.ones(plan.storage_shape[-1], bool)
    outside[lo:lo + dims[0] + 2 * r] = False
    expect = -3.0 if iters % 2 else 11.0
    assert np.all(full[..., outside] == expect), what + ": outside columns written"
    return plan


PITCHED = [  # dims, r, dtype, variant, (row_pitch, x_offset), tile
    ((70, 37, 29), 3, S.F64, S.STAR3D, (96, 16), (4, 2, 16, 0x221)),
    ((70, 37, 29), 3, S.F64, S.STAR3D, (96, 16), (4, 1, 16, 0x009)),  # hardware-cached
    ((70, 37, 29), 3, S.F32, S.STAR3D, (128, 32), (8, 2, 16, 0x021)),
    ((50, 21, 19), 2, S.BF16, S.STAR3D, (70, 9), (4, 4, 8, 0x001)),
    ((40, 33), 3, S.F64, S.GENERIC, (51, 5), None),
    ((23, 17, 11), 2, S.F32, S.GENERIC, (31, 4), None),
    ((1000,), 3, S.F64, S.LINE1D, (0, 16), (4, 1)),
    ((1000,), 3, S.BF16, S.LINE1D, (0, 64), (2, 1)),
]


@pytest.mark.parametrize("case", range(len(PITCHED)))
def test_pitched_layout(case):
    dims, r, dtype, variant, (pitch, ox), tile = PITCHED[case]
    g = rand_star(r, 6) if len(dims) == 3 else np.random.default_rng(6).uniform(
        -1, 1, (2 * r + 1,) * len(dims))
    run_pitched(dims, r, g, dtype, variant, pitch, ox, tile=tile)


@pytest.mark.parametrize("iters", [1, 6, 7])
def test_pitched_chained_star_and_temporal_line(iters):
    g = diffusion_star_exact(3, 3, 0.2)
    run_pitched((40, 33, 21), 3, g, S.F64, S.STAR3D, 64, 16, tile=(4, 2, 8, 0x221),
                iters=iters)
    g1 = np.array([0.1, 0.2, 0.4, 0.2, 0.1])
    run_pitched((4099,), 2, g1, S.F64, S.LINE1D, 0, 8, tile=(4, 8), iters=iters + 3)


def test_pitched_user_halo_and_plan_halo():
    dims, r = (45, 26, 17), 3
    run_pitched(dims, r, rand_star(3, 4), S.F64, S.STAR3D, 64, 8, tile=(4, 2, 8, 0x221),
                bc=S.USER_HALO)
    plan = S.LinearPlan(dims, r, rand_star(3, 4), row_pitch=64, x_offset=8)
    inner = inputs.uniform_field(dims, 8)
    store = np.full(plan.storage_shape, 5.0)
    pv = store[..., 5:5 + dims[0] + 2 * r]
    O.interior(pv, r)[...] = inner
    t = dev(store, S.F64)
    plan.halo(t)
    got = host(t)
    assert np.array_equal(got[..., 5:5 + dims[0] + 2 * r], O.pad_periodic(inner, r))
    assert np.all(got[..., :5] == 5.0) and np.all(got[..., 5 + dims[0] + 2 * r:] == 5.0)


def test_smoother_2pow20_ten_iterations():
    n = 2 ** 20
    g = W.smoother3()
    assert np.array_equal(g, np.array([0.25, 0.5, 0.25]))
    run_case((n,), 1, g, S.F64, S.VARIANT_AUTO, iters=10, autotune=True)


def sample_points(dims, count, seed):
    rng = np.random.default_rng(seed)
    pts = np.stack([rng.integers(0, d, count) for d in dims], axis=1)
    corners = np.array([[x, y, z] for x in (0, dims[0] - 1) for y in (0, dims[1] - 1)
                        for z in (0, dims[2] - 1)])
    return np.concatenate([pts, corners])


@pytest.mark.parametrize("dtype", [S.F64, S.F32])
@pytest.mark.parametrize("aligned", [False, True])
def test_star_512_cubed_sampled_points(dtype, aligned):
    # aligned: the cache-line-aligned row layout the benchmark times
    dims, r = (512, 512, 512), 3
    s = W.diffusion_number(512)
    g_prod = W.diffusion_star(3, 3, s)
    g_ref = diffusion_star_exact(3, 3, s)
    assert np.max(np.abs(g_prod - g_ref)) < 1e-15
    inner = to_storage_values(inputs.uniform_field(dims, 1), dtype)
    pitch, ox = W.aligned_layout(512, r, 8 if dtype == S.F64 else 4) if aligned else (0, 0)
    plan = S.LinearPlan(dims, r, g_prod, dtype=dtype, autotune=True, row_pitch=pitch,
                        x_offset=ox)
    a_host = np.zeros(O.padded_shape(dims, r))
    O.interior(a_host, r)[...] = inner
    del inner
    a = plan.empty(0.0)
    plan.padded(a).copy_(dev(a_host, dtype))
    b = plan.empty(0.0)
    plan.apply(a, b, 1)
    got = host(plan.padded(b))
    O.fill_periodic(a_host, r)
    pts = sample_points(dims, 4000, 2)
    ref = O.xcorr_at(a_host, r, g_ref, pts)
    vals = got[pts[:, 2] + r, pts[:, 1] + r, pts[:, 0] + r]
    if dtype == S.F64:
        assert np.max(np.abs(vals - ref)) <= 1e-12 * np.max(np.abs(ref))
    else:
        absconv = O.xcorr_at(np.abs(a_host), r, np.abs(g_ref), pts)
        assert np.all(np.abs(vals - ref) <= 2 * 20 * 2.0 ** -24 * absconv + 2.0 ** -24 * np.abs(ref))
    # the output halo is the periodic image of its interior
    assert np.array_equal(got[:r], got[512:512 + r]) and np.array_equal(got[:, :, -r:], got[:, :, r:2 * r])


@pytest.mark.parametrize("dtype", [S.F64, S.F32])
def test_star_512_cubed_two_iteration_launches(dtype):
    # 4 iterations = two launches of the two-iteration kernel: bitwise equal
    # to four one-iteration launches at full size, and (FP64) the oracle's
    # fourth iterate at sampled points
    dims, r, iters = (512, 512, 512), 3, 4
    s = W.diffusion_number(512)
    g_ref = diffusion_star_exact(3, 3, s)
    inner = to_storage_values(inputs.uniform_field(dims, 4), dtype)
    pitch, ox = W.aligned_layout(512, r, 4) if dtype == S.F32 else (0, 0)
    pad = np.zeros(O.padded_shape(dims, r))
    O.interior(pad, r)[...] = inner
    del inner
    outs = []
    # two-iteration (shifting window; register rings), one-iteration
    for tile in ((8, 2, 64, 0x2101), (4, 2, 32, 0x221), (12, 2, 64, 0x2101), (12, 2, 64, 0x12101)):
        plan = S.LinearPlan(dims, r, W.diffusion_star(3, 3, s), dtype=dtype, variant=S.STAR3D,
                            tile=tile, row_pitch=pitch, x_offset=ox)
        a = plan.empty(0.0)
        plan.padded(a).copy_(dev(pad, dtype))
        b = plan.empty(0.0)
        res = plan.apply(a, b, iters)
        outs.append(host(plan.padded(res)))
        del a, b, res, plan
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[2], outs[1])
    assert np.array_equal(outs[3], outs[1])
    if dtype == S.F64:
        O.fill_periodic(pad, r)
        cur = pad
        for _ in range(iters - 1):
            cur = O.fill_periodic(O.xcorr(cur, r, g_ref), r)
        pts = sample_points(dims, 2000, 7)
        ref = O.xcorr_at(cur, r, g_ref, pts)
        vals = outs[0][pts[:, 2] + r, pts[:, 1] + r, pts[:, 0] + r]
        assert np.max(np.abs(vals - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("autotune", [False, True])
def test_star_512_cubed_hundred_iterations_fourier_mode(autotune):
    # a single Fourier mode is an eigenvector: after N iterations it is scaled
    # by the symbol to the N-th power (closed form, any size); the default
    # plan is the one the benchmark times (50 two-iteration launches)
    dims, r, N = (512, 512, 512), 3, 100
    s = W.diffusion_number(512)
    k = (3, -5, 7)
    X = inputs.grid_coords(dims)
    inner = np.cos(sum(k[a] * X[a] for a in range(3)) + 0.25)
    lam = 1.0 + s * sum(laplacian_symbol_grid(k[a], 512, r) for a in range(3))
    plan = S.LinearPlan(dims, r, W.diffusion_star(3, 3, s), autotune=autotune)
    if not autotune:
        assert plan.launches(N) == (N // 2, 0)
    a_host = np.zeros(O.padded_shape(dims, r))
    O.interior(a_host, r)[...] = inner
    a = dev(a_host, S.F64)
    b = plan.empty(0.0)
    res = plan.apply(a, b, N)
    got = O.interior(host(res), r)
    err = np.max(np.abs(got - lam ** N * inner))
    assert err <= 1e-12, err


@pytest.mark.parametrize("n,r,e,T,iters", [(5000, 1, 4, 4, 10), (777, 4, 2, 16, 17),
                                           (3, 3, 1, 8, 5), (1000, 2, 8, 16, 2),
                                           (1 << 20, 1, 4, 10, 10), (4099, 1, 1, 3, 1)])
def test_line1d_temporal_blocking(n, r, e, T, iters):
    g = np.random.default_rng(13).uniform(-0.3, 0.3, 2 * r + 1)
    g[r] = 1.0 - (np.abs(g).sum() - abs(g[r]))  # keep the iteration bounded
    run_case((n,), r, g, S.F64, S.LINE1D, tile=(e, T), iters=iters)


# ---------------------------------------------------------------------------
# large radius (1-D lines up to r = 1024, the radius study of Sec. 5)
# ---------------------------------------------------------------------------

def bounded_taps(r, seed):
    g = np.random.default_rng(seed).uniform(-1, 1, 2 * r + 1)
    return g / np.abs(g).sum()  # sum |g| = 1: chained iterations stay bounded


@pytest.mark.parametrize("r", [16, 100, 1024])
@pytest.mark.parametrize("variant,tile", [(S.LINE1D, (1, 1)), (S.LINE1D, (8, 1)),
                                          (S.LINE1D, (4, 2)), (S.GENERIC, None),
                                          (S.LINE1D, (4, 1, 1)), (S.LINE1D, (8, 1, 1)),
                                          (S.LINE1D, (16, 1, 1))])
def test_line1d_large_radius(r, variant, tile):
    n = 65536 + 37
    g = bounded_taps(r, r)
    run_case((n,), r, g, S.F64, variant, tile=tile, iters=3)


@pytest.mark.parametrize("r", [64, 1024])
def test_line1d_large_radius_fp32(r):
    run_case((20011,), r, bounded_taps(r, 3), S.F32, S.LINE1D, tile=(4, 1))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("e,r,n", [(4, 2, 5000), (8, 4, 2049), (16, 7, 777), (16, 300, 4099),
                                   (8, 1024, 70000)])
def test_line1d_register_blocked_bitwise_equal_to_plain_line(dtype, e, r, n):
    g = bounded_taps(r, 11)
    inner = to_storage_values(inputs.uniform_field((n,), 2), dtype)
    outs = []
    for tile in ((1, 1), (e, 1, 1)):
        plan = S.LinearPlan((n,), r, g, dtype=dtype, variant=S.LINE1D, tile=tile)
        a = dev(O.pad_periodic(inner, r), dtype)
        b = plan.empty(0.0)
        outs.append(host(plan.apply(a, b, 2)))
    assert np.array_equal(outs[0], outs[1])
    if dtype == S.F64:
        ref = oracle_apply(inner, r, g, 2)
        assert_close(O.interior(outs[1], r), O.interior(ref, r), S.F64)


def test_line1d_register_blocking_validation():
    g = bounded_taps(1, 1)
    with pytest.raises(S.StencilError):
        S.LinearPlan((1000,), 1, g, variant=S.LINE1D, tile=(16, 1, 1)).apply(
            torch.zeros(1002, dtype=torch.float64, device="cuda"),
            torch.zeros(1002, dtype=torch.float64, device="cuda"))
    with pytest.raises(S.StencilError):
        S.LinearPlan((1000,), 8, bounded_taps(8, 1), variant=S.LINE1D, tile=(8, 4, 1))


def test_line1d_radius_equal_to_length():
    # periodic with n == r: every output reads each input several times
    r = n = 300
    run_case((n,), r, bounded_taps(r, 5), S.F64, S.LINE1D, tile=(2, 1), iters=2)
    run_case((n,), r, bounded_taps(r, 5), S.F64, S.GENERIC, iters=2)


def test_line1d_temporal_needs_periodic():
    with pytest.raises(S.StencilError):
        S.LinearPlan((100,), 1, W.smoother3(), bc=S.USER_HALO, variant=S.LINE1D, tile=(4, 8))


# ---------------------------------------------------------------------------
# window filters (max filter of Sec. 2.3, min, median of Sec. 1): bit-exact
# ---------------------------------------------------------------------------

def star_mask(ndim, r):
    m = np.zeros((2 * r + 1,) * ndim)
    for a in range(ndim):
        for k in range(2 * r + 1):
            idx = [r] * ndim
            idx[a] = k
            m[tuple(idx)] = 1.0
    return m


def holey_mask(ndim, r, seed, max_cells=None):
    rng = np.random.default_rng(seed)
    m = (rng.uniform(size=(2 * r + 1,) * ndim) < 0.45).astype(float)
    m[(r,) * ndim] = 1.0
    if max_cells is not None:
        on = np.flatnonzero(m.reshape(-1))
        for k in on[max_cells:]:
            m.reshape(-1)[k] = 0.0
        m[(r,) * ndim] = 1.0
    return m


def run_filter(dims, r, mask, op, dtype, variant=S.VARIANT_AUTO, tile=None, seed=4, inner=None,
               iters=1):
    """Periodic filter through the library (input halo garbage: the library
    fills it) and the oracle's iterate; returns interiors, plan, padded result."""
    if inner is None:
        inner = to_storage_values(inputs.uniform_field(dims, seed), dtype)
    plan = S.LinearPlan(dims, r, mask, dtype=dtype, variant=variant, tile=tile, op=op)
    a_h = np.full(O.padded_shape(dims, r), 7.0)
    O.interior(a_h, r)[...] = inner
    a = dev(a_h, dtype)
    b = plan.empty(fill=-3.0)
    res = host(plan.apply(a, b, iters))
    code = {S.OP_MAX: O.FILTER_MAX, S.OP_MIN: O.FILTER_MIN, S.OP_MEDIAN: O.FILTER_MEDIAN}[op]
    ref = O.pad_periodic(inner, r)
    for _ in range(iters):
        ref = O.fill_periodic(O.filter(ref, r, mask, code), r)
    return O.interior(res, r), O.interior(ref, r), plan, res


def same_bits(a, b):
    return np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(
        np.nan_to_num(a, nan=0.0), np.nan_to_num(b, nan=0.0)) and np.array_equal(
        np.signbit(a[~np.isnan(a)]), np.signbit(b[~np.isnan(b)]))


FILTER_CASES = [((1000,), 3, "box"), ((333,), 13, "box"), ((45, 37), 2, "box"), ((45, 37), 3, "star"),
                ((29, 17, 23), 1, "box"), ((29, 17, 23), 2, "star"), ((29, 17, 23), 3, "holey"),
                ((70, 33, 21), 2, "box"),
                # the windows whose median runs by forgetful selection: 9 and 7 cells
                ((45, 37), 1, "box"), ((29, 17, 23), 1, "star")]


@pytest.mark.parametrize("case", range(len(FILTER_CASES)))
@pytest.mark.parametrize("op", [S.OP_MAX, S.OP_MIN, S.OP_MEDIAN])
@pytest.mark.parametrize("dtype", DTYPES)
def test_filters_bit_exact(case, op, dtype):
    dims, r, shape = FILTER_CASES[case]
    nd = len(dims)
    mask = {"box": np.ones((2 * r + 1,) * nd), "star": star_mask(nd, r),
            "holey": holey_mask(nd, r, 3, max_cells=S.MEDIAN_MAX)}[shape]
    if op == S.OP_MEDIAN and int(np.count_nonzero(mask)) > S.MEDIAN_MAX:
        with pytest.raises(S.StencilError):
            S.LinearPlan(dims, r, mask, dtype=dtype, op=op)
        return
    got, ref, plan, res = run_filter(dims, r, mask, op, dtype)
    assert same_bits(got, ref), (dims, r, shape, op, plan.variant, plan.tile)
    assert np.array_equal(res, O.fill_periodic(res.copy(), r))


@pytest.mark.parametrize("op", [S.OP_MAX, S.OP_MIN])
@pytest.mark.parametrize("r", [1, 2, 3])
@pytest.mark.parametrize("tile", [(4, 0, 16, 0), (8, 0, 32, 0), (4, 0, 5, 0)])
def test_box_filter_z_march_bit_exact(op, r, tile):
    dims = (70, 33, 21)
    mask = np.ones((2 * r + 1,) * 3)
    got, ref, plan, _ = run_filter(dims, r, mask, op, S.F64, variant=S.STAR3D, tile=tile)
    assert plan.variant == S.STAR3D
    assert same_bits(got, ref)
    got2, _, _, _ = run_filter(dims, r, mask, op, S.F64, variant=S.GENERIC)
    assert same_bits(got, got2)


@pytest.mark.parametrize("op", [S.OP_MAX, S.OP_MIN, S.OP_MEDIAN])
@pytest.mark.parametrize("variant", [S.STAR3D, S.GENERIC])
def test_filters_signed_zeros_and_nan(op, variant):
    if op == S.OP_MEDIAN and variant == S.STAR3D:
        return
    dims, r = (40, 20, 12), 1
    rng = np.random.default_rng(5)
    inner = rng.choice(np.array([-0.0, 0.0, -1.0, 1.0]), size=dims[::-1])
    inner[5, 7, 9] = np.nan
    got, ref, _, _ = run_filter(dims, r, np.ones((3, 3, 3)), op, S.F64, variant=variant,
                                inner=inner)
    assert same_bits(got, ref)
    assert int(np.isnan(got).sum()) == 27


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("window", ["box27", "star7", "box9", "line5"])
def test_median_signed_zeros_nan_and_ties(window, dtype):
    # few distinct values (many ties, zeros of both signs): the selection
    # compares values, so the sign of a zero median is the total order's
    # (-0 below +0); windows with a NaN give NaN
    if window == "box9":
        dims, r, mask = (40, 36), 1, np.ones((3, 3))
    elif window == "line5":
        dims, r, mask = (4000,), 2, np.ones(5)  # rank counting, for comparison
    else:
        dims, r = (40, 20, 12), 1
        mask = np.ones((3, 3, 3)) if window == "box27" else star_mask(3, 1)
    rng = np.random.default_rng(11)
    inner = rng.choice(np.array([-0.0, 0.0, -0.0, 0.0, -1.0, 1.0, 0.5, -0.5]),
                       size=dims[::-1])
    inner.reshape(-1)[rng.integers(0, inner.size, 3)] = np.nan
    inner = to_storage_values(inner, dtype)
    got, ref, _, _ = run_filter(dims, r, mask, S.OP_MEDIAN, dtype, inner=inner)
    assert same_bits(got, ref)
    zeros = got[got == 0]
    assert np.signbit(zeros).any() and (~np.signbit(zeros)).any()


def test_filters_chained_and_user_halo():
    dims, r = (45, 26, 17), 1
    mask = np.ones((3, 3, 3))
    got, ref, _, _ = run_filter(dims, r, mask, S.OP_MAX, S.F32, iters=3)
    assert same_bits(got, ref)
    rng = np.random.default_rng(12)
    a_host = rng.uniform(-1, 1, O.padded_shape(dims, r))  # non-periodic halo
    for variant in (S.STAR3D, S.GENERIC):
        plan = S.LinearPlan(dims, r, mask, bc=S.USER_HALO, variant=variant, op=S.OP_MIN)
        b = plan.empty(fill=123.0)
        plan.apply(dev(a_host, S.F64), b, 1)
        out = host(b)
        want = O.filter(a_host, r, mask, O.FILTER_MIN)
        assert np.array_equal(O.interior(out, r), O.interior(want, r))


def test_filter_variant_validation():
    with pytest.raises(S.StencilError):  # median has no z-march form
        S.LinearPlan((32, 32, 32), 1, np.ones((3, 3, 3)), op=S.OP_MEDIAN, variant=S.STAR3D)
    with pytest.raises(S.StencilError):  # star window is not a box
        S.LinearPlan((32, 32, 32), 1, star_mask(3, 1), op=S.OP_MAX, variant=S.STAR3D)
    with pytest.raises(S.StencilError):
        S.LinearPlan((1000,), 1, np.ones(3), op=S.OP_MAX, variant=S.LINE1D)


@pytest.mark.parametrize("op", [S.OP_MAX, S.OP_MEDIAN])
def test_filter_512_cubed_sampled_points(op):
    dims, r = (512, 512, 512), 1
    mask = np.ones((3, 3, 3))
    inner = inputs.uniform_field(dims, 6)
    plan = S.LinearPlan(dims, r, mask, op=op)
    a_host = np.zeros(O.padded_shape(dims, r))
    O.interior(a_host, r)[...] = inner
    del inner
    b = plan.empty(0.0)
    plan.apply(dev(a_host, S.F64), b, 1)
    got = host(b)
    O.fill_periodic(a_host, r)
    pts = sample_points(dims, 3000, 8)
    ref = O.filter_at(a_host, r, mask, {S.OP_MAX: O.FILTER_MAX, S.OP_MEDIAN: O.FILTER_MEDIAN}[op],
                      pts)
    assert np.array_equal(got[pts[:, 2] + r, pts[:, 1] + r, pts[:, 0] + r], ref)
