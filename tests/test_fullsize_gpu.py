"""Full-size, element-wise GPU parity of the launches the benchmark times, and
the long-run anchor of the precision study, through the C ABI.

* 512^3 radius-3 diffusion star, FP64 and FP32, with the plan the benchmark
  builds (no autotuning, its row layout): four chained iterations are two
  launches of the two-iteration kernel (the first without periodic images,
  the last with them); every interior and halo point is compared with the
  oracle's fourth iterate.
* 256^3 8-field substep (proxy and full MHD), default FP64 plan, each of the
  three RK stages: every point of f_out (interior and halo) and of the
  register against one oracle substep on the same inputs.
* 1000 RK3 steps at 32^3 of both 8-field models: the FP64 path against the
  oracle at steps 1, 10, 100 and 1000, every point; the FP32/BF16 storage
  policies' error per field against the same oracle states (Sec. 5.1: the
  paper verifies on separate small runs).
* Arrays of 4 GiB or more: the default star plan at 1024 x 1024 x 520 FP64
  against the oracle at sampled points; RK plans of that size are refused at
  plan time.

FP64 bar: normwise max relative error <= 1e-12 per field. FP32 star: the
rounding bound of four chained FP32 iterations (derived below); the measured
error against the FP64 oracle is printed.
"""
import math

import numpy as np
import pytest

import oracle as O
from closed_forms import diffusion_star_exact
from paper_2406_08923_amd import inputs

torch = pytest.importorskip("torch")
import paper_2406_08923_amd as S  # noqa: E402
from paper_2406_08923_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

# constants of the full model in the benchmark: every closure term on
FULL = dict(zeta=3e-3, mu0=1.0, gamma=5.0 / 3.0, cp=1.0, lnrho0=0.0, K=4e-3, heat=2e-3,
            cool=5e-4)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def host(t):
    return t.to(torch.float64).cpu().numpy()


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------------------
# 512^3 star, the benchmark's plan
# ---------------------------------------------------------------------------

def fp32_chain_bound(gabs, ntaps, iters, fmax):
    """Max-norm bound of |FP32 chain - exact chain| after ``iters`` chained
    iterations of a cross-correlation with sum |g| = gabs from inputs
    |f| <= fmax that are exact in FP32: iteration k adds at most
    (ntaps + 1) u sum|g| max|f_k| from the FP32 multiply-add chain plus
    u max|f_{k+1}| from rounding the stored result, u = 2^-24, and carries
    the earlier error multiplied by at most gabs."""
    u = 2.0 ** -24
    err, fk = 0.0, fmax
    for _ in range(iters):
        err = gabs * err + (ntaps + 1) * u * gabs * fk + u * gabs * fk
        fk *= gabs
    return err


@pytest.mark.parametrize("dtype", [S.F64, S.F32])
def test_star_512_default_plan_every_point(dtype):
    dims, r, iters = (512, 512, 512), 3, 4
    s = W.diffusion_number(512)
    g_prod = W.diffusion_star(3, r, s)
    g_ref = diffusion_star_exact(3, r, s)
    aligned = dtype != S.F64  # the benchmark's layout per dtype
    pitch, ox = W.aligned_layout(512, r, 4) if aligned else (0, 0)
    plan = S.LinearPlan(dims, r, g_prod, dtype=dtype, row_pitch=pitch, x_offset=ox)
    assert plan.iterations_per_launch == 2 and plan.launches(iters) == (2, 0)
    inner = inputs.uniform_field(dims, 1)
    if dtype == S.F32:
        inner = inner.astype(np.float32).astype(np.float64)
    pad = O.pad_periodic(inner, r)
    del inner
    a = plan.empty(0.0)
    plan.padded(a).copy_(torch.from_numpy(pad).cuda().to(a.dtype))
    b = plan.empty(0.0)
    res = plan.apply(a, b, iters)
    assert res is a
    got = host(plan.padded(res))
    del a, b, res
    ref = O.xcorr_periodic_iterate(pad, r, g_ref, iters)
    del pad
    # halo: the periodic image of the result's interior, bit for bit
    assert np.array_equal(got, O.fill_periodic(got.copy(), r))
    err = relerr(got, ref)
    if dtype == S.F64:
        assert err <= 1e-12, err
    else:
        bound = fp32_chain_bound(float(np.abs(g_ref).sum()), int(np.count_nonzero(g_ref)),
                                 iters, 1.0)
        worst = float(np.max(np.abs(got - ref)))
        print("512^3 FP32 star, %d iterations: normwise error vs FP64 oracle %.2e "
              "(max abs %.2e, bound %.2e)" % (iters, err, worst, bound))
        assert worst <= bound


# ---------------------------------------------------------------------------
# 256^3 fused substep, every stage, every point
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("r", [1, 2])
def test_dense_box_512_default_plan_every_point(r):
    # the dense-box benchmark workloads: one periodic application of the
    # 27-point and the radius-2 (125-point) box to the 512^3 FP64 field on
    # the default plans (the LDS march), every interior and halo point
    # against the oracle
    dims, k = (512, 512, 512), 2 * r + 1
    g = np.random.default_rng(r).uniform(0.2, 1.0, (k, k, k))
    g /= g.sum()
    plan = S.LinearPlan(dims, r, g)
    assert plan.variant == S.BOX3D
    pad = O.pad_periodic(inputs.uniform_field(dims, 1), r)
    a = plan.empty(0.0)
    plan.padded(a).copy_(torch.from_numpy(pad).cuda())
    b = plan.empty(0.0)
    res = plan.apply(a, b, 1)
    got = host(plan.padded(res))
    del a, b, res
    ref = O.fill_periodic(O.xcorr(pad, r, g), r)
    del pad
    assert np.array_equal(got, O.fill_periodic(got.copy(), r))
    err = relerr(got, ref)
    assert err <= 1e-12, err


def test_dense_2d_box_16384_default_plan_every_point():
    # the 2-D dense-box benchmark workload: the radius-2 box on the 16384^2
    # FP64 field, default plan (the LDS march over row blocks), every point
    dims, r = (16384, 16384), 2
    g = np.random.default_rng(r).uniform(0.2, 1.0, (5, 5))
    g /= g.sum()
    plan = S.LinearPlan(dims, r, g)
    assert plan.variant == S.BOX3D
    pad = O.pad_periodic(inputs.uniform_field(dims, 1), r)
    a = plan.empty(0.0)
    plan.padded(a).copy_(torch.from_numpy(pad).cuda())
    b = plan.empty(0.0)
    got = host(plan.padded(plan.apply(a, b, 1)))
    del a, b
    ref = O.fill_periodic(O.xcorr(pad, r, g), r)
    del pad
    assert np.array_equal(got, O.fill_periodic(got.copy(), r))
    assert relerr(got, ref) <= 1e-12


@pytest.mark.parametrize("stage", [0, 1, 2])
@pytest.mark.parametrize("model", [S.MODEL_MHD8, S.MODEL_MHD_FULL])
def test_mhd_256_default_plan_every_point(model, stage):
    n = (256, 256, 256)
    ds = [2 * math.pi / v for v in n]
    dt = 0.1 * min(ds)
    mhd = FULL if model == S.MODEL_MHD_FULL else None
    f, _ = inputs.fourier_fields(n, 1, nf=8, modes=8, kmax=8, amp=0.01)
    plan = S.RkPlan(model, n, S.PREC_F64, mhd=mhd)
    b = plan.alloc()
    fin = []
    for k in range(8):
        fin.append(O.pad_periodic(f[k], 3))
        b["f_a"][k].copy_(torch.from_numpy(fin[k]).cuda())
        b["f_b"][k].fill_(-9.0)
    del f
    rng = np.random.default_rng(10 + stage)
    w0 = [rng.uniform(-1e-4, 1e-4, fin[0].shape) for _ in range(8)]
    for k in range(8):
        b["w"][k].copy_(torch.from_numpy(w0[k]).cuda())
    plan.step(b["f_a"], b["f_b"], b["w"], stage, dt)
    torch.cuda.synchronize()
    w_ref = [v.copy() for v in w0]
    omodel = O.MODEL_MHD_FULL if model == S.MODEL_MHD_FULL else O.MODEL_MHD8
    ref = O.rk3_substep(omodel, stage, fin, w_ref, ds, dt, mhd=mhd)
    del fin
    for k in range(8):
        got = host(b["f_b"][k])
        e = relerr(got, ref[k])
        assert e <= 1e-12, ("f", stage, k, e)
        gw = O.interior(host(b["w"][k]), 3)
        if stage < 2:
            e = relerr(gw, O.interior(w_ref[k], 3))
            assert e <= 1e-12, ("w", stage, k, e)
        else:
            assert np.array_equal(gw, O.interior(w0[k], 3))  # dead register: not written


# ---------------------------------------------------------------------------
# 1000 steps at 32^3: FP64 anchored to the oracle; mixed precision against it
# ---------------------------------------------------------------------------

CHECKPOINTS = (1, 10, 100, 1000)
POLICIES = (("f64", S.PREC_F64), ("f32_master64", S.PREC_F32_MASTER64),
            ("bf16_master64", S.PREC_BF16_MASTER64), ("f32_only", S.PREC_F32_ONLY),
            ("bf16_only", S.PREC_BF16_ONLY))


def gpu_checkpoints(model, n, prec, f, dt, mhd):
    plan = S.RkPlan(model, n, prec, mhd=mhd)
    b = plan.alloc()
    for k in range(8):
        pad = torch.from_numpy(O.pad_periodic(f[k], 3)).cuda()
        b["f_a"][k].copy_(pad.to(b["f_a"][k].dtype))
        if plan.master:
            b["f64"][k].copy_(pad)
    snaps, done, cur, nxt = {}, 0, b["f_a"], b["f_b"]
    for cp in CHECKPOINTS:
        res = plan.run(cur, nxt, b["w"], cp - done, dt, w2=b["w2"], f64=b["f64"])
        if res is nxt:
            cur, nxt = nxt, cur
        done = cp
        state = b["f64"] if plan.master else cur
        snaps[cp] = [O.interior(host(t), 3) for t in state]
        if not plan.master:
            snaps[cp, "halo"] = [host(t) for t in state]
    return snaps


@pytest.mark.parametrize("model", [S.MODEL_MHD8, S.MODEL_MHD_FULL])
def test_mhd_1000_steps_32_cubed_against_oracle(model):
    n = (32, 32, 32)
    ds = [2 * math.pi / v for v in n]
    dt = 0.1 * min(ds)
    mhd = FULL if model == S.MODEL_MHD_FULL else None
    omodel = O.MODEL_MHD_FULL if model == S.MODEL_MHD_FULL else O.MODEL_MHD8
    f, _ = inputs.fourier_fields(n, 1, nf=8, modes=8, kmax=8, amp=0.01)
    runs = {name: gpu_checkpoints(model, n, prec, f, dt, mhd) for name, prec in POLICIES}
    # the oracle, checkpointed
    cur = [O.pad_periodic(v, 3) for v in f]
    w = [np.zeros_like(cur[0]) for _ in range(8)]
    ref, done = {}, 0
    for cp in CHECKPOINTS:
        for _ in range(cp - done):
            for stage in range(3):
                cur = O.rk3_substep(omodel, stage, cur, w, ds, dt, mhd=mhd)
        done = cp
        ref[cp] = [v.copy() for v in cur]
    table = {}
    for name, _ in POLICIES:
        table[name] = {cp: [relerr(runs[name][cp][k], O.interior(ref[cp][k], 3))
                            for k in range(8)] for cp in CHECKPOINTS}
        print("model %d, %s: max-over-fields error vs the FP64 oracle at steps %s: %s"
              % (model, name, CHECKPOINTS,
                 " ".join("%.2e" % max(table[name][cp]) for cp in CHECKPOINTS)))
    # FP64: every point, halos included, at every checkpoint
    for cp in CHECKPOINTS:
        for k in range(8):
            e = relerr(runs["f64"][cp, "halo"][k], ref[cp][k])
            assert e <= 1e-12, (cp, k, e)
    # mixed precision: loose ceilings (the magnitudes are measured, not
    # pinned); the FP64 master keeps BF16 storage bounded where plain BF16
    # storage drifts
    assert max(table["f32_master64"][1000]) <= 2e-5
    assert max(table["bf16_master64"][1000]) <= 1e-1
    assert max(table["bf16_master64"][1000]) < max(table["bf16_only"][1000])


# ---------------------------------------------------------------------------
# arrays of 4 GiB or more
# ---------------------------------------------------------------------------

def test_star_beyond_4_gib_default_plan_sampled_points():
    # 1024 x 1024 x 520 FP64: 4.46 GB per padded buffer. The default plan
    # (two-iteration launches) reads its input plane by plane, so 32-bit
    # offsets never span the array; four iterations against the oracle's
    # fourth iterate at sampled points (and every point of the output halo
    # against the periodic image of its interior)
    dims, r, iters = (1024, 1024, 520), 3, 4
    s = W.diffusion_number(1024)
    g_ref = diffusion_star_exact(3, r, s)
    plan = S.LinearPlan(dims, r, W.diffusion_star(3, r, s))
    assert plan.iterations_per_launch == 2 and plan.launches(iters) == (2, 0)
    assert S.padded_elems(dims, r) * 8 >= 1 << 32
    pad = O.pad_periodic(inputs.uniform_field(dims, 3), r)
    a = plan.empty(0.0)
    a.copy_(torch.from_numpy(pad))
    b = plan.empty(0.0)
    res = plan.apply(a, b, iters)
    got = host(res)
    del a, b, res
    torch.cuda.empty_cache()
    cur = O.xcorr_periodic_iterate(pad, r, g_ref, iters - 1)
    del pad
    rng = np.random.default_rng(5)
    pts = np.stack([rng.integers(0, d, 3000) for d in dims], axis=1)
    corners = np.array([[x, y, z] for x in (0, dims[0] - 1) for y in (0, dims[1] - 1)
                        for z in (0, dims[2] - 1)])
    pts = np.concatenate([pts, corners, [[0, 0, 260], [1023, 511, 519]]])
    ref = O.xcorr_at(cur, r, g_ref, pts)
    del cur
    vals = got[pts[:, 2] + r, pts[:, 1] + r, pts[:, 0] + r]
    assert relerr(vals, ref) <= 1e-12
    assert np.array_equal(got[:r], got[dims[2]:dims[2] + r])
    assert np.array_equal(got[-r:], got[r:2 * r])
    assert np.array_equal(got[:, :, :r], got[:, :, dims[0]:dims[0] + r])


@pytest.mark.parametrize("kind", ["dense_box", "dense_box_lane_exchange", "dense_box_r2",
                                  "lane_exchange_star"])
def test_lane_exchange_kernels_beyond_4_gib_sampled_points(kind):
    # the z marches address the input plane by plane above 4 GiB (a buffer
    # resource per plane): one iteration of the dense 27-point box and of the
    # dense radius-2 box (default plans: the lane-exchange and the LDS march)
    # and of the radius-3 star's lane-exchange march at 1024 x 1024 x 520
    # FP64, sampled points against the oracle
    dims = (1024, 1024, 520)
    if kind.startswith("dense_box"):
        r = 2 if kind == "dense_box_r2" else 1
        k = 2 * r + 1
        g = np.random.default_rng(7).uniform(0.2, 1.0, (k, k, k)) / k ** 3
        # default plans (the LDS march), and radius 1 on the lane-exchange
        # march through an explicit tile
        tile = (4, 2, 8, 1) if kind == "dense_box_lane_exchange" else None
        plan = S.LinearPlan(dims, r, g, variant=S.BOX3D, tile=tile)
        assert plan.variant == S.BOX3D
    else:
        r = 3
        g = diffusion_star_exact(3, r, W.diffusion_number(1024))
        plan = S.LinearPlan(dims, r, g, variant=S.STAR3D, tile=(8, 2, 32, (1 << 17) | 1))
    assert S.padded_elems(dims, r) * 8 >= 1 << 32
    pad = O.pad_periodic(inputs.uniform_field(dims, 4), r)
    a = plan.empty(0.0)
    a.copy_(torch.from_numpy(pad))
    b = plan.empty(0.0)
    res = plan.apply(a, b, 1, halo_valid=True)
    got = host(res)
    del a, b, res
    torch.cuda.empty_cache()
    rng = np.random.default_rng(6)
    pts = np.stack([rng.integers(0, d, 3000) for d in dims], axis=1)
    corners = np.array([[x, y, z] for x in (0, dims[0] - 1) for y in (0, dims[1] - 1)
                        for z in (0, dims[2] - 1)])
    pts = np.concatenate([pts, corners, [[0, 0, 260], [1023, 511, 519], [61, 62, 300]]])
    ref = O.xcorr_at(pad, r, g, pts)
    del pad
    vals = got[pts[:, 2] + r, pts[:, 1] + r, pts[:, 0] + r]
    assert relerr(vals, ref) <= 1e-12
    assert np.array_equal(got[:r], got[dims[2]:dims[2] + r])
    assert np.array_equal(got[:, :, :r], got[:, :, dims[0]:dims[0] + r])


def test_rk_plans_beyond_4_gib_are_refused_at_plan_time():
    with pytest.raises(S.StencilError) as e:
        S.RkPlan(S.MODEL_MHD8, (1024, 1024, 520), S.PREC_F64)
    assert e.value.code == -3
    with pytest.raises(S.StencilError):
        S.RkPlan(S.MODEL_ADVDIFF, (1024, 1024, 520), S.PREC_F32_MASTER64)
