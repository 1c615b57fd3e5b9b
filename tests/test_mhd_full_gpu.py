"""GPU parity of the fused substep of the full non-ideal MHD equations (Eq.
A1-A4 with the ideal-gas closure) through the C ABI, against the CPU oracle.

FP64 bar: normwise max relative error <= 1e-12 per field (the same bar as the
proxy model: both sides evaluate the same sixth-order bank in FP64; only the
summation order and the exp implementation differ). Mixed-precision policies
are compared with the FP64 oracle; their asserted ceilings are sanity limits.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2406_08923_amd import inputs

torch = pytest.importorskip("torch")
import paper_2406_08923_amd as S  # noqa: E402

pytestmark = pytest.mark.gpu

NU, ETA, CS02 = 2e-3, 5e-3, 0.7
MHD = dict(zeta=3e-3, mu0=1.3, gamma=5.0 / 3.0, cp=1.7, lnrho0=0.2, K=4e-3, heat=2e-3,
           cool=5e-4)
KW = dict(nu=NU, eta=ETA, cs2=CS02)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def host(t):
    return t.to(torch.float64).cpu().numpy()


def put(t, a):
    t.copy_(torch.from_numpy(np.ascontiguousarray(a)).to(t.device).to(t.dtype))


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def fields(n, seed, amp=0.3, kmax=3):
    f, _ = inputs.fourier_fields(n, seed, nf=8, modes=4, kmax=kmax, amp=amp)
    return f


def ds_of(n):
    return [2 * math.pi / v for v in n]


BANKS = [(S.RK_CACHED, None), (S.RK_LDS, None), (S.RK_LDS, (16, 8, 4)), (S.RK_LDS, (16, 8, 8)),
         (S.RK_LDS, (32, 4, 4)), (S.RK_LDS, (8, 8, 8))]


@pytest.mark.parametrize("bank", range(len(BANKS)))
@pytest.mark.parametrize("stage", [0, 1, 2])
def test_full_mhd_substep_f64(stage, bank):
    n = (40, 24, 20)
    ds = ds_of(n)
    dt = 0.1 * min(ds)
    f = fields(n, 1)
    rng = np.random.default_rng(2)
    variant, block = BANKS[bank]
    print("full MHD substep stage %d bank %s %s" % (stage, variant, block), flush=True)
    plan = S.RkPlan(S.MODEL_MHD_FULL, n, S.PREC_F64, variant=variant, block=block, mhd=MHD, **KW)
    b = plan.alloc()
    fin = [O.pad_periodic(v, 3) for v in f]
    w0 = [rng.uniform(-1e-2, 1e-2, fin[0].shape) for _ in range(8)]
    for k in range(8):
        put(b["f_a"][k], fin[k])
        put(b["w"][k], w0[k] if stage else np.full(fin[0].shape, np.nan))
        b["f_b"][k].fill_(-9.0)
    plan.step(b["f_a"], b["f_b"], b["w"], stage, dt)
    torch.cuda.synchronize()
    w_ref = [a.copy() for a in w0]
    ref = O.rk3_substep(O.MODEL_MHD_FULL, stage, fin, w_ref, ds, dt, mhd=MHD, **KW)
    for k in range(8):
        got = host(b["f_b"][k])
        assert relerr(got, ref[k]) <= 1e-12, (stage, k, relerr(got, ref[k]))
        gw = O.interior(host(b["w"][k]), 3)
        if stage < 2:
            assert relerr(gw, O.interior(w_ref[k], 3)) <= 1e-12, (stage, k)
        else:
            assert np.array_equal(gw, O.interior(w0[k], 3))  # dead register not written


@pytest.mark.parametrize("model", [S.MODEL_MHD8, S.MODEL_MHD_FULL])
@pytest.mark.parametrize("n", [(20, 4, 5), (6, 7, 9)])
def test_lds_bank_short_axes_and_their_halo_images(n, model):
    # axes shorter than 2r (a point has two images along them: the general
    # image search) and axes of exactly 2r (one image each side: the images
    # found once per point); the whole padded output, halo included, against
    # the oracle at every stage
    ds = ds_of(n)
    dt = 0.1 * min(ds)
    f = fields(n, 5, kmax=1)
    rng = np.random.default_rng(6)
    mhd = MHD if model == S.MODEL_MHD_FULL else None
    for stage in (0, 1, 2):
        print("short axes %s model %d stage %d" % (n, model, stage), flush=True)
        plan = S.RkPlan(model, n, S.PREC_F64, variant=S.RK_LDS, mhd=mhd, **KW)
        b = plan.alloc()
        fin = [O.pad_periodic(v, 3) for v in f]
        w0 = [rng.uniform(-1e-2, 1e-2, fin[0].shape) for _ in range(8)]
        for k in range(8):
            put(b["f_a"][k], fin[k])
            put(b["w"][k], w0[k])
            b["f_b"][k].fill_(-9.0)
        plan.step(b["f_a"], b["f_b"], b["w"], stage, dt)
        torch.cuda.synchronize()
        w_ref = [a.copy() for a in w0]
        omodel = O.MODEL_MHD_FULL if model == S.MODEL_MHD_FULL else O.MODEL_MHD8
        ref = O.rk3_substep(omodel, stage, fin, w_ref, ds, dt, mhd=mhd, **KW)
        for k in range(8):
            got = host(b["f_b"][k])
            assert relerr(got, ref[k]) <= 1e-12, (n, stage, k, relerr(got, ref[k]))
            assert np.array_equal(got, O.fill_periodic(got.copy(), 3)), (n, stage, k)


def test_full_mhd_right_hand_side_terms_reach_the_update():
    # dt R is the stage-0 register: compare it with the oracle's right-hand
    # side directly, per field, on a state where every closure term is active
    n = (24, 20, 18)
    ds = ds_of(n)
    dt = 1e-3
    f = fields(n, 11)
    plan = S.RkPlan(S.MODEL_MHD_FULL, n, S.PREC_F64, mhd=MHD, **KW)
    b = plan.alloc()
    fin = [O.pad_periodic(v, 3) for v in f]
    for k in range(8):
        put(b["f_a"][k], fin[k])
    plan.step(b["f_a"], b["f_b"], b["w"], 0, dt)
    torch.cuda.synchronize()
    R = O.rhs(O.MODEL_MHD_FULL, fin, ds, mhd=MHD, **KW)
    for k in range(8):
        got = O.interior(host(b["w"][k]), 3) / dt
        assert relerr(got, O.interior(R[k], 3)) <= 1e-12, k


@pytest.mark.parametrize("n", [(3, 3, 3), (5, 4, 7), (17, 9, 33)])
@pytest.mark.parametrize("block", [(16, 8, 4), (8, 8, 8)])
def test_full_mhd_lds_bricks_on_tiny_and_ragged_grids(n, block):
    ds = ds_of(n)
    dt = 0.05 * min(ds)
    f = fields(n, 4, kmax=1)
    plan = S.RkPlan(S.MODEL_MHD_FULL, n, S.PREC_F64, variant=S.RK_LDS, block=block, mhd=MHD,
                    **KW)
    b = plan.alloc()
    for k in range(8):
        put(b["f_a"][k], O.pad_periodic(f[k], 3))
    res = plan.run(b["f_a"], b["f_b"], b["w"], 2, dt)
    ref = O.rk3_steps(O.MODEL_MHD_FULL, [O.pad_periodic(v, 3) for v in f], ds, dt, 2, mhd=MHD,
                      **KW)
    for k in range(8):
        assert relerr(host(res[k]), ref[k]) <= 1e-12, (n, block, k)


def test_full_mhd_three_steps_f64_pitched_layout():
    n = (33, 26, 21)
    ds = ds_of(n)
    dt = 0.1 * min(ds)
    f = fields(n, 3)
    plan = S.RkPlan(S.MODEL_MHD_FULL, n, S.PREC_F64, row_pitch=64, x_offset=16, mhd=MHD, **KW)
    b = plan.alloc()
    for k in range(8):
        b["f_a"][k].fill_(float("nan"))  # columns outside the padded field stay unread
        put(plan.padded(b["f_a"][k]), O.pad_periodic(f[k], 3))
    res = plan.run(b["f_a"], b["f_b"], b["w"], 3, dt)
    ref = O.rk3_steps(O.MODEL_MHD_FULL, [O.pad_periodic(v, 3) for v in f], ds, dt, 3, mhd=MHD,
                      **KW)
    for k in range(8):
        got = O.interior(host(plan.padded(res[k])), 3)
        assert relerr(got, O.interior(ref[k], 3)) <= 1e-12, k


def run_policy(n, prec, f, steps, dt, **kw):
    plan = S.RkPlan(S.MODEL_MHD_FULL, n, prec, **kw)
    b = plan.alloc()
    for k, v in enumerate(f):
        put(b["f_a"][k], O.pad_periodic(v, 3))
        if plan.master:
            put(b["f64"][k], O.pad_periodic(v, 3))
    res = plan.run(b["f_a"], b["f_b"], b["w"], steps, dt, w2=b["w2"], f64=b["f64"])
    lp = [host(t) for t in res]
    master = [host(t) for t in b["f64"]] if plan.master else None
    return lp, master


@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_full_mhd_mixed_precision_error_vs_fp64(store):
    n = (32, 24, 20)
    ds = ds_of(n)
    dt = 0.1 * min(ds)
    steps = 10
    f = fields(n, 7)
    ref = O.rk3_steps(O.MODEL_MHD_FULL, [O.pad_periodic(v, 3) for v in f], ds, dt, steps,
                      mhd=MHD, **KW)
    pm, po = ((S.PREC_F32_MASTER64, S.PREC_F32_ONLY) if store == "f32"
              else (S.PREC_BF16_MASTER64, S.PREC_BF16_ONLY))
    lp_m, master = run_policy(n, pm, f, steps, dt, mhd=MHD, **KW)
    lp_o, _ = run_policy(n, po, f, steps, dt, mhd=MHD, **KW)
    err = lambda a: [relerr(O.interior(a[k], 3), O.interior(ref[k], 3)) for k in range(8)]
    e_m, e_o = err(master), err(lp_o)
    for name, e in (("master (FP64)", e_m), ("no master", e_o)):
        print("full MHD, %s storage, %d steps, %s error per field: %s"
              % (store, steps, name, " ".join("%.2e" % v for v in e)))
    rnd = np.stack([O.interior(m, 3) for m in master]).astype(np.float32).astype(np.float64)
    if store == "bf16":
        rnd = inputs.to_bf16_values(rnd)
    assert np.array_equal(rnd, np.stack([O.interior(v, 3) for v in lp_m]))
    assert np.mean(e_m) < np.mean(e_o)
    assert max(e_m) <= (1e-5 if store == "f32" else 3e-2)


@pytest.mark.parametrize("prec", [S.PREC_F32_MASTER64, S.PREC_BF16_MASTER64])
def test_full_mhd_lds_and_cached_banks_agree_in_mixed_precision(prec):
    n = (40, 24, 20)
    ds = ds_of(n)
    dt = 0.1 * min(ds)
    f = fields(n, 9)
    outs = []
    for variant in (S.RK_CACHED, S.RK_LDS):
        _, master = run_policy(n, prec, f, 2, dt, variant=variant, mhd=MHD, **KW)
        outs.append(master)
    # the banks differ only in FP32 summation order; where that moves the
    # master across a rounding boundary of the stored state, the stored value
    # differs by one unit (2^-24 FP32, 2^-8 BF16, relative), which the next
    # step's update carries with weight about dt sum|w1| / ds = 0.18
    tol = 1e-5 if prec == S.PREC_F32_MASTER64 else 2.0 ** -8 * 0.18 * 1.5
    for k in range(8):
        e = relerr(outs[1][k], outs[0][k])
        print("full MHD banks, precision %d, field %d: rel diff %.2e" % (prec, k, e))
        assert e <= tol, (prec, k)


@pytest.mark.parametrize("prec", [S.PREC_F32_ONLY, S.PREC_BF16_ONLY])
def test_full_mhd_lds_and_cached_banks_agree_without_master(prec):
    # the no-master ablations: the stored states of the two banks after two
    # steps; a rounding of the stored state can differ by one unit (2^-24
    # FP32, 2^-8 BF16, relative) at any of the 6 substeps
    n = (40, 24, 20)
    ds = ds_of(n)
    dt = 0.1 * min(ds)
    f = fields(n, 9)
    outs = []
    for variant in (S.RK_CACHED, S.RK_LDS):
        lp, _ = run_policy(n, prec, f, 2, dt, variant=variant, mhd=MHD, **KW)
        outs.append(lp)
    tol = 1e-5 if prec == S.PREC_F32_ONLY else 6 * 2.0 ** -8
    for k in range(8):
        e = relerr(outs[1][k], outs[0][k])
        print("full MHD banks, precision %d, field %d: rel diff %.2e" % (prec, k, e))
        assert e <= tol, (prec, k)


def test_full_mhd_256_cubed_sampled_points():
    n = (256, 256, 256)
    ds = ds_of(n)
    dt = 0.1 * min(ds)
    f, _ = inputs.fourier_fields(n, 1, nf=8, modes=8, kmax=8, amp=0.01)
    rng = np.random.default_rng(3)
    plan = S.RkPlan(S.MODEL_MHD_FULL, n, S.PREC_F64, mhd=MHD, **KW)
    b = plan.alloc()
    fin = []
    for k in range(8):
        fin.append(O.pad_periodic(f[k], 3))
        put(b["f_a"][k], fin[k])
    del f
    w0 = [rng.uniform(-1e-4, 1e-4, fin[0].shape) for _ in range(8)]
    for k in range(8):
        put(b["w"][k], w0[k])
    plan.step(b["f_a"], b["f_b"], b["w"], 1, dt)
    torch.cuda.synchronize()
    pts = np.concatenate([np.stack([rng.integers(0, 256, 3000) for _ in range(3)], axis=1),
                          np.array([[x, y, z] for x in (0, 255) for y in (0, 255)
                                    for z in (0, 255)])])
    w_in = np.array([[w0[k][p[2] + 3, p[1] + 3, p[0] + 3] for p in pts] for k in range(8)])
    w_at, f_at = O.rk3_substep_at(O.MODEL_MHD_FULL, 1, fin, w_in, ds, dt, pts, mhd=MHD, **KW)
    for k in range(8):
        gf = host(b["f_b"][k])
        gw = host(b["w"][k])
        vf = gf[pts[:, 2] + 3, pts[:, 1] + 3, pts[:, 0] + 3]
        vw = gw[pts[:, 2] + 3, pts[:, 1] + 3, pts[:, 0] + 3]
        assert relerr(vf, f_at[k]) <= 1e-12, k
        assert relerr(vw, w_at[k]) <= 1e-12, k


# diagonal (12-tap) mixed derivatives in the bank, both models, both banks

DIAG_BANKS = [(S.RK_CACHED, None), (S.RK_LDS, (16, 8, 8)), (S.RK_LDS, (32, 4, 4)),
              (S.RK_LDS, (16, 8, 4)), (S.RK_LDS, (8, 8, 8))]


@pytest.mark.parametrize("model", [S.MODEL_MHD8, S.MODEL_MHD_FULL])
@pytest.mark.parametrize("bank", range(len(DIAG_BANKS)))
@pytest.mark.parametrize("stage", [0, 2])
def test_diagonal_mixed_substep_f64(model, bank, stage):
    n = (40, 24, 20)
    ds = ds_of(n)
    dt = 0.1 * min(ds)
    f = fields(n, 21)
    rng = np.random.default_rng(22)
    variant, block = DIAG_BANKS[bank]
    print("diagonal mixed: model %d stage %d bank %s %s" % (model, stage, variant, block),
          flush=True)
    mhd = MHD if model == S.MODEL_MHD_FULL else None
    plan = S.RkPlan(model, n, S.PREC_F64, variant=variant, block=block, mhd=mhd,
                    mixed=S.MIXED_DIAGONAL, **KW)
    b = plan.alloc()
    fin = [O.pad_periodic(v, 3) for v in f]
    w0 = [rng.uniform(-1e-2, 1e-2, fin[0].shape) for _ in range(8)]
    for k in range(8):
        put(b["f_a"][k], fin[k])
        put(b["w"][k], w0[k] if stage else np.full(fin[0].shape, np.nan))
    plan.step(b["f_a"], b["f_b"], b["w"], stage, dt)
    torch.cuda.synchronize()
    w_ref = [a.copy() for a in w0]
    ref = O.rk3_substep(model, stage, fin, w_ref, ds, dt, mhd=mhd, mixed=O.MIXED_DIAG, **KW)
    ref_t = O.rk3_substep(model, stage, fin, [a.copy() for a in w0], ds, dt, mhd=mhd, **KW)
    for k in range(8):
        got = host(b["f_b"][k])
        assert relerr(got, ref[k]) <= 1e-12, (stage, k, relerr(got, ref[k]))
    # the two forms differ (u and A carry mixed terms), so the test can tell
    assert max(relerr(ref[k], ref_t[k]) for k in range(8)) > 1e-9


@pytest.mark.parametrize("n", [(3, 3, 3), (5, 4, 7), (17, 9, 33)])
def test_diagonal_mixed_on_tiny_and_ragged_grids(n):
    ds = ds_of(n)
    dt = 0.05 * min(ds)
    f = fields(n, 4, kmax=1)
    for variant, block in ((S.RK_LDS, (16, 8, 4)), (S.RK_CACHED, None)):
        plan = S.RkPlan(S.MODEL_MHD_FULL, n, S.PREC_F64, variant=variant, block=block, mhd=MHD,
                        mixed=S.MIXED_DIAGONAL, **KW)
        b = plan.alloc()
        for k in range(8):
            put(b["f_a"][k], O.pad_periodic(f[k], 3))
        res = plan.run(b["f_a"], b["f_b"], b["w"], 2, dt)
        ref = O.rk3_steps(O.MODEL_MHD_FULL, [O.pad_periodic(v, 3) for v in f], ds, dt, 2,
                          mhd=MHD, mixed=O.MIXED_DIAG, **KW)
        for k in range(8):
            assert relerr(host(res[k]), ref[k]) <= 1e-12, (n, variant, k)


@pytest.mark.parametrize("prec", [S.PREC_F32_MASTER64, S.PREC_BF16_MASTER64])
def test_diagonal_mixed_lds_and_cached_agree_in_mixed_precision(prec):
    n = (40, 24, 20)
    ds = ds_of(n)
    dt = 0.1 * min(ds)
    f = fields(n, 9)
    outs = []
    for variant in (S.RK_CACHED, S.RK_LDS):
        _, master = run_policy(n, prec, f, 2, dt, variant=variant, mhd=MHD,
                               mixed=S.MIXED_DIAGONAL, **KW)
        outs.append(master)
    tol = 1e-5 if prec == S.PREC_F32_MASTER64 else 2.0 ** -8 * 0.18 * 1.5
    for k in range(8):
        assert relerr(outs[1][k], outs[0][k]) <= tol, (prec, k)
