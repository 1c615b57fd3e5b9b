"""GPU parity of the fused substep (sixth-order derivative bank, nonlinear
right-hand side, Williamson RK3) and of the FP64 diagnostics, through the C ABI.

FP64 bar: normwise max relative error <= 1e-12 per field against the CPU
oracle. Mixed-precision policies are compared with the FP64 oracle and their
error is printed per field; the asserted ceilings are loose sanity limits.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2406_08923_amd import inputs

torch = pytest.importorskip("torch")
import paper_2406_08923_amd as S  # noqa: E402

pytestmark = pytest.mark.gpu

NU, ETA, CS2 = 2e-3, 5e-3, 0.7


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


def mhd_fields(n, seed, amp=0.3, kmax=3):
    f, _ = inputs.fourier_fields(n, seed, nf=8, modes=4, kmax=kmax, amp=amp)
    return f


def ds_of(n):
    return [2 * math.pi / v for v in n]


BANKS = [(S.RK_CACHED, None), (S.RK_LDS, None), (S.RK_LDS, (16, 8, 8)), (S.RK_LDS, (32, 4, 4)),
         (S.RK_LDS, (8, 8, 8))]


@pytest.mark.parametrize("bank", range(len(BANKS)))
@pytest.mark.parametrize("stage", [0, 1, 2])
def test_mhd8_substep_f64(stage, bank):
    n = (40, 24, 20)
    ds = ds_of(n)
    dt = 0.1 * min(ds)
    f = mhd_fields(n, 1)
    rng = np.random.default_rng(2)
    variant, block = BANKS[bank]
    plan = S.RkPlan(S.MODEL_MHD8, n, S.PREC_F64, nu=NU, eta=ETA, cs2=CS2, variant=variant,
                    block=block)
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
    ref = O.rk3_substep(O.MODEL_MHD8, stage, fin, w_ref, ds, dt, nu=NU, eta=ETA, cs2=CS2)
    for k in range(8):
        got = host(b["f_b"][k])
        assert relerr(got, ref[k]) <= 1e-12, (stage, k, relerr(got, ref[k]))
        gw = O.interior(host(b["w"][k]), 3)
        if stage < 2:
            assert relerr(gw, O.interior(w_ref[k], 3)) <= 1e-12, (stage, k)
        else:
            assert np.array_equal(gw, O.interior(w0[k], 3))  # dead register not written


@pytest.mark.parametrize("n", [(3, 3, 3), (5, 4, 7), (17, 9, 33)])
@pytest.mark.parametrize("block", [(16, 8, 4), (8, 8, 8)])
def test_mhd8_lds_bricks_on_tiny_and_ragged_grids(n, block):
    ds = ds_of(n)
    dt = 0.05 * min(ds)
    f = mhd_fields(n, 4, kmax=1)
    plan = S.RkPlan(S.MODEL_MHD8, n, S.PREC_F64, nu=NU, eta=ETA, cs2=CS2, variant=S.RK_LDS,
                    block=block)
    b = plan.alloc()
    for k in range(8):
        put(b["f_a"][k], O.pad_periodic(f[k], 3))
    res = plan.run(b["f_a"], b["f_b"], b["w"], 2, dt)
    ref = O.rk3_steps(O.MODEL_MHD8, [O.pad_periodic(v, 3) for v in f], ds, dt, 2, nu=NU,
                      eta=ETA, cs2=CS2)
    for k in range(8):
        assert relerr(host(res[k]), ref[k]) <= 1e-12, (n, block, k)


@pytest.mark.parametrize("prec", [S.PREC_F32_MASTER64, S.PREC_BF16_MASTER64, S.PREC_F32_ONLY,
                                  S.PREC_BF16_ONLY])
def test_mhd8_lds_and_cached_banks_agree_in_mixed_precision(prec):
    # same arithmetic type, different summation order of the grad(div)
    # terms: the banks agree to a few units of the storage rounding
    n = (40, 24, 20)
    ds = ds_of(n)
    dt = 0.1 * min(ds)
    f = mhd_fields(n, 9)
    outs = []
    for variant in (S.RK_CACHED, S.RK_LDS):
        lp, master = run_policy(n, prec, f, 2, dt, nu=NU, eta=ETA, cs2=CS2, variant=variant)
        outs.append(master if master is not None else lp)
    tol = 1e-4 if prec in (S.PREC_BF16_MASTER64, S.PREC_BF16_ONLY) else 1e-5
    if prec == S.PREC_BF16_ONLY:
        # no master: a BF16 rounding of the two banks' states can differ by
        # one unit (2^-8 relative) after any of the 6 substeps
        tol = 6 * 2.0 ** -8
    for k in range(8):
        assert relerr(outs[1][k], outs[0][k]) <= tol, (prec, k)


@pytest.mark.parametrize("n", [(3, 3, 3), (5, 4, 7), (17, 9, 33)])
@pytest.mark.parametrize("block", [(32, 4, 4), (16, 8, 4)])
@pytest.mark.parametrize("prec", [S.PREC_F32_MASTER64, S.PREC_BF16_MASTER64])
def test_mhd8_lds_bricks_mixed_precision_on_tiny_and_ragged_grids(prec, block, n):
    # FP32 storage fills its tiles with 4-byte buffer loads straight into LDS,
    # BF16 through registers: bricks larger than the grid and ragged in every
    # axis, against the cached bank (same arithmetic type)
    ds = ds_of(n)
    dt = 0.05 * min(ds)
    f = mhd_fields(n, 5, kmax=1)
    _, ref = run_policy(n, prec, f, 2, dt, nu=NU, eta=ETA, cs2=CS2, variant=S.RK_CACHED)
    _, got = run_policy(n, prec, f, 2, dt, nu=NU, eta=ETA, cs2=CS2, variant=S.RK_LDS, block=block)
    tol = 1e-4 if prec == S.PREC_BF16_MASTER64 else 1e-5
    for k in range(8):
        assert relerr(got[k], ref[k]) <= tol, (prec, block, n, k)


def test_mhd8_three_steps_f64_run():
    n = (33, 26, 21)
    ds = ds_of(n)
    dt = 0.1 * min(ds)
    f = mhd_fields(n, 3)
    plan = S.RkPlan(S.MODEL_MHD8, n, S.PREC_F64, nu=NU, eta=ETA, cs2=CS2)
    b = plan.alloc()
    for k in range(8):
        put(b["f_a"][k], O.pad_periodic(f[k], 3))
    res = plan.run(b["f_a"], b["f_b"], b["w"], 3, dt)
    ref = O.rk3_steps(O.MODEL_MHD8, [O.pad_periodic(v, 3) for v in f], ds, dt, 3, nu=NU,
                      eta=ETA, cs2=CS2)
    for k in range(8):
        assert relerr(host(res[k]), ref[k]) <= 1e-12, k


@pytest.mark.parametrize("n", [(50, 37), (30, 20, 17), (3, 3, 3), (64, 4)])
def test_advdiff_steps_f64(n):
    ds = ds_of(n)
    c = (0.7, -0.4, 0.3)[:len(n)]
    dt = 0.1 * min(ds) / max(1.0, max(abs(v) for v in c))
    f0 = inputs.uniform_field(n, 5)
    plan = S.RkPlan(S.MODEL_ADVDIFF, n, S.PREC_F64, nu=0.01, adv=c)
    b = plan.alloc()
    put(b["f_a"][0], O.pad_periodic(f0, 3))
    res = plan.run(b["f_a"], b["f_b"], b["w"], 2, dt)
    ref = O.rk3_steps(O.MODEL_ADVDIFF, [O.pad_periodic(f0, 3)], ds, dt, 2, nu=0.01, c=c)
    assert relerr(host(res[0]), ref[0]) <= 1e-12


@pytest.mark.parametrize("n,layout", [((48, 40), (0, 0)), ((72, 72), (0, 0)), ((64, 6), (0, 0)),
                                      ((50, 37), (70, 8))])
@pytest.mark.parametrize("steps", [1, 2, 7])
def test_advdiff_resident_run_bitwise_equal_to_substep_launches(n, layout, steps):
    # a small 2-D FP64 plan with the automatic variant keeps the whole run in
    # LDS (one launch); the per-point variant launches every substep. Both
    # state buffers (with their halos) and the register must agree bitwise.
    ds = ds_of(n)
    c = (0.6, -0.8)
    dt = 0.1 * min(ds) / max(1.0, max(abs(v) for v in c))
    f0 = inputs.uniform_field(n, 9)
    outs = []
    for variant in (0, S.RK_CACHED):
        plan = S.RkPlan(S.MODEL_ADVDIFF, n, S.PREC_F64, nu=0.02, adv=c, variant=variant,
                        row_pitch=layout[0], x_offset=layout[1])
        b = plan.alloc()
        pad = O.pad_periodic(f0, 3)
        plan.padded(b["f_a"][0]).copy_(torch.from_numpy(pad).cuda())
        b["f_b"][0].fill_(-7.0)
        b["w"][0].fill_(0.0)
        res = plan.run(b["f_a"], b["f_b"], b["w"], steps, dt)
        torch.cuda.synchronize()
        outs.append([host(plan.padded(b["f_a"][0])), host(plan.padded(b["f_b"][0])),
                     O.interior(host(plan.padded(b["w"][0])), 3),
                     res[0].data_ptr() == b["f_b"][0].data_ptr()])
    for k in range(4):
        assert np.array_equal(outs[0][k], outs[1][k]), (n, steps, k)
    assert outs[0][3] == (steps % 2 == 1)
    ref = O.rk3_steps(O.MODEL_ADVDIFF, [O.pad_periodic(f0, 3)], ds, dt, steps, nu=0.02, c=c)
    last = outs[0][1] if steps % 2 else outs[0][0]
    assert relerr(last, ref[0]) <= 1e-12


def run_policy(n, prec, f, steps, dt, model=S.MODEL_MHD8, **kw):
    plan = S.RkPlan(model, n, prec, **kw)
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
def test_mhd8_mixed_precision_error_vs_fp64(store):
    # error of the stored state after 10 steps against the FP64 oracle, per
    # field, with the FP64 master and without it (ablation)
    n = (32, 24, 20)
    ds = ds_of(n)
    dt = 0.1 * min(ds)
    steps = 10
    f = mhd_fields(n, 7)
    ref = O.rk3_steps(O.MODEL_MHD8, [O.pad_periodic(v, 3) for v in f], ds, dt, steps, nu=NU,
                      eta=ETA, cs2=CS2)
    pm, po = ((S.PREC_F32_MASTER64, S.PREC_F32_ONLY) if store == "f32"
              else (S.PREC_BF16_MASTER64, S.PREC_BF16_ONLY))
    lp_m, master = run_policy(n, pm, f, steps, dt, nu=NU, eta=ETA, cs2=CS2)
    lp_o, _ = run_policy(n, po, f, steps, dt, nu=NU, eta=ETA, cs2=CS2)
    err = lambda a: [relerr(O.interior(a[k], 3), O.interior(ref[k], 3)) for k in range(8)]
    e_m, e_lp, e_o = err(master), err(lp_m), err(lp_o)
    for name, e in (("master (FP64)", e_m), ("stored", e_lp), ("no master", e_o)):
        print("%s storage, %d steps, %s error per field: %s"
              % (store, steps, name, " ".join("%.2e" % v for v in e)))
    # the stored state is exactly the rounding of the FP64 master (to FP32,
    # then for BF16 storage from FP32 to BF16, both to nearest even)
    rnd = np.stack([O.interior(m, 3) for m in master]).astype(np.float32).astype(np.float64)
    if store == "bf16":
        rnd = inputs.to_bf16_values(rnd)
    assert np.array_equal(rnd, np.stack([O.interior(v, 3) for v in lp_m]))
    # the master removes the accumulation of storage rounding in the state
    assert np.mean(e_m) < np.mean(e_o)
    assert max(e_m) <= (1e-5 if store == "f32" else 3e-2)


def test_mhd8_256_cubed_sampled_points():
    n = (256, 256, 256)
    ds = ds_of(n)
    dt = 0.1 * min(ds)
    f, _ = inputs.fourier_fields(n, 1, nf=8, modes=8, kmax=8, amp=0.01)
    rng = np.random.default_rng(3)
    plan = S.RkPlan(S.MODEL_MHD8, n, S.PREC_F64)
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
                          np.array([[x, y, z] for x in (0, 255) for y in (0, 255) for z in (0, 255)])])
    w_in = np.array([[w0[k][p[2] + 3, p[1] + 3, p[0] + 3] for p in pts] for k in range(8)])
    w_at, f_at = O.rk3_substep_at(O.MODEL_MHD8, 1, fin, w_in, ds, dt, pts)
    for k in range(8):
        gf = host(b["f_b"][k])
        gw = host(b["w"][k])
        vf = gf[pts[:, 2] + 3, pts[:, 1] + 3, pts[:, 0] + 3]
        vw = gw[pts[:, 2] + 3, pts[:, 1] + 3, pts[:, 0] + 3]
        assert relerr(vf, f_at[k]) <= 1e-12, k
        assert relerr(vw, w_at[k]) <= 1e-12, k


@pytest.mark.parametrize("dtype", [S.F64, S.F32, S.BF16])
def test_reduce_matches_oracle_and_is_deterministic(dtype):
    n = (70, 37, 29)
    plan = S.RkPlan(S.MODEL_MHD8, n, S.PREC_F64)
    rng = np.random.default_rng(6)
    fields, pads = [], []
    for k in range(3):
        v = rng.uniform(-1, 1, tuple(reversed(n)))
        if dtype == S.F32:
            v = v.astype(np.float32).astype(np.float64)
        elif dtype == S.BF16:
            v = inputs.to_bf16_values(v)
        pad = np.full(O.padded_shape(n, 3), 1e6)  # halo must not count
        O.interior(pad, 3)[...] = v
        pads.append(pad)
        t = torch.from_numpy(pad).cuda().to(S.torch_dtype(dtype))
        fields.append(t)
    got = plan.reduce(fields, dtype)
    again = plan.reduce(fields, dtype)
    assert np.array_equal(got, again)
    for k in range(3):
        ref = O.reduce(pads[k], 3)
        absum = math.fsum(np.abs(O.interior(pads[k], 3)).ravel())
        assert abs(got[k, 0] - math.fsum(O.interior(pads[k], 3).ravel())) <= 1e-13 * absum
        assert abs(got[k, 1] - ref[1]) <= 1e-13 * ref[1]
        assert got[k, 2] == ref[2]


def test_step_validation():
    plan = S.RkPlan(S.MODEL_ADVDIFF, (16, 16), S.PREC_F64)
    b = plan.alloc()
    with pytest.raises(S.StencilError):
        plan.step(b["f_a"], b["f_a"], b["w"], 0, 0.1)  # in == out
    with pytest.raises(S.StencilError):
        plan.step(b["f_a"], b["f_b"], b["w"], 3, 0.1)
    with pytest.raises(S.StencilError):
        S.RkPlan(S.MODEL_MHD8, (16, 16), S.PREC_F64)
    with pytest.raises(S.StencilError):
        S.RkPlan(S.MODEL_ADVDIFF, (2, 16), S.PREC_F64)
    mp = S.RkPlan(S.MODEL_ADVDIFF, (16, 16), S.PREC_F32_MASTER64)
    mb = mp.alloc()
    with pytest.raises(S.StencilError):
        mp.step(mb["f_a"], mb["f_b"], mb["w"], 2, 0.1)  # master policy needs w2 and f64


# ---------------------------------------------------------------------------
# pitched layout: interior at column x_offset of rows of row_pitch elements
# ---------------------------------------------------------------------------

def run_layout(model, n, prec, f, steps, dt, layout, **kw):
    plan = S.RkPlan(model, n, prec, row_pitch=layout[0], x_offset=layout[1], **kw)
    b = plan.alloc()
    for k, v in enumerate(f):
        b["f_a"][k].fill_(11.0)  # columns outside the padded rows
        plan.padded(b["f_a"][k]).copy_(
            torch.from_numpy(O.pad_periodic(v, 3)).cuda().to(b["f_a"][k].dtype))
        if plan.master:
            plan.padded(b["f64"][k]).copy_(torch.from_numpy(O.pad_periodic(v, 3)).cuda())
    res = plan.run(b["f_a"], b["f_b"], b["w"], steps, dt, w2=b["w2"], f64=b["f64"])
    state = b["f64"] if plan.master else res
    out = [host(plan.padded(t)) for t in state]
    lo, hi = plan.x_offset - 3, plan.x_offset + n[0] + 3
    untouched = all(bool((host(t)[..., :lo] == 11.0).all() and (host(t)[..., hi:] == 11.0).all())
                    for t in b["f_a"])
    red = plan.reduce(state, dtype=S.F64 if plan.master else None)
    return out, untouched, red


@pytest.mark.parametrize("bank", [S.RK_LDS, S.RK_CACHED])
def test_mhd8_pitched_layout_f64_matches_oracle(bank):
    n = (40, 24, 20)
    ds = ds_of(n)
    dt = 0.1 * min(ds)
    f = mhd_fields(n, 5)
    out, untouched, red = run_layout(S.MODEL_MHD8, n, S.PREC_F64, f, 2, dt, (64, 16),
                                     nu=NU, eta=ETA, cs2=CS2, variant=bank)
    ref = O.rk3_steps(O.MODEL_MHD8, [O.pad_periodic(v, 3) for v in f], ds, dt, 2, nu=NU,
                      eta=ETA, cs2=CS2)
    for k in range(8):
        assert relerr(out[k], ref[k]) <= 1e-12, k
        assert np.array_equal(out[k], O.fill_periodic(out[k].copy(), 3))
        want = O.reduce(ref[k], 3)
        assert abs(red[k][0] - want[0]) <= 1e-12 * np.sum(np.abs(O.interior(ref[k], 3)))
    assert untouched


@pytest.mark.parametrize("prec", [S.PREC_F32_MASTER64, S.PREC_BF16_MASTER64])
def test_mhd8_pitched_layout_bitwise_equal_to_compact(prec):
    n = (40, 24, 20)
    dt = 0.1 * min(ds_of(n))
    f = mhd_fields(n, 6)
    a, _, _ = run_layout(S.MODEL_MHD8, n, prec, f, 2, dt, (0, 0))
    b, untouched, _ = run_layout(S.MODEL_MHD8, n, prec, f, 2, dt, (96, 32))
    for k in range(8):
        assert np.array_equal(a[k], b[k]), k
    assert untouched


@pytest.mark.parametrize("n", [(50, 37), (30, 20, 17)])
def test_advdiff_pitched_layout(n):
    ds = ds_of(n)
    c = (0.7, -0.4, 0.3)[:len(n)]
    dt = 0.1 * min(ds) / max(1.0, max(abs(v) for v in c))
    f0 = inputs.uniform_field(n, 5)
    out, untouched, _ = run_layout(S.MODEL_ADVDIFF, n, S.PREC_F64, [f0], 2, dt,
                                   (n[0] + 20, 8), nu=0.01, adv=c)
    ref = O.rk3_steps(O.MODEL_ADVDIFF, [O.pad_periodic(f0, 3)], ds, dt, 2, nu=0.01, c=c)
    assert relerr(out[0], ref[0]) <= 1e-12
    assert untouched


@pytest.mark.parametrize("prec", [S.PREC_F64, S.PREC_F32_MASTER64])
@pytest.mark.parametrize("lz", [0, 5, 64])
def test_advdiff_zmarch_matches_oracle_and_cached(prec, lz):
    n = (70, 37, 41)  # ragged against the 64 x 16 tiles
    ds = ds_of(n)
    c = (0.7, -0.4, 0.3)
    dt = 0.1 * min(ds) / max(1.0, max(abs(v) for v in c))
    f0 = inputs.uniform_field(n, 5)
    outs = []
    for variant, block in ((S.RK_LDS, (0, 0, lz)), (S.RK_CACHED, None)):
        lp, master = run_policy(n, prec, [f0], 3, dt, model=S.MODEL_ADVDIFF, nu=0.01, adv=c,
                                variant=variant, block=block)
        # the FP64 master holds interior values only (its halo is never read)
        outs.append(O.interior(master[0] if master is not None else lp[0], 3))
    ref = O.interior(O.rk3_steps(O.MODEL_ADVDIFF, [O.pad_periodic(f0, 3)], ds, dt, 3, nu=0.01,
                                 c=c)[0], 3)
    tol = 1e-12 if prec == S.PREC_F64 else 1e-5
    assert relerr(outs[0], ref) <= tol
    assert relerr(outs[0], outs[1]) <= tol


@pytest.mark.parametrize("prec", [S.PREC_BF16_MASTER64, S.PREC_F32_ONLY, S.PREC_BF16_ONLY])
def test_advdiff_zmarch_other_policies(prec):
    # the z march's prefetched registers per policy: no master (F32/BF16
    # only) and the BF16 master; compared with the FP64 oracle and with the
    # per-point kernel (same arithmetic type, other summation order)
    n = (70, 37, 41)
    ds = ds_of(n)
    c = (0.7, -0.4, 0.3)
    dt = 0.1 * min(ds) / max(1.0, max(abs(v) for v in c))
    f0 = inputs.uniform_field(n, 5)
    outs = []
    for variant, block in ((S.RK_LDS, (0, 0, 8)), (S.RK_CACHED, None)):
        lp, master = run_policy(n, prec, [f0], 3, dt, model=S.MODEL_ADVDIFF, nu=0.01, adv=c,
                                variant=variant, block=block)
        outs.append(O.interior(master[0] if master is not None else lp[0], 3))
    ref = O.interior(O.rk3_steps(O.MODEL_ADVDIFF, [O.pad_periodic(f0, 3)], ds, dt, 3, nu=0.01,
                                 c=c)[0], 3)
    bf16 = prec in (S.PREC_BF16_MASTER64, S.PREC_BF16_ONLY)
    # storage rounding (2^-8 BF16, 2^-24 FP32, relative) entering each of the
    # 9 substeps, amplified by at most the step operator's norm (< 2 here)
    u = 2.0 ** -8 if bf16 else 2.0 ** -24
    print("advdiff z march, precision %d: error vs FP64 %.2e, vs per-point kernel %.2e"
          % (prec, relerr(outs[0], ref), relerr(outs[0], outs[1])))
    assert relerr(outs[0], ref) <= 9 * 2 * u
    assert relerr(outs[0], outs[1]) <= 9 * 2 * u
