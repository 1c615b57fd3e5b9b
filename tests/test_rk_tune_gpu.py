"""GPU checks of the RK plans' schedule search (Sec. 5.1: launch parameters
searched at runtime, failed launches dropped; Sec. 5.4: register allocation
as a tuning knob), through the C ABI.

Every schedule the search can pick (LDS bricks with their occupancy targets,
cached-bank lane tiles, z-march depths) must match the oracle to 1e-12 in
FP64; schedules that differ only in occupancy or z-march depth compute the
same arithmetic per point and must agree bit for bit; an autotuned plan must
give bitwise the result of the plan pinned to the schedule it chose.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2406_08923_amd import inputs

torch = pytest.importorskip("torch")
import paper_2406_08923_amd as S  # noqa: E402

pytestmark = pytest.mark.gpu

NU, ETA, CS2 = 2e-3, 5e-3, 0.7
MHD = dict(zeta=3e-3, mu0=1.3, gamma=5.0 / 3.0, cp=1.7, lnrho0=0.2, K=4e-3, heat=2e-3,
           cool=5e-4)
BRICKS = [(16, 8, 4, 0), (16, 8, 4, 4), (16, 8, 8, 0), (32, 4, 4, 0), (32, 4, 4, 4),
          (8, 8, 8, 0), (8, 8, 8, 4)]
TILES = [(64, 4), (64, 2), (128, 2), (256, 1), (64, 1)]
N = (40, 24, 20)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def host(t):
    return t.to(torch.float64).cpu().numpy()


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def mhd_kw(model):
    kw = dict(nu=NU, eta=ETA, cs2=CS2)
    if model == S.MODEL_MHD_FULL:
        kw["mhd"] = MHD
    return kw


def run(model, prec, f, steps, dt, **plan_kw):
    plan = S.RkPlan(model, N, prec, **mhd_kw(model), **plan_kw)
    b = plan.alloc()
    for k, v in enumerate(f):
        pad = torch.from_numpy(O.pad_periodic(v, 3)).cuda()
        b["f_a"][k].copy_(pad.to(b["f_a"][k].dtype))
        if plan.master:
            b["f64"][k].copy_(pad)
    res = plan.run(b["f_a"], b["f_b"], b["w"], steps, dt, w2=b["w2"], f64=b["f64"])
    state = b["f64"] if plan.master else res
    return [host(t) for t in state], plan.schedule


@pytest.fixture(scope="module")
def case():
    f, _ = inputs.fourier_fields(N, 11, nf=8, modes=4, kmax=3, amp=0.3)
    ds = [2 * math.pi / v for v in N]
    dt = 0.1 * min(ds)
    refs = {}
    for model, om in ((S.MODEL_MHD8, O.MODEL_MHD8), (S.MODEL_MHD_FULL, O.MODEL_MHD_FULL)):
        kw = mhd_kw(model)
        refs[model] = O.rk3_steps(om, [O.pad_periodic(v, 3) for v in f], ds, dt, 2, **kw)
    return f, dt, refs


@pytest.mark.parametrize("model", [S.MODEL_MHD8, S.MODEL_MHD_FULL])
@pytest.mark.parametrize("sched", BRICKS + TILES)
def test_every_tuner_schedule_matches_the_oracle_f64(model, sched, case):
    f, dt, refs = case
    if len(sched) == 4:
        kw = dict(variant=S.RK_LDS, block=sched[:3], occupancy=sched[3])
    else:
        kw = dict(variant=S.RK_CACHED, block=sched)
    out, got_sched = run(model, S.PREC_F64, f, 2, dt, **kw)
    assert got_sched[1:4] == (tuple(sched[:3]) if len(sched) == 4 else tuple(sched) + (1,))
    for k in range(8):
        assert relerr(out[k], refs[model][k]) <= 1e-12, (sched, k)


@pytest.mark.parametrize("prec", [S.PREC_F64, S.PREC_F32_MASTER64, S.PREC_BF16_MASTER64])
@pytest.mark.parametrize("brick", [(16, 8, 4), (32, 4, 4), (8, 8, 8)])
@pytest.mark.parametrize("model", [S.MODEL_MHD8, S.MODEL_MHD_FULL])
def test_occupancy_targets_change_no_bit(model, brick, prec, case):
    f, dt, _ = case
    a, _ = run(model, prec, f, 2, dt, variant=S.RK_LDS, block=brick, occupancy=0)
    b, _ = run(model, prec, f, 2, dt, variant=S.RK_LDS, block=brick, occupancy=4)
    for k in range(8):
        assert np.array_equal(a[k], b[k]), (brick, prec, k)


def test_zmarch_depths_change_no_bit():
    n = (70, 37, 41)
    ds = [2 * math.pi / v for v in n]
    c = (0.7, -0.4, 0.3)
    dt = 0.1 * min(ds) / max(1.0, max(abs(v) for v in c))
    f0 = inputs.uniform_field(n, 5)
    outs = []
    for lz in (8, 16, 32, 64):
        plan = S.RkPlan(S.MODEL_ADVDIFF, n, S.PREC_F64, nu=0.01, adv=c, variant=S.RK_LDS,
                        block=(0, 0, lz))
        assert plan.schedule[3] == lz
        b = plan.alloc()
        b["f_a"][0].copy_(torch.from_numpy(O.pad_periodic(f0, 3)).cuda())
        outs.append(host(plan.run(b["f_a"], b["f_b"], b["w"], 3, dt)[0]))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    ref = O.rk3_steps(O.MODEL_ADVDIFF, [O.pad_periodic(f0, 3)], ds, dt, 3, nu=0.01, c=c)[0]
    assert relerr(outs[0], ref) <= 1e-12


@pytest.mark.parametrize("model,prec", [(S.MODEL_MHD8, S.PREC_F64),
                                        (S.MODEL_MHD_FULL, S.PREC_F32_MASTER64)])
def test_autotuned_plan_is_bitwise_its_pinned_schedule(model, prec, case, tmp_path,
                                                       monkeypatch):
    f, dt, refs = case
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("STENCIL_TUNE_CACHE", str(cache))
    tuned, sched = run(model, prec, f, 2, dt, autotune=True)
    variant, bx, by, bz, occ = sched
    assert variant in (S.RK_CACHED, S.RK_LDS)
    if variant == S.RK_LDS:
        assert (bx, by, bz, occ) in BRICKS
        kw = dict(variant=S.RK_LDS, block=(bx, by, bz), occupancy=occ)
    else:
        assert (bx, by) in TILES
        kw = dict(variant=S.RK_CACHED, block=(bx, by))
    pinned, _ = run(model, prec, f, 2, dt, **kw)
    for k in range(8):
        assert np.array_equal(tuned[k], pinned[k]), k
    if prec == S.PREC_F64:
        for k in range(8):
            assert relerr(tuned[k], refs[model][k]) <= 1e-12
    # the choice was recorded under its shape class in the cache file
    lines = cache.read_text().splitlines()
    assert any(l.startswith("rk|m%d|" % model) and l.split()[1:] == [str(v) for v in sched]
               for l in lines), lines
    print("autotuned schedule, model %d precision %d: %s" % (model, prec, sched))


def test_rk_plan_rejects_unbuilt_schedules():
    with pytest.raises(S.StencilError):
        S.RkPlan(S.MODEL_MHD8, N, S.PREC_F64, variant=S.RK_LDS, block=(16, 8, 8), occupancy=4)
    with pytest.raises(S.StencilError):
        S.RkPlan(S.MODEL_MHD8, N, S.PREC_F64, variant=S.RK_CACHED, occupancy=4)
    with pytest.raises(S.StencilError):
        S.RkPlan(S.MODEL_ADVDIFF, (32, 32), S.PREC_F64, occupancy=4)
