"""GPU tests of the batched job kernel and the continuous-batching server.

* a job's result is bitwise the same alone, in a mix, with and without graph
  replay, and through the solo fused-substep path (same per-point code);
* FP64 results match the CPU oracle within 1e-12 (normwise, per job) and the
  per-mode RK3 amplification closed form;
* failure handling forced from the host: a job larger than the budget fails
  with ENOMEM, cancellation, a NaN-poisoned job stays isolated, queue cap.
"""
import math

import numpy as np
import pytest

import oracle as O
from closed_forms import kappa, lam, rk3_stability
from paper_2406_08923_amd import inputs

torch = pytest.importorskip("torch")
import paper_2406_08923_amd as S  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def job_dt(n, c):
    return 0.1 * min(2 * math.pi / v for v in n) / max(1.0, max(abs(v) for v in c))


JOBS = [  # (dims (x[, y[, z]]), steps, precision, velocity, nu, seed)
    ((48, 40), 7, S.PREC_F64, (0.6, -0.3), 0.01, 1),
    ((21, 18, 15), 5, S.PREC_F64, (0.2, 0.5, -0.7), 0.02, 2),
    ((64, 33), 9, S.PREC_F32_MASTER64, (-0.4, 0.8), 0.005, 3),
    ((17, 16, 19), 4, S.PREC_F32_MASTER64, (0.1, 0.0, 0.3), 0.01, 4),
    ((130, 67), 3, S.PREC_F32_ONLY, (0.9, 0.9), 0.001, 5),
]


def make_init(dims, seed):
    return inputs.uniform_field(dims, seed)


def run_server(jobs, **kw):
    srv = S.Server(**kw)
    tickets = []
    for dims, steps, prec, c, nu, seed in jobs:
        tickets.append(srv.submit(make_init(dims, seed), steps, prec, nu=nu, adv=c,
                                  dt=job_dt(dims, c)))
    out = []
    for t in tickets:
        st = srv.wait(t, 120000)
        assert st["state"] == S.JOB_DONE, st
        assert 0 <= st["t_submit"] <= st["t_admit"] <= st["t_first_tick"] <= st["t_done"]
        out.append(srv.result(t).copy())
    stats = srv.stats()
    srv.close()
    return out, stats


def solo_path(dims, steps, prec, c, nu, seed):
    """The same job through stencil_plan_rk + stencil_rk_run (no batching)."""
    plan = S.RkPlan(S.MODEL_ADVDIFF, dims, prec, nu=nu, adv=c)
    b = plan.alloc()
    init = make_init(dims, seed)
    pad = O.pad_periodic(init, 3)
    b["f_a"][0].copy_(torch.from_numpy(pad).cuda().to(b["f_a"][0].dtype))
    if plan.master:
        b["f64"][0].copy_(torch.from_numpy(pad).cuda())
    res = plan.run(b["f_a"], b["f_b"], b["w"], steps, job_dt(dims, c), w2=b["w2"], f64=b["f64"])
    src = b["f64"][0] if plan.master else res[0]
    return O.interior(src.to(torch.float64).cpu().numpy(), 3)


def test_batch_matches_solo_mix_and_graph_bitwise():
    mix, stats = run_server(JOBS, tick_steps=3, use_graph=True, max_slots=16)
    assert stats["completed"] == len(JOBS) and stats["failed"] == 0
    nograph, _ = run_server(JOBS, tick_steps=2, use_graph=False, max_slots=2)
    for k, job in enumerate(JOBS):
        alone, _ = run_server([job], tick_steps=4, use_graph=True, max_slots=1)
        assert np.array_equal(mix[k], alone[0]), k
        assert np.array_equal(mix[k], nograph[k]), k
        assert np.array_equal(mix[k], solo_path(*job)), k


@pytest.mark.parametrize("min_points", [0, 3000, 1 << 40])
def test_both_policies_give_the_same_results(min_points):
    # the policy only changes which resident jobs a tick takes: every job's
    # result is bitwise that of the other policy and of the solo path, with
    # a tick size that fits all jobs, some, or one at a time
    ref, _ = run_server(JOBS, tick_steps=3, max_slots=16, policy=S.SERVE_SHORTEST)
    old, stats = run_server(JOBS, tick_steps=3, max_slots=16, min_points=min_points,
                            policy=S.SERVE_OLDEST)
    assert stats["completed"] == len(JOBS) and stats["failed"] == 0
    for k, job in enumerate(JOBS):
        assert np.array_equal(old[k], ref[k]), k
        assert np.array_equal(old[k], solo_path(*job)), k


@pytest.mark.parametrize("k", range(len(JOBS)))
def test_server_jobs_match_oracle(k):
    dims, steps, prec, c, nu, seed = JOBS[k]
    out, _ = run_server([JOBS[k]], tick_steps=4)
    ds = [2 * math.pi / v for v in dims]
    ref = O.rk3_steps(O.MODEL_ADVDIFF, [O.pad_periodic(make_init(dims, seed), 3)], ds,
                      job_dt(dims, c), steps, nu=nu, c=c)[0]
    err = relerr(out[0], O.interior(ref, 3))
    print("job %d precision %d: error vs FP64 oracle %.2e" % (k, prec, err))
    assert err <= (1e-12 if prec == S.PREC_F64 else 1e-5)


@pytest.mark.parametrize("ndim", [2, 3])
def test_server_fourier_modes_closed_form(ndim):
    # each Fourier mode is amplified by the RK3 stability polynomial of dt
    # times its symbol, per step (any grid size)
    n = (96, 80, 40)[:ndim]
    c = (0.5, -0.25, 0.75)[:ndim]
    nu, steps = 0.02, 12
    dt = job_dt(n, c)
    rng = np.random.default_rng(9)
    modes = inputs.draw_modes(rng, 3, ndim, 4, 1.0)
    init = inputs.eval_modes(n, modes)
    srv = S.Server(tick_steps=5)
    t = srv.submit(init, steps, S.PREC_F64, nu=nu, adv=c, dt=dt)
    assert srv.wait(t, 60000)["state"] == S.JOB_DONE
    got = srv.result(t)
    srv.close()
    X = inputs.grid_coords(n)
    ref = np.zeros_like(init)
    for kv, a, ph in modes:
        sym = complex(nu * sum(lam(kv[d], n[d]) for d in range(ndim)),
                      -sum(c[d] * kappa(kv[d], n[d]) for d in range(ndim)))
        G = rk3_stability(dt * sym) ** steps
        arg = ph + sum(kv[d] * X[d] for d in range(ndim))
        ref += a * np.real(G * np.exp(1j * arg))
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref)) + 1e-13


def test_job_larger_than_budget_fails_others_run():
    small = ((32, 32), 3, S.PREC_F64, (0.1, 0.2), 0.01, 1)
    srv = S.Server(hbm_budget=200_000, max_slots=4, tick_steps=2)
    big = srv.submit(make_init((100, 100), 2), 3, S.PREC_F64, nu=0.01)
    t = srv.submit(make_init(small[0], 1), 3, S.PREC_F64, nu=0.01, adv=small[3],
                   dt=job_dt(small[0], small[3]))
    sb = srv.wait(big, 30000)
    assert sb["state"] == S.JOB_FAILED and sb["error"] == -2
    assert srv.wait(t, 30000)["state"] == S.JOB_DONE
    srv.close()


def test_budget_admits_in_waves():
    # budget for about two jobs at a time: all still complete
    jobs = [((40, 40), 6, S.PREC_F64, (0.3, 0.1), 0.01, s) for s in range(6)]
    per = 46 * 46 * 24
    out, stats = run_server(jobs, hbm_budget=2 * per + 100, tick_steps=2)
    assert stats["completed"] == 6
    alone, _ = run_server(jobs[:1], tick_steps=2)
    assert np.array_equal(out[0], alone[0])


def test_cancel_running_and_queued():
    srv = S.Server(max_slots=1, tick_steps=1)
    long_job = srv.submit(make_init((64, 64, 64), 1), 100000, S.PREC_F64, nu=0.01)
    queued = srv.submit(make_init((16, 16), 2), 5, S.PREC_F64, nu=0.01)
    srv.cancel(queued)
    srv.cancel(long_job)
    assert srv.wait(long_job, 60000)["state"] == S.JOB_CANCELLED
    assert srv.wait(queued, 60000)["state"] == S.JOB_CANCELLED
    srv.close()


def test_nan_job_is_isolated():
    jobs = [((48, 40), 6, S.PREC_F64, (0.6, -0.3), 0.01, 1),
            ((21, 18, 15), 5, S.PREC_F64, (0.2, 0.5, -0.7), 0.02, 2)]
    ref, _ = run_server(jobs, tick_steps=3)
    srv = S.Server(tick_steps=3)
    bad = make_init((40, 40), 7)
    bad[3, 5] = np.nan
    tb = srv.submit(bad, 6, S.PREC_F64, nu=0.01)
    ts = [srv.submit(make_init(d, s), st, p, nu=nu, adv=c, dt=job_dt(d, c))
          for d, st, p, c, nu, s in jobs]
    for k, t in enumerate(ts):
        assert srv.wait(t, 60000)["state"] == S.JOB_DONE
        assert np.array_equal(srv.result(t), ref[k])
    assert srv.wait(tb, 60000)["state"] == S.JOB_DONE
    assert np.isnan(srv.result(tb)).any()
    srv.close()


def test_submit_validation_and_queue_cap():
    with pytest.raises(S.StencilError):
        S.Server(max_slots=1, tick_steps=1, policy=2)
    srv = S.Server(max_slots=1, tick_steps=1, queue_cap=1)
    with pytest.raises(S.StencilError):
        srv.submit(np.zeros((2, 8)), 3)  # dims < 3
    with pytest.raises(S.StencilError):
        srv.submit(np.zeros((8, 8)), 0)  # no steps
    with pytest.raises(S.StencilError):
        srv.submit(np.zeros((8, 8)), 3, precision=S.PREC_BF16_MASTER64)
    first = srv.submit(make_init((64, 64, 64), 1), 100000, S.PREC_F64)
    # wait until the first job is admitted, then fill the one queue place
    for _ in range(2000):
        if srv.poll(first)["state"] == S.JOB_RUNNING:
            break
        import time
        time.sleep(0.001)
    second = srv.submit(make_init((8, 8), 1), 2)
    with pytest.raises(S.StencilError) as ei:
        srv.submit(make_init((8, 8), 2), 2)
    assert ei.value.code == -5
    srv.cancel(first)
    srv.cancel(second)
    srv.close()


# 3-D jobs of at least 2^20 points run as z-march tiles in the batch (and in
# the solo plan); smaller ones keep the per-point kernel
BIG = [((128, 96, 96), 3, S.PREC_F64, (0.4, -0.6, 0.2), 0.01, 11),
       ((112, 100, 96), 2, S.PREC_F32_MASTER64, (-0.3, 0.5, 0.9), 0.02, 12),
       ((100, 104, 101), 2, S.PREC_F32_ONLY, (0.7, 0.1, -0.2), 0.005, 13)]


def test_zmarch_jobs_bitwise_alone_mixed_graph_and_solo():
    jobs = BIG + JOBS[:2]
    mix, stats = run_server(jobs, tick_steps=2, use_graph=True, max_slots=8)
    assert stats["completed"] == len(jobs)
    nograph, _ = run_server(jobs, tick_steps=1, use_graph=False, max_slots=2)
    for k, job in enumerate(BIG):
        alone, _ = run_server([job], tick_steps=3, use_graph=True, max_slots=1)
        assert np.array_equal(mix[k], alone[0]), k
        assert np.array_equal(mix[k], nograph[k]), k
        assert np.array_equal(mix[k], solo_path(*job)), k


def test_zmarch_job_matches_oracle():
    dims, steps, prec, c, nu, seed = BIG[0]
    out, _ = run_server([BIG[0]], tick_steps=2)
    ds = [2 * math.pi / v for v in dims]
    ref = O.rk3_steps(O.MODEL_ADVDIFF, [O.pad_periodic(make_init(dims, seed), 3)], ds,
                      job_dt(dims, c), steps, nu=nu, c=c)[0]
    assert relerr(out[0], O.interior(ref, 3)) <= 1e-12


def test_tuned_batch_schedules_change_no_bit(tmp_path, monkeypatch):
    # the server's per-class schedule search (z-march depth, per-point tile
    # shape) picks among launches that compute the same arithmetic per point:
    # every job's result is bitwise that of the fixed schedule and of the solo
    # path, and each class is searched once
    cache = tmp_path / "batch_tune.txt"
    monkeypatch.setenv("STENCIL_TUNE_CACHE", str(cache))
    jobs = BIG + JOBS
    fixed, _ = run_server(jobs, tick_steps=2, max_slots=16)
    tuned, stats = run_server(jobs, tick_steps=2, max_slots=16, tune=True)
    assert stats["completed"] == len(jobs) and stats["failed"] == 0
    assert stats["tuned_classes"] == len(jobs)  # every job here is its own class
    for k, job in enumerate(jobs):
        assert np.array_equal(tuned[k], fixed[k]), k
        assert np.array_equal(tuned[k], solo_path(*job)), k
    lines = [l for l in cache.read_text().splitlines() if l.startswith("batch|")]
    assert len(lines) == len(jobs)
    for l in lines:
        a, b = (int(v) for v in l.split()[1:])
        assert (a in (8, 16, 32, 64) and b == 0) or (a, b) in ((64, 4), (128, 2), (256, 1),
                                                                (32, 8)), l
    # a second server reads the choices back: no new search
    again, stats2 = run_server(jobs[:2], tick_steps=2, max_slots=16, tune=True)
    assert stats2["tuned_classes"] == 0
    for k in range(2):
        assert np.array_equal(again[k], fixed[k])
