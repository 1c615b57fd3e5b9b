"""Replay a seeded job trace against the continuous-batching server and
against a plain first-in-first-out per-job FP64 path on the same GPU.

Jobs are scalar advection-diffusion integrations (radius-3 sixth-order
stencils, RK3), 2-D or 3-D, with the trace's grid edge, step count, velocity
and per-request storage precision (FP32 requests run with FP32 storage and an
FP64 master; the FIFO baseline runs every job in FP64). Latency = completion
time - arrival time; throughput = sum of points x steps / makespan.
"""
import math
import threading
import time

import numpy as np

from . import PREC_F32_MASTER64, PREC_F64, MODEL_ADVDIFF, JOB_DONE, SERVE_OLDEST, RkPlan, Server
from . import inputs


def job_dims(job):
    return (job["edge"],) * job["ndim"]


def job_dt(job):
    n = job_dims(job)
    return 0.1 * min(2 * math.pi / v for v in n) / max(1.0, max(abs(v) for v in job["c"]))


def make_inits(jobs):
    """Initial fields (sum of the job's Fourier modes), generated once, on the
    GPU (the host takes minutes for a 384^3 job)."""
    return [inputs.eval_modes_device(job_dims(j), j["modes"]) for j in jobs]


def _percentiles(lat):
    a = np.sort(np.asarray(lat))
    return {"p50_s": float(np.percentile(a, 50)), "p99_s": float(np.percentile(a, 99)),
            "max_s": float(a[-1]), "mean_s": float(a.mean())}


def _by_dtype(jobs, lat, makespan):
    """p50/p99 latency and point-steps/s (over the whole makespan) of the FP32
    and the FP64 requests separately."""
    out = {}
    for dt in ("f32", "f64"):
        idx = [k for k, j in enumerate(jobs) if j["dtype"] == dt]
        if not idx:
            continue
        ps = sum(int(np.prod(job_dims(jobs[k]))) * jobs[k]["steps"] for k in idx)
        a = np.asarray([lat[k] for k in idx])
        out[dt] = {"jobs": len(idx), "p50_s": float(np.percentile(a, 50)),
                   "p99_s": float(np.percentile(a, 99)), "point_steps_per_s": ps / makespan}
    return out


def run_served(jobs, inits, tick_steps=16, max_slots=512, use_graph=True, min_points=0,
               policy=SERVE_OLDEST, tune=False):
    srv = Server(max_slots=max_slots, tick_steps=tick_steps, use_graph=use_graph,
                 min_points=min_points, policy=policy, tune=tune)
    tickets = [None] * len(jobs)
    start = srv.clock()

    def feeder():
        for k, j in enumerate(jobs):
            delay = start + j["arrival"] - srv.clock()
            if delay > 0:
                time.sleep(delay)
            prec = PREC_F32_MASTER64 if j["dtype"] == "f32" else PREC_F64
            tickets[k] = srv.submit(inits[k], j["steps"], prec, nu=j["nu"], adv=j["c"],
                                    dt=job_dt(j))

    th = threading.Thread(target=feeder)
    th.start()
    th.join()
    lat, results, done_t = [], [], []
    for k, t in enumerate(tickets):
        st = srv.wait(t)
        if st["state"] != JOB_DONE:
            raise RuntimeError("job %d ended in state %d (error %d)" % (k, st["state"],
                                                                       st["error"]))
        lat.append(st["t_done"] - (start + jobs[k]["arrival"]))
        done_t.append(st["t_done"])
        results.append(srv.result(t))
    stats = srv.stats()
    srv.close()
    makespan = max(done_t) - start
    out = _percentiles(lat)
    out.update({"makespan_s": makespan, "point_steps": stats["point_steps"],
                "point_steps_per_s": stats["point_steps"] / makespan,
                "ticks": stats["ticks"], "launches": stats["launches"],
                "busy_s": stats["busy_s"], "tuned_classes": stats["tuned_classes"],
                "by_dtype": _by_dtype(jobs, lat, makespan)})
    return out, results


def run_fifo_f64(jobs, inits):
    """One job at a time in arrival order, FP64, per-job kernels."""
    import torch
    t0 = time.perf_counter()
    lat, results = [], []
    pts_steps = 0
    for k, j in enumerate(jobs):
        now = time.perf_counter() - t0
        if now < j["arrival"]:
            time.sleep(j["arrival"] - now)
        n = job_dims(j)
        plan = RkPlan(MODEL_ADVDIFF, n, PREC_F64, nu=j["nu"], adv=j["c"])
        b = plan.alloc()
        r = 3
        sl = tuple(slice(r, r + v) for v in reversed(n))
        b["f_a"][0][sl] = torch.from_numpy(inits[k]).cuda()
        res = plan.run(b["f_a"], b["f_b"], b["w"], j["steps"], job_dt(j))
        out = res[0][sl].cpu().numpy()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0 - j["arrival"])
        results.append(out)
        pts_steps += int(np.prod(n)) * j["steps"]
        del b, plan
    makespan = time.perf_counter() - t0
    o = _percentiles(lat)
    o.update({"makespan_s": makespan, "point_steps": pts_steps,
              "point_steps_per_s": pts_steps / makespan,
              "by_dtype": _by_dtype(jobs, lat, makespan)})
    return o, results


def compare(jobs, served_res, fifo_res):
    """Max normwise relative difference of served results vs the FP64 path,
    separately for FP32-storage and FP64 requests."""
    e32, e64 = [0.0], [0.0]
    for j, a, b in zip(jobs, served_res, fifo_res):
        e = float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
        (e32 if j["dtype"] == "f32" else e64).append(e)
    return {"max_rel_err_f32_requests_vs_fp64": max(e32),
            "max_rel_err_f64_requests_vs_fp64": max(e64)}
