#!/usr/bin/env python3
"""Benchmark of the stencil hot path on one MI355X.

Headline workload: the 3-D linear cross-correlation with the 19-point radius-3
star (one forward-Euler step of the sixth-order diffusion operator, Eq. 5/7),
512^3 FP64, periodic halo, 100 chained iterations. One step = one iteration;
the default plan runs two iterations per kernel launch (temporal blocking,
bitwise equal to one-iteration launches), so 100 steps are 50 launches.
Input: seeded uniform [-1, 1), resident in HBM before timing starts.

Prints one JSON line (kept short): grid-point updates/s, the HBM roofline of
the dominant kernel (algorithmic bytes per launch / average launch duration
from HIP events recorded on the launch stream), the measured HBM traffic of
that kernel, the CPU oracle timed on a bounded sample, and one compact entry
per other workload (1-D radius-1 smoother; FP32 star with its error against
FP64; radius-4 star; fused 8-field RK3 step in FP64 and with FP32/BF16
storage, with the storage policies' error after 1/10/100/1000 steps; the
serving trace). The full record (per-field errors, radius sweep, filters,
serving rate sweep) goes to stderr and, with --detail-out, to a file.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DTYPES = {"f64": (0, 8), "f32": (1, 4), "bf16": (2, 2)}
METRIC = "grid-point updates/s + % HBM roofline; served p50/p99 latency vs plain FP64"
# constants of the full non-ideal model in the benchmark: every closure term on
FULL_MHD = dict(zeta=3e-3, mu0=1.0, gamma=5.0 / 3.0, cp=1.0, lnrho0=0.0, K=4e-3, heat=2e-3,
                cool=5e-4)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dtype", choices=sorted(DTYPES), default="f64")
    ap.add_argument("--n", type=int, default=512, help="grid edge")
    ap.add_argument("--radius", type=int, default=3)
    ap.add_argument("--tile", default=None,
                    help="star3d launch shape TY,NY,LZ,FLAGS (FLAGS may be hex)")
    ap.add_argument("--autotune", action="store_true",
                    help="time the launch candidates first (default: the plan's default "
                         "shape, the one measured fastest for this workload)")
    ap.add_argument("--layout", choices=("auto", "compact", "aligned"), default="auto",
                    help="field rows: compact (n + 2r cells) or padded so each interior row "
                         "starts a 128-byte line; auto = compact for FP64, aligned for the "
                         "narrower types (what measured faster for each)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--no-copy", action="store_true", help="skip the copy-bandwidth probe")
    ap.add_argument("--no-secondary", action="store_true", help="headline workload only")
    ap.add_argument("--no-precision-error", action="store_true",
                    help="skip the 1000-step mixed-precision error measurement")
    ap.add_argument("--precision-n", type=int, default=256,
                    help="grid edge of the 1000-step mixed-precision error measurement")
    ap.add_argument("--serve-rates", default="10,25,50",
                    help="mean arrival rates (jobs/s) of the sustainable-load replays of the "
                         "serving trace (empty: none)")
    ap.add_argument("--serve-jobs", type=int, default=400,
                    help="jobs in the serving trace (0 skips the serving comparison)")
    ap.add_argument("--serve-sweep-jobs", type=int, default=48,
                    help="jobs of the trace replayed at the sustainable rates")
    ap.add_argument("--detail-out", default=None,
                    help="also write the full record (JSON) to this file")
    ap.add_argument("--only", default=None,
                    help="comma list of secondary sections to run (stars, lines, filters, box, "
                         "mhd, precision, serving); default: all")
    return ap.parse_args()


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2406_08923_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(name, files):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != source_hash(files):
        return None
    return d.get("hbm_bytes_per_launch")


def timed(torch, fn, reps, warm=2):
    """Average ms per call of fn over reps calls (HIP events on the current
    stream)."""
    for _ in range(warm):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def copy_bandwidth(torch, S, nbytes=2 << 30, reps=20):
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    ms = timed(torch, lambda: S.copy(src, dst), reps, warm=3)
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(n, r, g, seconds):
    """The oracle as it stands (dense (2r+1)^3 tap loop, OpenMP over z) on an
    n x n x nz slab of the same workload; nz grown until the run takes about
    `seconds`."""
    import oracle as O
    from paper_2406_08923_amd import inputs
    nz, t = 2, 0.0
    while True:
        a = O.pad_periodic(inputs.uniform_field((n, n, nz), 1), r)
        t0 = time.perf_counter()
        O.xcorr(a, r, g)
        t = time.perf_counter() - t0
        if t >= seconds / 4 or nz >= n:
            break
        nz = min(n, max(nz * 2, int(nz * seconds / 4 / max(t, 1e-3))))
    if t < seconds / 2 and nz < n:
        reps = max(1, int(seconds / max(t, 1e-3)))
        t0 = time.perf_counter()
        for _ in range(reps):
            O.xcorr(a, r, g)
        t = (time.perf_counter() - t0) / reps
    return {"value": n * n * nz / t, "unit": "grid-point updates/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": "oracle FP64 dense %d-tap loop, one iteration on a %dx%dx%d periodic slab "
                      "(same row length and input distribution), %.2f s per run"
                      % ((2 * r + 1) ** 3, n, n, nz, t)}


def star_run(torch, S, W, inputs, n, r, dtype, steps, warmup, tile=None, layout="auto",
             autotune=False):
    """Chained iterations of the star workload: `warmup` untimed iterations,
    then `steps` iterations in one apply call bracketed by HIP events on the
    launch stream (the library issues the launches back to back). Returns
    (plan, coefficients, total ms, mean ms per launch, launch counts).
    layout: "compact", "aligned" (each interior row starts a 128-byte line) or
    "auto" (compact for FP64, aligned otherwise)."""
    dims = (n, n, n)
    g = W.diffusion_star(3, r, W.diffusion_number(n))
    es = {S.F64: 8, S.F32: 4, S.BF16: 2}[dtype]
    aligned = layout == "aligned" or (layout == "auto" and dtype != S.F64)
    pitch, ox = W.aligned_layout(n, r, es) if aligned else (0, 0)
    if tile:
        plan = S.LinearPlan(dims, r, g, dtype=dtype, variant=S.STAR3D, tile=tile,
                            row_pitch=pitch, x_offset=ox)
    else:
        plan = S.LinearPlan(dims, r, g, dtype=dtype, autotune=autotune, row_pitch=pitch,
                            x_offset=ox)
    a = plan.empty(0.0)
    plan.padded(a)[r:r + n, r:r + n, r:r + n] = torch.from_numpy(
        inputs.uniform_field(dims, 1)).to("cuda").to(a.dtype)
    b = plan.empty(0.0)
    plan.halo(a)
    res = plan.apply(a, b, warmup) if warmup else a
    cur, nxt = (res, b if res is a else a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    res = plan.apply(cur, nxt, steps, halo_valid=True)
    e1.record()
    torch.cuda.synchronize()
    total = e0.elapsed_time(e1)
    n_multi, n_single = plan.launches(steps)
    nlaunch = n_multi + n_single
    del a, b, cur, nxt, res
    return plan, g, total, total / max(1, nlaunch), (n_multi, n_single)


def paper_ideal_ms(points):
    """The paper's ideal time of one fused MHD substep (Sec. 5.4): the 8 FP64
    fields read and written exactly once at peak HBM bandwidth."""
    return 2 * 8 * 8 * points / (HBM_PEAK_GBS * 1e9) * 1e3


def progress(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def sig(v, digits=4):
    """v rounded to a few significant digits (keeps the result line short)."""
    if isinstance(v, float):
        return float("%.*g" % (digits, v)) if math.isfinite(v) else None
    if isinstance(v, dict):
        return {k: sig(x, digits) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [sig(x, digits) for x in v]
    return v


def star_f32_error(torch, S, W, inputs, n, r, iters=100):
    """Normwise relative error of the FP32-storage star after ``iters``
    chained iterations against the FP64 path on the same FP32-exact input
    (the FP64 path matches the CPU oracle to 1e-12 at this size)."""
    dims = (n, n, n)
    g = W.diffusion_star(3, r, W.diffusion_number(n))
    x = torch.from_numpy(inputs.uniform_field(dims, 1)).cuda().to(torch.float32)
    outs = []
    for dtype in (S.F64, S.F32):
        es = 8 if dtype == S.F64 else 4
        pitch, ox = W.aligned_layout(n, r, es) if dtype == S.F32 else (0, 0)
        p = S.LinearPlan(dims, r, g, dtype=dtype, row_pitch=pitch, x_offset=ox)
        a = p.empty(0.0)
        p.padded(a)[r:r + n, r:r + n, r:r + n] = x.to(a.dtype)
        b = p.empty(0.0)
        res = p.apply(a, b, iters)
        outs.append(p.padded(res)[r:r + n, r:r + n, r:r + n].to(torch.float64))
        del a, b, res, p
    err = float((outs[1] - outs[0]).abs().max() / outs[0].abs().max())
    del outs, x
    torch.cuda.empty_cache()
    return err


def secondary(torch, S, W, inputs, args):
    """The other configurations. Returns (compact, detail): compact goes into
    the result line, detail to stderr and --detail-out."""
    comp, det = {}, {}
    n, r = args.n, args.radius
    only = set(args.only.split(",")) if args.only else None
    want = lambda k: only is None or k in only  # noqa: E731
    if want("stars"):
        progress("FP32 star")
        # FP32 storage of the same star workload, and its error against FP64
        p32, _, tot, per, nl = star_run(torch, S, W, inputs, n, r, S.F32, 100, 4)
        ipl = p32.iterations_per_launch if nl[1] == 0 else 1
        det["star_%d_f32" % n] = {"updates_per_s": n ** 3 / (tot / 100 * 1e-3),
                                  "ms_per_iteration": tot / 100, "iterations_per_launch": ipl,
                                  "hbm_frac": ipl * 8 * n ** 3 / (per * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                  "avg_launch_ms": per, "tile": list(p32.tile),
                                  "layout": [p32.row_pitch, p32.x_offset]}
        del p32
        err32 = star_f32_error(torch, S, W, inputs, n, r)
        d = det["star_%d_f32" % n]
        d["rel_err_vs_f64_100_iterations"] = err32
        comp["c1_star512_f32"] = {"gups": d["updates_per_s"] / 1e9, "ms_it": d["ms_per_iteration"],
                                  "frac": d["hbm_frac"], "err_vs_f64_100it": err32}
        progress("radius-4 star")
        # the secondary star of the same workload: 25 points, radius 4, FP64
        p4, _, tot, per, nl = star_run(torch, S, W, inputs, n, 4, S.F64, 100, 4)
        ipl = p4.iterations_per_launch if nl[1] == 0 else 1
        d = det["star_%d_f64_r4" % n] = {
            "updates_per_s": n ** 3 / (tot / 100 * 1e-3), "ms_per_iteration": tot / 100,
            "iterations_per_launch": ipl,
            "hbm_frac": ipl * 16 * n ** 3 / (per * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "avg_launch_ms": per, "tile": list(p4.tile)}
        comp["c1_star512_f64_r4"] = {"gups": d["updates_per_s"] / 1e9, "ms_it": d["ms_per_iteration"],
                                     "frac": d["hbm_frac"]}
        del p4
    if want("lines"):
        progress("1-D lines")
        # 1-D radius-1 smoother at 2^28 points (2 GiB per buffer): 10 chained
        # iterations per call, autotuned plan (temporal blocking allowed)
        N = 1 << 28
        pl = S.LinearPlan((N,), 1, W.smoother3(), autotune=True)
        a = pl.empty(0.0)
        a[1:N + 1] = torch.from_numpy(inputs.uniform_field((N,), 1)).cuda()
        b = pl.empty(0.0)
        ms = timed(torch, lambda: pl.apply(a, b, 10), 3, warm=1)
        det["line_2^28_f64_10iter"] = {"updates_per_s": N * 10 / (ms * 1e-3), "ms_per_call": ms,
                                       "algorithmic_frac": 16 * N * 10 / (ms * 1e-3) / 1e9 /
                                       HBM_PEAK_GBS,
                                       "iterations_per_launch": pl.iterations_per_launch,
                                       "variant": pl.variant, "tile": list(pl.tile)}
        del a, b, pl
        # 1-D radius-1 smoother, 2^20 points, 10 chained iterations per call
        N = 1 << 20
        p1 = S.LinearPlan((N,), 1, W.smoother3(), autotune=True)
        a = p1.empty(0.0)
        a[1:N + 1] = torch.from_numpy(inputs.uniform_field((N,), 1)).cuda()
        b = p1.empty(0.0)
        ms = timed(torch, lambda: p1.apply(a, b, 10), 50)
        d = det["line_2^20_f64_10iter"] = {"updates_per_s": N * 10 / (ms * 1e-3), "ms_per_call": ms,
                                           "us_per_iteration": ms * 100.0,
                                           "variant": p1.variant, "tile": list(p1.tile)}
        comp["c0_line2^20_f64_10it"] = {"gups": d["updates_per_s"] / 1e9, "us_it": d["us_per_iteration"]}
        del a, b
    if want("lines"):
        progress("radius sweep")
        det["line_radius_sweep_2^24_f64"] = radius_sweep(torch, S, inputs)
    if want("filters"):
        progress("filters")
        det["filters_512_f64"] = filters(torch, S, inputs, args.n)
        f = det["filters_512_f64"]
        comp["f4_filters_512_f64"] = {"max_ms": f["max_3x3x3"]["ms_per_launch"],
                                      "max_frac": f["max_3x3x3"]["hbm_frac"],
                                      "median_ms": f["median_3x3x3"]["ms_per_launch"]}
    if want("box"):
        progress("dense box")
        det["box27_512"] = dense_box(torch, S, inputs, args.n)
        b = det["box27_512"]
        comp["f3_box27_512"] = {"f64_ms": b["f64"]["ms_per_launch"], "f64_frac": b["f64"]["hbm_frac"],
                                "f64_gather_ms": b["f64_gather"]["ms_per_launch"],
                                "f32_ms": b["f32"]["ms_per_launch"]}
        det["box_r2_r3_512"] = dense_box_r(torch, S, inputs, args.n)
        b = det["box_r2_r3_512"]
        comp["f3_box_r23_512"] = {k: [b[k]["ms_per_launch"], b[k]["valu_frac"]]
                                  for k in ("r2_f64", "r3_f64", "r2_f32", "r2_f64_gather")}
        det["box_r5_r8_256"] = dense_box_r(torch, S, inputs, 256, radii=(5, 8), gather=True)
        det["box2d_16384_f64"] = dense_box2d(torch, S, inputs)
        b = det["box2d_16384_f64"]
        comp["f3_box2d_16k_f64"] = {k: [b[k]["ms_per_launch"], b[k]["hbm_frac"]] for k in b}
    if want("mhd"):
        progress("fused 8-field steps")
        # fused 8-field RK3 step, 256^3
        nm = 256
        f, _ = inputs.fourier_fields((nm, nm, nm), 1, nf=8, modes=8, kmax=8, amp=0.01)
        ds = 2 * math.pi / nm
        dt = 0.1 * ds
        bytes_step = {S.PREC_F64: 640, S.PREC_F32_MASTER64: 480, S.PREC_BF16_MASTER64: 384}
        for model, mname, prec, name in (
                (S.MODEL_MHD8, "mhd8", S.PREC_F64, "f64"),
                (S.MODEL_MHD8, "mhd8", S.PREC_F32_MASTER64, "f32_master64"),
                (S.MODEL_MHD8, "mhd8", S.PREC_BF16_MASTER64, "bf16_master64"),
                (S.MODEL_MHD_FULL, "mhd_full", S.PREC_F64, "f64"),
                (S.MODEL_MHD_FULL, "mhd_full", S.PREC_F32_MASTER64, "f32_master64"),
                # 12-tap diagonal mixed derivatives instead of the tensor product
                (S.MODEL_MHD8, "mhd8_diag", S.PREC_F64, "f64"),
                (S.MODEL_MHD_FULL, "mhd_full_diag", S.PREC_F64, "f64")):
            plan = S.RkPlan(model, (nm, nm, nm), prec,
                            mhd=FULL_MHD if model == S.MODEL_MHD_FULL else None,
                            mixed=S.MIXED_DIAGONAL if mname.endswith("_diag") else S.MIXED_TENSOR)
            bufs = plan.alloc()
            for k in range(8):
                bufs["f_a"][k][3:nm + 3, 3:nm + 3, 3:nm + 3] = torch.from_numpy(f[k]).cuda().to(
                    bufs["f_a"][k].dtype)
                if plan.master:
                    bufs["f64"][k][3:nm + 3, 3:nm + 3, 3:nm + 3] = torch.from_numpy(f[k]).cuda()
            steps = 5
            ms = timed(torch, lambda: plan.run(bufs["f_a"], bufs["f_b"], bufs["w"], steps, dt,
                                               w2=bufs["w2"], f64=bufs["f64"]), 2, warm=1) / steps
            pts = nm ** 3
            flops = mhd_flops(model == S.MODEL_MHD_FULL, mname.endswith("_diag"))
            peak = VALU_PEAK_TFLOPS["f64" if prec == S.PREC_F64 else "f32"]
            d = det["%s_%d_%s" % (mname, nm, name)] = {
                "point_steps_per_s": pts / (ms * 1e-3),
                "point_substeps_per_s": 3 * pts / (ms * 1e-3),
                "ms_per_step": ms,
                "hbm_frac": bytes_step[prec] * pts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "valu_roof": {"flops_per_point_substep": flops, "peak_tflops": peak,
                              "frac": 3 * pts / (ms * 1e-3) * flops / (peak * 1e12)}}
            key = ("c2_" if prec == S.PREC_F64 else "c3_") + "%s_256_%s" % (mname, name)
            comp[key] = {"ms_step": ms, "hbm_frac": d["hbm_frac"],
                         "valu_frac": d["valu_roof"]["frac"]}
            if mname in ("mhd8", "mhd_full") and prec in (S.PREC_F64, S.PREC_F32_MASTER64):
                # the same step with the plan-time schedule search
                tp = S.RkPlan(model, (nm, nm, nm), prec,
                              mhd=FULL_MHD if model == S.MODEL_MHD_FULL else None, autotune=True)
                tms = timed(torch, lambda: tp.run(bufs["f_a"], bufs["f_b"], bufs["w"], steps, dt,
                                                  w2=bufs["w2"], f64=bufs["f64"]), 2, warm=1) / steps
                d["autotuned"] = {"ms_per_step": tms, "schedule": list(tp.schedule),
                                  "default_schedule": list(plan.schedule)}
                comp[key]["tuned_ms"] = tms
                del tp
            if mname in ("mhd8", "mhd_full") and prec == S.PREC_F64:
                # the paper's measure (Sec. 5.4): the final RK3 substep against
                # the 8 fields read and written once at peak bandwidth
                fin = timed(torch, lambda: plan.step(bufs["f_a"], bufs["f_b"], bufs["w"], 2, dt,
                                                     w2=bufs["w2"], f64=bufs["f64"]), 10, warm=2)
                d["final_substep"] = {"ms": fin, "paper_ideal_frac": paper_ideal_ms(pts) / fin}
                comp[key]["final_substep_ms"] = fin
                comp[key]["paper_ideal_frac"] = paper_ideal_ms(pts) / fin
            if mname == "mhd8" and prec == S.PREC_F64:
                # FP64 diagnostics of the 8 fields (a7): sums, sums of squares,
                # maxima; one read of each field (8 B per point and field)
                state = bufs["f_a"]
                rms = timed(torch, lambda: plan.reduce(state), 5, warm=1)
                nms = timed(torch, lambda: plan.reduce_noalloc(state), 5, warm=1)
                gb = 8 * 8 * pts / 1e9
                det["reduce_256_f64_8fields"] = {"ms": rms, "noalloc_ms": nms,
                                                 "hbm_frac": gb / (rms * 1e-3) / HBM_PEAK_GBS,
                                                 "noalloc_hbm_frac":
                                                     gb / (nms * 1e-3) / HBM_PEAK_GBS}
                comp["a7_reduce_256_f64_8f"] = {"ms": rms, "noalloc_ms": nms,
                                                "hbm_frac": gb / (rms * 1e-3) / HBM_PEAK_GBS}
            del bufs, plan
        del f
        # the same measure at the paper's own grid, 128^3
        n2 = 128
        f2, _ = inputs.fourier_fields((n2,) * 3, 1, nf=8, modes=8, kmax=8, amp=0.01)
        for model, mname in ((S.MODEL_MHD8, "mhd8"), (S.MODEL_MHD_FULL, "mhd_full")):
            plan = S.RkPlan(model, (n2,) * 3, S.PREC_F64,
                            mhd=FULL_MHD if model == S.MODEL_MHD_FULL else None)
            bufs = plan.alloc()
            for k in range(8):
                bufs["f_a"][k][3:n2 + 3, 3:n2 + 3, 3:n2 + 3] = torch.from_numpy(f2[k]).cuda()
            dt2 = 0.1 * 2 * math.pi / n2
            fin = timed(torch, lambda: plan.step(bufs["f_a"], bufs["f_b"], bufs["w"], 2, dt2,
                                                 w2=bufs["w2"], f64=bufs["f64"]), 20, warm=3)
            det["%s_128_f64_final_substep" % mname] = {
                "ms": fin, "paper_ideal_frac": paper_ideal_ms(n2 ** 3) / fin}
            key = "c2_%s_256_f64" % mname
            if key in comp:
                comp[key]["final128_frac"] = paper_ideal_ms(n2 ** 3) / fin
            del bufs, plan
        del f2
        torch.cuda.empty_cache()
    if want("precision"):
        if not args.no_precision_error:
            for model, mname in ((S.MODEL_MHD8, "mhd8"), (S.MODEL_MHD_FULL, "mhd_full")):
                progress("precision study %s" % mname)
                res = mixed_precision_error(torch, S, inputs, n=args.precision_n, model=model,
                                            mhd=FULL_MHD if model == S.MODEL_MHD_FULL else None)
                det["%s_mixed_precision_error_%d" % (mname, args.precision_n)] = res
                comp["c3_err_%s_%d" % (mname, args.precision_n)] = {
                    "steps": res["steps"],
                    # max over the 8 fields, two significant digits (the
                    # per-field values are in the detail output)
                    **{k: [float("%.2g" % max(res[k][str(cp)])) for cp in res["steps"]]
                       for k in ("f32_master64", "bf16_master64", "f32_only", "bf16_only")}}
    if want("serving"):
        if args.serve_jobs > 0:
            rates = tuple(float(v) for v in args.serve_rates.split(",") if v)
            progress("serving trace (%d jobs)" % args.serve_jobs)
            sv = serving(torch, args.serve_jobs, rates=rates, sweep_jobs=args.serve_sweep_jobs)
            det["serving"] = sv
            # throughput in 1e9 point-steps/s (keeps the result line short)
            comp["c4_serving"] = {
                "jobs": args.serve_jobs, "rate_per_s": 200,
                "served": {"p50_s": sv["served"]["p50_s"], "p99_s": sv["served"]["p99_s"],
                           "gpts_s": sv["served"]["point_steps_per_s"] / 1e9},
                "fifo_f64": {"p50_s": sv["fifo_f64"]["p50_s"], "p99_s": sv["fifo_f64"]["p99_s"],
                             "gpts_s": sv["fifo_f64"]["point_steps_per_s"] / 1e9},
                # per request dtype: [jobs, p50 s, p99 s, 1e9 point-steps/s]
                "served_by_dtype": {d: [v["jobs"], v["p50_s"], v["p99_s"], v["point_steps_per_s"] / 1e9]
                                    for d, v in sv["served"]["by_dtype"].items()},
                "fifo_by_dtype": {d: [v["jobs"], v["p50_s"], v["p99_s"], v["point_steps_per_s"] / 1e9]
                                  for d, v in sv["fifo_f64"]["by_dtype"].items()},
                "speedup": sv["speedup_point_steps_per_s"],
                "p99_ratio_fifo_over_served": sv["p99_ratio_fifo_over_served"],
                # max relative error of the f32 / f64 requests against FP64 runs
                "err_vs_f64": {"f32": sv["error_vs_fp64"]["max_rel_err_f32_requests_vs_fp64"],
                               "f64": sv["error_vs_fp64"]["max_rel_err_f64_requests_vs_fp64"]},
                "sweep_p99_served_vs_fifo": {k: [v["served"]["p99_s"], v["fifo_f64"]["p99_s"]]
                                             for k, v in sv["rate_sweep"].items()}}
    return comp, det


def filters(torch, S, inputs, n):
    """Window filters on the n^3 FP64 field: 3x3x3 max (the default
    lane-exchange z march, and the LDS z march for comparison) and 3x3x3
    median (gather kernel, forgetful selection among the 27 values), one
    periodic application per launch; 16 B per point (read once, write once)."""
    import numpy as np
    dims, r = (n, n, n), 1
    out = {}
    x = torch.from_numpy(inputs.uniform_field(dims, 1)).cuda()
    for name, op, tile in (("max_3x3x3", S.OP_MAX, None), ("median_3x3x3", S.OP_MEDIAN, None),
                           # the LDS z march the lane-exchange default replaced
                           ("max_3x3x3_lds_march", S.OP_MAX, (8, 1, 32, 0))):
        p = S.LinearPlan(dims, r, np.ones((3, 3, 3)), op=op,
                         variant=S.STAR3D if tile else S.VARIANT_AUTO, tile=tile)
        a = p.empty(0.0)
        p.padded(a)[r:r + n, r:r + n, r:r + n] = x
        b = p.empty(0.0)
        p.halo(a)
        ms = timed(torch, lambda: p.apply(a, b, 1, halo_valid=True), 20, warm=2)
        out[name] = {"ms_per_launch": ms, "updates_per_s": n ** 3 / (ms * 1e-3),
                     "hbm_frac": 16 * n ** 3 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "variant": p.variant, "tile": list(p.tile)}
        del a, b, p
    return out


def dense_box(torch, S, inputs, n):
    """Dense 27-point box (every tap of the radius-1 box nonzero, seeded
    coefficients) on the n^3 field, one periodic application per launch: the
    default BOX3D march (LDS, outputs stored as whole rows) in FP64 and FP32,
    the lane-exchange march (FP64) and the gather kernel. 2 x storage bytes
    per point; 27 multiply-adds per point."""
    import numpy as np
    dims = (n, n, n)
    g = np.random.default_rng(1).uniform(0.2, 1.0, (3, 3, 3)) / 27
    x = torch.from_numpy(inputs.uniform_field(dims, 1)).cuda()
    out = {}
    for name, dtype, es, variant, tile in (
            ("f64", S.F64, 8, S.VARIANT_AUTO, None), ("f32", S.F32, 4, S.VARIANT_AUTO, None),
            ("f64_lane_exchange", S.F64, 8, S.BOX3D, (4, 2, 8, 1)),
            ("f64_gather", S.F64, 8, S.GENERIC, None)):
        p = S.LinearPlan(dims, 1, g, dtype=dtype, variant=variant, tile=tile)
        a = p.empty(0.0)
        p.padded(a)[1:n + 1, 1:n + 1, 1:n + 1] = x.to(a.dtype)
        b = p.empty(0.0)
        p.halo(a)
        ms = timed(torch, lambda: p.apply(a, b, 1, halo_valid=True), 10, warm=2)
        out[name] = {"ms_per_launch": ms, "updates_per_s": n ** 3 / (ms * 1e-3),
                     "hbm_frac": 2 * es * n ** 3 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "variant": p.variant, "tile": list(p.tile)}
        del a, b, p
    return out


def dense_box_r(torch, S, inputs, n, radii=(2, 3), gather=False):
    """Dense boxes of radius 2 and 3 (all 125 / 343 taps nonzero, seeded
    coefficients with sum |g| = 1) on the n^3 field, one periodic application
    per launch (halo refresh included): the default BOX3D LDS march in FP64
    and FP32 and, at radius 2, the gather kernel it replaces. (2R+1)^3
    multiply-adds per point, so the bound is the vector FMA rate: valu_frac =
    2 (2R+1)^3 n^3 flops per launch over the vector peak of the type. With
    gather=True every radius also runs FP32 and the gather kernel (the
    radius 5 and 8 boxes at 256^3)."""
    import numpy as np
    dims = (n, n, n)
    x = torch.from_numpy(inputs.uniform_field(dims, 1)).cuda()
    out = {}
    for r in radii:
        K = 2 * r + 1
        g = np.random.default_rng(r).uniform(0.2, 1.0, (K, K, K)) * \
            np.random.default_rng(r + 10).choice([-1.0, 1.0], (K, K, K))
        g /= np.abs(g).sum()
        runs = [("f64", S.F64, S.VARIANT_AUTO)]
        if r == 2 or gather:
            runs += [("f32", S.F32, S.VARIANT_AUTO), ("f64_gather", S.F64, S.GENERIC)]
        for name, dtype, variant in runs:
            p = S.LinearPlan(dims, r, g, dtype=dtype, variant=variant)
            a = p.empty(0.0)
            p.padded(a)[r:n + r, r:n + r, r:n + r] = x.to(a.dtype)
            b = p.empty(0.0)
            p.halo(a)
            ms = timed(torch, lambda: p.apply(a, b, 1, halo_valid=True), 5, warm=1)
            peak = VALU_PEAK_TFLOPS["f64" if dtype == S.F64 else "f32"]
            out["r%d_%s" % (r, name)] = {
                "ms_per_launch": ms, "updates_per_s": n ** 3 / (ms * 1e-3),
                "valu_frac": 2 * K ** 3 * n ** 3 / (ms * 1e-3) / 1e12 / peak,
                "variant": p.variant, "tile": list(p.tile)}
            del a, b, p
    return out


def dense_box2d(torch, S, inputs, n=16384, radii=(2, 4)):
    """Dense 2-D boxes of radius 2 and 4 (all 25 / 81 taps nonzero, seeded,
    sum |g| = 1) on an n^2 FP64 field, one periodic application per launch
    (halo refresh included): the default plan (the LDS march over one plane)
    and, at radius 2, the gather kernel. 16 B per point of HBM traffic."""
    import numpy as np
    dims = (n, n)
    x = torch.from_numpy(inputs.uniform_field(dims, 1)).cuda()
    out = {}
    for r in radii:
        K = 2 * r + 1
        g = np.random.default_rng(r).uniform(0.2, 1.0, (K, K))
        g /= g.sum()
        for name, variant in (("r%d" % r, S.VARIANT_AUTO),) + \
                ((("r%d_gather" % r, S.GENERIC),) if r == 2 else ()):
            p = S.LinearPlan(dims, r, g, variant=variant)
            a = p.empty(0.0)
            p.padded(a)[r:n + r, r:n + r] = x
            b = p.empty(0.0)
            p.halo(a)
            ms = timed(torch, lambda: p.apply(a, b, 1, halo_valid=True), 5, warm=1)
            out[name] = {"ms_per_launch": ms, "updates_per_s": n * n / (ms * 1e-3),
                         "hbm_frac": 16 * n * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "variant": p.variant, "tile": list(p.tile)}
            del a, b, p
    return out


def radius_sweep(torch, S, inputs, n=1 << 24, radii=(1, 2, 4, 8, 16, 64, 256, 1024)):
    """1-D FP64 lines of 2^24 points (the paper's 1-D size), radius 1..1024,
    random taps with sum |g| = 1, autotuned plan; 10 chained iterations per
    timed call. Reports updates/s and the effective bandwidth 16 B per update
    (the radius study of Sec. 5, Fig. 8: bandwidth-bound at small r, on-chip
    bound at large r)."""
    import numpy as np
    res = {}
    x = torch.from_numpy(inputs.uniform_field((n,), 1)).cuda()
    for r in radii:
        g = np.random.default_rng(r).uniform(-1, 1, 2 * r + 1)
        g /= np.abs(g).sum()
        p = S.LinearPlan((n,), r, g, autotune=True)
        a = p.empty(0.0)
        a[r:r + n] = x
        b = p.empty(0.0)
        ms = timed(torch, lambda: p.apply(a, b, 10), 5, warm=1) / 10
        res[str(r)] = {"ms_per_iteration": ms, "updates_per_s": n / (ms * 1e-3),
                       "effective_gbs": 16 * n / (ms * 1e-3) / 1e9,
                       "variant": p.variant, "tile": list(p.tile)}
        del a, b, p
    return res


def mixed_precision_error(torch, S, inputs, n=256, checkpoints=(1, 10, 100, 1000), model=None,
                          mhd=None):
    """Normwise relative error per field of the FP32- and BF16-storage states
    (FP64 master, and the no-master ablation) against the FP64 path after 1,
    10, 100 and 1000 RK3 steps of an 8-field model (default: the proxy) at
    n^3 (Fourier-mode initial data, amplitude 0.01, |k| <= 8; dt = 0.1 ds).
    The FP64 path is the reference: it matches the CPU oracle to 1e-12 at
    every point at 256^3 for each substep, and over 1000 steps at 32^3. The
    differences are taken on the GPU; the FP64 snapshots stay in HBM."""
    model = S.MODEL_MHD8 if model is None else model
    dims = (n, n, n)
    dt = 0.1 * 2 * math.pi / n
    f, _ = inputs.fourier_fields(dims, 1, nf=8, modes=8, kmax=8, amp=0.01)
    f = [torch.from_numpy(v).cuda() for v in f]
    ref = {}
    out = {"grid": n, "reference": "GPU FP64 path (oracle-anchored)", "steps": list(checkpoints)}
    t0 = time.perf_counter()
    for name, prec in (("f64", S.PREC_F64), ("f32_master64", S.PREC_F32_MASTER64),
                       ("bf16_master64", S.PREC_BF16_MASTER64), ("f32_only", S.PREC_F32_ONLY),
                       ("bf16_only", S.PREC_BF16_ONLY)):
        plan = S.RkPlan(model, dims, prec, mhd=mhd)
        b = plan.alloc()
        for k in range(8):
            b["f_a"][k][3:n + 3, 3:n + 3, 3:n + 3] = f[k].to(b["f_a"][k].dtype)
            if plan.master:
                b["f64"][k][3:n + 3, 3:n + 3, 3:n + 3] = f[k]
        per, done, cur, nxt = {}, 0, b["f_a"], b["f_b"]
        for cp in checkpoints:
            res = plan.run(cur, nxt, b["w"], cp - done, dt, w2=b["w2"], f64=b["f64"])
            if res is nxt:
                cur, nxt = nxt, cur
            done = cp
            state = b["f64"] if plan.master else cur
            snap = [t[3:n + 3, 3:n + 3, 3:n + 3].to(torch.float64) for t in state]
            if name == "f64":
                ref[cp] = [s.clone() for s in snap]
            else:
                per[str(cp)] = [float((snap[k] - ref[cp][k]).abs().max() /
                                      ref[cp][k].abs().max()) for k in range(8)]
            del snap
        if name != "f64":
            out[name] = per
        del b, plan
    out["seconds"] = time.perf_counter() - t0
    del ref, f
    torch.cuda.empty_cache()
    return out


# dense vector peaks of one MI355X (FP64, FP32 arithmetic), TFLOP/s
VALU_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}


def mhd_flops(full, diagonal):
    """Algorithmic flops per point and substep of the fused 8-field step: 24
    first derivatives (3 antisymmetric differences, 3 multiply-adds and the
    1/ds scale: 9), 24 second derivatives (3 sums, 3 multiply-adds, the centre
    tap and the scale: 11), 12 mixed derivatives (tensor product with the
    antisymmetry folded: 9 four-point differences of 3 adds plus 9
    multiply-adds, 45; diagonal form: 3 four-point differences plus 3
    multiply-adds and the scale, 16), about 200 for the proxy right-hand side
    (about 260 for the full model), and 4 per field for the RK update."""
    return 24 * 9 + 24 * 11 + 12 * (16 if diagonal else 45) + (260 if full else 200) + 8 * 4


def serving(torch, count, seed=1, rates=(10.0, 25.0, 50.0), sweep_jobs=48):
    """Seeded Poisson trace (mean 200 jobs/s) of 2-D/3-D radius-3 advection-
    diffusion jobs, edges {64..384}, 10-500 steps, FP32/FP64 per request:
    continuous-batching server vs plain FIFO per-job FP64 on the same GPU.
    The 200/s trace overloads the GPU (its offered work exceeds the HBM roof);
    the first ``sweep_jobs`` jobs are also replayed at lower mean rates
    (arrival times stretched by 200/rate) for latencies under a load the GPU
    can sustain. The server runs its default policy (oldest first); the
    shortest-remaining-work policy is timed beside it."""
    import numpy as np

    import paper_2406_08923_amd as S_
    from paper_2406_08923_amd import inputs, serving as SV
    jobs = inputs.serving_trace(seed, count)
    inits = SV.make_inits(jobs)
    progress("serving: inits ready")
    served, res_s = SV.run_served(jobs, inits)
    torch.cuda.synchronize()
    progress("serving: served run %.1f s" % served["makespan_s"])
    fifo, res_f = SV.run_fifo_f64(jobs, inits)
    progress("serving: FIFO run %.1f s" % fifo["makespan_s"])
    err = SV.compare(jobs, res_s, res_f)
    del res_f
    torch.cuda.synchronize()
    tuned, res_t = SV.run_served(jobs, inits, tune=True)
    tuned_bitwise = all(np.array_equal(a, b) for a, b in zip(res_t, res_s)) if res_s else None
    del res_t, res_s
    progress("serving: served with batch-schedule search %.1f s" % tuned["makespan_s"])
    shortest, _ = SV.run_served(jobs, inits, policy=S_.SERVE_SHORTEST)
    keep = ("p50_s", "p99_s", "makespan_s", "point_steps_per_s")
    sweep = {}
    sj, si = jobs[:sweep_jobs], inits[:sweep_jobs]
    for rate in rates:
        jr = [dict(j, arrival=j["arrival"] * 200.0 / rate) for j in sj]
        row = {}
        for name, fn in (("served", lambda: SV.run_served(jr, si)),
                         ("fifo_f64", lambda: SV.run_fifo_f64(jr, si)),
                         ("served_shortest_first",
                          lambda: SV.run_served(jr, si, policy=S_.SERVE_SHORTEST))):
            torch.cuda.synchronize()
            res, _ = fn()
            row[name] = {k: res[k] for k in keep}
        sweep["%g_per_s" % rate] = row
        print("serving at %g jobs/s (%d jobs): p99 served %.3f s, fifo %.3f s, shortest-first "
              "%.3f s" % (rate, len(sj), row["served"]["p99_s"], row["fifo_f64"]["p99_s"],
                          row["served_shortest_first"]["p99_s"]), file=sys.stderr, flush=True)
    return {"trace": "seed %d, %d jobs, Poisson 200/s, 50%% 3-D, edges 64..384, steps "
                     "10..500, 50%% FP32 requests; rate sweep on the first %d jobs"
                     % (seed, count, len(sj)),
            "policy": "oldest submission first, shorter jobs filling up to a quarter more",
            "served": served, "fifo_f64": fifo, "error_vs_fp64": err,
            "served_shortest_first": {k: shortest[k] for k in keep},
            "served_tuned": dict({k: tuned[k] for k in keep},
                                 tuned_classes=tuned["tuned_classes"],
                                 bitwise_equal_to_untuned=tuned_bitwise),
            "speedup_point_steps_per_s": served["point_steps_per_s"] / fifo["point_steps_per_s"],
            "p99_ratio_fifo_over_served": fifo["p99_s"] / served["p99_s"],
            "rate_sweep": sweep}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this stencil build has no multi-GPU path "
              "(--gpus %d requested)" % max(args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np  # noqa: F401
    import torch

    import paper_2406_08923_amd as S
    from paper_2406_08923_amd import inputs
    from paper_2406_08923_amd import workloads as W

    torch.cuda.set_device(0)
    n, r = args.n, args.radius
    dtype, esize = DTYPES[args.dtype]
    tile = tuple(int(v, 0) for v in args.tile.split(",")) if args.tile else None
    K = args.steps
    t0 = time.perf_counter()
    plan, g, total_ms, avg_launch_ms, (n_multi, n_single) = star_run(
        torch, S, W, inputs, n, r, dtype, K, args.warmup, tile, layout=args.layout,
        autotune=args.autotune)
    wall = time.perf_counter() - t0
    ms_per_step = total_ms / K
    points = n ** 3
    value = points / (ms_per_step * 1e-3)
    # iterations one launch performs (all launches alike when n_single == 0)
    ipl = plan.iterations_per_launch if n_single == 0 else 1
    if n_multi and n_single:
        print("note: %d iterations mix %d two-iteration and %d one-iteration launches; "
              "use a multiple of 4 for a single kernel in the roofline" % (K, n_multi, n_single),
              file=sys.stderr)
    # per iteration each point's value is read once and written once
    alg_bytes = ipl * 2 * esize * points
    achieved = alg_bytes / (avg_launch_ms * 1e-3) / 1e9
    kern_files = ("star3d.hpp", "star3d_t2.hpp", "star3d_t2p.hpp", "star3d_t2q.hpp",
                  "star3d_dpp.hpp", "star3d_%s.hip" % args.dtype, "common.hpp",
                  "linear_kernels.hpp", "linear_api.hip")
    traffic = load_traffic("traffic_star3d_%d_%s.json" % (n, args.dtype), kern_files)
    traffic_gbs = traffic / (avg_launch_ms * 1e-3) / 1e9 if traffic else None
    copy_gbs = None if args.no_copy else copy_bandwidth(torch, S)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic: seeded uniform [-1,1) field, periodic halo",
        "config": {
            "workload": "3-D linear cross-correlation, %d-point radius-%d star (6th-order "
                        "diffusion step, s=%.4f), %d^3 %s, periodic halo, %d chained iterations"
                        % (int((g != 0).sum()), r, W.diffusion_number(n), n,
                           args.dtype.upper(), K),
            "tile": list(plan.tile),
            "iterations_per_launch": ipl,
            "launches": n_multi + n_single,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "avg_launch_ms": avg_launch_ms,
            "basis": "achieved: algorithmic %d B/pt/iteration x %d iterations per launch; "
                     "traffic: measured HBM B/launch (rocprofv3, copy-calibrated)"
                     % (2 * esize, ipl),
        },
        # the share of the HBM roof the kernel's measured traffic uses (one
        # pass of bytes, not the algorithmic bytes of both iterations)
        "hbm_traffic_pct": 100.0 * traffic_gbs / HBM_PEAK_GBS if traffic_gbs else None,
        "effective_bandwidth_gbs": achieved,
        "copy_bandwidth_gbs": copy_gbs,
        "wall_s_star_phase": wall,
    }
    detail = {}
    if not args.no_secondary:
        comp, detail = secondary(torch, S, W, inputs, args)
        out["workloads"] = sig(comp, 3)
    if not args.no_cpu_baseline:
        progress("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(n, r, g, args.cpu_seconds)
    if detail:
        detail["headline"] = {k: out[k] for k in ("value", "ms_per_step", "roofline")}
        text = json.dumps(detail)
        print("detail: " + text, file=sys.stderr, flush=True)
        if args.detail_out:
            with open(args.detail_out, "w") as fh:
                fh.write(text + "\n")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
