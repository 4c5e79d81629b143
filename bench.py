"""Benchmark of the hot path.

Headline: fused NLL + gradient evaluations per second.  A step is one
evaluation of -sum_i ln P(x_i|theta) and its gradient over every event of one
dataset (the per-minimiser-step work of an unbinned fit): constant staging,
the fused PDF/log/gradient event kernel, the deterministic two-pass reduction
and the FP64 epilogue -- one kernel launch.  The workload is the 4-D angular x
mass model (P-wave x Gauss signal, Chebyshev^3 x Exp background, 17 free
parameters, mu fixed) at 1e6 synthetic events in mixed precision (FP32
per-event arithmetic, FP64 accumulation), events resident in HBM.

Serving: a toy study of the same model.  Requests of log-uniform size in
[500, 50000] events arrive as a Poisson stream at 500 fits/s (open loop) or
all at once (saturated); each is fitted from the generating values with BFGS
to EDM < 1e-6 and its covariance taken from the analytic Hessian.  The batched
server (continuous batching, memory-budget admission, graph replays) is
compared with a loop that runs one fit after another through uml_fit.

Prints one JSON line (see the repository's benchmark contract).
"""
import argparse
import hashlib
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP32 vector peak: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz x 2 (FMA) = 78.6
# TFLOP/s with one FP32 operation per lane and cycle.  The library is built
# without packed FP32, whose 157.3 TFLOP/s is reported beside it.
PEAK_FP32_TFLOPS = 78.6
PEAK_FP32_PACKED_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# Algorithmic FP32 work per event of the 4-D model: the operations of the
# fused per-event formula (FMA and multiply-add count 2, every other
# operation including each transcendental counts 1).
FLOP_PER_EVENT_4D = 137

# Sources of the event kernels: HBM traffic measured with hardware counters
# (profiles/) is reported only while these are unchanged.
KERNEL_SOURCES = ["paper_2505_12414_amd/csrc/eval.hip", "paper_2505_12414_amd/csrc/prologue.h",
                  "paper_2505_12414_amd/csrc/devmath.h", "paper_2505_12414_amd/csrc/uml_internal.h",
                  "paper_2505_12414_amd/build.py"]  # the build flags shape the kernel too
COPY_MB = 512

SEED_DATA = 20250512
SEED_STREAM = 20250513
SEED_POOL = 20250514
SEED_TOY0 = 1_000_000


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counted_traffic(workload):
    """HBM bytes per launch from the committed counter summary of this
    workload, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(workload)
    if not rec or rec.get("kernel_sources") != kernel_source_hash():
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def copy_check(torch, stream, reps=20):
    """A plain device copy of known size (COPY_MB read + COPY_MB written per
    launch, beyond the 256 MB last-level cache): the measured HBM rate, and
    the calibration kernel for the hardware traffic counters."""
    n = (COPY_MB << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    with torch.cuda.stream(stream):
        for _ in range(3):
            torch.add(src, 1.0, out=dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record(stream)
        for _ in range(reps):
            torch.add(src, 1.0, out=dst)
        e1.record(stream)
    torch.cuda.synchronize()
    gbs = 2 * (COPY_MB << 20) * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


def theta_points(torch, model, truth, dev, count=64):
    """count parameter points near truth, all different: free parameter k of
    point j is truth_k (1 + 1e-7 (j + 1) (k + 1)).  Device-resident rows."""
    t = np.asarray(truth, dtype=np.float64)
    free = [i for i, p in enumerate(model.desc["params"]) if not p.get("fixed", False)]
    pts = np.repeat(t[None, :], count, axis=0)
    for j in range(count):
        for r, k in enumerate(free):
            pts[j, k] = t[k] * (1.0 + 1e-7 * (j + 1) * (r + 1)) if t[k] != 0.0 else 1e-9 * (j + 1)
    bank = torch.tensor(pts, dtype=torch.float64, device=dev)
    return [bank[j] for j in range(count)]


def time_evals(torch, uml, model, data, points, out, stream, steps, warmup, graph=True):
    """Microseconds per evaluation of `steps` back-to-back evaluations at the
    device-resident points in turn (each launch a new point), timed with HIP
    events on the launch stream.  graph=True: the launches are captured once
    in a HIP graph and replayed, so the host's per-launch cost does not pace
    the device; the device work is the same launches."""
    with torch.cuda.stream(stream):
        for i in range(warmup):
            uml.uml_eval_nll_grad_dev(model, data, points[i % len(points)], out, stream=stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    if graph:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            for i in range(steps):
                uml.uml_eval_nll_grad_dev(model, data, points[i % len(points)], out, stream=stream)
        with torch.cuda.stream(stream):
            g.replay()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            ev0.record(stream)
            g.replay()
            ev1.record(stream)
    else:
        with torch.cuda.stream(stream):
            ev0.record(stream)
            for i in range(steps):
                uml.uml_eval_nll_grad_dev(model, data, points[i % len(points)], out, stream=stream)
            ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) * 1e3 / steps


def time_rotated(torch, uml, model, datasets, points, out, stream, steps, graph=True):
    """As time_evals, with launch i over datasets[i % len(datasets)]."""
    nd = len(datasets)
    with torch.cuda.stream(stream):
        for i in range(2 * nd):
            uml.uml_eval_nll_grad_dev(model, datasets[i % nd], points[i % len(points)], out, stream=stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)

    def issue():
        for i in range(steps):
            uml.uml_eval_nll_grad_dev(model, datasets[i % nd], points[i % len(points)], out, stream=stream)
    if graph:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            issue()
        with torch.cuda.stream(stream):
            g.replay()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            ev0.record(stream)
            g.replay()
            ev1.record(stream)
    else:
        with torch.cuda.stream(stream):
            ev0.record(stream)
            issue()
            ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) * 1e3 / steps


def headline(args, torch, uml, G, W):
    n = args.events
    dtype = np.float32 if args.precision == "mixed" else np.float64
    if args.model == "angmass4d":
        desc = W.angmass4d()
        x = G.gen_angmass4d(n, seed=SEED_DATA, dtype=dtype)
        truth = W.angmass4d_truth_vector()
    else:
        desc = W.mass1d()
        x = G.gen_mass1d(n, seed=SEED_DATA, dtype=dtype)
        truth = [5.28, 0.02, -1.5, 0.3]
    dev = torch.device("cuda:0")
    model = uml.Model(desc, args.precision, precompute=args.precompute)
    data = uml.Data(model, x)
    theta = torch.tensor(truth, dtype=torch.float64, device=dev)
    # Every step evaluates a new parameter point, as a minimiser's steps do:
    # consecutive launches never share a point, so each one runs the
    # parameter-only prologue (no step reuses the previous step's constants).
    points = theta_points(torch, model, truth, dev)
    out = torch.empty(1 + model.n_free, dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream(device=dev)
    copy_gbs = copy_check(torch, stream)

    t0 = time.perf_counter()
    us_step = time_evals(torch, uml, model, data, points, out, stream, args.steps, args.warmup,
                         graph=not args.no_graph)
    wall = time.perf_counter() - t0
    ms_per_step = us_step * 1e-3
    value = n / (ms_per_step * 1e-3)
    # the same launches issued one by one from the host (no graph)
    us_eager = time_evals(torch, uml, model, data, points, out, stream, args.steps, 0, graph=False)

    esize = 4 if args.precision == "mixed" else 8
    kname = f"eval_kernel ({args.model}, {args.precision}{', precomputed terms' if args.precompute else ''})"
    if args.precompute:   # 4 columns + 9 precomputed terms per event: a streaming kernel
        nbytes = 13 * esize * n
        achieved = nbytes / (ms_per_step * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                    "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                    "kernel": kname, "bytes_per_event": 13 * esize}
    elif args.model == "angmass4d" and args.precision == "mixed":
        achieved = FLOP_PER_EVENT_4D * n / (ms_per_step * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                    "traffic": None, "kernel": kname, "flop_per_event": FLOP_PER_EVENT_4D,
                    "frac_of_packed_fp32": round(achieved / PEAK_FP32_PACKED_TFLOPS, 4),
                    "bytes_per_event": 4 * esize}
    elif args.model == "angmass4d":
        achieved = FLOP_PER_EVENT_4D * n / (ms_per_step * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                    "traffic": None, "kernel": kname, "flop_per_event": FLOP_PER_EVENT_4D,
                    "bytes_per_event": 4 * esize}
    else:
        achieved = esize * n / (ms_per_step * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                    "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                    "kernel": kname, "bytes_per_event": esize}
    if args.model == "angmass4d" and args.marginal_events > n and not args.precompute:
        # the per-event cost alone: a second, larger dataset timed the same
        # way; the difference removes the fixed cost of a launch (dispatch,
        # constant check, reduction chain), which dominates at 1e6 events
        n2 = args.marginal_events
        x2 = G.gen_angmass4d(n2, seed=SEED_DATA + 1, dtype=dtype)
        data2 = uml.Data(model, x2)
        steps2 = max(10, args.steps // 4)
        us2 = time_evals(torch, uml, model, data2, points, out, stream, steps2, args.warmup,
                         graph=not args.no_graph)
        us1 = ms_per_step * 1e3
        per_event_s = (us2 - us1) * 1e-6 / (n2 - n)
        peak = PEAK_FP32_TFLOPS if args.precision == "mixed" else PEAK_FP64_TFLOPS
        tf = FLOP_PER_EVENT_4D / per_event_s / 1e12
        roofline["marginal"] = {"events": [n, n2], "us_per_step": [round(us1, 3), round(us2, 3)],
                                "fixed_us": round(us1 - n * per_event_s * 1e6, 3),
                                "achieved": round(tf, 3), "frac": round(tf / peak, 4)}
        del data2, x2
    if args.rotate > 1:
        # the same evaluations over `rotate` distinct datasets of the same
        # shape, one per launch in turn: with a working set beyond the 256 MB
        # last-level cache each launch reads its events from HBM ("cold");
        # the main figure above is the fit loop's own, one dataset ("hot")
        gen = G.gen_angmass4d if args.model == "angmass4d" else G.gen_mass1d
        ds = [data] + [uml.Data(model, gen(n, seed=SEED_DATA + 100 + r, dtype=dtype))
                       for r in range(args.rotate - 1)]
        steps_c = max(args.rotate * 4, (args.steps // args.rotate) * args.rotate)
        us_c = time_rotated(torch, uml, model, ds, points, out, stream, steps_c, not args.no_graph)
        cold = {"datasets": args.rotate, "working_set_mb": round(args.rotate * n * esize * len(desc["dims"]) / 1e6, 1),
                "steps": steps_c, "us_per_step": round(us_c, 3)}
        if roofline["bound"] == "hbm":
            ach = roofline["bytes_per_event"] * n / (us_c * 1e-6) / 1e9
        else:
            ach = FLOP_PER_EVENT_4D * n / (us_c * 1e-6) / 1e12
        cold["achieved"] = round(ach, 3)
        cold["frac"] = round(ach / roofline["peak"], 4)
        roofline["cold"] = cold
        del ds
    with torch.cuda.stream(stream):  # the reported NLL: at the generating point
        uml.uml_eval_nll_grad_dev(model, data, theta, out, stream=stream)
    torch.cuda.synchronize()
    wl_key = f"{args.model}-{n}-{args.precision}" + ("-precomputed" if args.precompute else "")
    traffic = counted_traffic(wl_key)
    roofline["traffic"] = traffic
    roofline["traffic_key"] = wl_key
    roofline["measured_copy_gbs"] = round(copy_gbs, 1)
    return {"desc": desc, "x": x, "truth": truth, "n": n, "model": model, "value": value,
            "ms_per_step": ms_per_step, "wall": wall, "roofline": roofline,
            "us_per_step_eager": us_eager,
            "nll": float(out[0].item())}


# ---------------------------------------------------------------------------
# Further measurements of the same path: the 4-D model in FP64, the 1-D model
# (HBM-bound by intent) hot and cold, a 1-D FP64 fit at 1e4 events, and a
# large weighted 4-D fit with its Hessian (mixed against FP64).


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def leg_eval(torch, uml, desc, x, precision, truth, steps, warmup, graph, rotate=1, gen=None,
             seed=SEED_DATA, flop=None):
    """us per evaluation at a new point per launch, hot (one dataset) and,
    with rotate > 1, cold (rotate datasets in turn)."""
    dev = torch.device("cuda:0")
    model = uml.Model(desc, precision)
    data = uml.Data(model, x)
    points = theta_points(torch, model, truth, dev)
    out = torch.empty(1 + model.n_free, dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream(device=dev)
    n = x.shape[1]
    esize = 4 if precision == "mixed" else 8
    us = time_evals(torch, uml, model, data, points, out, stream, steps, warmup, graph)
    r = {"events": n, "precision": precision, "us_per_step": round(us, 3),
         "events_per_s": round(n / (us * 1e-6), 1)}
    if flop is None:   # HBM-bound: the event columns' bytes per evaluation
        gbs = esize * x.shape[0] * n / (us * 1e-6) / 1e9
        r.update({"achieved_gbs": round(gbs, 1), "frac_of_hbm": round(gbs / PEAK_HBM_GBS, 4)})
    else:
        tf = flop * n / (us * 1e-6) / 1e12
        peak = PEAK_FP32_TFLOPS if precision == "mixed" else PEAK_FP64_TFLOPS
        r.update({"achieved_tflops": round(tf, 3), "peak_tflops": peak, "frac": round(tf / peak, 4)})
        if precision == "mixed":
            r["frac_of_packed_fp32"] = round(tf / PEAK_FP32_PACKED_TFLOPS, 4)
    if rotate > 1:
        dt = np.float32 if precision == "mixed" else np.float64
        ds = [data] + [uml.Data(model, gen(n, seed=seed + 100 + k, dtype=dt)) for k in range(rotate - 1)]
        us_c = time_rotated(torch, uml, model, ds, points, out, stream,
                            max(rotate * 4, (steps // rotate) * rotate), graph)
        gbs = esize * x.shape[0] * n / (us_c * 1e-6) / 1e9
        r["cold"] = {"datasets": rotate, "working_set_mb": round(rotate * esize * x.shape[0] * n / 1e6, 1),
                     "us_per_step": round(us_c, 3), "achieved_gbs": round(gbs, 1),
                     "frac_of_hbm": round(gbs / PEAK_HBM_GBS, 4)}
        del ds
    return r


def legs(args, torch, uml, G, W):
    sel = set(args.legs.split(",")) if args.legs not in ("all", "none") else (
        set() if args.legs == "none" else {"fp64_4d", "mass1d", "fit1d", "weighted4d"})
    graph = not args.no_graph
    steps, warm = max(20, args.steps), max(5, args.warmup)
    out = {}
    if "fp64_4d" in sel:
        x = G.gen_angmass4d(1_000_000, seed=SEED_DATA, dtype=np.float64)
        out["angmass4d_fp64_1e6"] = leg_eval(torch, uml, W.angmass4d(), x, "fp64",
                                             W.angmass4d_truth_vector(), steps, warm, graph,
                                             flop=FLOP_PER_EVENT_4D)
        print("# leg fp64_4d done", file=sys.stderr, flush=True)
    if "mass1d" in sel:
        truth = [5.28, 0.02, -1.5, 0.3]
        for n in (1_000_000, 10_000_000):
            for prec in ("mixed", "fp64"):
                dt = np.float32 if prec == "mixed" else np.float64
                x = G.gen_mass1d(n, seed=SEED_DATA, dtype=dt)
                out[f"mass1d_{prec}_{n:.0e}".replace("+0", "")] = leg_eval(
                    torch, uml, W.mass1d(), x, prec, truth, steps, warm, graph,
                    rotate=8 if n >= 10_000_000 else 1, gen=G.gen_mass1d)
        print("# leg mass1d done", file=sys.stderr, flush=True)
    if "fit1d" in sel:
        # 1e4 events, FP64 throughout: NLL + gradient, and a BFGS fit from the
        # start point 5% off truth to EDM < 1e-6 (with its covariance)
        x = G.gen_mass1d(10_000, seed=SEED_DATA, dtype=np.float64)
        r = leg_eval(torch, uml, W.mass1d(), x, "fp64", [5.28, 0.02, -1.5, 0.3], steps, warm, graph)
        model = uml.Model(W.mass1d(), "fp64")
        data = uml.Data(model, x)
        start = W.mass1d_start()
        uml.uml_fit(model, data, start)
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            f = uml.uml_fit(model, data, start)
            ts.append(time.perf_counter() - t0)
        r.update({"fit_ms": round(1e3 * float(np.median(ts)), 3), "fit_iterations": f["n_iter"],
                  "fit_evaluations": f["n_eval"], "fit_edm": f["edm"], "fit_status": f["status_name"]})
        out["mass1d_fp64_1e4"] = r
        print("# leg fit1d done", file=sys.stderr, flush=True)
    if "weighted4d" in sel:
        # 1e7 events drawn on the device, weights U(0.5, 1.5): mixed and FP64
        # fits with the Hessian covariance, and the Hessian pass alone
        n = 10_000_000
        desc = W.angmass4d()
        mm = uml.Model(desc, "mixed")
        g = uml.Data.generate(mm, n, SEED_DATA + 7)
        x = g.download()
        g.close()
        w = np.random.default_rng(SEED_DATA + 8).uniform(0.5, 1.5, n).astype(np.float32)
        truth = np.array(W.angmass4d_truth_vector())
        res = {}
        for prec in ("mixed", "fp64"):
            model = mm if prec == "mixed" else uml.Model(desc, "fp64")
            xx, ww = (x, w) if prec == "mixed" else (x.astype(np.float64), w.astype(np.float64))
            data = uml.Data(model, xx, weights=ww)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f = uml.uml_fit(model, data, truth)
            t_fit = time.perf_counter() - t0
            t0 = time.perf_counter()
            uml.uml_eval_hessian(model, data, f["theta"])
            t_h = time.perf_counter() - t0
            res[prec] = (f, t_fit, t_h)
            del data
        fm, f6 = res["mixed"][0], res["fp64"][0]
        free = np.array([not p.get("fixed", False) for p in desc["params"]])
        dth = np.abs(fm["theta"][free] - f6["theta"][free]) / f6["errors"][free]
        dsg = np.abs(fm["errors"][free] - f6["errors"][free]) / f6["errors"][free]
        out["angmass4d_weighted_1e7"] = {
            "events": n, "weights": "U(0.5, 1.5)",
            "fit_ms": {k: round(1e3 * v[1], 2) for k, v in res.items()},
            "hessian_ms": {k: round(1e3 * v[2], 2) for k, v in res.items()},
            "fit_iterations": {k: v[0]["n_iter"] for k, v in res.items()},
            "status": {k: v[0]["status_name"] for k, v in res.items()},
            "max_dtheta_over_sigma_mixed_vs_fp64": float(dth.max()),
            "max_rel_dsigma_mixed_vs_fp64": float(dsg.max())}
        print("# leg weighted4d done", file=sys.stderr, flush=True)
    return out


# ---------------------------------------------------------------------------
# Serving toy study


class Stream:
    """The request stream: sizes, arrival times and events.  Toy i is the
    pseudo-experiment with seed SEED_TOY0 + i.  With device generation (the
    default) each request is drawn on the GPU from its seed.  With host
    events, the first n_indep requests carry independently generated events
    and the others are seeded windows of one large pool from the same model;
    pulls then come from the first n_indep toys only."""

    def __init__(self, args, G):
        rng = np.random.default_rng(SEED_STREAM)
        k = args.serving_fits
        self.device = args.serving_source == "device"
        self.sizes = np.floor(np.exp(rng.uniform(np.log(500), np.log(50000), k))).astype(np.int64)
        gaps = rng.exponential(1.0 / args.rate, k)
        self.arrivals = np.cumsum(gaps) - gaps[0]
        self.offsets = rng.integers(0, max(args.pool_events, 60000) - 50000, k)
        if self.device:
            self.n_indep = k
            return
        self.n_indep = min(args.pull_fits, k)
        pool_n = max(args.pool_events, 60000)
        self.pool = G.gen_angmass4d(pool_n, SEED_POOL, dtype=np.float32)
        self.indep = [G.gen_angmass4d(int(self.sizes[i]), SEED_TOY0 + i, dtype=np.float32)
                      for i in range(self.n_indep)]

    def seed(self, i):
        return SEED_TOY0 + i

    def events(self, i):
        if i < self.n_indep:
            return self.indep[i]
        o = int(self.offsets[i])
        return self.pool[:, o:o + int(self.sizes[i])]

    def submit(self, srv, i):
        if self.device:
            return srv.submit_generated(int(self.sizes[i]), self.seed(i))
        return srv.submit(self.events(i))

    def data(self, uml, um, i):
        if self.device:
            return uml.Data.generate(um, int(self.sizes[i]), self.seed(i))
        return uml.Data(um, self.events(i))


def _pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


def run_server(uml, um, st, k, open_loop, slots, budget):
    srv = uml.Server(um, max_slots=slots, hbm_budget=budget)
    t_recv, res = {}, {}
    idx = {}
    done = threading.Event()

    def collect():
        got = 0
        while got < k:
            rs = srv.poll(max_results=256, timeout_us=20000)
            t = time.perf_counter()
            for r in rs:
                t_recv[r["ticket"]] = t
                res[r["ticket"]] = r
            got += len(rs)
        done.set()

    th = threading.Thread(target=collect, daemon=True)
    th.start()
    t0 = time.perf_counter()
    for i in range(k):
        if open_loop:
            d = t0 + st.arrivals[i] - time.perf_counter()
            if d > 0:
                time.sleep(d)
        idx[st.submit(srv, i)] = i
    th.join()
    t_end = max(t_recv.values())
    stats = srv.stats()
    srv.close()
    lat = np.empty(k)
    out = [None] * k
    for tk, i in idx.items():
        lat[i] = t_recv[tk] - (t0 + (st.arrivals[i] if open_loop else 0.0))
        out[i] = res[tk]
    return {"fits_per_s": k / (t_end - t0), "p50_ms": 1e3 * _pct(lat, 50),
            "p99_ms": 1e3 * _pct(lat, 99), "elapsed_s": t_end - t0, "stats": stats,
            "results": out}


def run_loop(uml, um, st, k, open_loop):
    lat = np.empty(k)
    out = []
    t0 = time.perf_counter()
    for i in range(k):
        if open_loop:
            d = t0 + st.arrivals[i] - time.perf_counter()
            if d > 0:
                time.sleep(d)
        data = st.data(uml, um, i)
        r = uml.uml_fit(um, data)
        data.close()
        t = time.perf_counter()
        lat[i] = t - (t0 + (st.arrivals[i] if open_loop else 0.0))
        out.append(r)
    t_end = time.perf_counter()
    return {"fits_per_s": k / (t_end - t0), "p50_ms": 1e3 * _pct(lat, 50),
            "p99_ms": 1e3 * _pct(lat, 99), "elapsed_s": t_end - t0, "results": out}


def pulls(results, truth, free):
    ok = [r for r in results if r["status"] == 0]
    if not ok:
        return None
    p = np.array([(r["theta"][free] - truth[free]) / r["errors"][free] for r in ok])
    return {"fits": len(ok), "mean": [round(float(v), 3) for v in p.mean(0)],
            "width": [round(float(v), 3) for v in p.std(0, ddof=1)] if len(ok) > 1 else None}


def serving(args, uml, G, W):
    desc = W.angmass4d()
    um = uml.Model(desc, "mixed")
    truth = np.array(W.angmass4d_truth_vector())
    free = np.array([not p.get("fixed", False) for p in desc["params"]])
    st = Stream(args, G)
    k = args.serving_fits
    kl = min(args.loop_fits, k)
    budget = args.budget_mb << 20
    s_open = run_server(uml, um, st, k, True, args.slots, budget)
    s_sat = run_server(uml, um, st, k, False, args.slots, budget)
    # the same saturated stream under a budget below the natural footprint, so
    # that admission waits for memory
    s_tight = (run_server(uml, um, st, k, False, args.slots, args.tight_budget_mb << 20)
               if args.tight_budget_mb > 0 else None)
    empty = {"fits_per_s": 0.0, "p50_ms": 0.0, "p99_ms": 0.0, "elapsed_s": 0.0, "results": []}
    l_sat = run_loop(uml, um, st, kl, False) if kl else empty
    l_open = run_loop(uml, um, st, kl, True) if kl else empty
    # equal accuracy: the fits of both paths on the requests both ran
    dev = 0.0
    for a, b in zip(s_sat["results"][:kl], l_sat["results"]):
        if a["status"] == 0 and b["status"] == 0:
            dev = max(dev, float(np.max(np.abs(a["theta"][free] - b["theta"][free])
                                        / b["errors"][free])))
    statuses = {}
    for r in s_sat["results"]:
        statuses[r["status_name"]] = statuses.get(r["status_name"], 0) + 1

    def summary(d):
        o = {key: round(d[key], 3) for key in ("fits_per_s", "p50_ms", "p99_ms", "elapsed_s")}
        if "stats" in d:
            s = d["stats"]
            o["peak_resident_mb"] = round(s["peak_resident_bytes"] / 2**20, 1)
            o["budget_waits"] = s["budget_waits"]
            o["iterations"] = s["iterations"]
            o["worker_s"] = {"admit": round(s["t_admit_s"], 3), "iterate": round(s["t_iterate_s"], 3),
                             "retire": round(s["t_retire_s"], 3)}
        return o

    return {"desc": desc, "stream": st, "truth": truth, "free": free,
            "server_results": s_open["results"],
            "record": {
                "workload": (f"4-D toy fits, sizes log-uniform in [500, 50000], Poisson arrivals "
                             f"at {args.rate:g}/s, mixed precision, start at the generating values, "
                             "EDM < 1e-6"),
                "fits": k, "loop_fits": kl, "slots": args.slots, "hbm_budget_mb": args.budget_mb,
                "server_open_loop": summary(s_open), "server_saturated": summary(s_sat),
                "server_saturated_tight_budget": (dict(summary(s_tight), hbm_budget_mb=args.tight_budget_mb)
                                                  if s_tight else None),
                "loop_open_loop": summary(l_open), "loop_saturated": summary(l_sat),
                "capacity_ratio": (round(s_sat["fits_per_s"] / l_sat["fits_per_s"], 2)
                                   if l_sat["fits_per_s"] else None),
                "max_dtheta_over_sigma_server_vs_loop": dev,
                "statuses": statuses,
                "pulls": pulls(s_open["results"][:st.n_indep], truth, free),
                "events": ("every request drawn on the GPU from its own seed %d+i" % SEED_TOY0
                           if st.device else
                           "first %d requests independently generated (seed %d+i); the rest are "
                           "seeded windows of a %d-event pool from the same model"
                           % (st.n_indep, SEED_TOY0, st.pool.shape[1]))}}


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on a bounded sample of the same work


def fp32_storage(x64, desc):
    """FP32 storage of FP64 event values: the nearest value, moved one step
    inwards where rounding left the dimension's range."""
    out = x64.astype(np.float32)
    for d, dim in enumerate(desc["dims"]):
        f = out[d]
        up = f.astype(np.float64) > dim["hi"]
        f[up] = np.nextafter(f[up], np.float32(-np.inf))
        dn = f.astype(np.float64) < dim["lo"]
        f[dn] = np.nextafter(f[dn], np.float32(np.inf))
    return out


def cpu_baseline(args, H, S):
    import oracle
    om = oracle.Model(H["desc"])
    k = min(H["n"], 100_000)
    xs = H["x"][:, :k].astype(np.float64)
    th = np.array(H["truth"])
    reps, t = 0, 0.0
    t0 = time.perf_counter()
    while t < args.cpu_seconds:
        om.nll(xs, th, order=1)
        reps += 1
        t = time.perf_counter() - t0
    base = {"value": round(k * reps / t, 1), "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} events of the benchmark dataset, NLL+gradient, {reps} evaluations "
                      f"in {t:.1f} s, one thread", "host": host_info()}
    if S is None:
        return base, None
    # the oracle's own fits of the independently generated toys, in order,
    # for a bounded time; compared with the server's fits of the same toys
    st, free = S["stream"], S["free"]
    om4 = oracle.Model(S["desc"])
    n_fit, t, dmax, emax, nev = 0, 0.0, 0.0, 0.0, 0
    t0 = time.perf_counter()
    while n_fit < st.n_indep and t < args.cpu_seconds:
        if st.device:   # the oracle draws the same toy; stored in FP32 as the GPU stores it
            xg, _ = om4.generate(int(st.sizes[n_fit]), st.seed(n_fit))
            x = fp32_storage(xg, S["desc"]).astype(np.float64)
        else:
            x = st.indep[n_fit].astype(np.float64)
        r = om4.fit(x, S["truth"])
        g = S["server_results"][n_fit]
        if r["status"] == 0 and g["status"] == 0:
            sig = r["errors"]
            dmax = max(dmax, float(np.max(np.abs(g["theta"][free] - r["theta"][free]) / sig)))
            emax = max(emax, float(np.max(np.abs(g["errors"][free] - sig) / sig)))
        nev += x.shape[1]
        n_fit += 1
        t = time.perf_counter() - t0
    fits = {"value": round(n_fit / t, 2), "unit": "fits/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_fit} toys of the stream ({nev} events), FP64 BFGS "
                      f"to EDM < 1e-6 and Hessian, {t:.1f} s, one thread",
            "max_dtheta_over_sigma_vs_server": dmax,
            "max_rel_error_of_sigma_vs_server": emax}
    return base, fits


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--events", type=int, default=1_000_000)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--model", default="angmass4d", choices=["angmass4d", "mass1d"])
    ap.add_argument("--serving-fits", type=int, default=20000,
                    help="requests in the toy study (0: skip it)")
    ap.add_argument("--loop-fits", type=int, default=5000,
                    help="requests of the same stream run through the per-fit loop")
    ap.add_argument("--rate", type=float, default=500.0, help="open-loop arrival rate, fits/s")
    ap.add_argument("--slots", type=int, default=512,
                    help="server fit slots (512: about 140 MB resident in the toy study)")
    ap.add_argument("--budget-mb", type=int, default=256, help="server device-memory budget")
    ap.add_argument("--pull-fits", type=int, default=200,
                    help="host events only: independently generated toys for the pulls")
    ap.add_argument("--serving-source", default="device", choices=["device", "host"],
                    help="toy events drawn on the GPU from each request's seed, or uploaded")
    ap.add_argument("--pool-events", type=int, default=1 << 22)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precompute", action="store_true",
                    help="4-D model with the P-wave's event-only terms stored per event")
    ap.add_argument("--marginal-events", type=int, default=4_000_000,
                    help="second dataset size for the per-event (marginal) rate; 0: skip")
    ap.add_argument("--tight-budget-mb", type=int, default=16,
                    help="budget of a second saturated server run, below the natural footprint; 0: skip")
    ap.add_argument("--no-graph", action="store_true",
                    help="time launches issued one by one instead of graph replays")
    ap.add_argument("--legs", default="all",
                    help="comma list of extra measurements (fp64_4d, mass1d, fit1d, weighted4d) "
                         "or 'all' or 'none'")
    ap.add_argument("--rotate", type=int, default=1,
                    help="also time the evaluations over this many distinct datasets in turn "
                         "(a working set beyond the last-level cache); 1: skip")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this implementation runs on one GPU (asked for {args.gpus}); "
              "how the path would shard over several is described in DESIGN.md.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2505_12414_amd import datagen as G
    from paper_2505_12414_amd import uml
    from paper_2505_12414_amd import workloads as W

    torch.cuda.init()
    H = headline(args, torch, uml, G, W)
    print(f"# headline done: {H['ms_per_step'] * 1e3:.2f} us/step", file=sys.stderr, flush=True)
    L = legs(args, torch, uml, G, W)
    S = None
    if args.serving_fits > 0:
        S = serving(args, uml, G, W)
        print("# serving done", file=sys.stderr, flush=True)
    cpu, cpu_fits = (None, None)
    if not args.no_cpu_baseline:
        cpu, cpu_fits = cpu_baseline(args, H, S)

    if args.model == "angmass4d":
        metric = "NLL+grad events/s at 1e6 events (4D); toy fits/s with p50/p99 latency"
        wl = "4-D angular x mass NLL+gradient"
    else:
        metric = "NLL+grad events/s (1D mass model)"
        wl = "1-D mass-model NLL+gradient"
    prec = "FP32 compute / FP64 accumulate" if args.precision == "mixed" else "FP64"
    rec = {"metric": metric, "value": round(H["value"], 1), "unit": "events/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(H["ms_per_step"], 6), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f32" if args.precision == "mixed" else "f64", "data": "synthetic",
           "config": {"workload": f"{wl}, {H['n']} events, {prec}", "events": H["n"],
                      "free_params": H["model"].n_free, "precision": args.precision},
           "roofline": H["roofline"], "cpu_baseline": cpu,
           "nll": H["nll"], "wall_s": round(H["wall"], 4),
           "timing": "graph replay of the steps" if not args.no_graph else "launches issued one by one",
           "us_per_step_eager": round(H["us_per_step_eager"], 3), "host": host_info()}
    if L:
        rec["legs"] = L
    if S is not None:
        rec["serving"] = S["record"]
        if cpu_fits is not None:
            rec["serving"]["cpu_baseline"] = cpu_fits
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
