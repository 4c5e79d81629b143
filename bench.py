"""Benchmark of the hot path: fused NLL + gradient evaluations per second.

A step is one evaluation of -sum_i ln P(x_i|theta) and its gradient over every
event of one dataset (the per-minimiser-step work of an unbinned fit): the
constant staging, the fused PDF/log/gradient event kernel, the deterministic
two-pass reduction and the FP64 epilogue -- one kernel launch.  The workload
is the 4-D angular x mass model (P-wave x Gauss signal, Chebyshev^3 x Exp
background, 17 free parameters) at 1e6 synthetic events in mixed precision
(FP32 per-event arithmetic, FP64 accumulation), events resident in HBM.

Prints one JSON line (see the repository's benchmark contract).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peaks derived in the design doc: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3e12
# VALU lane-instructions/s; FP32 FMA = 2 FLOP -> 78.6 TFLOP/s without packed
# FP32 (packed FP32 instructions are not used by this library).
PEAK_FP32_UNPACKED_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# Algorithmic FP32 work per event of the 4-D model (counted from the fused
# per-event formula in the design doc: FMA = 2, transcendental = 1).
FLOP_PER_EVENT_4D = 145


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--events", type=int, default=1_000_000)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--model", default="angmass4d", choices=["angmass4d", "mass1d"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); "
              "the multi-GPU path is a design in DESIGN.md, not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2505_12414_amd import datagen as G
    from paper_2505_12414_amd import uml
    from paper_2505_12414_amd import workloads as W

    n = args.events
    dtype = np.float32 if args.precision == "mixed" else np.float64
    if args.model == "angmass4d":
        desc = W.angmass4d()
        x = G.gen_angmass4d(n, seed=20250512, dtype=dtype)
        truth = W.angmass4d_truth_vector()
    else:
        desc = W.mass1d()
        x = G.gen_mass1d(n, seed=20250512, dtype=dtype)
        truth = [5.28, 0.02, -1.5, 0.3]
    torch.cuda.init()
    dev = torch.device("cuda:0")
    model = uml.Model(desc, args.precision)
    data = uml.Data(model, x)
    theta = torch.tensor(truth, dtype=torch.float64, device=dev)
    out = torch.empty(1 + model.n_free, dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream(device=dev)

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            uml.uml_eval_nll_grad_dev(model, data, theta, out, stream=stream)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        ev0.record(stream)
        for _ in range(args.steps):
            uml.uml_eval_nll_grad_dev(model, data, theta, out, stream=stream)
        ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)          # HIP events on the kernels' stream
    ms_per_step = gpu_ms / args.steps
    value = n * args.steps / (gpu_ms * 1e-3)
    nll = float(out[0].item())

    esize = 4 if args.precision == "mixed" else 8
    kname = f"eval_kernel<{args.model}, {args.precision}>"
    if args.model == "angmass4d":
        flop = FLOP_PER_EVENT_4D * n
        achieved = flop / (ms_per_step * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 3),
                    "peak": PEAK_FP32_UNPACKED_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / PEAK_FP32_UNPACKED_TFLOPS, 4), "traffic": None,
                    "kernel": kname, "flop_per_event": FLOP_PER_EVENT_4D,
                    "bytes_per_event": 4 * esize}
    else:
        nbytes = esize * n
        achieved = nbytes / (ms_per_step * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                    "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                    "kernel": kname, "bytes_per_event": esize}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        om = oracle.Model(desc)
        k = min(n, 100_000)
        xs = x[:, :k].astype(np.float64)
        th = np.array(truth)
        reps, t = 0, 0.0
        t0 = time.perf_counter()
        while t < 10.0:
            om.nll(xs, th, order=1)
            reps += 1
            t = time.perf_counter() - t0
        cpu = {"value": round(k * reps / t, 1), "unit": "events/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{k} events of the same dataset, NLL+gradient, {reps} evaluations, "
                         f"{t:.1f} s, single thread"}

    metric = ("NLL+grad events/s at 1e6 events (4D)" if args.model == "angmass4d"
              else "NLL+grad events/s (1D mass model)")
    wl = ("4-D angular x mass NLL+gradient" if args.model == "angmass4d"
          else "1-D mass-model NLL+gradient")
    rec = {"metric": metric, "value": round(value, 1),
           "unit": "events/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms_per_step, 6), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32" if args.precision == "mixed" else "f64",
           "data": "synthetic",
           "config": {"workload": f"{wl}, {n} events, "
                                  f"{'FP32 compute / FP64 accumulate' if args.precision == 'mixed' else 'FP64'}",
                      "events": n, "free_params": model.n_free, "precision": args.precision},
           "roofline": roofline, "cpu_baseline": cpu,
           "nll": nll, "wall_s": round(wall, 4)}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
