"""Throughput benchmark of the network-dynamics hot path on one MI355X.

Default workload: FitzHugh-Nagumo rings of N = 65536 elements, coupling radius
P = floor(0.35 N) = 22937, eps = 0.05, a = 0.5, sigma = 0.1, phi = pi/2 - 0.1,
initial (u, v) on the circle of radius 2 at seeded random angles, classical RK4
with dt = 0.01 over a horizon of 10^4 steps.  One benchmark step integrates a
batch of B such rings (distinct seeds) over the full horizon with one batched
launch sequence; `value` is the aggregate oscillator-steps per second in FP64,
the FP32-bulk figure is reported beside it.  Inputs are synthetic and resident
on the GPU before timing starts.

Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
FHN_PRM = [0.05, 0.5, 0.1, math.pi / 2 - 0.1]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed benchmark steps")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=64, help="rings per benchmark step")
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--horizon", type=int, default=10000, help="RK4 steps per benchmark step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=1)
    ap.add_argument("--tile", type=int, default=0, help="ring tile override (0 = library default)")
    ap.add_argument("--grid", type=int, default=0, help="persistent grid override (0 = one block per tile)")
    ap.add_argument("--chunk", type=int, default=0, help="steps per captured graph chunk (0 = default)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (for scaling HBM counters)")
    return ap.parse_args()


def bytes_alg_per_elem_step(nvars, prec):
    """13 state-vector accesses per element and RK4 step (no window scratch):
    y read 4x, acc written and read, y written (doubles) and k1..k3 written and
    read once each (bulk type)."""
    kb = 8 if prec == "fp64" else 4
    return nvars * (7 * 8 + 6 * kb)


def run_fhn(nd, torch, args, prec_code, stream):
    n, P = args.n, int(0.35 * args.n)
    from paper_2410_19075_amd import inputs
    hs = []
    for b in range(args.batch):
        h = nd.nd_create(nd.problem(nd.ND_FHN, nd.ND_RING, n, FHN_PRM, precision=prec_code, radius=P))
        if args.tile or args.grid or args.chunk:
            c = nd.nd_get_config(h)
            c.tile = args.tile or c.tile
            c.grid = args.grid or c.grid
            c.chunk = args.chunk or c.chunk
            nd.nd_set_config(h, c)
        y0 = torch.from_numpy(inputs.fhn_circle(1000 + b, n)).cuda()
        nd.nd_set_state(h, y0, stream=stream)
        hs.append(h)
    torch.cuda.synchronize()
    dts = [0.01] * len(hs)
    steps = [args.horizon] * len(hs)

    def one():
        nd.nd_run_batch(hs, dts, steps, stream=stream)

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    times = []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev_total = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        ev0.record(stream)
        one()
        ev1.record(stream)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        ev_total += ev0.elapsed_time(ev1) / 1e3
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    y = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    nd.nd_get_state(hs[0], y, stream=stream)
    torch.cuda.synchronize()
    finite = bool(torch.isfinite(y).all().item())
    for h in hs:
        nd.nd_destroy(h)
    return wall, times, ev_total, finite


def cpu_baseline(args):
    from oracle import oracle as O
    from paper_2410_19075_amd import inputs
    n, P = args.n, int(0.35 * args.n)
    y0 = inputs.fhn_circle(1000, n)
    net = O.ring(O.FHN, n, P, FHN_PRM)
    O.lib()
    t0 = time.perf_counter()
    O.run(net, y0, 0.01, args.cpu_sample_steps)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n * args.cpu_sample_steps / dt, "unit": "oscillator-steps/s", "cores": cores,
            "kind": "oracle", "sample": f"one FHN ring N={n} P={P}, {args.cpu_sample_steps} RK4 step(s), FP64, "
                                        f"direct neighbour sums, {dt:.2f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (every box here has one GPU)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2410_19075_amd import nd
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    stream = torch.cuda.current_stream()
    if args.copy_calibration:
        nbytes = args.copy_calibration
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 3}))
        return
    n, P = args.n, int(0.35 * args.n)
    osc_per_step = args.batch * n * args.horizon

    wall, times, ev_total, finite = run_fhn(nd, torch, args, nd.ND_FP64, stream)
    value = osc_per_step * args.steps / wall
    n_stage = 4 * args.horizon * args.steps
    stage_s = ev_total / n_stage
    balg64 = bytes_alg_per_elem_step(2, "fp64")
    per_launch = args.batch * n * balg64 / 4.0
    achieved = per_launch / stage_s / 1e9
    out = {
        "metric": "oscillator-steps/s",
        "value": value,
        "unit": "oscillator-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FitzHugh-Nagumo ring N={n} P={P} (0.35N), eps=0.05 a=0.5 sigma=0.1 "
                               f"phi=pi/2-0.1, RK4 dt=0.01, {args.horizon} steps per ring, {args.batch} rings "
                               f"(seeds 1000..) per benchmark step",
                   "global_batch": args.batch, "seq_len": args.horizon, "parallelism": "single-gpu"},
        "coupling_terms_per_s": value * 2 * P * 4,
        "batch_latency_ms": {"p50": 1e3 * float(np.percentile(times, 50)),
                             "p99": 1e3 * float(np.percentile(times, 99))},
        "state_finite": finite,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_ring_stage<FHN,double>", "bytes_per_launch": per_launch,
                     "avg_launch_us": stage_s * 1e6},
    }
    if not args.no_fp32:
        wall32, times32, ev32, fin32 = run_fhn(nd, torch, args, nd.ND_FP32_BULK, stream)
        v32 = osc_per_step * args.steps / wall32
        s32 = ev32 / n_stage
        pl32 = args.batch * n * bytes_alg_per_elem_step(2, "fp32") / 4.0
        out["fp32_bulk"] = {"value": v32, "unit": "oscillator-steps/s", "ms_per_step": 1e3 * wall32 / args.steps,
                            "roofline": {"bound": "hbm", "achieved": pl32 / s32 / 1e9, "peak": HBM_PEAK_GBS,
                                         "unit": "GB/s", "frac": pl32 / s32 / 1e9 / HBM_PEAK_GBS,
                                         "avg_launch_us": s32 * 1e6},
                            "state_finite": fin32}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
