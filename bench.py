"""Throughput benchmark of the network-dynamics hot path on one MI355X.

Default workload (--workload cube): 3D Kuramoto-Sakaguchi on the periodic
200^3 lattice (8e6 oscillators), cube neighbourhood of half-width 4 (728
neighbours), alpha = 0.8, mu = 1, omega = 0, uniform phases plus a planted
coherent ball, classical RK4 with dt = 0.05 over 2000 steps.  One benchmark
step integrates the lattice over the full horizon; `value` is oscillator-steps
per second in FP64, the FP32-bulk figure (FP32 maps and RHS, FP64 window sums
and state) is reported beside it.  --n 400 runs the 400^3 lattice (6.4e7
oscillators, beyond the 256 MB Infinity Cache).

Other workloads (one JSON line each, same fields):
  --workload fhn       FitzHugh-Nagumo rings of N = 65536 elements, coupling
                       radius P = floor(0.35 N) = 22937, eps = 0.05, a = 0.5,
                       sigma = 0.1, phi = pi/2 - 0.1, (u, v) on the circle of
                       radius 2 at seeded random angles, dt = 0.01, 10^4 steps;
                       a batch of B rings (distinct seeds, --batch, default 64)
                       per benchmark step in one batched launch sequence
  --workload hh        Hodgkin-Huxley, 10^6 neurons, random directed graph with
                       out-degree 100, weights U[0, 0.1], I_app U[8, 12],
                       dt = 0.01 ms, 5000 steps
  --workload kuramoto  Kuramoto rings N = 1024, P = 256, alpha = 1.46, 200 steps
  --workload inertia   3D Kuramoto-Sakaguchi with inertia, 100^3 periodic lattice,
                       m = 1, eps = 0.05, mu = 0.01, alpha = 0.45 (the paper's
                       performance state), cube half-width 2 (124 neighbours),
                       dt = 0.05, 1000 steps (50 time units), psi = 0 initially
  --workload ball      the same state with the paper's ball neighbourhood of
                       radius --radius (2: 33 links, the default; 6: 925 links),
                       centre included
  --workload links     the same 100^3 inertia state with the ball of radius
                       --radius given as an arbitrary binary coupling matrix
                       (33 links per row at P = 2), held in the paper's
                       differentially compressed form and extracted per row on
                       the fly
  --workload adaptive  Dormand-Prince 5(4) with step-size control on the device:
                       4096 Kuramoto rings N = 1024, P = 256, alpha = 1.46,
                       omega = 0, integrated over t = 100 at rtol = 1e-8,
                       atol = 1e-10, each ring controlling its own step from
                       h0 = 1e-3; value counts accepted steps.  With --n above
                       1024: FHN rings of that size (P = floor(0.35 N), the
                       default workload's parameters and inputs) integrated over
                       t = 10, 16 rings, on the tiled path
  --workload adaptive3d  the paper's 3D performance state (Kuramoto with inertia,
                       100^3 lattice, ball of radius 2 as a compressed coupling
                       matrix) integrated with Dormand-Prince over the paper's
                       50 time units at rtol = 1e-6, atol = 1e-8
  --workload serve     continuous-batching server fed by seeded Poisson arrivals of
                       Kuramoto-ring and FHN-ring requests (50/50), N log-uniform in
                       [2^10, 2^22], P/N uniform in [0.05, 0.4], alpha uniform in
                       [1.3, 1.55], horizons log-uniform in [--hmin, --hmax] RK4 steps,
                       arrival rate = rho x measured capacity; reports p50/p99 request
                       and chunk latency, aggregate oscillator-steps/s, and the FP32-bulk
                       results' error against the FP64 run of the same requests

Inputs are synthetic (seeded) and resident on the GPU before timing starts.
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
FP64_PEAK_TFLOPS = 78.6  # MI355X vector FP64 (FMA = 2 flops), vendor figure
# FP64 flops per element and RK4 step of the resident Kuramoto ring kernel, per
# stage: sin+cos by reduction and two Horner polynomials (37), window sums from
# the prefix sums and the self term (8), the rotated RHS (15), stage value and
# RK bookkeeping (4)
KURAMOTO_RESIDENT_FLOPS = 4 * (37 + 8 + 15 + 4)
PROFILES = os.path.join(ROOT, "profiles")
FHN_PRM = [0.05, 0.5, 0.1, math.pi / 2 - 0.1]
HH_PRM = [1.0, 120.0, 36.0, 0.3, 50.0, -77.0, -54.387, 0.0, 0.0, 2.0]

DEFAULTS = {  # workload: (batch, horizon, dt, n)
    "fhn": (64, 10000, 0.01, 65536),
    "kuramoto": (4096, 200, 0.01, 1024),
    "cube": (1, 2000, 0.05, 200),
    "hh": (1, 5000, 0.01, 1000000),
    "inertia": (1, 1000, 0.05, 100),
    "ball": (1, 1000, 0.05, 100),
    "links": (1, 1000, 0.05, 100),
    "serve": (200, 0, 0.01, 0),
    "adaptive": (4096, 0, 0.0, 1024),
    "adaptive3d": (1, 0, 0.0, 100),
}
DEFAULTS_N = {"fhn": 65536, "kuramoto": 1024, "cube": 200 ** 3, "hh": 1000000, "inertia": 100 ** 3,
              "ball": 100 ** 3, "links": 100 ** 3}
INERTIA_PRM = [0.0, 0.01, 0.45, 1.0, 0.05]  # omega, mu, alpha, m, eps (Sec. V, Fig. 6c)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed benchmark steps")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(DEFAULTS), default="cube")
    ap.add_argument("--batch", type=int, default=0, help="networks per benchmark step (0 = workload default)")
    ap.add_argument("--n", type=int, default=0, help="elements (cube: edge) per network (0 = default)")
    ap.add_argument("--radius", type=int, default=2, help="ball: neighbourhood radius P")
    ap.add_argument("--horizon", type=int, default=0, help="RK4 steps per benchmark step (0 = workload default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=1)
    ap.add_argument("--tile", type=int, default=0, help="tile override (0 = library default)")
    ap.add_argument("--tile-y", type=int, default=0)
    ap.add_argument("--tile-z", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0, help="persistent grid override (0 = one block per work item)")
    ap.add_argument("--block", type=int, default=0, help="ball: workgroup size override (256 or 1024: gather form; 512: plane-scatter form)")
    ap.add_argument("--chunk", type=int, default=0, help="steps per captured graph chunk (0 = default)")
    ap.add_argument("--hmin", type=float, default=1e3, help="serve: shortest horizon (RK4 steps)")
    ap.add_argument("--hmax", type=float, default=1e5, help="serve: longest horizon (RK4 steps)")
    ap.add_argument("--probe", type=int, default=40, help="serve: requests of the closed-loop capacity probe")
    ap.add_argument("--floor-checks", type=int, default=8,
                    help="serve: FP64 floor runs for the requests with the largest FP32-bulk R gaps")
    ap.add_argument("--rho", type=float, default=0.8, help="serve: offered load / capacity")
    ap.add_argument("--budget-gb", type=float, default=8.0, help="serve: HBM budget of the server")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (for scaling HBM counters)")
    a = ap.parse_args()
    b, hz, dt, n = DEFAULTS[a.workload]
    if a.workload == "adaptive" and a.n > 1024:
        b = 16  # rings beyond one workgroup (the FHN ring of the default workload)
    a.batch = a.batch or b
    a.horizon = a.horizon or hz
    a.n = a.n or n
    a.dt = dt
    return a


# ----------------------------------------------------------------- workloads
class Workload:
    """Network descriptions, synthetic inputs and per-element algorithmic bytes."""

    def __init__(self, args, nd):
        self.a, self.nd = args, nd
        w = args.workload
        if w == "fhn":
            self.n, self.P = args.n, int(0.35 * args.n)
            self.nvars, self.links = 2, 2 * self.P
            self.name = (f"FitzHugh-Nagumo ring N={self.n} P={self.P} (0.35N), eps=0.05 a=0.5 sigma=0.1 "
                         f"phi=pi/2-0.1, RK4 dt=0.01, {args.horizon} steps per ring, {args.batch} rings "
                         f"(seeds 1000..) per benchmark step")
            self.kernel = "k_ring_stage<FHN>"
            self.prof = ("ring_stage_fhn_65536_x64.md", "k_ring_stage", ["ring.hip", "models.h", "nd_dev.h", "runtime.hip"])
        elif w == "kuramoto":
            self.n, self.P = args.n, args.n // 4
            self.nvars, self.links = 1, 2 * self.P
            self.name = (f"Kuramoto-Sakaguchi ring N={self.n} P={self.P}, alpha=1.46 mu=1 omega=0, RK4 dt=0.01, "
                         f"{args.horizon} steps, {args.batch} rings per benchmark step")
            self.kernel = "k_ring_resident<Kuramoto>"
            self.prof = None
        elif w == "inertia":
            self.n1 = args.n
            self.n, self.P = args.n ** 3, 2
            self.nvars, self.links = 2, 124
            self.name = (f"Kuramoto-Sakaguchi with inertia, 3D lattice {args.n}^3 periodic, cube half-width 2 "
                         f"(124 neighbours), m=1 eps=0.05 mu=0.01 alpha=0.45 omega=0, RK4 dt=0.05, "
                         f"{args.horizon} steps, planted coherent ball, psi=0")
            self.kernel = "k_cube_stage<inertia>"
            self.prof = (f"cube_stage_inertia_{args.n}cubed_h2.md", "k_cube_stage",
                         ["cube.hip", "models.h", "nd_dev.h", "runtime.hip"])
        elif w == "ball":
            self.n1 = args.n
            self.n, self.P = args.n ** 3, args.radius
            r = np.arange(-args.radius, args.radius + 1)
            X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
            self.nvars, self.links = 2, int(np.sum(X ** 2 + Y ** 2 + Z ** 2 <= args.radius ** 2))
            self.name = (f"Kuramoto-Sakaguchi with inertia, 3D lattice {args.n}^3 periodic, ball of radius "
                         f"{args.radius} ({self.links} links incl. the element), m=1 eps=0.05 mu=0.01 alpha=0.45 "
                         f"omega=0, RK4 dt=0.05, {args.horizon} steps, planted coherent ball, psi=0")
            self.kernel = "k_ball_stage<inertia>"
            self.prof = (f"ball_stage_inertia_{args.n}cubed_p{args.radius}.md", "k_ball_stage",
                         ["cube.hip", "models.h", "nd_dev.h", "runtime.hip"])
        elif w == "links":
            from paper_2410_19075_amd import inputs
            self.n1 = args.n
            self.n, self.P = args.n ** 3, args.radius
            self.rows = inputs.lattice_ball_links(args.n, args.n, args.n, args.radius)
            self.nvars, self.links = 2, int(self.rows[0][1])
            self.name = (f"Kuramoto-Sakaguchi with inertia, 3D lattice {args.n}^3 periodic, ball of radius "
                         f"{args.radius} ({self.links} links incl. the element) given as a binary coupling "
                         f"matrix in compressed form (Alg. 2), m=1 eps=0.05 mu=0.01 alpha=0.45 omega=0, "
                         f"RK4 dt=0.05, {args.horizon} steps, planted coherent ball, psi=0")
            self.kernel = "k_links_stage<inertia>"
            self.prof = (f"links_stage_inertia_{args.n}cubed_ball{args.radius}.md", "k_links_stage",
                         ["links.hip", "models.h", "nd_dev.h", "runtime.hip"])
        elif w == "cube":
            self.n1 = args.n
            self.n, self.P = args.n ** 3, 4
            self.nvars, self.links = 1, 728
            self.name = (f"Kuramoto-Sakaguchi 3D lattice {args.n}^3 periodic, cube half-width 4 (728 neighbours), "
                         f"alpha=0.8 mu=1 omega=0, RK4 dt=0.05, {args.horizon} steps, planted coherent ball")
            self.kernel = "k_cube_stage"
            self.prof = ("cube_stage_200cubed_h4.md", "k_cube_stage", ["cube.hip", "models.h", "nd_dev.h", "runtime.hip"])
        else:
            self.n = args.n
            self.nvars, self.links = 4, 100
            self.name = (f"Hodgkin-Huxley N={self.n}, random directed graph out-degree 100 (nnz={self.n * 100}), "
                         f"w U[0,0.1], I_app U[8,12], RK4 dt=0.01 ms, {args.horizon} steps")
            self.kernel = "k_csr_gather + k_csr_update"
            self.prof = ("csr_hh_1e6_deg100.md", "k_csr_gather|k_csr_update", ["csr.hip", "nd_dev.h", "runtime.hip"])
            from paper_2410_19075_amd import inputs
            self.graph = inputs.random_out_graph(1, self.n, 100)
            self.iapp = inputs.hh_iapp(1, self.n)

    def kernel_form(self, cfg):
        """Ball workloads: the plane-scatter form runs where the configuration's
        workgroup is 512 threads."""
        if self.a.workload == "ball" and cfg.get("block") == 512:
            self.kernel = "k_ball_scatter<inertia>"
            self.prof = (f"ball_scatter_inertia_{self.n1}cubed_p{self.a.radius}.md", "k_ball_scatter",
                         ["ball.hip", "models.h", "nd_dev.h", "runtime.hip"])

    def problem(self, prec):
        nd, w = self.nd, self.a.workload
        if w == "fhn":
            return nd.problem(nd.ND_FHN, nd.ND_RING, self.n, FHN_PRM, precision=prec, radius=self.P)
        if w == "kuramoto":
            return nd.problem(nd.ND_KURAMOTO, nd.ND_RING, self.n, [0.0, 1.0, 1.46], precision=prec, radius=self.P)
        if w == "cube":
            return nd.problem(nd.ND_KURAMOTO, nd.ND_CUBE3D, self.n, [0.0, 1.0, 0.8], precision=prec, radius=4,
                              dims=(self.n1,) * 3)
        if w == "inertia":
            return nd.problem(nd.ND_KURAMOTO_INERTIA, nd.ND_CUBE3D, self.n, INERTIA_PRM, precision=prec, radius=2,
                              dims=(self.n1,) * 3)
        if w == "ball":
            return nd.problem(nd.ND_KURAMOTO_INERTIA, nd.ND_BALL3D, self.n, INERTIA_PRM, precision=prec,
                              radius=self.P, dims=(self.n1,) * 3)
        if w == "links":
            return nd.problem(nd.ND_KURAMOTO_INERTIA, nd.ND_LINKS, self.n, INERTIA_PRM, precision=prec,
                              row_ptr=self.rows[0], col=self.rows[1])
        rp, col, wt = self.graph
        return nd.problem(nd.ND_HH, nd.ND_CSR, self.n, HH_PRM, precision=prec, row_ptr=rp, col=col, weight=wt,
                          per_elem=self.iapp)

    def state(self, b):
        from paper_2410_19075_amd import inputs
        w = self.a.workload
        if w == "fhn":
            return inputs.fhn_circle(1000 + b, self.n)
        if w == "kuramoto":
            return inputs.kuramoto_phases(1000 + b, self.n)
        if w == "cube":
            return inputs.cube_phases_with_patch(1000 + b, self.n1)
        if w in ("inertia", "ball", "links"):
            return np.concatenate([inputs.cube_phases_with_patch(1000 + b, self.n1), np.zeros(self.n)])
        return inputs.hh_state(1000 + b, self.n)

    def bytes_alg_per_elem_step(self, prec):
        """13 state-vector accesses per element and RK4 step (no scratch): y read
        4x, acc written and read, y written (doubles), k1..k3 written and read
        once each (bulk type); the CSR path adds its edge stream (col + w) once
        per stage."""
        kb = 8 if prec == 0 else 4
        b = self.nvars * (7 * 8 + 6 * kb)
        if self.a.workload == "hh":
            b += 4 * self.links * (4 + kb)
        if self.a.workload == "links":
            # per stage: the row's table index, and the exchanged map (cos, sin)
            # written once and read once (its gathers by the neighbours hit cache)
            b += 4 * (4 + 2 * (16 if prec == 0 else 8))
        return b


def run(nd, torch, wl, args, prec, stream):
    hs = []
    for b in range(args.batch):
        h = nd.nd_create(wl.problem(prec))
        if args.tile or args.grid or args.chunk or args.tile_y or args.tile_z or args.block:
            c = nd.nd_get_config(h)
            c.tile = args.tile or c.tile
            c.tile_y = args.tile_y or c.tile_y
            c.tile_z = args.tile_z or c.tile_z
            c.grid = args.grid or c.grid
            c.chunk = args.chunk or c.chunk
            c.block = args.block or c.block
            nd.nd_set_config(h, c)
        y0 = torch.from_numpy(wl.state(b)).cuda()
        nd.nd_set_state(h, y0, stream=stream)
        hs.append(h)
    torch.cuda.synchronize()
    dts = [args.dt] * len(hs)
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
    y = torch.empty(wl.nvars * wl.n, dtype=torch.float64, device="cuda")
    nd.nd_get_state(hs[0], y, stream=stream)
    torch.cuda.synchronize()
    finite = bool(torch.isfinite(y).all().item())
    cfg = nd.nd_get_config(hs[0])
    cfgd = {k: getattr(cfg, k) for k, _ in cfg._fields_}
    for h in hs:
        nd.nd_destroy(h)
    return wall, times, ev_total, finite, cfgd


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, args):
    """The FP64 oracle on a bounded sample of the same workload, on the host cores."""
    from oracle import oracle as O
    O.lib()
    y0 = wl.state(0)
    w = args.workload
    if w == "fhn":
        net, steps, what = O.ring(O.FHN, wl.n, wl.P, FHN_PRM), args.cpu_sample_steps, f"one FHN ring N={wl.n} P={wl.P}"
    elif w == "kuramoto":
        net, steps, what = O.ring(O.KURAMOTO, wl.n, wl.P, [0.0, 1.0, 1.46]), 200, f"one Kuramoto ring N={wl.n}"
    elif w == "cube":
        net, steps, what = O.cube(wl.n1, 4, [0.0, 1.0, 0.8]), 1, f"the {wl.n1}^3 lattice, h=4"
    elif w == "inertia":
        net, steps, what = (O.cube(wl.n1, 2, INERTIA_PRM, model=O.INERTIA), 2,
                            f"the {wl.n1}^3 lattice with inertia, h=2")
    elif w == "ball":
        net, steps, what = (O.ball(wl.n1, wl.P, INERTIA_PRM, model=O.INERTIA), 1,
                            f"the {wl.n1}^3 lattice with inertia, ball radius {wl.P}")
    elif w == "links":
        net, steps, what = (O.links(O.INERTIA, wl.n, wl.rows[0], wl.rows[1], np.array(INERTIA_PRM)), 20,
                            f"the {wl.n1}^3 lattice with inertia, ball radius {wl.P} as row lists")
    else:
        rp, col, wt = wl.graph
        net, steps, what = O.csr(wl.n, rp, col, wt, HH_PRM, wl.iapp), args.cpu_sample_steps, f"HH N={wl.n} deg 100"
    t0 = time.perf_counter()
    O.run(net, y0, args.dt, steps)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": wl.n * steps / dt, "unit": "oscillator-steps/s", "cores": cores, "kind": "oracle",
            "cpu": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"{what}, {steps} RK4 step(s), FP64, direct neighbour sums, {dt:.2f} s"}


def roofline(wl, args, prec, ev_total, cfg):
    """Algorithmic bytes of one stage launch over the measured average stage time
    (HIP events on the launch stream; the chunk's few small bookkeeping kernels
    are included, so the stage time is an upper bound).  `traffic` is the HBM
    bytes per launch from the committed rocprofv3 counter summary, when that was
    taken on the current kernel sources (else null)."""
    from paper_2410_19075_amd import profsum
    if args.workload == "kuramoto" and cfg["tile"] < 0:
        # rings resident in one workgroup for a whole chunk: no HBM traffic
        # between stages, so the bound is the FP64 ALU rate
        launches = args.steps * -(-args.horizon // max(1, cfg["chunk"]))
        flops = args.batch * wl.n * args.horizon * args.steps * KURAMOTO_RESIDENT_FLOPS
        achieved = flops / ev_total / 1e12
        return {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None, "kernel": wl.kernel,
                "flops_per_launch": flops / launches, "avg_launch_us": ev_total / launches * 1e6}
    n_stage = 4 * args.horizon * args.steps
    stage_s = ev_total / n_stage
    per_launch = args.batch * wl.n * wl.bytes_alg_per_elem_step(prec) / 4.0
    achieved = per_launch / stage_s / 1e9
    traffic = None
    if wl.prof:
        md, kf, files = wl.prof
        t = profsum.read_traffic(os.path.join(PROFILES, md), kf, "f64" if prec == 0 else "f32", files)
        # the summary's workload is the default one; other sizes scale with the elements
        default_shape = (args.batch == DEFAULTS[args.workload][0] and wl.n == DEFAULTS_N[args.workload]
                         and not (args.tile or args.tile_y or args.tile_z or args.grid or args.chunk or args.block))
        if t is not None and default_shape:
            traffic = t
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": wl.kernel,
            "bytes_per_launch": per_launch, "avg_launch_us": stage_s * 1e6}


LDS_PEAK_GBS = 256 * 128 * 2.4  # 256 CUs x 128 bytes per clock x 2.4 GHz


def ball_prefix_reads(P, n1, n3, cfg):
    """16-byte prefix reads of one ball stage launch over an n1 x n1 x n3 lattice.
    Gather form: every output reads two prefix values per (dy, dz) run of the
    ball.  Plane-scatter form (block 512): per mapped plane every output thread
    reads two values per (|dz|, dy) run pair whose two output planes include one
    of its work item's outputs (the pair serves dz and -dz)."""
    rz = [int(np.floor(np.sqrt(P * P - a * a) + 1e-9)) for a in range(P + 1)]
    if cfg.get("block") != 512:
        runs = sum(2 * rz[abs(dz)] + 1 for dz in range(-P, P + 1))
        return n1 * n1 * n3 * 2 * runs
    cx, cy, cz = cfg["tile"], cfg["tile_y"], cfg["tile_z"]
    per_thread = 0
    for z0 in range(0, n3, cz):
        nz = min(cz, n3 - z0)
        for q in range(nz + 2 * P):
            for a in range(P + 1):
                o1, o2 = q - P - a, q - P + a
                if 0 <= o1 < nz or (a > 0 and 0 <= o2 < nz):
                    per_thread += 2 * (2 * rz[a] + 1)
    return n1 * n1 * per_thread  # every xy column is one output thread of one tile


def lds_roofline(wl, args, ev_total, cfg):
    """The ball kernel's prefix reads against the LDS bandwidth (16 bytes each)."""
    reads = args.batch * ball_prefix_reads(args.radius, wl.n1, wl.n1, cfg)
    per_launch = reads * 16
    stage_s = ev_total / (4 * args.horizon * args.steps)
    achieved = per_launch / stage_s / 1e9
    return {"bound": "lds", "achieved": achieved, "peak": LDS_PEAK_GBS, "unit": "GB/s", "frac": achieved / LDS_PEAK_GBS,
            "bytes_per_launch": per_launch, "reads_per_output": reads / (args.batch * wl.n)}


# ------------------------------------------------------------------- serving
def serve_requests(args):
    """The request stream: model, N, P, alpha, horizon, seed and arrival gap per request."""
    from paper_2410_19075_amd import inputs
    m = args.batch
    u = inputs.uniform(77, inputs.TAG_MISC, 6 * m).reshape(6, m)
    reqs = []
    for i in range(m):
        model = "kur" if u[0, i] < 0.5 else "fhn"
        n = int(2 ** (10 + 12 * u[1, i]))
        P = max(1, int(n * (0.05 + 0.35 * u[2, i])))
        P = min(P, (n - 1) // 2)
        alpha = 1.3 + 0.25 * u[3, i]
        steps = int(10 ** (math.log10(args.hmin) + (math.log10(args.hmax) - math.log10(args.hmin)) * u[4, i]))
        reqs.append(dict(model=model, n=n, P=P, alpha=alpha, steps=steps, seed=5000 + i, gap=-math.log(1 - u[5, i])))
    return reqs


SERVE_R_EVERY = 10  # R recorded every 10 steps for the FP32-bulk statistics


def serve_run(nd, torch, args, reqs, states, prec, rate, stream):
    """Feed the requests at their arrival times (rate = requests per second) and pump
    the server until all are done; returns per-request latencies, chunk times,
    makespan and the results (final state and R every SERVE_R_EVERY steps)."""
    s = nd.nd_server_create(int(args.budget_gb * 2 ** 30), max_slots=256, chunk_steps=64)
    obs = nd.observe(SERVE_R_EVERY, -1)
    try:
        arrivals, t = [], 0.0
        for r in reqs:
            t += r["gap"] / rate
            arrivals.append(t)
        ids = [None] * len(reqs)
        chunk_ms = []
        i = 0
        t0 = nd.nd_server_now(s)
        pending = 0
        last_note = time.perf_counter()
        while i < len(reqs) or pending:
            if time.perf_counter() - last_note > 15.0:  # progress for long streams
                last_note = time.perf_counter()
                st_ = nd.nd_server_stats(s)
                print(f"serve: {st_.completed}/{len(reqs)} done, {st_.running} running, {st_.queued} queued, "
                      f"t={nd.nd_server_now(s) - t0:.0f} s", file=sys.stderr, flush=True)
            now = nd.nd_server_now(s) - t0
            while i < len(reqs) and arrivals[i] <= now:
                r = reqs[i]
                if r["model"] == "kur":
                    p = nd.problem(nd.ND_KURAMOTO, nd.ND_RING, r["n"], [0.0, 1.0, r["alpha"]], precision=prec,
                                   radius=r["P"])
                else:
                    p = nd.problem(nd.ND_FHN, nd.ND_RING, r["n"], FHN_PRM, precision=prec, radius=r["P"])
                ids[i] = nd.nd_server_submit(s, p, states[i], 0.01, r["steps"], obs, arrival=t0 + arrivals[i])
                i += 1
            if pending == 0 and i < len(reqs) and nd.nd_server_stats(s).queued == 0:
                time.sleep(max(0.0, min(0.05, arrivals[i] - now)))
            a = time.perf_counter()
            pending = nd.nd_server_pump(s, stream)
            if nd.nd_server_stats(s).running or pending:
                chunk_ms.append(1e3 * (time.perf_counter() - a))
        makespan = nd.nd_server_now(s) - t0
        lat, results = [], []
        for rid, r, st in zip(ids, reqs, states):
            info = nd.nd_server_info(s, rid)
            assert info.state == nd.ND_REQ_DONE, (r, info.state, info.status)
            lat.append(info.finished - info.arrival)
            y = np.empty_like(st)
            R = np.empty(r["steps"] // SERVE_R_EVERY + 1)
            nd.nd_server_result(s, rid, y, R)
            results.append((y, R))
        stats = nd.nd_server_stats(s)
        return dict(lat=lat, chunk_ms=chunk_ms, makespan=makespan, results=results, osc=stats.osc_steps,
                    gpu_s=stats.gpu_seconds, active_s=stats.active_seconds)
    finally:
        nd.nd_server_destroy(s)


def main_serve(nd, torch, args, stream):
    from paper_2410_19075_amd import inputs
    reqs = serve_requests(args)
    states = [inputs.kuramoto_phases(r["seed"], r["n"]) if r["model"] == "kur" else inputs.fhn_circle(r["seed"], r["n"])
              for r in reqs]
    work = sum(r["n"] * r["steps"] for r in reqs)
    # capacity probe: the first --probe requests submitted at once (closed loop), FP64
    k = min(args.probe, len(reqs))
    probe = serve_run(nd, torch, args, reqs[:k], states[:k], nd.ND_FP64, 1e9, stream)
    capacity = sum(r["n"] * r["steps"] for r in reqs[:k]) / probe["makespan"]
    rate = args.rho * capacity / (work / len(reqs))
    out = {"metric": "oscillator-steps/s", "unit": "oscillator-steps/s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"serving: {len(reqs)} Poisson requests (50/50 Kuramoto/FHN rings, N log-uniform "
                                  f"2^10..2^22, P/N U[0.05,0.4], alpha U[1.3,1.55], horizons log-uniform "
                                  f"[{args.hmin:g}, {args.hmax:g}] RK4 steps, dt=0.01), offered load "
                                  f"rho={args.rho} of the capacity measured on the first {min(args.probe, len(reqs))} "
                                  f"requests in closed loop, HBM budget {args.budget_gb} GB, chunks of 64 steps, "
                                  f"R recorded every {SERVE_R_EVERY} steps"},
           "capacity_osc_steps_per_s": capacity}
    ref = None
    for prec, key in ((nd.ND_FP64, "fp64"), (nd.ND_FP32_BULK, "fp32_bulk")):
        r = serve_run(nd, torch, args, reqs, states, prec, rate, stream)
        lat = np.array(r["lat"]) * 1e3
        rec = {"value": work / r["makespan"], "latency_ms": {"p50": float(np.percentile(lat, 50)),
                                                           "p99": float(np.percentile(lat, 99))},
               "chunk_ms": {"p50": float(np.percentile(r["chunk_ms"], 50)),
                            "p99": float(np.percentile(r["chunk_ms"], 99))},
               "makespan_s": r["makespan"], "gpu_busy_frac": r["gpu_s"] / r["makespan"],
               "gpu_busy_frac_while_active": r["gpu_s"] / max(r["active_s"], 1e-9)}
        if key == "fp64":
            ref = r["results"]
            out["value"] = rec["value"]
            out["ms_per_step"] = 1e3 * r["makespan"]
            out.update({"latency_ms": rec["latency_ms"], "batch_latency_ms": rec["chunk_ms"],
                        "makespan_s": rec["makespan_s"], "gpu_busy_frac": rec["gpu_busy_frac"],
                        "gpu_busy_frac_while_active": rec["gpu_busy_frac_while_active"]})
        else:
            # horizons reach 10^5 steps, past the point where chaotic trajectories
            # decorrelate, so the FP32-bulk results are judged on statistics: the
            # second-half mean of R (recorded every SERVE_R_EVERY steps) against the
            # FP64 run of the same request; the pointwise state error is reported too
            errs, dR = [], []
            for (y, R), (yr, Rr), q in zip(r["results"], ref, reqs):
                nv = 1 if q["model"] == "kur" else 2
                a, b = y.reshape(nv, -1), yr.reshape(nv, -1)
                errs.append(max(float(np.max(np.abs(a[v] - b[v])) / np.max(np.abs(b[v]))) for v in range(nv)))
                h = len(R) // 2
                dR.append(abs(float(R[h:].mean() - Rr[h:].mean())))
            rec["max_mean_R_gap_vs_fp64"] = max(dR)
            rec["p99_mean_R_gap_vs_fp64"] = float(np.percentile(dR, 99))
            rec["max_normwise_state_error_vs_fp64"] = max(errs)
            # the FP64 floor of the requests whose gap exceeds 1e-3: the same request
            # in FP64 from its initial state with one element moved by one ulp
            over = sorted((i for i in range(len(reqs)) if dR[i] > 1e-3), key=lambda i: -dR[i])
            floors = []
            for i in over[:args.floor_checks]:
                print(f"serve: FP64 floor of request {i} (gap {dR[i]:.2e})", file=sys.stderr, flush=True)
                q, y0 = reqs[i], states[i].copy()
                y0[3] = np.nextafter(y0[3], np.inf)
                if q["model"] == "kur":
                    p = nd.problem(nd.ND_KURAMOTO, nd.ND_RING, q["n"], [0.0, 1.0, q["alpha"]], radius=q["P"])
                else:
                    p = nd.problem(nd.ND_FHN, nd.ND_RING, q["n"], FHN_PRM, radius=q["P"])
                _, Rp, _ = nd.simulate(p, y0, 0.01, q["steps"], record_every=SERVE_R_EVERY)
                Rr = ref[i][1]
                h = len(Rr) // 2
                floor = abs(float(Rp[h:].mean() - Rr[h:].mean()))
                # and with every element moved by 1e-7 relative (FP32's rounding scale)
                sgn = np.where(inputs.uniform(900 + i, inputs.TAG_MISC, states[i].size) < 0.5, -1.0, 1.0)
                _, Rq, _ = nd.simulate(p, states[i] * (1.0 + 1e-7 * sgn), 0.01, q["steps"],
                                       record_every=SERVE_R_EVERY)
                floor32 = abs(float(Rq[h:].mean() - Rr[h:].mean()))
                floors.append({"request": i, "model": q["model"], "n": q["n"], "P": q["P"], "steps": q["steps"],
                               "fp32_gap": dR[i], "fp64_floor_1ulp": floor, "fp64_floor_1e-7": floor32,
                               "within_1ulp_floor": dR[i] <= max(1e-3, 2 * floor),
                               "within_1e-7_floor": dR[i] <= max(1e-3, 2 * floor32)})
            rec["requests_over_1e-3"] = len(over)
            rec["floor_checks"] = floors
            out["fp32_bulk"] = rec
    print(json.dumps(out), flush=True)


def main_adaptive(nd, torch, args, stream):
    """One call integrates every ring to t_end with its own step control."""
    from paper_2410_19075_amd import inputs
    n, rtol, atol = args.n, 1e-8, 1e-10
    tiled = n > 1024 or args.workload == "adaptive3d"
    if args.workload == "adaptive3d":  # the paper's 3D inertia state as a compressed coupling matrix
        n1 = args.n
        n = n1 ** 3
        rows = inputs.lattice_ball_links(n1, n1, n1, 2)
        P, t_end, prm, model, rtol, atol = 2, 50.0, INERTIA_PRM, nd.ND_KURAMOTO_INERTIA, 1e-6, 1e-8
        state = lambda b: np.concatenate([inputs.cube_phases_with_patch(1000 + b, n1), np.zeros(n)])
        nv = 2
    elif tiled:  # the FHN ring of the default workload, on the tiled path
        P, t_end, prm, model = int(0.35 * n), 10.0, FHN_PRM, nd.ND_FHN
        state = lambda b: inputs.fhn_circle(1000 + b, n)
        nv = 2
    else:
        P, t_end, prm, model = n // 4, 100.0, [0.0, 1.0, 1.46], nd.ND_KURAMOTO
        state = lambda b: inputs.kuramoto_phases(1000 + b, n)
        nv = 1
    if args.workload == "adaptive3d":
        hs = [nd.nd_create(nd.problem(model, nd.ND_LINKS, n, prm, row_ptr=rows[0], col=rows[1]))
              for _ in range(args.batch)]
    else:
        hs = [nd.nd_create(nd.problem(model, nd.ND_RING, n, prm, radius=P)) for _ in range(args.batch)]
    y0s = [torch.from_numpy(state(b)).cuda() for b in range(args.batch)]

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    Rs = []

    def one():
        for h, y0 in zip(hs, y0s):
            nd.nd_set_state(h, y0, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        if args.workload == "adaptive3d":  # with R at every time unit from the dense output
            st, Rout, _ = nd.nd_run_adaptive_dense(hs, [t_end] * len(hs), [1e-3] * len(hs), rtol, atol, 1.0,
                                                   stream=stream)
            Rs.append(Rout[0])
        else:
            st = nd.nd_run_adaptive(hs, [t_end] * len(hs), [1e-3] * len(hs), rtol, atol, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, ev0.elapsed_time(ev1) / 1e3, st

    for _ in range(args.warmup):
        one()
    times, ev_total, acc, rej = [], 0.0, 0, 0
    for _ in range(args.steps):
        dt_s, ev_s, st = one()
        times.append(dt_s)
        ev_total += ev_s
        acc += sum(s.accepted for s in st)
        rej += sum(s.rejected for s in st)
    wall = sum(times)
    value = acc * n / wall
    if tiled:
        # algorithmic bytes per element and accepted step: stage s (1..6) reads y and
        # k_1..k_s and writes k_{s+1}; the fifth-order solution is written once
        bpe = (sum(s + 2 for s in range(1, 7)) + 1) * 8 * nv
        if args.workload == "adaptive3d":
            bpe += 6 * (4 + 2 * 16)  # per stage: the row's table index, the exchanged map written and read
        achieved = acc * n * bpe / ev_total / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "kernel": "k_dt_map + k_dt_rhs + k_dt_control" + (" + k_dt_emit" if args.workload == "adaptive3d" else ""),
                "bytes_per_element_step": bpe}
        what = f"{args.batch} FitzHugh-Nagumo rings N={n} P={P} (0.35N), eps=0.05 a=0.5 sigma=0.1 phi=pi/2-0.1"
        if args.workload == "adaptive3d":
            what = (f"Kuramoto-Sakaguchi with inertia, 3D lattice {args.n}^3 periodic, ball of radius 2 (33 links) "
                    f"as a compressed coupling matrix, m=1 eps=0.05 mu=0.01 alpha=0.45, planted coherent ball, psi=0")
    else:
        # algorithmic FP64 flops per element and accepted step: 7 stages of the resident
        # kernel's per-stage work (KURAMOTO_RESIDENT_FLOPS / 4 each, sin/cos included)
        # plus the stage combinations (2 flops per coefficient, 27 + 7 coefficients)
        flops = acc * n * (7 * KURAMOTO_RESIDENT_FLOPS / 4 + 2 * 34)
        achieved = flops / ev_total / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None, "kernel": "k_ring_dopri<Kuramoto>"}
        what = f"{args.batch} Kuramoto rings N={n} P={P} alpha=1.46"
    roof["avg_launch_us"] = ev_total / args.steps * 1e6
    out = {"metric": "oscillator-steps/s", "value": value, "unit": "oscillator-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"Dormand-Prince 5(4), {what}, t=0..{t_end}, rtol={rtol} atol={atol}, "
                                  f"per-network step control",
                      "global_batch": args.batch, "parallelism": "single-gpu"},
           "accepted_steps": acc, "rejected_steps": rej, "roofline": roof}
    if Rs:
        out["R_every_10_time_units"] = [float(x) for x in Rs[-1][::10]]
    for h in hs:
        nd.nd_destroy(h)
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        O.lib()
        y0 = state(0)
        # a bounded sample: the Kuramoto ring to t_end, the large FHN ring to t = 0.01,
        # the lattice to t = 1
        ts = t_end if not tiled else 0.01
        net = O.ring(O.FHN if tiled else O.KURAMOTO, n, P, prm) if args.workload != "adaptive3d" else None
        if args.workload == "adaptive3d":
            ts, net = 1.0, O.links(O.INERTIA, n, rows[0], rows[1], np.array(prm))
        t0 = time.perf_counter()
        _, _, oacc, orej, _ = O.run_dopri(net, y0, ts, rtol, atol, 1e-3)
        sec = time.perf_counter() - t0
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        out["cpu_baseline"] = {"value": oacc * n / sec, "unit": "oscillator-steps/s", "cores": cores,
                               "kind": "oracle", "cpu": cpu_model(), "nproc": os.cpu_count(),
                               "sample": f"one network of {n} elements, Dormand-Prince 5(4) to t={ts}, "
                                         f"{oacc} accepted / {orej} rejected steps, FP64, {sec:.2f} s"}
    print(json.dumps(out), flush=True)


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
        dst.copy_(src)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(3):
            dst.copy_(src)
        ev1.record(stream)
        torch.cuda.synchronize()
        sec = ev0.elapsed_time(ev1) / 1e3 / 3
        print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 4, "copy_GBps": 2 * nbytes / sec / 1e9}))
        return
    if args.workload == "serve":
        main_serve(nd, torch, args, stream)
        return
    if args.workload in ("adaptive", "adaptive3d"):
        main_adaptive(nd, torch, args, stream)
        return
    wl = Workload(args, nd)
    osc_per_step = args.batch * wl.n * args.horizon
    wall, times, ev_total, finite, cfg = run(nd, torch, wl, args, nd.ND_FP64, stream)
    wl.kernel_form(cfg)
    value = osc_per_step * args.steps / wall
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
        "config": {"workload": wl.name, "global_batch": args.batch, "seq_len": args.horizon,
                   "parallelism": "single-gpu", "kernel_config": cfg},
        "coupling_terms_per_s": value * wl.links * 4,
        "batch_latency_ms": {"p50": 1e3 * float(np.percentile(times, 50)),
                             "p99": 1e3 * float(np.percentile(times, 99))},
        "state_finite": finite,
        "roofline": roofline(wl, args, 0, ev_total, cfg),
    }
    if args.workload == "ball":
        out["lds_roofline"] = lds_roofline(wl, args, ev_total, cfg)
    if not args.no_fp32:
        wall32, times32, ev32, fin32, cfg32 = run(nd, torch, wl, args, nd.ND_FP32_BULK, stream)
        v32 = osc_per_step * args.steps / wall32
        out["fp32_bulk"] = {"value": v32, "unit": "oscillator-steps/s", "ms_per_step": 1e3 * wall32 / args.steps,
                            "coupling_terms_per_s": v32 * wl.links * 4,
                            "roofline": roofline(wl, args, 1, ev32, cfg32), "state_finite": fin32}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
