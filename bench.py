"""Benchmark: 3D acoustic finite-difference time stepping on one MI355X.

Workload: the 512^3 physical grid (h = 10 m) with a 40-point damping layer
(592^3 = 207.5 M points updated per step), two-layer velocity 1.5 / 3.5 km/s
with a smooth +-5 % perturbation, 10 Hz Ricker point source, 512 x 512
surface receivers, swept over space orders 4, 8, 12 and 16.

A step is one time step of the whole path for one order: the stencil update
with damping, the source injection and the receiver sampling.  Each order runs
``--warmup`` untimed steps and then ``--steps`` timed steps (inputs resident
in HBM, timed with events on the launch stream between two synchronisations).
A zero-step call first uploads the point tables; then, before the warm-up
steps, the full step runs untimed for 60 ms of wall time (`settle`): host
work that leaves the GPU idle for milliseconds (a problem's setup, building
the point tables of 262,144 receivers) makes the next ~25 launches run 4-10 %
slower while the GPU leaves its idle state.

Printed (one JSON line): value = Gpt/s over the sweep (total point updates /
total time), the per-order figures, the roofline of the stencil kernel
(algorithmic 16 bytes per point update / the kernel's average launch time,
measured in a second timed loop that launches only the stencil), the STREAM
triad bandwidth measured the same way (the practical ceiling of section 3.1),
and the FP64 CPU oracle timed on a bounded sample of the same workload.
`roofline.traffic` is the calibrated HBM traffic per launch from the committed
rocprofv3 counter summary, reported only while the kernel source is unchanged.

`--profile-pass` is the driver for counter collection: it launches 3 triads of
2^26 floats and then 3 stencil-only steps per order, and prints nothing else.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFLOPS = 78.6        # MI355X FP32 vector arithmetic without packed instructions
TRAFFIC_SUMMARY = ROOT / "profiles" / "acoustic3d_tiled_592cubed_traffic.md"
KERNEL_SOURCES = [ROOT / "paper_1608_03984_amd" / "csrc" / f
                  for f in ("fd_acoustic_tiled.h", "fd_acoustic.hip", "fd_acoustic_hi.hip",
                            "fd_acoustic_top.hip")]
BYTES_PER_POINT = 16           # read u^n, u^{n-1}, dt^2 v^2; write u^{n+1}
ORDERS = (4, 8, 12, 16)


def paper_flops(so: int) -> int:
    """FLOPs per point update of the acoustic stencil, 6k + 4 with k = so + 1
    points per 1D stencil (Table 1)."""
    return 6 * (so + 1) + 4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--orders", type=str, default=",".join(map(str, ORDERS)))
    ap.add_argument("--phys", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--profile-pass", action="store_true")
    ap.add_argument("--workload",
                    choices=("acoustic", "2d", "tti", "vti", "gradient", "fwi", "shots", "cost",
                             "learned"),
                    default="acoustic")
    ap.add_argument("--interval", type=int, default=0)
    ap.add_argument("--group", type=int, default=4)
    ap.add_argument("--fwi-steps", type=int, default=1200)
    ap.add_argument("--models", type=int, default=200)
    ap.add_argument("--windows", type=int, default=4)
    ap.add_argument("--iters", type=int, default=3000)
    return ap.parse_args()


def kernel_source_hash() -> str:
    """sha256[:16] of the acoustic kernel's sources, concatenated in order,
    followed by the per-source compiler flags they are built with (the
    path-free additions of the build script)."""
    from paper_1608_03984_amd import _build

    h = hashlib.sha256(b"".join(f.read_bytes() for f in KERNEL_SOURCES))
    h.update(repr([_build.EXTRA.get(f.name, []) for f in KERNEL_SOURCES]).encode())
    return h.hexdigest()[:16]


# (waves per block, rows per lane) of the tiled acoustic kernel's tile
# configurations, as FD_OPT_TILE numbers them
ACOUSTIC_TILES = {0: (4, 2), 1: (4, 4), 2: (8, 1), 3: (8, 2), 4: (12, 2)}


def committed_traffic(phys: int):
    """Per-order (kernel, HBM bytes per launch) from the committed counter
    summary, or None when the summary is missing, for another size, or older
    than the kernel source."""
    if phys != 512 or not TRAFFIC_SUMMARY.exists():
        return None
    m = re.search(r"<!-- machine-readable: (.*) -->", TRAFFIC_SUMMARY.read_text())
    if not m:
        return None
    data = json.loads(m.group(1))
    if data["source_sha256_16"] != kernel_source_hash():
        return None
    return {int(k): (v["kernel"], v["traffic_bytes"]) for k, v in data["per_order"].items()}


def traffic_of(traffic, so: int, tile: int):
    """The committed bytes of order so if they were counted for the kernel
    the context launches (radius, waves, rows of its tile, one shot), else
    None."""
    if not traffic or so not in traffic or tile not in ACOUSTIC_TILES:
        return None
    kernel, nbytes = traffic[so]
    nw, vy = ACOUSTIC_TILES[tile]
    return nbytes if kernel.startswith(f"acoustic3d_tiled<{so // 2}, {nw}, {vy}, 1,") else None


TRIAD_SWEEP = [(u, b, f) for f in (0, 1) for u in (1, 2, 4, 8) for b in (0, 2048, 4096, 8192)]


def triad_gbs(torch, P):
    """STREAM-style triad bandwidth (2^28 floats per array, 3 GiB moved per
    launch), events on the launch stream: the best of a sweep over the
    triad's unroll depth, grid and load kind (fd_triad_config).  Returns
    (GB/s, {"unroll", "blocks", "temporal", "default_gbs"}) or (None, None)
    when a result is wrong."""
    n = 1 << 28
    dev = torch.device("cuda:0")
    a = torch.empty(n, device=dev)
    b = torch.ones(n, device=dev)
    c = torch.ones(n, device=dev)
    st = torch.cuda.current_stream().cuda_stream
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    ptrs = (a.data_ptr(), b.data_ptr(), c.data_ptr())
    best, cfg = 0.0, None
    for u, blocks, flags in TRIAD_SWEEP:
        P.fd_triad_config(*ptrs, 2.0, n, u, blocks, flags, st)
        t = timed(lambda: [P.fd_triad_config(*ptrs, 2.0, n, u, blocks, flags, st)
                           for _ in range(10)], ev) / 10
        gbs = 12 * n / t / 1e9
        if gbs > best:
            best, cfg = gbs, {"unroll": u, "blocks": blocks, "temporal": bool(flags)}
    P.fd_triad(*ptrs, 2.0, n, st)
    t = timed(lambda: [P.fd_triad(*ptrs, 2.0, n, st) for _ in range(10)], ev) / 10
    cfg["default_gbs"] = round(12 * n / t / 1e9, 1)
    a.zero_()
    P.fd_triad(*ptrs, 2.0, n, st)
    ok = bool((a == 3.0).all().item())
    del a, b, c
    torch.cuda.empty_cache()
    return (best, cfg) if ok else (None, None)


def profile_pass(args):
    import torch

    import paper_1608_03984_amd as P
    from paper_1608_03984_amd.solver import Solver
    from workloads import DT, acoustic_3d

    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    n = 1 << 26
    a = torch.empty(n, device=dev)
    b = torch.ones(n, device=dev)
    c = torch.ones(n, device=dev)
    for _ in range(3):
        P.fd_triad(a.data_ptr(), b.data_ptr(), c.data_ptr(), 2.0, n, st)
    torch.cuda.synchronize()
    del a, b, c
    prob = acoustic_3d(so=8, phys=args.phys, nbl=40, nt=1, receivers="none")
    for so in [int(x) for x in args.orders.split(",")]:
        s = Solver(3, prob.shape, prob.spacing, prob.nbl, so, DT[("acoustic_3d", so)], prob.vel,
                   prob.eta, max_points=4, device=dev)
        s.forward(3, zero_state=False)
        torch.cuda.synchronize()
        print(f"# profile pass so{so} done", file=sys.stderr, flush=True)
        s.close()
        del s
        torch.cuda.empty_cache()


def settle(step, seconds: float = 0.06):
    """Untimed GPU work after a problem's setup and point upload: `step` (a
    few steps) repeated, with a synchronisation after each, for `seconds` of
    wall time, so that the warm-up and timed steps that follow run at the
    GPU's working clocks (after milliseconds of host work with the GPU idle
    the next ~25 stencil launches run 4-10 % slower)."""
    import torch

    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        step()
        torch.cuda.synchronize()


def timed(fn, stream_events):
    import torch

    start, end = stream_events
    torch.cuda.synchronize()
    start.record()
    fn()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / 1e3


def cpu_baseline(problem, seconds: float):
    """The FP64 oracle on a z-slab of the workload (full x-y extent)."""
    import oracle

    threads = max(1, min(os.cpu_count() or 1, 16))
    oracle.set_threads(threads)
    p = problem
    slab = 48
    vel = np.ascontiguousarray(p.vel[:slab])
    eta = np.ascontiguousarray(p.eta[:slab])
    pts = vel.size
    rates = {}
    t_total = 0.0
    budget = seconds / len(ORDERS)
    for so in ORDERS:
        from workloads import DT
        dt = DT[("acoustic_3d", so)]
        up = np.zeros(vel.shape)
        uc = np.zeros(vel.shape)
        uc[slab // 2, vel.shape[1] // 2, vel.shape[2] // 2] = 1.0
        steps = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget:
            _, up, uc = oracle.acoustic_forward(3, 0, p.spacing, dt, so, vel, eta, [],
                                                np.zeros((1, 0)), [], 1, up, uc)
            steps += 1
        el = time.perf_counter() - t0
        t_total += el
        rates[so] = pts * steps / el / 1e9
    # one thread, on the first 8 planes of the slab (about 0.5 s per order)
    oracle.set_threads(1)
    thin = 8
    rates1 = {}
    for so in ORDERS:
        from workloads import DT
        dt = DT[("acoustic_3d", so)]
        v1 = np.ascontiguousarray(vel[:thin])
        up = np.zeros(v1.shape)
        uc = np.zeros(v1.shape)
        uc[thin // 2, v1.shape[1] // 2, v1.shape[2] // 2] = 1.0
        steps = 0
        t0 = time.perf_counter()
        while steps < 1 or time.perf_counter() - t0 < 0.5:
            _, up, uc = oracle.acoustic_forward(3, 0, p.spacing, dt, so, v1,
                                                np.ascontiguousarray(eta[:thin]), [],
                                                np.zeros((1, 0)), [], 1, up, uc)
            steps += 1
        rates1[so] = v1.size * steps / (time.perf_counter() - t0) / 1e9
    agg = len(ORDERS) / sum(1.0 / r for r in rates.values())
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")),
                         None)
    except OSError:
        pass
    return {
        "value": round(agg, 5), "unit": "Gpt/s", "cores": threads, "kind": "oracle",
        "cpu_model": model, "host_cpus": os.cpu_count(),
        "sample": (f"FP64 oracle, {vel.shape[2]}x{vel.shape[1]}x{slab} slab of the workload, "
                   f"so 4/8/12/16, ~{seconds:.0f} s total; per order Gpt/s "
                   + ", ".join(f"so{k} {v:.4f}" for k, v in rates.items())),
        "single_thread_gpts": {f"so{k}": round(v, 5) for k, v in rates1.items()},
    }


def tti_bench(args, physics="tti"):
    """TTI pseudo-acoustic, 384^3 + 40-point layer (464^3), space order 8:
    60 algorithmic bytes and 964 paper FLOPs per point update (Table 1).
    With physics "vti": the same model without tilt, 36 bytes and
    2 (6k + 8) = 124 paper FLOPs per point update."""
    import torch

    from paper_1608_03984_amd.solver import Solver
    from workloads import tti_3d, vti_3d

    phys = 384 if args.phys == 512 else args.phys
    gen = tti_3d if physics == "tti" else vti_3d
    p = gen(so=8, phys=phys, nbl=40, nt=1, receivers="line")
    nbytes, nflops = (60, 964) if physics == "tti" else (36, 12 * 9 + 16)
    npts = p.npoints
    dev = torch.device("cuda:0")
    nt = args.warmup + args.steps
    from workloads import ricker
    wav = torch.from_numpy(ricker(10.0, p.dt, nt)[:, None]).to(dev)
    traces = torch.empty((nt, p.rec.shape[0]), dtype=torch.float32, device=dev)
    s = Solver(3, p.shape, p.spacing, p.nbl, 8, p.dt, p.vel, p.eta, physics=physics,
               epsilon=p.eps, delta=p.delta, theta=p.theta, phi=p.phi,
               max_points=1 + p.rec.shape[0], device=dev)
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    s.forward(0, p.src, wav[:0], p.rec)
    settle(lambda: s.forward(4, p.src, wav[:4], p.rec, zero_state=False, traces=traces[:4],
                             keep_points=True))
    s.forward(args.warmup, p.src, wav[:args.warmup], p.rec, traces=traces[:args.warmup],
              keep_points=True)
    tw = timed(lambda: s.forward(args.steps, p.src, wav[args.warmup:], p.rec, zero_state=False,
                                 traces=traces[args.warmup:], keep_points=True), ev)
    s.forward(args.warmup, zero_state=False)
    tk = timed(lambda: s.forward(args.steps, zero_state=False), ev)
    ok = bool(torch.isfinite(traces).all().item())
    s.close()
    kernel_s = tk / args.steps
    ach = nbytes * npts / kernel_s / 1e9
    name = physics.upper()
    line = {
        "metric": f"Gpt/s (3D {name} so8)", "value": round(npts * args.steps / tw / 1e9, 3),
        "unit": "Gpt/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(tw / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"3D {name}, {phys}^3 + 40-pt layer ({p.padded[0]}^3 points), "
                               "h=12.5 m, layered v, smooth eps/delta"
                               + ("/theta/phi" if physics == "tti" else "") + ", so 8",
                   "points": npts},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": f"{name} stencil ({nbytes} B per point update)"},
        "gflops_paper": round(nflops * npts / kernel_s / 1e9, 1),
        # the paper's FLOP count against the FP32 vector roofs (non-packed,
        # as built, and packed): above 1 means the kernel does less arithmetic
        # than the count (symmetric pairs summed first, first derivatives of
        # the mixed terms formed once and reused)
        "alu": {"flops_per_pt_paper": nflops,
                "tflops_paper": round(nflops * npts / kernel_s / 1e12, 2),
                "peak_fp32_tflops": FP32_PEAK_TFLOPS, "peak_packed_fp32_tflops": 157.3,
                "frac": round(nflops * npts / kernel_s / 1e12 / FP32_PEAK_TFLOPS, 4),
                "frac_packed": round(nflops * npts / kernel_s / 1e12 / 157.3, 4)},
        "stencil_ms": round(kernel_s * 1e3, 4), "finite": ok,
    }
    print(json.dumps(line), flush=True)


def acoustic2d_bench(args):
    """The 2D workload (201 x 201 physical + 20-point layer = 241^2 points, so
    4, 500 steps, one source, 101 receivers): cache-resident and bound by
    launches (three per step), so the 500-step loop is also captured once in
    a HIP graph and replayed; both rates are reported (no roofline: the
    0.9 MB of a step never leaves the caches)."""
    import torch

    from paper_1608_03984_amd.solver import Solver
    from workloads import acoustic_2d

    p = acoustic_2d()
    nt, nrec = p.nt, p.rec.shape[0]
    dev = torch.device("cuda:0")
    s = Solver(2, p.shape, p.spacing, p.nbl, p.so, p.dt, p.vel, p.eta, max_points=1 + nrec,
               device=dev)
    q = torch.from_numpy(p.wavelet.astype(np.float32)).to(dev)
    traces = torch.empty((nt, nrec), dtype=torch.float32, device=dev)
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

    def run():
        s.forward(nt, p.src, q, p.rec, traces=traces)

    run()
    reps = 20
    t_eager = timed(lambda: [run() for _ in range(reps)], ev) / reps
    ref = traces.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    g.replay()
    torch.cuda.synchronize()
    same = bool(torch.equal(traces, ref))
    t_graph = timed(lambda: [g.replay() for _ in range(reps)], ev) / reps
    torch.cuda.synchronize()
    same = same and bool(torch.equal(traces, ref))
    s.close()
    npts = p.npoints
    line = {
        "metric": "Gpt/s (2D acoustic so4)", "value": round(npts * nt / t_graph / 1e9, 3),
        "unit": "Gpt/s", "n_gpus": 1, "steps": nt, "warmup": 1,
        "ms_per_step": round(t_graph / nt * 1e3, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "2D isotropic acoustic, 201^2 + 20-pt layer (241^2 points), "
                               "h=10 m, v=1500 m/s, so 4, 500 steps, 15 Hz Ricker, 101 receivers",
                   "points": npts},
        "eager_gpts": round(npts * nt / t_eager / 1e9, 3),
        "graph_gpts": round(npts * nt / t_graph / 1e9, 3),
        "eager_us_per_step": round(t_eager / nt * 1e6, 2),
        "graph_us_per_step": round(t_graph / nt * 1e6, 2),
        "graph_traces_equal_eager": same,
    }
    print(json.dumps(line), flush=True)


def gradient_bytes(nt, I):
    """Algorithmic bytes per point of a checkpointed forward run plus its
    gradient (nt steps, checkpoint interval I): forward 16 per step (the last
    segment also stores its accelerations, 4 more); the other segments
    recomputed storing the accelerations, 20; adjoint steps 16 with the
    imaging term fused in, 12 more (acceleration and partial sum read, partial
    sum written), except one term per segment imaged by the separate kernel,
    16 (adjoint field read as well); 16 per flush of the partial sums into the
    total (every 32 terms)."""
    last = nt - (nt - 1) // I * I           # steps of the last segment (not recomputed)
    nseg = (nt + I - 1) // I
    flushes = (nt + 31) // 32
    return (16 * nt + 4 * last + 20 * (nt - last) + 16 * nt + 12 * (nt - nseg) + 16 * nseg
            + 16 * flushes)


def gradient_bench(args):
    """FWI gradient of the 3D acoustic workload (so 8, 592^3 points, 1 shot):
    checkpointed forward run of ``--steps`` steps, then the adjoint run with
    segment recomputation and the imaging condition (fused into the adjoint
    steps).  Algorithmic bytes: gradient_bytes()."""
    import torch

    from paper_1608_03984_amd.solver import Solver
    from workloads import DT, acoustic_3d, ricker

    so = 8
    p = acoustic_3d(so=so, phys=args.phys, nbl=40, nt=1, receivers="surface")
    npts = p.npoints
    dev = torch.device("cuda:0")
    dt = DT[("acoustic_3d", so)]
    s = Solver(3, p.shape, p.spacing, p.nbl, so, dt, p.vel, p.eta,
               max_points=1 + p.rec.shape[0], device=dev)
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

    def run(nt):
        wav = torch.from_numpy(ricker(10.0, dt, nt)[:, None]).to(dev)
        out = {}
        out["t_fwd"] = timed(lambda: out.__setitem__(
            "tr", s.forward_checkpointed(nt, p.src, wav, p.rec, interval=args.interval)), ev)
        adj = out["tr"] * 0.5  # trace sensitivities of a synthetic misfit
        out["t_grad"] = timed(lambda: out.__setitem__("g", s.gradient(adj, wrt="vel")), ev)
        out["finite"] = bool(torch.isfinite(out["g"][0]).all().item())
        out["interval"] = s.checkpoint_interval
        out["store_gb"] = s._ck["bytes"] / 1e9
        s._ck = None
        return out

    run(max(args.warmup, 4))
    torch.cuda.empty_cache()
    r = run(args.steps)
    nt = args.steps
    t_all = r["t_fwd"] + r["t_grad"]
    I = r["interval"]
    alg = npts * gradient_bytes(nt, I)
    ach = alg / t_all / 1e9
    s.close()
    line = {
        "metric": "FWI gradient Gpt/s (3D acoustic so8)", "value": round(npts * nt / t_all / 1e9, 3),
        "unit": "Gpt/s", "n_gpus": 1, "steps": nt, "warmup": args.warmup,
        "ms_per_step": round(t_all / nt * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"FWI gradient, 3D acoustic {args.phys}^3 + 40-pt layer "
                               f"({p.padded[0]}^3 points), so 8, 1 shot, {p.rec.shape[0]} "
                               "receivers", "points": npts, "interval": I,
                   "store_gb": round(r["store_gb"], 1)},
        "forward_s": round(r["t_fwd"], 4), "gradient_s": round(r["t_grad"], 4),
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "whole gradient (algorithmic bytes of every pass / wall time)"},
        "finite": r["finite"],
    }
    print(json.dumps(line), flush=True)


def fwi_bench(args):
    """FWI gradient of the 16-shot survey (256^3 + 40-point layer = 336^3
    points, h = 15 m, so 8, 1200 steps, one 8 Hz Ricker per shot on a 4 x 4
    grid at z = 30 m, 256 x 256 receivers).  Observed data: the true model,
    all 16 shots advanced in one launch per step.  Timed: for each shot, the
    checkpointed forward run in the smoothed start model, its residual and
    misfit (fd_misfit) and the gradient of J = 1/2 sum_shots |d - d_obs|^2
    with respect to v, summed over the shots into one buffer
    (FD_GRAD_ACCUMULATE).  Checked: central differences of J
    (16-shot launches) along the normalised gradient against <g, dir>.
    Algorithmic bytes per point and step as in the single-shot gradient."""
    import torch

    from paper_1608_03984_amd.solver import Solver
    from workloads import fwi_3d

    S, nt = 16, args.fwi_steps
    p = fwi_3d(so=8, phys=256 if args.phys == 512 else args.phys, nbl=40, nt=nt, nshots=S,
               receivers="surface")
    npts = p.npoints
    dev = torch.device("cuda:0")
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    srcs = [p.src[k:k + 1] for k in range(S)]
    wav = torch.from_numpy(p.wavelet.astype(np.float32)).to(dev)
    nrec = p.rec.shape[0]
    say = lambda m: print(m, file=sys.stderr, flush=True)

    def survey(vel):
        """Traces of all shots in `vel` (one launch per step for the 16 shots)."""
        sv = Solver(3, p.shape, p.spacing, p.nbl, p.so, p.dt, vel, p.eta, nshots=S,
                    max_points=S * (1 + nrec), device=dev)
        # per-shot traces are column blocks of one [nt][S nrec] array: made
        # contiguous for fd_misfit
        tr = [t.contiguous() for t in sv.forward_shots(nt, srcs, [wav] * S, [p.rec] * S)]
        torch.cuda.synchronize()
        sv.close()
        return tr

    import paper_1608_03984_amd as P
    st = torch.cuda.current_stream().cuda_stream
    Jdev = torch.zeros(P.FD_MISFIT_DOUBLES, dtype=torch.float64, device=dev)

    def misfit(tr, dobs):
        """J = 1/2 sum over shots |d - d_obs|^2 (fd_misfit, residuals in place)."""
        Jdev.zero_()
        for a, b in zip(tr, dobs):
            P.fd_misfit(a.data_ptr(), b.data_ptr(), a.numel(), a.data_ptr(), Jdev.data_ptr(), st)
        return float(Jdev[0].item())

    t0 = time.perf_counter()
    dobs = survey(p.vel)
    t_obs = time.perf_counter() - t0
    say(f"# observed data: {S} shots x {nt} steps in {t_obs:.2f} s")
    vel0 = p.extra["vel_start"]
    s = Solver(3, p.shape, p.spacing, p.nbl, p.so, p.dt, vel0, p.eta, max_points=1 + nrec,
               device=dev)
    g = torch.zeros(s.field_shape, dtype=torch.float32, device=dev)
    info = {}

    def gradient():
        g.zero_()
        for k in range(S):
            tr = s.forward_checkpointed(nt, srcs[k], wav, p.rec, interval=args.interval)
            # residual in place (the trace sensitivities of J)
            P.fd_misfit(tr.data_ptr(), dobs[k].data_ptr(), tr.numel(), tr.data_ptr(),
                        Jdev.data_ptr(), st)
            s.gradient(tr, wrt="vel", wavelet_grad=False, accumulate_into=g)
            info["interval"] = s.checkpoint_interval
            info["store_gb"] = s._ck["bytes"] / 1e9

    # warm-up: one shot
    tr = s.forward_checkpointed(nt, srcs[0], wav, p.rec, interval=args.interval)
    P.fd_misfit(tr.data_ptr(), dobs[0].data_ptr(), tr.numel(), tr.data_ptr(), Jdev.data_ptr(), st)
    s.gradient(tr, wrt="vel", wavelet_grad=False)
    Jdev.zero_()
    t_grad = timed(gradient, ev)
    J_grad = float(Jdev[0].item())
    say(f"# gradient of {S} shots in {t_grad:.2f} s (one shot at a time)")
    finite = bool(torch.isfinite(g).all().item())
    s.close()
    del s
    torch.cuda.empty_cache()
    # the same gradient with G shots per context: each group's checkpointed
    # forward runs, adjoints and imaging advance G shots in shared launches
    G = args.group
    grouped = None
    if G > 1 and S % G == 0:
        sg = Solver(3, p.shape, p.spacing, p.nbl, p.so, p.dt, vel0, p.eta, nshots=G,
                    max_points=G * (1 + nrec), device=dev)
        g2 = torch.zeros(sg.field_shape, dtype=torch.float32, device=dev)
        dobs_g = [torch.cat(dobs[k:k + G], dim=1).contiguous() for k in range(0, S, G)]

        def gradient_grouped():
            g2.zero_()
            for j, k in enumerate(range(0, S, G)):
                sg.forward_checkpointed_shots(nt, srcs[k:k + G], [wav] * G, [p.rec] * G,
                                              interval=args.interval)
                tr = sg._ck_traces   # [nt][G nrec], shot k's columns k nrec .. (k+1) nrec
                P.fd_misfit(tr.data_ptr(), dobs_g[j].data_ptr(), tr.numel(), tr.data_ptr(),
                            Jdev.data_ptr(), st)
                sg.gradient_shots(tr, wrt="vel", accumulate_into=g2)
                info["group_store_gb"] = sg._ck["bytes"] / 1e9

        Jdev.zero_()
        t_g = timed(gradient_grouped, ev)
        grouped = {"shots_per_context": G, "gradient_s": round(t_g, 3),
                   "gpts": round(S * npts * nt / t_g / 1e9, 3),
                   "speedup_vs_one_at_a_time": round(t_grad / t_g, 3),
                   "store_gb_per_context": round(info["group_store_gb"], 1),
                   "bitwise_equal_to_one_at_a_time": bool(torch.equal(g, g2)),
                   "misfit": float(Jdev[0].item())}
        say(f"# gradient of {S} shots in {t_g:.2f} s ({G} shots per context), "
            f"equal bits: {grouped['bitwise_equal_to_one_at_a_time']}")
        sg.close()
        del sg, g2, dobs_g
        torch.cuda.empty_cache()
    # central differences along the normalised gradient
    d = (g / g.abs().max()).cpu().numpy()
    J0 = misfit(survey(vel0), dobs)
    say(f"# misfit of the gradient runs {J_grad:.6e}, of the 16-shot launch {J0:.6e}")
    gd = float(torch.sum(g.double() * torch.from_numpy(d).to(dev).double()))
    eps = 1e-3 * J0 / abs(gd) if gd != 0 else 1.0
    Jp = misfit(survey((vel0 + eps * d).astype(np.float32)), dobs)
    Jm = misfit(survey((vel0 - eps * d).astype(np.float32)), dobs)
    fd = (Jp - Jm) / (2 * eps)
    say(f"# J {J0:.6e}, central difference {fd:.6e} vs <g, dir> {gd:.6e} (eps {eps:.3e} m/s)")
    I = info["interval"]
    alg = S * npts * gradient_bytes(nt, I)
    ach = alg / t_grad / 1e9
    line = {
        "metric": "FWI gradient Gpt/s (3D acoustic so8, 16-shot survey)",
        "value": round(S * npts * nt / t_grad / 1e9, 3), "unit": "Gpt/s", "n_gpus": 1,
        "steps": nt, "warmup": 1, "ms_per_step": round(t_grad / nt * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"FWI gradient of a {S}-shot survey, 3D acoustic {p.shape[0]}^3 + "
                               f"40-pt layer ({p.padded[0]}^3 points), h=15 m, so 8, {nt} steps, "
                               f"8 Hz Ricker per shot, {nrec} receivers, true vs smoothed model",
                   "points": npts, "shots": S, "interval": I,
                   "store_gb_per_shot": round(info["store_gb"], 1)},
        "gradient_s": round(t_grad, 3), "observed_data_s": round(t_obs, 3),
        "misfit": J0, "misfit_gradient_runs": J_grad, "fd_check": {"central_difference": fd, "gradient_dot_dir": gd,
                                   "eps_m_per_s": eps, "rel_err": abs(fd - gd) / abs(gd)},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "whole gradient (algorithmic bytes of every pass / wall time)"},
        "finite": finite,
        "grouped": grouped,
    }
    print(json.dumps(line), flush=True)


def shots_bench(args):
    """Survey of 16 shots on the 256^3 + 40-point-layer grid (336^3 points),
    so 8, one source per shot, 256 x 256 receivers shared by the shots: all
    shots advance in one launch per step, a group of shots sharing each read
    of the model.  Algorithmic bytes per step and point: 12 per shot (read
    u^n and u^(n-1), write u^(n+1)) plus 4 for dt^2 v^2 read once."""
    import torch

    from paper_1608_03984_amd.solver import Solver
    from workloads import fwi_3d

    S = 16
    p = fwi_3d(so=8, phys=256 if args.phys == 512 else args.phys, nbl=40, nt=1, nshots=S,
               receivers="surface")
    npts = p.npoints
    dev = torch.device("cuda:0")
    from workloads import ricker
    nt = args.warmup + args.steps
    wav = ricker(8.0, p.dt, nt)[:, None].astype(np.float32)
    srcs = [p.src[k:k + 1] for k in range(S)]
    recs = [p.rec] * S
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    s = Solver(3, p.shape, p.spacing, p.nbl, p.so, p.dt, p.vel, p.eta, nshots=S,
               max_points=S * (1 + p.rec.shape[0]), device=dev)
    none, w0 = [None] * S, [np.zeros((1, 0), np.float32)] * S
    s.forward_shots(0, srcs, [wav[:0]] * S, recs)
    settle(lambda: s.forward_shots(2, srcs, [wav[:2]] * S, recs, zero_state=False,
                                   keep_points=True))
    s.forward_shots(args.warmup, srcs, [wav[:args.warmup]] * S, recs, keep_points=True)
    tw = timed(lambda: s.forward_shots(args.steps, srcs, [wav[args.warmup:]] * S, recs,
                                       zero_state=False, keep_points=True), ev)
    s.forward_shots(args.warmup, none, w0, none, zero_state=False)
    tk = timed(lambda: s.forward_shots(args.steps, none, w0, none, zero_state=False), ev)
    s.close()
    del s
    torch.cuda.empty_cache()
    # one shot at a time (a single-shot context, same kernels with one shot per block)
    s1 = Solver(3, p.shape, p.spacing, p.nbl, p.so, p.dt, p.vel, p.eta,
                max_points=1 + p.rec.shape[0], device=dev)
    s1.forward(0, srcs[0], wav[:0], p.rec)
    settle(lambda: s1.forward(4, srcs[0], wav[:4], p.rec, zero_state=False, keep_points=True))
    s1.forward(args.warmup, srcs[0], wav[:args.warmup], p.rec, keep_points=True)
    t1 = timed(lambda: s1.forward(args.steps, srcs[0], wav[args.warmup:], p.rec,
                                  zero_state=False, keep_points=True), ev)
    s1.close()
    kernel_s = tk / args.steps
    ach = (12 * S + 4) * npts / kernel_s / 1e9
    value = S * npts * args.steps / tw / 1e9
    single = npts * args.steps / t1 / 1e9
    line = {
        "metric": "Gshot-pt/s (3D acoustic so8, 16 shots per launch)", "value": round(value, 3),
        "unit": "Gpt/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(tw / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"survey of {S} shots, 3D acoustic {p.shape[0]}^3 + 40-pt layer "
                               f"({p.padded[0]}^3 points), h=15 m, so 8, one source per shot, "
                               f"{p.rec.shape[0]} receivers per shot", "points": npts,
                   "shots": S},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "acoustic3d_tiled, 16 shots per launch "
                               "((12 S + 4) B per point / launch time)"},
        "stencil_ms": round(kernel_s * 1e3, 4),
        "single_shot_gpts": round(single, 3), "speedup_vs_single_shot": round(value / single, 3),
    }
    print(json.dumps(line), flush=True)


def cost_bench(args):
    """Cost-to-solution of section 6 measured: the fixed physical problem of
    Tables 2 and 3 (500^3 points at second order, p points per wavelength
    from 6 down, the same final time) run for real at orders 2, 6, 12 and 16
    (16 with p interpolated between the printed rows), against the MI355X
    roofline prediction of the perfmodel module (Table 1 FLOPs, 16 B per
    point, 8 TB/s).  Homogeneous v = 1500 m/s, h = 10 m at second order, no
    absorbing layer, a 10 Hz Ricker source at the centre, 64 receivers."""
    import torch

    from paper_1608_03984_amd import perfmodel as M
    from paper_1608_03984_amd.solver import Solver
    from workloads import ricker

    dev = torch.device("cuda:0")
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    rows = []
    for order in (2, 6, 12, 16):
        r = M.cost_row(order)
        n = r.n_axis
        h = 10.0 * r.h
        v = 1500.0
        dt = r.dt * 10.0 / v * (1.0 - 1e-6)     # inside the CFL bound by 1e-6
        vel = np.full((n, n, n), v, np.float32)
        src = np.array([[n * h / 2, n * h / 2, n * h / 2]])
        xs = np.linspace(0.0, (n - 1) * h, 64)
        rec = np.stack([xs, np.full(64, n * h / 2), np.full(64, 2 * h)], 1)
        wav = ricker(10.0, dt, r.nt)[:, None].astype(np.float32)
        s = Solver(3, (n, n, n), (h, h, h), 0, order, dt, vel, None, max_points=65, device=dev)
        s.forward(5, src, wav[:5], rec)                         # warm-up
        t = timed(lambda: s.forward(r.nt, src, wav, rec), ev)
        s.close()
        del s
        torch.cuda.empty_cache()
        # the model's N is (500/h)^3; the run uses n_axis^3 points
        pred = r.runtime_s(M.MI355X_HBM_GBS, M.MI355X_FP32_GFLOPS) * n ** 3 / r.N
        rows.append({"order": order, "p": round(r.p, 4), "h_m": round(h, 3), "n_axis": n,
                     "N_model": r.N, "points": n ** 3, "nt": r.nt,
                     "gflop_paper": round(r.gflop, 1), "oi": round(r.oi(), 4),
                     "predicted_s": round(pred, 4), "measured_s": round(t, 4),
                     "frac_of_roofline": round(pred / t, 4),
                     "gpts": round(n ** 3 * r.nt / t / 1e9, 2)})
        print(f"# order {order}: {n}^3 x {r.nt} steps: {t:.3f} s (roofline {pred:.3f} s)",
              file=sys.stderr, flush=True)
    best = min(rows, key=lambda x: x["measured_s"])
    line = {
        "metric": "cost-to-solution s (3D acoustic, fixed physics of Tables 2-3)",
        "value": best["measured_s"], "unit": "s", "n_gpus": 1, "steps": None,
        "warmup": 5, "ms_per_step": None, "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "fixed physical problem of Tables 2-3: 500^3 points at order 2, "
                               "p points per wavelength 6/5/4/3.33 at orders 2/6/12/16, common "
                               "final time of 1000 second-order steps, homogeneous 1500 m/s",
                   "best_order": best["order"]},
        "rows": rows,
    }
    print(json.dumps(line), flush=True)


def learned_bench(args):
    """Learned coarse-grid correction at the configuration of its design: fine
    space order 16 on 256^3 + 40-point layer (h = 10 m, 1000 steps), coarse
    space order 4 on every second point (128^3 + 20, h = 20 m, 500 steps),
    correction every 8 coarse steps after the source has radiated.  Trains on
    --models random layered models (solver-generated pairs) with libfd's
    kernels, then times and scores on 3 held-out models: the fine solve (the
    reference), the plain coarse solve, the corrected coarse solve, the coarse
    solve corrected by the exact residual (the scheme's best case), and plain
    coarse solves of space order 8 and 16.  Errors are relative L2 of the
    receiver traces against the fine solve, over all receivers and samples
    ("err") and over receivers outside the source ball after the first
    correction ("late").  The headline compares the learned solve's time with
    the cheapest plain solve whose error is no larger."""
    import torch

    from paper_1608_03984_amd import learned as Lm
    from paper_1608_03984_amd.solver import Solver
    from workloads import learned_model

    K = 8
    say = lambda m: print(m, file=sys.stderr, flush=True)
    m0 = learned_model(100)
    start = Lm.correction_start(m0)
    nt_f, nt_c = m0["nt_f"], m0["nt_c"]
    shape_c = tuple(s + 2 * m0["nbl_c"] for s in m0["shape_c"])
    times = list(range(start + K, nt_c + 1, 8))
    t0 = time.perf_counter()
    samples = []
    # --windows per model (evenly spaced over the run, shifted from model to
    # model so that together they cover every window time)
    nw = min(args.windows, len(times)) if args.windows > 0 else len(times)
    for i in range(args.models):
        pair = Lm.make_pair(learned_model(100 + i))
        sel = sorted({times[(i + j * len(times) // nw) % len(times)] for j in range(nw)})
        samples += Lm.training_pairs(pair, sel, K)
        pair.close()
        if (i + 1) % 10 == 0 or i + 1 == args.models:
            say(f"# training model {i + 1}/{args.models}: {len(samples)} samples")
    t_data = time.perf_counter() - t0
    net = Lm.CorrectionNet(seed=1, out_scale=0.01)
    none_loss = Lm.sample_loss(None, samples, shape_c)
    (hist, t_train) = Lm.timed(lambda: Lm.train(net, samples, shape_c, args.iters, lr=1e-3,
                                                lr_end=1e-4))
    train_loss = Lm.sample_loss(net, samples, shape_c)
    say(f"# trained {args.iters} iterations in {t_train:.1f} s: window loss {none_loss:.3e} "
        f"-> {train_loss:.3e}")
    n_samples = len(samples)
    del samples
    rows = []
    for seed in (900, 901, 902):
        m = learned_model(seed)
        pair = Lm.make_pair(m)
        far = Lm.far_receivers(pair, Lm.SRC_RADIUS * m["h_c"][0])
        held = Lm.training_pairs(pair, times, K)
        win = (Lm.sample_loss(None, held, shape_c), Lm.sample_loss(net, held, shape_c))
        del held
        Lm.solve_fine(pair, 20)                                   # warm-up
        tf, t_fine = Lm.timed(lambda: Lm.solve_fine(pair, nt_f).clone())
        runs = {"plain_so4": Lm.timed(lambda: Lm.solve_coarse(pair, nt_c).clone()),
                "learned_so4": Lm.timed(lambda: Lm.solve_coarse(pair, nt_c, K, net,
                                                                start=start).clone()),
                "exact_so4": Lm.timed(lambda: Lm.solve_coarse_exact(pair, nt_c, K,
                                                                    start=start).clone())}
        for so in (8, 16):
            s = Solver(3, m["shape_c"], m["h_c"], m["nbl_c"], so, m["dt_c"], m["vel_c"],
                       m["eta_c"], max_points=1 + len(m["rec"]))
            alt = Lm.PairSetup(pair.fine, s, m["src"], m["rec"], m["wav_f"], m["wav_c"], nt_c)
            runs[f"plain_so{so}"] = Lm.timed(lambda: Lm.solve_coarse(alt, nt_c).clone())
            s.close()
        pair.close()
        row = {"seed": seed, "fine_s": round(t_fine, 4),
               "window_loss_none": win[0], "window_loss_learned": win[1]}
        for k, (tr, t) in runs.items():
            row[f"{k}_s"] = round(t, 4)
            row[f"err_{k}"] = round(Lm.trace_error(tr, tf), 5)
            row[f"late_{k}"] = round(Lm.trace_error(tr, tf, far, start), 5)
        plain = [(row["fine_s"], 0.0)] + [(row[f"plain_so{so}_s"], row[f"err_plain_so{so}"])
                                          for so in (4, 8, 16)]
        row["plain_at_equal_error_s"] = min(t for t, e in plain if e <= row["err_learned_so4"])
        rows.append(row)
        say(f"# held-out {seed}: {row}")
    mean = lambda k: float(np.mean([r[k] for r in rows]))
    t_learn = mean("learned_so4_s")
    line = {
        "metric": "learned vs plain s at equal L2 error (3D acoustic coarse-grid correction)",
        "value": round(t_learn, 4), "unit": "s", "n_gpus": 1, "steps": nt_c,
        "warmup": 1, "ms_per_step": round(t_learn / nt_c * 1e3, 4),
        "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "fine so16 256^3+40 (h 10 m, 1000 steps) as reference; coarse so4 "
                               "128^3+20 (h 20 m, 500 steps) corrected every 8 steps by a "
                               "3-layer 3x3x3 conv net (16 channels, BF16, FP32 accumulation)",
                   "train_models": args.models, "windows_per_model": nw,
                   "train_samples": n_samples,
                   "train_iters": args.iters,
                   "data_s": round(t_data, 1), "train_s": round(t_train, 2),
                   "window_loss_train": [none_loss, train_loss]},
        "plain_at_equal_error_s": round(mean("plain_at_equal_error_s"), 4),
        "speedup_vs_plain_at_equal_error": round(mean("plain_at_equal_error_s") / t_learn, 3),
        "speedup_vs_fine": round(mean("fine_s") / t_learn, 3),
        "mean": {k: float(f"{mean(k):.5g}") for k in rows[0] if k != "seed"},
        "rows": rows,
    }
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus above 1 is not "
                                   "supported (the solver has no multi-GPU path)"}))
        sys.exit(2)
    if args.profile_pass:
        profile_pass(args)
        return
    if args.workload in ("tti", "vti"):
        tti_bench(args, args.workload)
        return
    if args.workload == "gradient":
        gradient_bench(args)
        return
    if args.workload == "shots":
        shots_bench(args)
        return
    if args.workload == "fwi":
        fwi_bench(args)
        return
    if args.workload == "2d":
        acoustic2d_bench(args)
        return
    if args.workload == "cost":
        cost_bench(args)
        return
    if args.workload == "learned":
        learned_bench(args)
        return
    import torch

    import paper_1608_03984_amd as P
    from paper_1608_03984_amd.solver import Solver
    from workloads import DT, acoustic_3d

    orders = [int(s) for s in args.orders.split(",")]
    traffic = committed_traffic(args.phys)
    t0 = time.perf_counter()
    prob = acoustic_3d(so=8, phys=args.phys, nbl=40, nt=1, receivers="surface")
    print(f"# model generated in {time.perf_counter() - t0:.1f} s, padded {prob.padded}",
          file=sys.stderr, flush=True)
    npts = prob.npoints
    dev = torch.device("cuda:0")
    rec = prob.rec
    per = []
    tot_pts = 0.0
    tot_time = 0.0
    tot_kernel = 0.0
    for so in orders:
        dt = DT[("acoustic_3d", so)]
        from workloads import ricker
        nt = args.warmup + args.steps
        wav = torch.from_numpy(ricker(10.0, dt, nt)[:, None]).to(dev)
        traces = torch.empty((nt, rec.shape[0]), dtype=torch.float32, device=dev)
        s = Solver(3, prob.shape, prob.spacing, prob.nbl, so, dt, prob.vel, prob.eta,
                   max_points=1 + rec.shape[0], device=dev)
        tile = s.get_option(P.FD_OPT_TILE)
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        # upload the point tables (no steps), settle the GPU, warm up
        s.forward(0, prob.src, wav[:0], rec)
        settle(lambda: s.forward(4, prob.src, wav[:4], rec, zero_state=False, traces=traces[:4],
                                 keep_points=True))
        s.forward(args.warmup, prob.src, wav[:args.warmup], rec, traces=traces[:args.warmup],
                  keep_points=True)
        tw = timed(lambda: s.forward(args.steps, prob.src, wav[args.warmup:], rec,
                                     zero_state=False, traces=traces[args.warmup:],
                                     keep_points=True), ev)
        # the stencil kernel alone (no sparse points): its average launch time
        s.forward(args.warmup, zero_state=False)
        tk = timed(lambda: s.forward(args.steps, zero_state=False), ev)
        ok = bool(torch.isfinite(traces).all().item())
        s.close()
        del s, traces
        torch.cuda.empty_cache()
        gpts = npts * args.steps / tw / 1e9
        kernel_ms = tk / args.steps * 1e3
        achieved = BYTES_PER_POINT * npts / (kernel_ms / 1e3) / 1e9
        per.append({"so": so, "gpts": round(gpts, 2), "ms_per_step": round(tw / args.steps * 1e3, 4),
                    "stencil_ms": round(kernel_ms, 4), "stencil_gbs": round(achieved, 1),
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic_of(traffic, so, tile),
                    "gflops_paper": round(paper_flops(so) * npts / (kernel_ms / 1e3) / 1e9, 1),
                    "finite": ok})
        print(f"# so{so}: {gpts:.1f} Gpt/s, stencil {kernel_ms:.3f} ms = {achieved:.0f} GB/s",
              file=sys.stderr, flush=True)
        tot_pts += npts * args.steps
        tot_time += tw
        tot_kernel += tk
    value = tot_pts / tot_time / 1e9
    ach = BYTES_PER_POINT * tot_pts / tot_kernel / 1e9
    tgbs, tcfg = triad_gbs(torch, P)
    counted = [o["traffic"] for o in per]
    mean_traffic = (round(sum(counted) / len(counted))
                    if counted and all(c is not None for c in counted) else None)
    line = {
        "metric": "Gpt/s, % roofline (3D acoustic SO4-16)",
        "value": round(value, 3),
        "unit": "Gpt/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(tot_time / (args.steps * len(orders)) * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"3D isotropic acoustic, {args.phys}^3 + 40-pt layer "
                               f"({prob.padded[0]}^3 points), h=10 m, two-layer v with +-5% "
                               f"smooth perturbation, 1 Ricker source, {rec.shape[0]} receivers",
                   "space_orders": orders, "points": npts},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": mean_traffic,
                     "kernel": "acoustic3d_tiled (sweep aggregate; traffic = mean bytes per "
                               "launch over the orders)"},
        "triad_gbs": round(tgbs, 1) if tgbs else None,
        "triad_config": tcfg,
        "frac_of_triad": round(ach / tgbs, 4) if tgbs else None,
        "per_order": per,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
