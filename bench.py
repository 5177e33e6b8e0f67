"""Benchmark of the fused lattice-Boltzmann step on one MI355X.

    python bench.py [--gpus 1] [--steps 500] [--warmup 50] [--workload spinodal4096]

A "step" is one time step of the whole update (pull-stream, moments,
pseudo-potential forces, wall forces, EDM-BGK collision, store) on the
workload lattice, with the diagnostic pass (FP64 totals, residual, non-finite
check) every 100 steps inside the timed region.  Inputs are resident in HBM
before timing starts.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % peak HBM GB/s (1 GPU); batched solves/s, p50/p99 latency vs plain"
HBM_PEAK_GBS = 8000.0
DIAG_EVERY = 100


def bytes_per_update(storage):
    # 9 populations read + 9 written per lattice update
    return {"f32": 72, "f16dev": 36, "f64": 144}[storage]


WORKLOADS = {
    # name: (nx, ny, description)
    "spinodal4096": (4096, 4096, "periodic 4096x4096 phase separation from seeded Gaussian-smoothed "
                                 "noise (sigma 4), 50% liquid, G=-5, tau=1, no solid"),
    "drop1024": (1024, 512, "sessile drop 1024x512, radius 160, flat solid band of 8 rows, "
                            "seeded wall amplitudes"),
}


def make_lattice(name, storage, seg_rows):
    from paper_1202_6130_amd import inputs as I
    from paper_1202_6130_amd import lbm
    st = {"f32": lbm.STORE_F32, "f16dev": lbm.STORE_F16DEV, "f64": lbm.STORE_F64}[storage]
    nx, ny, _ = WORKLOADS[name]
    if name == "spinodal4096":
        rho0 = I.spinodal_field(nx, seed=0)
        p = lbm.lbm_params_default(nx=nx, ny=ny, storage=st, diag_interval=DIAG_EVERY, seg_rows=seg_rows,
                                   rho_ref=float(rho0.mean()))
    else:
        gr, ga = I.draw_wall_amplitudes(0)
        rho0 = I.drop_field(nx, ny, 160.0)
        p = lbm.lbm_params_default(nx=nx, ny=ny, storage=st, wall_kind=lbm.WALL_FLAT_SLAB, G_R=float(gr[0]),
                                   G_A=float(ga[0]), diag_interval=DIAG_EVERY, seg_rows=seg_rows,
                                   rho_ref=float(rho0.mean()))
    return lbm.Lattice(p, rho0), p


def time_gpu(name, storage, steps, warmup, seg_rows):
    import torch
    L, p = make_lattice(name, storage, seg_rows)
    nodes = p.nx * p.ny
    L.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    # per-launch events on the launch stream for steps without a diagnostic pass
    ev = []
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    start_idx = L.step_index
    for s in range(steps):
        diag_here = (start_idx + s + 1) % DIAG_EVERY == 0
        if not diag_here:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            L.step(1)
            b.record(stream)
            ev.append((a, b))
        else:
            L.step(1)
    t1.record(stream)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    kern_ms = np.array([a.elapsed_time(b) for a, b in ev])
    d = L.diagnostics()
    L.close()
    return {
        "nodes": nodes, "ms_total": total_ms, "ms_per_step": total_ms / steps,
        "kernel_ms_mean": float(kern_ms.mean()), "kernel_ms_median": float(np.median(kern_ms)),
        "mass": float(d[1]), "nonfinite": float(d[5]), "seg_rows": p.seg_rows,
    }


COPY_REF_BYTES = 1 << 30


def copy_reference():
    """One device-to-device copy of COPY_REF_BYTES (reads and writes that many
    bytes once): the known-size dispatch the memory counters are scaled by."""
    import torch
    src = torch.ones(COPY_REF_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def cpu_baseline(seconds_hint=15.0):
    """The FP64 oracle (single thread, as it stands) on a bounded sample of the
    same workload recipe: a 1024x1024 periodic spinodal lattice."""
    import oracle as O
    from paper_1202_6130_amd import inputs as I
    n = 1024
    rho0 = I.spinodal_field(n, seed=0)
    p = O.make_params(n, n, tau=1.0, G=-5.0)
    w = O.Walls.none(n, n)
    f = O.init(p, rho0)
    f = O.run(p, w, f, 1)            # page in
    t = time.perf_counter()
    steps = 0
    while True:
        f = O.run(p, w, f, 2)
        steps += 2
        if time.perf_counter() - t > seconds_hint:
            break
    dt = time.perf_counter() - t
    return {"value": n * n * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"FP64 oracle, 1 thread, 1024x1024 periodic spinodal lattice (same recipe), "
                      f"{steps} steps in {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="spinodal4096", choices=sorted(WORKLOADS))
    ap.add_argument("--storage", default="f32", choices=["f32", "f16dev", "f64"])
    ap.add_argument("--seg-rows", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--copy-ref", action="store_true",
                    help="after timing, run one plain device copy of 1 GiB (reference dispatch for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the update is measured on a "
              "single MI355X and no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)

    r = time_gpu(args.workload, args.storage, args.steps, args.warmup, args.seg_rows)
    if args.copy_ref:
        copy_reference()
    mlups = r["nodes"] * args.steps / (r["ms_total"] * 1e-3) / 1e6
    bpu = bytes_per_update(args.storage)
    achieved = bpu * r["nodes"] / (r["kernel_ms_mean"] * 1e-3) / 1e9
    traffic = None
    key = f"{args.workload}:{args.storage}"
    if os.path.exists(args.traffic_json):
        with open(args.traffic_json) as fh:
            traffic = json.load(fh).get(key)
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.storage, "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload][2], "nx": WORKLOADS[args.workload][0],
                   "ny": WORKLOADS[args.workload][1], "storage": args.storage, "seg_rows": r["seg_rows"],
                   "diag_every": DIAG_EVERY},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_step", "kernel_ms_mean": round(r["kernel_ms_mean"], 5),
                     "bytes_per_update": bpu},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
