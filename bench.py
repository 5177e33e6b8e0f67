"""Benchmark of the fused lattice-Boltzmann step on one MI355X.

    python bench.py [--gpus 1] [--steps 500] [--warmup 300] [--workload spinodal4096]

A "step" is one time step of the whole update (pull-stream, moments,
pseudo-potential forces, wall forces, EDM-BGK collision, store) on the
workload lattice, with the diagnostic pass (FP64 totals, residual, non-finite
check) every 100 steps inside the timed region.  Inputs are resident in HBM
before timing starts.  On D2Q9 lattices (F32, F16DEV or F64 storage) the
warm-up autotunes the tile shape and then the choice between one step per
launch and two steps per launch (temporal blocking: the populations between
the two steps stay in LDS; bitwise the same fields).  Prints one JSON line.
"""
import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % peak HBM GB/s (1 GPU); batched solves/s, p50/p99 latency vs plain"
HBM_PEAK_GBS = 8000.0
DIAG_EVERY = 100
SAMPLE_EVERY = 10          # timed launches per per-launch event pair
KERNEL_SAMPLES = 50        # event-timed launches right after the timed region


KERNEL_SOURCES = {
    9: ("paper_1202_6130_amd/csrc/kernels.hip", "paper_1202_6130_amd/csrc/lbm_device.hpp",
        "paper_1202_6130_amd/csrc/launch.hpp"),
    21: ("paper_1202_6130_amd/csrc/kernels_q21.hip", "paper_1202_6130_amd/csrc/lbm_device.hpp",
         "paper_1202_6130_amd/csrc/launch.hpp"),
}


def kernel_sources_digest(q=9):
    """SHA-256 over the device sources of the step kernel of D2Q<q>; a stored
    traffic figure is used only while the kernel it was counted on is
    unchanged."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[q]:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def q21_kernel(variant):
    return "k_march_q21" if variant == 1 else "k_tile_q21"


def q21_label(variant):
    """Kernel and tiling of a D2Q21 step variant (variants 0 and 2 are the
    two-row and one-row instances of k_tile_q21)."""
    return {0: "k_tile_q21", 1: "k_march_q21", 2: "k_tile_q21_r1"}[variant]


def traffic_key(workload, storage, shape):
    """shape: the D2Q9 tile shape, "pass2v<V>" for two steps per pass with
    variant V, or the D2Q21 step variant."""
    if isinstance(shape, str):
        return f"{workload}:{storage}:{shape}"
    return f"{workload}:{storage}:" + (f"shape{shape}" if workload_q(workload) == 9 else q21_label(shape))


# (strips, output rows, waves per strip) of the two-steps-per-pass variants, as
# in lbm_two_step_variants (strips, rows, waves per workgroup)
PASS2_GEOMETRY = [(1, 8, 4), (1, 8, 8), (2, 8, 4), (1, 12, 6), (1, 12, 12), (1, 16, 8), (1, 16, 16), (1, 24, 8),
                  (1, 24, 12)]


def pass2_desc(v):
    ts, oh, wps = PASS2_GEOMETRY[v]
    return (f"two steps per pass, variant {v}: {64 * ts} x {oh} output nodes per workgroup "
            f"({ts * wps} waves), populations between the steps in LDS")


def stored_traffic(path, key, field="bytes_per_launch"):
    """HBM bytes per launch of the step kernel (workload:storage:shape) from
    rocprofv3 FETCH_SIZE + WRITE_SIZE runs, scaled by a 1 GiB copy (or another
    field of the same record: "valu_insts"); None if absent or counted on
    other kernels."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(key)
    if not rec or rec.get("kernel_sources_sha256") != kernel_sources_digest(workload_q(key.split(":")[0])):
        return None
    return rec.get(field)


# VALU issue peak from the FP32 vector rate (157.3 TFLOP/s = 256 CUs x 2.4 GHz
# x 2 wave64 FMA instructions per CU and cycle x 64 lanes x 2 flops): two
# wave64 VALU instructions per CU and cycle; binary64 arithmetic issues at half
# that rate (78.6 TFLOP/s), so a mix with binary64 work tops out lower
VALU_PEAK_WAVE_INSTS = 256 * 2.4e9 * 2


def alu_roofline(valu_insts, kernel_ms):
    rate = valu_insts / (kernel_ms * 1e-3)
    return {"bound": "alu", "achieved": round(rate / 1e9, 2), "peak": VALU_PEAK_WAVE_INSTS / 1e9,
            "unit": "G VALU wave-instructions/s", "frac": round(rate / VALU_PEAK_WAVE_INSTS, 4),
            "valu_insts_per_launch": valu_insts,
            "note": "VALU instructions per launch from a rocprofv3 SQ_INSTS_VALU run (profiles/traffic.json) "
                    "over the live launch time"}


def _counter_rows(run_dir):
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(run_dir, "**", "*_counter_collection.csv"), recursive=True))
    if not files:
        sys.exit(f"no *_counter_collection.csv under {run_dir}")
    with open(files[-1]) as fh:
        return list(csv.DictReader(fh))


def _step_dispatch_key(name):
    """Tile shape (D2Q9), or the D2Q21 step variant (0 two-row tiles, 1
    marching, 2 one-row tiles), of a dispatch of a step kernel; None for any
    other kernel (the diagnostic variant of k_tile_q21 included)."""
    if "k_step_tiles<" in name and "k_step_tiles_batch" not in name:
        # <S, C, WALL, SHAPE, ONE>
        return int(name.split("k_step_tiles<")[1].split(">")[0].split(",")[3])
    if "k_step_pass2<" in name:
        # <S, C, WALL, TS, OH, WPS, ONE>
        args = [a.strip() for a in name.split("k_step_pass2<")[1].split(">")[0].split(",")]
        return f"pass2v{PASS2_GEOMETRY.index((int(args[3]), int(args[4]), int(args[5])))}"
    if "k_step_pass2_batch<" in name:
        # <TS, OH, WPS>
        args = [int(a) for a in name.split("k_step_pass2_batch<")[1].split(">")[0].split(",")]
        return f"batch_pass2v{PASS2_GEOMETRY.index(tuple(args))}"
    if "k_march_q21<" in name:
        return 1
    if "k_tile_q21<" in name:
        args = [a.strip() for a in name.split("k_tile_q21<")[1].split(">")[0].split(",")]
        if args[-3] == "0":                           # <S, C, WALL, PSI, DIAG, ONE, rows per wave>
            return 0 if args[-1] == "2" else 2
    return None


def ingest_counters(fetch_dir, write_dir, workload, storage, out_json, valu_dir=None):
    """Per-launch HBM bytes of the step kernel from one rocprofv3 FETCH_SIZE
    run and one WRITE_SIZE run of `bench.py --copy-ref` on the same workload:
    each counter's KiB scaled by what it reads for the 1 GiB reference copy.
    With valu_dir (a run that counted SQ_INSTS_VALU), also the VALU wave
    instructions per launch.  Updates out_json and prints a markdown table."""
    import collections
    valu = collections.defaultdict(list)
    if valu_dir is not None:
        for r in _counter_rows(valu_dir):
            k = _step_dispatch_key(r["Kernel_Name"])
            if k is not None and r["Counter_Name"] == "SQ_INSTS_VALU":
                valu[k].append(float(r["Counter_Value"]))

    def per_key(run_dir):
        by = collections.defaultdict(list)
        copy = None
        for r in _counter_rows(run_dir):
            k = _step_dispatch_key(r["Kernel_Name"])
            if k is not None:
                by[k].append(float(r["Counter_Value"]))
            if r["Kernel_Name"] == "__amd_rocclr_copyBuffer" and int(r["Grid_Size"]) >= 65536:
                copy = float(r["Counter_Value"])
        if copy is None:
            sys.exit(f"{run_dir}: no reference copy dispatch (run bench.py with --copy-ref)")
        return by, copy

    fb, fc = per_key(fetch_dir)
    wb, wc = per_key(write_dir)
    fs, ws = COPY_REF_BYTES / 1024 / fc, COPY_REF_BYTES / 1024 / wc
    q = workload_q(workload)
    alg = bytes_per_update(storage, q) // 2 * workload_nodes(workload)
    data = {}
    if os.path.exists(out_json):
        with open(out_json) as fh:
            data = json.load(fh)
    print(f"FETCH_SIZE copy {fc:,.1f} KiB (scale {fs:.4f}), WRITE_SIZE copy {wc:,.1f} KiB (scale {ws:.4f}); "
          f"compulsory {alg:,} B each way per launch (every stored population read once and written once, "
          f"for one time step or two)\n")
    print("| Kernel / shape | dispatches | FETCH_SIZE KiB | read bytes (scaled) | read / compulsory | "
          "WRITE_SIZE KiB | write / compulsory | total / compulsory |")
    print("|---|---|---|---|---|---|---|---|")
    for k in sorted(fb, key=str):
        if (workload == "ensemble256") != str(k).startswith("batch_"):
            continue        # the ensemble's batch kernel only; single lattices' kernels only
        f = sum(fb[k]) / len(fb[k])
        w = sum(wb[k]) / len(wb[k])
        rd, wr = f * fs * 1024, w * ws * 1024
        data[traffic_key(workload, storage, k)] = {
            "bytes_per_launch": round(rd + wr), "read_bytes": round(rd), "write_bytes": round(wr),
            "fetch_kib": round(f, 2), "write_kib": round(w, 2), "fetch_scale": round(fs, 5),
            "write_scale": round(ws, 5), "kernel_sources_sha256": kernel_sources_digest(q)}
        if valu.get(k):
            data[traffic_key(workload, storage, k)]["valu_insts"] = round(sum(valu[k]) / len(valu[k]))
        a = alg
        print(f"| {k if q == 9 else q21_label(k)} | {len(fb[k])} | {f:,.0f} | {rd:,.0f} | {rd / a:.3f} | {w:,.0f} | {wr / a:.3f} | "
              f"{(rd + wr) / (2 * a):.3f} |")
    with open(out_json, "w") as fh:
        json.dump(data, fh, indent=1)


def _short_kernel(name):
    n = name.replace("void lbmwet::", "").replace("(anonymous namespace)::", "")
    return n.split("(")[0] if "(" in n else n


def counter_table(run_dirs, workload=None):
    """Markdown table of rocprofv3 --pmc runs: per kernel, the mean of each
    counter per dispatch.  With a single-lattice workload, the SQ instruction
    counts per lattice update (wave instructions x 64 lanes / (nodes x
    updates per launch)) and the VALU issue fraction: SQ_INSTS_VALU over
    (GRBM_GUI_ACTIVE / 8 XCDs) x 256 CUs x 2, a CU issuing at most two wave64
    VALU instructions per cycle (the FP32 vector rate).  Prints the table;
    returns {kernel: {counter: mean}}."""
    import collections
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for d in run_dirs:
        for r in _counter_rows(d):
            vals[_short_kernel(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    nodes = None
    if workload is not None and (workload in WORKLOADS or workload == "ensemble256"):
        nodes = workload_nodes(workload)
    out = {}
    print("| Kernel | counter | dispatches | mean per dispatch | per lattice update |")
    print("|---|---|---|---|---|")
    for k in sorted(vals):
        if not (k.startswith("k_step") or k.startswith("k_march") or k.startswith("k_tile")):
            continue
        ups = 2 if k.startswith("k_step_pass2") else 1
        # per lattice update: single-lattice kernels of a single-lattice
        # workload, or the two-step batch kernel (one launch over every
        # lattice) of the ensemble
        whole = ("batch" in k) == (workload == "ensemble256") and not k.startswith("k_step_tiles_batch")
        out[k] = {}
        for c in sorted(vals[k]):
            v = vals[k][c]
            m = sum(v) / len(v)
            out[k][c] = m
            per = ""
            if nodes and c.startswith("SQ_INSTS") and whole:
                per = f"{m * 64 / (nodes * ups):.1f}"
            print(f"| `{k}` | {c} | {len(v)} | {m:,.0f} | {per} |")
        if "SQ_INSTS_VALU" in out[k] and "GRBM_GUI_ACTIVE" in out[k]:
            frac = out[k]["SQ_INSTS_VALU"] / (out[k]["GRBM_GUI_ACTIVE"] / 8 * 256 * 2)
            out[k]["valu_issue_fraction"] = frac
            print(f"| `{k}` | VALU issue fraction | | {frac:.3f} | |")
    return out


def trace_table(run_dir, top=25):
    """Markdown table of a rocprofv3 --kernel-trace --stats run (the
    *_kernel_stats.csv under run_dir): calls and durations per kernel."""
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(run_dir, "**", "*_kernel_stats.csv"), recursive=True))
    if not files:
        sys.exit(f"no *_kernel_stats.csv under {run_dir}")
    with open(files[-1]) as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print("| Kernel | Calls | Avg (us) | Min (us) | Max (us) | % time |")
    print("|---|---|---|---|---|---|")
    out = {}
    for r in rows[:top]:
        k = _short_kernel(r["Name"])
        out[k] = float(r["AverageNs"]) / 1e3
        print(f"| `{k}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
              f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return out


def bytes_per_update(storage, q=9):
    # q populations read + q written per lattice update
    return 2 * q * {"f32": 4, "f16dev": 2, "f64": 8}[storage]


def tile_desc(shape):
    from paper_1202_6130_amd import lbm
    w, r, s = lbm.lbm_tile_shapes()[shape]
    return (f"shape {shape}: {64 * s} columns x {w // s * r - 2} rows per workgroup ({w} waves: {s} strip(s) x "
            f"{w // s} waves x {r} rows, 2 halo rows)")

WORKLOADS = {
    # name: (nx, ny, description)
    "spinodal4096": (4096, 4096, "periodic 4096x4096 phase separation from seeded Gaussian-smoothed "
                                 "noise (sigma 4), 50% liquid, G=-5, tau=1, no solid"),
    "drop1024": (1024, 512, "sessile drop 1024x512, radius 160, flat solid band of 8 rows, "
                            "seeded wall amplitudes"),
    # the paper's own lattice and fluid: D2Q21 (Tab. I) with the EOS pseudo-potential, G = -1
    "spinodal4096_q21": (4096, 4096, "D2Q21, EOS pseudo-potential (G=-1, rho_1=0.222, rho_2=0.869): periodic "
                                     "4096x4096 phase separation from seeded Gaussian-smoothed noise (sigma 4), "
                                     "50% at rho 1.0 / 0.1, tau=1, no solid"),
    "drop1024_q21": (1024, 512, "D2Q21, EOS pseudo-potential (G=-1): sessile drop 1024x512 at rho 1.0 / 0.1, "
                                "radius 160, flat solid band of 8 rows, seeded wall amplitudes"),
    "paper650x150_q21": (650, 150, "D2Q21, EOS pseudo-potential (G=-1): the paper's 650x150 domain, drop of "
                                   "radius 50 at rho 1.0 / 0.1 on the lower wall, recursive-filter walls with the "
                                   "outer rows solid, G_R=1.33, G_A=0.5, eps=1"),
}
Q21_TILE = {0: "tiles of 16 waves x 2 rows: 58 output columns x 26 output rows per workgroup (3 halo columns/rows "
               "each side)",
            1: "marching: 256 aligned output columns per workgroup over 128-row segments (6 halo rows per segment)",
            2: "tiles of 16 waves x 1 row: 58 output columns x 10 output rows per workgroup (3 halo columns/rows "
               "each side)"}


def workload_q(name):
    return 21 if name.endswith("_q21") else 9


ENSEMBLE_SEED, ENSEMBLE_COUNT = 0, 256


def workload_nodes(name):
    """Lattice nodes of a single-lattice workload, or of all lattices of the
    256-drop ensemble."""
    if name == "ensemble256":
        from paper_1202_6130_amd import inputs as I
        return sum(c.nx * c.ny for c in I.ensemble_cases(seed=ENSEMBLE_SEED, count=ENSEMBLE_COUNT))
    nx, ny, _ = WORKLOADS[name]
    return nx * ny


def make_lattice(name, storage, seg_rows, tau=1.0, collision=0):
    from paper_1202_6130_amd import inputs as I
    from paper_1202_6130_amd import lbm
    st = {"f32": lbm.STORE_F32, "f16dev": lbm.STORE_F16DEV, "f64": lbm.STORE_F64}[storage]
    nx, ny, _ = WORKLOADS[name]
    if workload_q(name) == 21:
        fluid = dict(lattice=lbm.D2Q21, psi_kind=lbm.PSI_EOS, G=-1.0)
        dens = dict(rho_l=1.0, rho_g=0.1)
    else:
        fluid, dens = {}, {}
    if name.startswith("spinodal"):
        rho0 = I.spinodal_field(nx, seed=0, **dens)
        p = lbm.lbm_params_default(nx=nx, ny=ny, storage=st, diag_interval=DIAG_EVERY, seg_rows=seg_rows,
                                   rho_ref=float(rho0.mean()), tau=tau, collision=collision, **fluid)
    elif name.startswith("paper650x150"):
        H = np.zeros((ny, nx))
        H[0, :] = 1.0
        H[ny - 1, :] = 1.0
        rho0 = I.drop_field(nx, ny, 50.0, slab_rows=1, **dens)
        p = lbm.lbm_params_default(nx=nx, ny=ny, storage=st, wall_kind=lbm.WALL_MASK, G_R=1.33, G_A=0.5, eps=1.0,
                                   diag_interval=DIAG_EVERY, seg_rows=seg_rows, rho_ref=float(rho0.mean()), tau=tau,
                                   collision=collision, **fluid)
        return lbm.Lattice(p, rho0, wall_fields=np.stack([H, H])), p
    else:
        gr, ga = I.draw_wall_amplitudes(0)
        rho0 = I.drop_field(nx, ny, 160.0, **dens)
        p = lbm.lbm_params_default(nx=nx, ny=ny, storage=st, wall_kind=lbm.WALL_FLAT_SLAB, G_R=float(gr[0]),
                                   G_A=float(ga[0]), diag_interval=DIAG_EVERY, seg_rows=seg_rows,
                                   rho_ref=float(rho0.mean()), tau=tau, collision=collision, **fluid)
    return lbm.Lattice(p, rho0), p


def _timed(L, steps, upl):
    """Times `steps` steps in blocks of SAMPLE_EVERY: the first launch of a
    block (unless a diagnostic pass follows its first step) between a pair of
    events on the launch stream, the rest in one lbm_step call, so that host
    work per step never starves the GPU on small lattices.  upl: time steps
    per launch (2 with two steps per pass).  Returns (total ms, per-launch ms
    of the sampled launches)."""
    import torch
    stream = torch.cuda.current_stream()
    pool = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range((steps + SAMPLE_EVERY - 1) // SAMPLE_EVERY)]
    ev = []
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    start_idx = L.step_index
    s = 0
    while s < steps:
        n = min(SAMPLE_EVERY, steps - s)
        if (start_idx + s + 1) % DIAG_EVERY != 0 and n >= upl:
            a, b = pool[len(ev)]
            a.record(stream)
            L.step(upl)
            b.record(stream)
            ev.append((a, b))
            if n > upl:
                L.step(n - upl)
        else:
            L.step(n)
        s += n
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1), np.array([a.elapsed_time(b) for a, b in ev])


def _sample_launches(L, upl, count):
    """Per-launch kernel time (ms) of `count` launches after the timed region:
    each sampled launch (upl steps, no diagnostic pass inside) between a pair
    of events on the launch stream, followed by one unsampled launch so that
    the GPU never idles between samples."""
    import torch
    stream = torch.cuda.current_stream()
    ev = []
    torch.cuda.synchronize()
    while len(ev) < count:
        t = L.step_index
        if any((t + k) % DIAG_EVERY == 0 for k in range(1, 2 * upl + 1)):
            L.step(1)                 # move past the diagnostic pass, unsampled
            continue
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        L.step(upl)
        b.record(stream)
        L.step(upl)
        ev.append((a, b))
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in ev])


def time_gpu(name, storage, steps, warmup, seg_rows, tile=None, tau=1.0, collision=0, two_step=None):
    """tile None: the autotuner picks the D2Q9 tile shape during the
    warm-up (its steps count as warm-up), and a D2Q21 lattice keeps the step
    variant a new context starts with; else the given shape or variant.
    two_step None: for D2Q9 with F32, F16DEV or F64 storage, a second autotuner
    chooses between single steps and two steps per pass; -1: single steps;
    V >= 0: that two-step variant.  With two steps per pass, the same number
    of single steps is timed afterwards as well (the "single" entry)."""
    import torch
    from paper_1202_6130_amd import lbm
    L, p = make_lattice(name, storage, seg_rows, tau, collision)
    nodes = p.nx * p.ny
    q = workload_q(name)
    tune_ms = two_ms = None
    pass2_ok = q == 9 and storage in ("f32", "f16dev", "f64")
    budget = warmup // 2 if (two_step is None and pass2_ok) else warmup
    if tile is not None:
        L.tile_shape = tile
    elif q == 21:
        pass                      # the context's default step variant
    else:
        # 3 * tune_steps + 1 trial steps per shape, within the warm-up when it is long enough
        tune_steps = max(2, (budget // len(lbm.lbm_tile_shapes()) - 1) // 3)
        shape, tune_ms = L.tune(tune_steps)
        tune_ms = [round(float(v), 5) for v in tune_ms]
    if pass2_ok and two_step is None:
        # 6 * steps + 2 trial steps per candidate (the variants and single steps)
        cand = len(lbm.lbm_two_step_variants()) + 1
        steps2 = max(1, ((warmup - budget) // cand - 2) // 6)
        _, two_ms = L.tune_two_step(steps2)
        two_ms = [round(float(v), 5) for v in two_ms]
    elif two_step is not None and two_step >= 0:
        L.two_step = two_step
    variant = L.two_step if q == 9 else -1
    upl = 2 if variant >= 0 else 1
    L.step(max(0, warmup - L.step_index))
    total_ms, kern_in = _timed(L, steps, upl)
    # kernel durations: the sampled launches of the timed region plus
    # KERNEL_SAMPLES more right after it (short timed regions sample few)
    kern_ms = np.concatenate([kern_in, _sample_launches(L, upl, KERNEL_SAMPLES)])
    single = None
    if upl == 2:
        L.two_step = -1
        s_total, s_kern = _timed(L, steps, 1)
        s_kern = np.concatenate([s_kern, _sample_launches(L, 1, KERNEL_SAMPLES)])
        single = {"ms_total": s_total, "kernel_ms_mean": float(s_kern.mean()), "kernel_samples": len(s_kern)}
    d = L.diagnostics()
    shape = L.tile_shape
    L.close()
    return {
        "nodes": nodes, "ms_total": total_ms, "ms_per_step": total_ms / steps,
        "kernel_ms_mean": float(kern_ms.mean()), "kernel_ms_median": float(np.median(kern_ms)),
        "kernel_samples": len(kern_ms),
        "mass": float(d[1]), "nonfinite": float(d[5]), "seg_rows": p.seg_rows, "tile_shape": shape,
        "tune_ms": tune_ms, "two_step_ms": two_ms, "updates_per_launch": upl, "two_step": variant,
        "single": single,
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


def copy_ceiling(reps=20):
    """HBM rate of lbm_device_copy (16-byte non-temporal loads and stores) on
    COPY_REF_BYTES, read + write bytes over time, events on the launch stream:
    the measured plain-copy ceiling next to the nominal peak."""
    import torch
    from paper_1202_6130_amd import lbm
    src = torch.ones(COPY_REF_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        lbm.lbm_device_copy(src.data_ptr(), dst.data_ptr(), COPY_REF_BYTES, stream.cuda_stream)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        lbm.lbm_device_copy(src.data_ptr(), dst.data_ptr(), COPY_REF_BYTES, stream.cuda_stream)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    ok = bool(torch.equal(src, dst))
    del src, dst
    return {"value": round(2 * COPY_REF_BYTES / (ms * 1e-3) / 1e9, 1), "unit": "GB/s", "copied_exactly": ok,
            "kind": "lbm_device_copy: 1 GiB device-to-device copy with 16-byte non-temporal loads and stores, "
                    "read + write bytes"}


def device_copy(reps=20):
    """HBM rate of a plain 1 GiB device-to-device copy with torch's copy kernel
    (read + write bytes over time), timed with events in this process: a
    reference point next to the nominal peak (not a bound: hand-written copies
    with 16-byte non-temporal accesses run faster)."""
    import torch
    n = COPY_REF_BYTES // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return {"value": round(2 * COPY_REF_BYTES / (ms * 1e-3) / 1e9, 1), "unit": "GB/s",
            "kind": "1 GiB device-to-device copy (torch), read + write bytes"}


def cpu_baseline(seconds_hint=15.0, q=9):
    """The FP64 oracle (single thread, as it stands) on a bounded sample of the
    same workload recipe: a 1024x1024 periodic spinodal lattice of the same
    velocity set and pseudo-potential."""
    import oracle as O
    from paper_1202_6130_amd import inputs as I
    n = 1024
    if q == 21:
        rho0 = I.spinodal_field(n, seed=0, rho_l=1.0, rho_g=0.1)
        p = O.make_params(n, n, tau=1.0, G=-1.0, lattice=21, psi_kind=1)
        what = "D2Q21 EOS"
    else:
        rho0 = I.spinodal_field(n, seed=0)
        p = O.make_params(n, n, tau=1.0, G=-5.0)
        what = "D2Q9"
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
            "sample": f"FP64 oracle, 1 thread, 1024x1024 periodic {what} spinodal lattice (same recipe), "
                      f"{steps} steps in {dt:.1f} s"}


def cpu_baseline_omp(q=9, threads=None, seconds_hint=10.0):
    """The same oracle built with OpenMP over rows (bitwise the serial
    result), timed on the same sample in a child process (the oracle module
    loads one build per process)."""
    threads = threads or min(16, os.cpu_count() or 1)
    code = ("import sys, time; sys.path.insert(0, %r)\n"
            "import oracle as O\n"
            "O.use_threads(%d)\n"
            "from paper_1202_6130_amd import inputs as I\n"
            "n = 1024\n"
            "if %d == 21:\n"
            "    rho0 = I.spinodal_field(n, seed=0, rho_l=1.0, rho_g=0.1)\n"
            "    p = O.make_params(n, n, tau=1.0, G=-1.0, lattice=21, psi_kind=1)\n"
            "else:\n"
            "    rho0 = I.spinodal_field(n, seed=0)\n"
            "    p = O.make_params(n, n, tau=1.0, G=-5.0)\n"
            "w = O.Walls.none(n, n)\n"
            "f = O.run(p, w, O.init(p, rho0), 2)\n"
            "t = time.perf_counter(); s = 0\n"
            "while time.perf_counter() - t < %f:\n"
            "    f = O.run(p, w, f, 4); s += 4\n"
            "print(n * n * s / (time.perf_counter() - t) / 1e6, s)\n") % (ROOT, threads, q, seconds_hint)
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    try:
        outp = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
        v, s = outp.stdout.split()
    except Exception as e:  # the baseline is reported, never required
        return {"error": str(e)[:200]}
    return {"value": round(float(v), 2), "unit": "MLUPS", "threads": threads, "kind": "oracle, OpenMP over rows",
            "sample": f"same 1024x1024 lattice, {s} steps"}


def ensemble(steps, seq_steps, seed=ENSEMBLE_SEED, count=ENSEMBLE_COUNT, chunk=100, tune_steps=5, two_step=None,
             traffic_json=None, copy_ref=False):
    """Batched ensemble of `count` sessile drops of uneven size and wall
    parameters: one launch per time step over all lattices, replayed from a
    HIP graph, against the same lattices stepped one after another alone.
    With two steps per launch (one kernel over every lattice) the roofline's
    traffic is the HBM bytes of one launch recorded from rocprofv3 counters of
    the same ensemble, when current."""
    import torch
    from paper_1202_6130_amd import inputs as I
    from paper_1202_6130_amd import lbm
    cases = I.ensemble_cases(seed=seed, count=count)
    ps = [lbm.lbm_params_default(nx=c.nx, ny=c.ny, wall_kind=lbm.WALL_FLAT_SLAB, G=c.G, G_R=c.G_R, G_A=c.G_A)
          for c in cases]
    rhos = [I.drop_field(c.nx, c.ny, c.radius) for c in cases]
    nodes = sum(c.nx * c.ny for c in cases)
    B = lbm.Batch(ps, rhos)
    stream = B._stream_obj
    shapes, tune_ms = B.tune(tune_steps)
    two_ms = None
    if two_step is None:
        variant, two_ms = B.tune_two_step(2)
    else:
        B.two_step = variant = two_step
    B.step(chunk, chunk=chunk)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True); b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    B.step(steps, chunk=chunk)
    b.record(stream)
    torch.cuda.synchronize()
    ms_batch = a.elapsed_time(b)
    upl = 2 if variant >= 0 else 1
    launches = steps // upl
    ens_gbs = 72 * nodes / (ms_batch / launches * 1e-3) / 1e9
    diag = B.diagnostics()
    bad = int(diag[:, 5].sum())
    B.close()
    if copy_ref:
        copy_reference()
    traffic = None
    if traffic_json and (seed, count) == (ENSEMBLE_SEED, ENSEMBLE_COUNT) and variant >= 0:
        traffic = stored_traffic(traffic_json, traffic_key("ensemble256", "f32", f"batch_pass2v{variant}"))
    # sequential baseline: each lattice alone, plain launches, seq_steps steps
    seq_ms = 0.0
    for p, rho, shape in zip(ps, rhos, shapes):
        L = lbm.Lattice(p, rho)
        L.tile_shape = int(shape)      # same tile shape and step variant as in the batch:
        L.two_step = variant           # the speedup is batching alone
        L.step(2)
        torch.cuda.synchronize()
        t = time.perf_counter()
        L.step(seq_steps)
        torch.cuda.synchronize()
        seq_ms += (time.perf_counter() - t) * 1e3
        L.close()
    seq_ms_full = seq_ms * steps / seq_steps
    return {
        "metric": "batched solves/s (ensemble of sessile drops)", "value": round(count / (ms_batch * 1e-3), 2),
        "unit": "solves/s", "n_gpus": 1, "steps": steps, "higher_is_better": True, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{count} sessile drops, nx in 128..1024, ny in 64..512 (multiples of 32), "
                               "radius 0.3*min(nx,ny), G~U[-5.5,-4.5], G_R~U[0,1], G_A~U[0,0.6], "
                               f"{steps} steps each, one launch per step (or per two steps) over all lattices, "
                               f"graph chunks of {chunk}",
                   "lattices": count, "nodes": nodes,
                   "two_step": variant if variant < 0 else pass2_desc(variant),
                   "two_step_tuner_ms_per_step_variants_then_single":
                       None if two_ms is None else [round(float(v), 4) for v in two_ms]},
        "mlups": round(nodes * steps / (ms_batch * 1e-3) / 1e6, 1),
        "roofline": {"bound": "hbm", "achieved": round(ens_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ens_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_step_pass2_batch" if variant >= 0 else "k_step_tiles_batch",
                     "updates_per_launch": upl, "launch_ms_mean": round(ms_batch / launches, 5),
                     "algorithmic_bytes_per_launch": 72 * nodes,
                     "note": "compulsory bytes of one launch over every lattice (one read and one write of every "
                             "stored population, 72 B per node) over the mean launch time of the graph "
                             "replays (launch gaps inside a replay included)"},
        "batched_s": round(ms_batch * 1e-3, 3),
        "sequential": {"solves_per_s": round(count / (seq_ms_full * 1e-3), 2), "s": round(seq_ms_full * 1e-3, 2),
                       "measured_steps_per_lattice": seq_steps, "extrapolated_to": steps},
        "speedup_vs_sequential": round(seq_ms_full / ms_batch, 2),
        "nonfinite_nodes": bad,
        "tiles": {"tuner_ms_per_step": [None if np.isnan(v) else round(float(v), 4) for v in tune_ms],
                  "shape_counts": np.bincount(shapes, minlength=len(tune_ms) - 1).tolist()},
    }


CS = 1.0 / np.sqrt(3.0)


def field_errors(test, ref, iso=1.07):
    """Error of one run's (rho, ux, uy, totals) against the FP64 run's."""
    rho, ux, uy, tot = test
    r0, x0, y0, t0 = ref
    du = np.hypot(ux - x0, uy - y0)
    return {
        "rho_maxrel": float(np.abs(rho - r0).max() / np.abs(r0).max()),
        "rho_l2rel": float(np.linalg.norm(rho - r0) / np.linalg.norm(r0)),
        "u_max_over_cs": float(du.max() / CS),
        "u_l2rel": float(np.linalg.norm(du) / max(np.linalg.norm(np.hypot(x0, y0)), 1e-300)),
        "mass_rel": float(abs(tot[0] - t0[0]) / t0[0]),
        "phase_flip_frac": float(np.mean((rho > iso) != (r0 > iso))),
    }


def precision_study(steps=5000, checkpoints=(100, 500, 1000, 2000, 5000)):
    """4096x4096 spinodal lattice from one initial state with populations
    stored in FP32 and as FP16 deviations (rho_ref = mean density), both with
    FP32 arithmetic, against FP64 storage and arithmetic (the configuration
    the FP64 parity tests pin to the oracle); fields compared at checkpoints."""
    from paper_1202_6130_amd import inputs as I
    from paper_1202_6130_amd import lbm
    n = 4096
    rho0 = I.spinodal_field(n, seed=0)
    runs = {}
    for name, st in (("f64", lbm.STORE_F64), ("f32", lbm.STORE_F32), ("f16dev", lbm.STORE_F16DEV)):
        p = lbm.lbm_params_default(nx=n, ny=n, storage=st, rho_ref=float(rho0.mean()), diag_interval=0)
        runs[name] = lbm.Lattice(p, rho0)
    out = {"metric": "field error vs FP64 storage (precision study)", "n_gpus": 1, "dtype": "f32/f16dev vs f64",
           "data": "synthetic",
           "config": {"workload": "periodic 4096x4096 phase separation from seeded Gaussian-smoothed noise "
                                  "(sigma 4), 50% liquid, G=-5, tau=1, no solid", "steps": steps},
           "checkpoints": []}
    t_prev = 0
    for t in [c for c in checkpoints if c <= steps]:
        for L in runs.values():
            L.step(t - t_prev)
        t_prev = t
        ref = runs["f64"].moments()
        row = {"t": t}
        for name in ("f32", "f16dev"):
            row[name] = field_errors(runs[name].moments(), ref)
        out["checkpoints"].append(row)
        print(json.dumps({"precision_checkpoint": row}), file=sys.stderr, flush=True)
    for L in runs.values():
        L.close()
    return out


GOLDEN = os.path.join(ROOT, "tests", "golden")


def wetting(drop_steps=20000, channel_steps=600000):
    """The 1024x512 sessile drop (radius 160, seeded wall amplitudes, 20000
    steps): contact angle from the rho = 1.07 isoline, in FP32 and FP64
    storage; and the 32x256 channel driven by a body force 1e-6: slip length
    against a Poiseuille fit.  Compared with the FP64 oracle's stored results
    when tests/golden holds them."""
    import torch
    from paper_1202_6130_amd import inputs as I
    from paper_1202_6130_amd import lbm
    gr, ga = I.draw_wall_amplitudes(0)
    res = {"metric": "contact angle and slip length (wetting model)", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "sessile drop 1024x512 radius 160, 20000 steps; channel 32x256, body force 1e-6, "
                                  "600000 steps; G=-5, tau=1, wall amplitudes seed 0",
                      "G_R": float(gr[0]), "G_A": float(ga[0])}}
    gold_drop = os.path.join(GOLDEN, "drop_1024x512_fp64.json")
    gold_chan = os.path.join(GOLDEN, "channel_32x256_fp64.json")
    for name, st in (("f32", lbm.STORE_F32), ("f64", lbm.STORE_F64)):
        p = lbm.lbm_params_default(nx=1024, ny=512, storage=st, wall_kind=lbm.WALL_FLAT_SLAB, G_R=float(gr[0]),
                                   G_A=float(ga[0]), diag_interval=0)
        L = lbm.Lattice(p, I.drop_field(1024, 512, 160.0))
        torch.cuda.synchronize()
        t = time.perf_counter()
        L.step(drop_steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        ang = L.contact_angle(I.ISO, 0.0)
        rho, ux, uy, tot = L.moments()
        d = {"angle_deg": None if ang is None else float(ang[0]), "fit": None if ang is None else ang.tolist(),
             "mlups": round(1024 * 512 * drop_steps / dt / 1e6, 1), "totals": tot.tolist()}
        if os.path.exists(gold_drop):
            g = json.load(open(gold_drop))
            ys = np.array([s["y"] for s in g["samples"]]); xs = np.array([s["x"] for s in g["samples"]])
            rg = np.array([s["rho"] for s in g["samples"]])
            ug = np.hypot([s["ux"] for s in g["samples"]], [s["uy"] for s in g["samples"]])
            d["vs_oracle"] = {
                "angle_diff_deg": None if ang is None or g["contact_angle"] is None
                else float(ang[0] - g["contact_angle"][0]),
                "rho_maxrel_samples": float(np.abs(rho[ys, xs] - rg).max() / np.abs(rg).max()),
                "u_max_over_cs_samples": float(np.abs(np.hypot(ux[ys, xs], uy[ys, xs]) - ug).max() / CS),
                "mass_rel": float(abs(tot[0] - g["totals"][0]) / g["totals"][0]),
            }
        res["drop_" + name] = d
        L.close()
        p = lbm.lbm_params_default(nx=32, ny=256, storage=st, wall_kind=lbm.WALL_FLAT_SLAB, G_R=float(gr[0]),
                                   G_A=float(ga[0]), F_ext=(1e-6, 0.0), diag_interval=0)
        L = lbm.Lattice(p, I.uniform_field(32, 256, 2.0))
        t = time.perf_counter()
        L.step(channel_steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        slip = L.slip_length()
        rho, ux, uy, tot = L.moments()
        c = {"slip": slip.tolist(), "seconds": round(dt, 2)}
        if os.path.exists(gold_chan):
            g = json.load(open(gold_chan))
            prof = ux.mean(axis=1)
            c["vs_oracle"] = {"slip_rel": float(abs(slip[0] - g["slip"][0]) / abs(g["slip"][0])),
                              "ux_profile_maxrel": float(np.abs(prof - np.array(g["ux_profile"])).max()
                                                         / np.abs(g["ux_profile"]).max())}
        res["channel_" + name] = c
        L.close()
        print(json.dumps({name: [d, c]}), file=sys.stderr, flush=True)
    return res


def _serve_record(r):
    return {"rid": r.rid, "kind": r.kind, "nx": r.nx, "ny": r.ny, "arrival": r.arrival,
            "solve_s": r.finished - r.admitted, "steps": r.steps, "converged": bool(r.converged),
            "floor": bool(r.floor), "rest": bool(r.rest), "residual": r.residual,
            "value": [float(v) for v in r.value], "error": r.error}


def fifo_schedule(records):
    """Latencies of one server taking requests in arrival order, each solved
    alone for its measured solve time: finish = max(arrival, previous finish)
    + solve time.  The plain sequential baseline, rebuilt from solves that may
    have been timed in several runs."""
    free, out = 0.0, []
    for r in sorted(records, key=lambda r: (r["arrival"], r["rid"])):
        start = max(r["arrival"], free)
        free = start + r["solve_s"]
        out.append(dict(r, finished=free, latency=free - r["arrival"]))
    return out


def summarize_records(recs):
    done = [r for r in recs if not r["error"]]
    lat = np.array([r["latency"] for r in done])
    elapsed = max(r["finished"] for r in recs)
    return {"requests": len(recs), "completed": len(done), "failed": len(recs) - len(done),
            "converged": sum(r["converged"] for r in done),
            "converged_below_tol": sum(r["converged"] and not (r["floor"] or r["rest"]) for r in done),
            "converged_at_floor": sum(r["floor"] for r in done),
            "converged_at_rest": sum(r["rest"] for r in done),
            "at_step_cap": sum(not r["converged"] for r in done),
            "solves_per_s": len(done) / elapsed, "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "elapsed_s": elapsed,
            "lattice_updates": int(sum(r["steps"] * r["nx"] * r["ny"] for r in done))}


def serving(count, max_steps, seed=0, rate=20.0, max_nodes=16 << 20, tol=1e-5, legs=("continuous", "sequential"),
            part=None):
    """Served stream of contact-angle and slip-length queries (Poisson
    arrivals): continuous batching against plain sequential solves.

    The sequential leg solves the requests one at a time in arrival order; its
    latencies follow from the solve times (fifo_schedule), so it can also be
    timed in parts: part = (i, n) solves the i-th of n contiguous slices and
    returns its records, and serving_combine() joins the parts."""
    from paper_1202_6130_amd import inputs as I
    from paper_1202_6130_amd import serve
    reqs = I.request_stream(seed=seed, rate=rate, count=count)
    out = {}
    if "continuous" in legs:
        srv = serve.Server(max_steps=max_steps, tol=tol, batched=True, max_nodes=max_nodes)
        res = srv.run(reqs, realtime=True, log=sys.stderr)
        out["continuous"] = serve.summarize(res, srv.elapsed)
        out["continuous"]["two_step"] = srv.two_step
        out["continuous_records"] = [dict(_serve_record(r), finished=r.finished, latency=r.latency) for r in res]
        print(json.dumps({"continuous": out["continuous"]}), file=sys.stderr, flush=True)
    if "sequential" in legs:
        sub = reqs
        if part is not None:
            i, n = part
            sub = reqs[i * count // n:(i + 1) * count // n]
        srv = serve.Server(max_steps=max_steps, tol=tol, batched=False, max_resident=1)
        res = srv.run(sub, realtime=False, log=sys.stderr)
        out["sequential_records"] = [dict(_serve_record(r), arrival=q.arrival) for r, q in zip(res, sub)]
        out["sequential_two_step"] = srv.two_step
        if part is None:
            recs = fifo_schedule(out["sequential_records"])
            out["sequential"] = summarize_records(recs)
            out["sequential"]["two_step"] = srv.two_step
    if "continuous" in out and "sequential" in out:
        return serving_result(out["continuous"], out["sequential"], count, rate, max_steps, tol, max_nodes)
    return out


def serving_result(c, q, count, rate, max_steps, tol, max_nodes):
    return {
        "metric": "served solves/s and p50/p99 latency (contact angle + slip queries)",
        "value": round(c["solves_per_s"], 3), "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{count} requests, Poisson arrivals at {rate}/s, lattices 128x128..2048x1024 "
                               "(multiples of 32), half sessile drops (angle), half body-force channels (slip), "
                               f"until the velocity residual (relative change over 100 steps) is below {tol}, "
                               "at its binary32 floor, or at rest (rounding noise), "
                               f"or {max_steps} steps",
                   "max_resident_nodes": max_nodes},
        "continuous": c, "sequential": q,
        "p99_speedup": round(q["p99_s"] / c["p99_s"], 2) if c["p99_s"] else None,
    }


def serving_combine(paths, count, max_steps, tol, max_nodes, rate=20.0):
    """Joins a continuous run and sequential parts (JSON lines written by the
    serve workload) into the serving result."""
    c, seq, two = None, [], None
    for p in paths:
        d = json.load(open(p))
        c = d.get("continuous", c)
        seq += d.get("sequential_records", [])
        two = d.get("sequential_two_step", two)
    rids = sorted(r["rid"] for r in seq)
    if c is None or rids != list(range(count)):
        raise SystemExit("serve-combine: need one continuous run and sequential records of every request")
    q = summarize_records(fifo_schedule(seq))
    q["two_step"] = two
    return serving_result(c, q, count, rate, max_steps, tol, max_nodes)


def laplace_gamma_q21(storage, n=96, radii=(12.0, 16.0, 24.0), steps=4000):
    """Surface tension of the D2Q21 EOS fluid from pressure jumps across free
    discs (Sec. II.B's measurement): dp = p_EOS(rho_in) - p_EOS(rho_out)
    against 1/R (R from the liquid area), least-squares slope."""
    from paper_1202_6130_amd import inputs as I
    from paper_1202_6130_amd import lbm
    th = 2.0 / 3.0
    tV, tU, tL, r1, r2 = 0.25 * th, -0.25 * th, th, 0.222, 0.869     # eq. EOS, the paper's parameters

    def p_eos(r):
        p1 = r1 * tV
        return r * tV if r <= r1 else (p1 + (r - r1) * tU if r <= r2 else p1 + (r2 - r1) * tU + (r - r2) * tL)
    pts = []
    for R in radii:
        p = lbm.lbm_params_default(nx=n, ny=n, storage=storage, lattice=lbm.D2Q21, psi_kind=lbm.PSI_EOS, G=-1.0)
        L = lbm.Lattice(p, I.disc_field(n, n, R, rho_l=1.0, rho_g=0.1))
        L.step(steps)
        rho = L.moments()[0]
        L.close()
        rin = rho[n // 2 - 2:n // 2 + 2, n // 2 - 2:n // 2 + 2].mean()
        rout = rho[:3, :3].mean()
        req = np.sqrt(((rho - rout).sum() / (rin - rout)) / np.pi)
        pts.append((1.0 / req, p_eos(rin) - p_eos(rout)))
    x, y = np.array(pts).T
    return float(np.polyfit(x, y, 1)[0])


def paper_dynamic(steps=50000, dp=5.25e-4):
    """The paper's own model and geometry (Sec. III.B-C): D2Q21 (Tab. I), EOS
    pseudo-potential with G = -1, wall functions from the recursive filter of
    Appendix A with the domain's top and bottom rows as solid outer boundary,
    G_R = 1.33, G_A = 0.5, eps = 1, tau = 1, on 650x150 with a drop of radius
    50 on the lower wall.  A static run (no force) gives the equilibrium angle;
    a run driven by the largest pressure difference of Sec. III.C, applied
    across the domain length as a uniform force density dp / L_x, gives the
    advancing and receding angles, the mean drop speed U and Ca = U mu_L /
    gamma, with gamma measured in the same process from Laplace pressure
    jumps.  The step rate is the
    binary32 rate of the static run."""
    import torch
    from paper_1202_6130_amd import inputs as I
    from paper_1202_6130_amd import lbm
    nx, ny = 650, 150
    H = np.zeros((ny, nx))
    H[0, :] = 1.0
    H[ny - 1, :] = 1.0
    rho0 = I.drop_field(nx, ny, 50.0, rho_l=1.0, rho_g=0.1, slab_rows=1)
    iso = 0.55
    force = dp / nx
    res = {"metric": "MLUPS and contact angles (paper's model)", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "650x150, D2Q21, EOS psi (G=-1), recursive-filter walls (psiR=G^5, phi=G^22, "
                                  "outer rows solid), G_R=1.33, G_A=0.5, eps=1, tau=1, drop radius 50, binary32",
                      "steps": steps, "dp": dp, "force_density": force, "iso": iso, "y_ref": 0.0}}
    gamma = laplace_gamma_q21(lbm.STORE_F32)
    res["gamma"] = gamma
    for name, F in (("static", 0.0), ("driven", force)):
        p = lbm.lbm_params_default(nx=nx, ny=ny, storage=lbm.STORE_F32, wall_kind=lbm.WALL_MASK, lattice=lbm.D2Q21,
                                   psi_kind=lbm.PSI_EOS, G=-1.0, G_R=1.33, G_A=0.5, eps=1.0, tau=1.0,
                                   F_ext=(F, 0.0))
        L = lbm.Lattice(p, rho0, wall_fields=np.stack([H, H]))
        res["config"]["step_variant"] = Q21_TILE[L.tile_shape]
        L.step(100)
        torch.cuda.synchronize()
        t = time.perf_counter()
        L.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        d = {"mlups": round(nx * ny * steps / dt / 1e6, 1), "seconds": round(dt, 3)}
        if name == "static":
            ang = L.contact_angle(iso, 0.0)
            d["theta_deg"] = None if ang is None else float(ang[0])
        else:
            dyn = L.dynamic_angles(iso, 0.0)
            d["dynamic_fit"] = dyn is not None
            if dyn is not None:
                mu_l = dyn[7] * (2.0 / 3.0) * (1.0 - 0.5)
                d.update({"theta_A_deg": float(dyn[0]), "theta_R_deg": float(dyn[1]), "U": float(dyn[2]),
                          "Ca": float(dyn[2] * mu_l / gamma)})
        res[name] = d
        L.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--workload", default="spinodal4096",
                    choices=sorted(WORKLOADS) + ["ensemble256", "serve", "precision4096", "wetting1024",
                                                 "paper650x150"])
    ap.add_argument("--tile", type=int, default=None,
                    help="D2Q9 tile shape index (default: autotuned in the warm-up), or D2Q21 step variant "
                         "(default: the one a new context starts with)")
    ap.add_argument("--two-step", type=int, default=None,
                    help="D2Q9 F32/F16DEV/F64: two time steps per launch with this variant (lbm_two_step_variants), "
                         "-1 for single steps (default: autotuned in the warm-up)")
    ap.add_argument("--seq-steps", type=int, default=500, help="ensemble: steps per lattice of the sequential leg")
    ap.add_argument("--requests", type=int, default=300, help="serve: number of requests")
    ap.add_argument("--max-steps", type=int, default=1000000, help="serve: step cap per request")
    ap.add_argument("--serve-tol", type=float, default=1e-5, help="serve: residual tolerance")
    ap.add_argument("--serve-legs", default="continuous,sequential",
                    help="serve: which legs to run (continuous, sequential)")
    ap.add_argument("--serve-max-nodes", type=int, default=16 << 20, help="serve: resident lattice nodes cap")
    ap.add_argument("--serve-part", default="", help="serve, sequential leg: I/N solves the I-th of N slices")
    ap.add_argument("--serve-combine", nargs="+", default=None,
                    help="join serve JSON outputs (one continuous run, sequential parts) into the serving line "
                         "(no GPU work)")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16dev", "f64"])
    ap.add_argument("--seg-rows", type=int, default=0)
    ap.add_argument("--tau", type=float, default=1.0, help="relaxation time (the workloads are defined at 1)")
    ap.add_argument("--collision", default="bgk", choices=["bgk", "projected"],
                    help="projected: the projection step onto eq. f2 before the collision")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--trace-table", default=None,
                    help="print the kernel statistics of a rocprofv3 --kernel-trace --stats run (directory) as a "
                         "markdown table (no GPU work)")
    ap.add_argument("--counter-table", nargs="+", default=None,
                    help="print the per-kernel means of rocprofv3 --pmc runs (directories) as a markdown table, "
                         "per lattice update for --workload (no GPU work)")
    ap.add_argument("--copy-ref", action="store_true",
                    help="after timing, run one plain device copy of 1 GiB (reference dispatch for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--ingest-counters", nargs="+", metavar="DIR",
                    help="no GPU work: FETCH_DIR WRITE_DIR [VALU_DIR]: read the rocprofv3 --pmc FETCH_SIZE and "
                         "WRITE_SIZE output directories of `bench.py --copy-ref` runs on --workload/--storage (and "
                         "optionally a run that counted SQ_INSTS_VALU) and record the step kernel's HBM bytes "
                         "(and VALU instructions) per launch in --traffic-json")
    args = ap.parse_args()
    if args.ingest_counters:
        if len(args.ingest_counters) not in (2, 3):
            sys.exit("--ingest-counters FETCH_DIR WRITE_DIR [VALU_DIR]")
        fd, wd = args.ingest_counters[:2]
        vd = args.ingest_counters[2] if len(args.ingest_counters) == 3 else None
        ingest_counters(fd, wd, args.workload, args.storage, args.traffic_json, valu_dir=vd)
        return
    if args.counter_table:
        counter_table(args.counter_table, args.workload)
        return
    if args.trace_table:
        trace_table(args.trace_table)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the update is measured on a "
              "single MI355X and no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "ensemble256":
        print(json.dumps(ensemble(args.steps, args.seq_steps, two_step=args.two_step, traffic_json=args.traffic_json,
                                  copy_ref=args.copy_ref)), flush=True)
        return
    if args.serve_combine:
        print(json.dumps(serving_combine(args.serve_combine, args.requests, args.max_steps, args.serve_tol,
                                         args.serve_max_nodes)), flush=True)
        return
    if args.workload == "serve":
        part = tuple(int(v) for v in args.serve_part.split("/")) if args.serve_part else None
        print(json.dumps(serving(args.requests, args.max_steps, max_nodes=args.serve_max_nodes, tol=args.serve_tol,
                                 legs=tuple(args.serve_legs.split(",")), part=part)), flush=True)
        return
    if args.workload == "precision4096":
        print(json.dumps(precision_study()), flush=True)
        return
    if args.workload == "paper650x150":
        print(json.dumps(paper_dynamic()), flush=True)
        return
    if args.workload == "wetting1024":
        print(json.dumps(wetting()), flush=True)
        return
    coll = 1 if args.collision == "projected" else 0
    r = time_gpu(args.workload, args.storage, args.steps, args.warmup, args.seg_rows, args.tile, args.tau, coll,
                 args.two_step)
    if args.copy_ref:
        copy_reference()
    mlups = r["nodes"] * args.steps / (r["ms_total"] * 1e-3) / 1e6
    q = workload_q(args.workload)
    if q == 21 and args.storage == "f16dev":
        sys.exit("D2Q21 runs with f32 or f64 storage")
    bpu = bytes_per_update(args.storage, q)
    upl = r["updates_per_launch"]
    # compulsory HBM bytes of one launch: every stored population read once
    # and written once, whatever the number of time steps the launch takes
    compulsory = bpu * r["nodes"]
    achieved = compulsory / (r["kernel_ms_mean"] * 1e-3) / 1e9
    key = f"pass2v{r['two_step']}" if upl == 2 else r["tile_shape"]
    traffic = stored_traffic(args.traffic_json, traffic_key(args.workload, args.storage, key))
    if upl == 2:
        kernel, tile = "k_step_pass2", pass2_desc(r["two_step"])
    elif q == 9:
        kernel, tile = "k_step_tiles", tile_desc(r["tile_shape"])
    else:
        kernel, tile = q21_kernel(r["tile_shape"]), Q21_TILE[r["tile_shape"]]
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.storage, "data": "synthetic",
        "dtype_note": (("storage type of the populations; per-node arithmetic in binary32 except the momentum after "
                        "the force and the equilibrium's rest and momentum terms, formed in binary64 and rounded once "
                        "per population") if args.storage in ("f32", "f16dev") and q == 9 else
                       ("storage type of the populations; per-node arithmetic in binary32 except the momentum after "
                        "the force, formed in binary64 and rounded once") if args.storage == "f32" else
                       "storage and arithmetic type"),
        "config": {"workload": WORKLOADS[args.workload][2], "nx": WORKLOADS[args.workload][0],
                   "ny": WORKLOADS[args.workload][1], "storage": args.storage,
                   "lattice": f"D2Q{q}", "tau": args.tau, "collision": args.collision,
                   "tile": tile, "tile_tuned": args.tile is None and q == 9,
                   "tune_ms_per_shape": r["tune_ms"], "two_step_tuned": args.two_step is None and q == 9,
                   "tune_ms_per_two_step_variant_then_single": r["two_step_ms"], "diag_every": DIAG_EVERY},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_unit": "bytes per launch", "algorithmic_bytes_per_launch": compulsory,
                     "updates_per_launch": upl,
                     "kernel": kernel, "kernel_ms_mean": round(r["kernel_ms_mean"], 5),
                     "kernel_timing": f"HIP events around {r['kernel_samples']} launches on the launch stream "
                                      f"({r['kernel_samples'] - KERNEL_SAMPLES} in the timed region, every "
                                      f"{SAMPLE_EVERY}th step, and {KERNEL_SAMPLES} right after it; none with a "
                                      "diagnostic pass)",
                     "bytes_per_update": bpu},
    }
    if upl == 2:
        out["roofline"]["note"] = ("achieved = the compulsory bytes of one launch (one read and one write of every "
                                   "stored population, bytes_per_update x nodes) over its duration; the launch "
                                   "advances 2 time steps with the populations between them kept in LDS")
        # the same launch counted as two single steps' algorithmic bytes (can exceed the peak)
        out["roofline"]["equiv_single_step_gbs"] = round(upl * achieved, 1)
    valu = stored_traffic(args.traffic_json, traffic_key(args.workload, args.storage, key), "valu_insts")
    if valu is not None:
        out["roofline"]["alu"] = alu_roofline(valu, r["kernel_ms_mean"])
    if traffic is not None:
        # bytes that actually crossed to memory per second (counters), beside the algorithmic rate
        out["roofline"]["hbm_gbs_from_traffic"] = round(traffic / (r["kernel_ms_mean"] * 1e-3) / 1e9, 1)
        out["roofline"]["hbm_frac_from_traffic"] = round(out["roofline"]["hbm_gbs_from_traffic"] / HBM_PEAK_GBS, 4)
    if r["single"] is not None:
        sg = r["single"]
        s_ach = bpu * r["nodes"] / (sg["kernel_ms_mean"] * 1e-3) / 1e9
        out["single_step"] = {
            "value": round(r["nodes"] * args.steps / (sg["ms_total"] * 1e-3) / 1e6, 1), "unit": "MLUPS",
            "kernel": "k_step_tiles", "tile": tile_desc(r["tile_shape"]), "kernel_ms_mean": round(sg["kernel_ms_mean"], 5),
            "achieved": round(s_ach, 1), "frac": round(s_ach / HBM_PEAK_GBS, 4),
            "traffic": stored_traffic(args.traffic_json, traffic_key(args.workload, args.storage, r["tile_shape"])),
            "note": "the same lattice stepped one step per launch right after the timed region, same step count"}
        sv = stored_traffic(args.traffic_json, traffic_key(args.workload, args.storage, r["tile_shape"]), "valu_insts")
        if sv is not None:
            out["single_step"]["alu"] = alu_roofline(sv, sg["kernel_ms_mean"])
    out["copy_ceiling"] = copy_ceiling()
    out["copy_ceiling"]["step_fraction"] = round(achieved / out["copy_ceiling"]["value"], 4)
    out["device_copy"] = device_copy()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(q=q)
        out["cpu_baseline"]["nproc"] = os.cpu_count()
        out["cpu_baseline"]["omp"] = cpu_baseline_omp(q=q)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
