"""Benchmark: walker-steps/s of the MI355X walker on one GPU.

One benchmark step is one rms_run of the whole hot path (start, walk, signal
and moment reductions, results in host memory) over the permeable ellipsoid
packing: 200^3 uint16 labels at 0.1 um, 120 cells (D 2 intra / 2.5 extra,
kappa 0.02 um/ms, T2 80/60 ms), 1e6 walkers x 1e4 steps at dt = 2e-4 ms, PGSE
(delta 0.5, Delta 1.5 ms), 30 directions x 6 b values.  The substrate is
resident in HBM before the timed region starts.

Prints one JSON line (see the keys below) with a roofline entry for the walk
kernel (timed with HIP events on the run's stream) and the CPU oracle timed on
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic VALU lane-operations of one walker-step of the double-precision
# walk (the per-unit work of the roofline), counted as the instructions an
# ideal gfx950 implementation of the method needs:
OPS_PER_WALKER_STEP = {
    "philox_half_block": 40,  # 10 rounds x (2 mul_lo + 2 mul_hi + 4 xor) / 2 steps per block
    "direction": 50,          # 2 cvt + 2 fma, v_z, rho (3 + sqrt ~8), sincospi ~33, 2 mul
    "face_distances": 36,     # 3 x (gap select/sub/max 4 + |v| 1 + divide ~7)
    "event_order": 9,         # 3 compare-and-swap
    "events": 22,             # 0.73 events/step x (neighbour index + wrap ~12, gather, compare,
                              #   flags, voxel update ~18)
    "end_point": 24,          # 3 x (closed-form end offset ~5, clamp 2, displacement 1)
    "phase_t2_counters": 9,   # 3 fma per active shape, R fma, counters
}
OPS_TOTAL = sum(OPS_PER_WALKER_STEP.values())
# MI355X VALU issue peak: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz lane-operations/s
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

WORKLOADS = ("ellipsoids200", "cylinder32", "axons")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(name):
    from rms_inputs import configs
    if name == "ellipsoids200":
        return configs.ellipsoid_case()
    if name == "cylinder32":
        return configs.cylinder_case()
    if name == "axons":
        return configs.axon_case()
    raise ValueError(name)


def kernel_sha() -> str:
    h = hashlib.sha256()
    for f in ("rms_walk.hip", "rms_device.h", "rms_internal.h"):
        with open(os.path.join(ROOT, "paper_2012_06478_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(name: str, precision: str):
    """HBM bytes per launch of the walk kernel, from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"walk_{precision}_{name}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_sha") != kernel_sha():
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(c, sample_walkers: int):
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    n = min(sample_walkers, c["n_walkers"])
    t0 = time.perf_counter()
    oracle.run(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"], c.get("dead"),
               seed=c["seed"], n_walkers=n, n_steps=c["n_steps"], dt=c["dt"],
               waveform=c["waveform"], dirs=c["dirs"], bvals=c["bvals"], n_threads=threads)
    el = time.perf_counter() - t0
    return {"value": n * c["n_steps"] / el, "unit": "walker-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"walkers 0..{n - 1} of the same run (all {c['n_steps']} steps), "
                      f"{el:.1f} s on {threads} threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64")
    ap.add_argument("--workload", choices=WORKLOADS, default="ellipsoids200")
    ap.add_argument("--cpu-sample-walkers", type=int, default=250_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device copy (3 times), to scale the "
                         "FETCH_SIZE/WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the walk needs no communication, and each "
              "GPU would run the same kernel on its own share of walkers.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2012_06478_amd as rms

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.calibrate_copy:
        a = torch.ones(2**30 // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] copied 1 GiB three times")
        return
    log(f"[bench] building workload {args.workload}")
    c = workload(args.workload)
    prec = rms.RMS_FP64 if args.precision == "fp64" else rms.RMS_MIXED
    t0 = time.perf_counter()
    sub = rms.rms_create_substrate(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"],
                                   c.get("dead"))
    torch.cuda.synchronize()
    log(f"[bench] substrate resident ({c['labels'].nbytes / 1e6:.1f} MB) in "
        f"{time.perf_counter() - t0:.2f} s")
    run = dict(seed=c["seed"], n_walkers=c["n_walkers"], n_steps=c["n_steps"], dt=c["dt"],
               waveform=c["waveform"], dirs=c["dirs"], bvals=c["bvals"], precision=prec,
               stream=stream)
    for i in range(args.warmup):
        r = rms.rms_run(sub, **run)
        log(f"[bench] warmup {i}: {r['wall_s']:.3f} s, walk kernel {r['kernel_ms']:.1f} ms")
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = rms.rms_run(sub, **run)
        kms.append(r["kernel_ms"])
        log(f"[bench] step {i}: {r['wall_s']:.3f} s, walk kernel {r['kernel_ms']:.1f} ms")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sub.close()
    ws = c["n_walkers"] * c["n_steps"]
    value = ws * args.steps / el
    kernel_s = float(np.mean(kms)) / 1e3
    achieved = OPS_TOTAL * ws / kernel_s / 1e12
    line = {
        "metric": "walker-steps/s",
        "value": value,
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == rms.RMS_FP64 else "f32+i32 walk, f64 reductions",
        "data": "synthetic",
        "config": {"workload": c["name"], "n_walkers": c["n_walkers"], "n_steps": c["n_steps"],
                   "dt_ms": c["dt"], "voxel_um": c["voxel_um"], "n_labels": int(c["D"].size),
                   "n_signals": int(c["waveform"].shape[0] * len(c["bvals"]) * len(c["dirs"])),
                   "precision": args.precision},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS,
                     "traffic": traffic_from_profile(c["name"], args.precision),
                     "kernel": "walk_fp64_kernel" if prec == rms.RMS_FP64 else "walk_mixed_kernel",
                     "kernel_ms": kernel_s * 1e3, "ops_per_walker_step": OPS_TOTAL},
        "last_signal_b_max_dir0": [float(r["signal"][0, -1, 0].real),
                                   float(r["signal"][0, -1, 0].imag)],
    }
    if not args.no_cpu_baseline:
        log(f"[bench] timing the CPU oracle on {args.cpu_sample_walkers} walkers")
        line["cpu_baseline"] = cpu_baseline(c, args.cpu_sample_walkers)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
