"""Benchmark: walker-steps/s of the MI355X walker on one GPU.

One benchmark step is one rms_run of the whole hot path (start, walk, signal
and moment reductions, results in host memory) over the synthetic axon
bundle: 400x400x1000 uint16 labels at 0.1 um, 300 beaded undulating tubes
(D 2 intra / 1.8 extra, kappa 0.01 um/ms), 1e7 walkers x 2e4 steps at
dt = 2e-4 ms, FP64, two gradient shapes (PGSE delta 1 / Delta 3 ms and a
cosine OGSE), 30 directions x 6 b values.  The substrate is resident in HBM
before the timed region starts.

Prints one JSON line (see the keys below) with a roofline entry for the walk
kernel (timed with HIP events on the run's stream), the CPU oracle timed on a
bounded sample of the same workload (on the host's cores, and on one core),
and the signal error of the GPU run of the oracle's walker sample against the
oracle (same seed, walkers 0..N-1).
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
    "direction": 36,          # 2 cvt + 2 fma, v_z, rho (3 + sqrt ~8), sincos 2 pi u by
                              #   table + short series ~19, 2 mul
    "face_events": 12,        # 3 x (gap select 2 + budget x |v| 1 + compare 1)
    "event_order": 13,        # 3 x (cross products mul + fma + compare) + table lookup 4
    "events": 22,             # 0.73 events/step x (neighbour index + wrap ~12, gather, compare,
                              #   flags, voxel update ~18)
    "end_point": 24,          # 3 x (closed-form end offset ~5, clamp 2, displacement 1)
    "phase_t2_counters": 9,   # 3 fma per active shape, R fma, counters
}
OPS_TOTAL = sum(OPS_PER_WALKER_STEP.values())
# MI355X VALU issue peak: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz lane-operations/s
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# MI355X HBM3E peak, GB/s
HBM_PEAK_GBPS = 8000.0

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


def walk_kernel_name(fp64: bool, c: dict, kind: str) -> str:
    """Template name of the walk kernel a run launched (``kind`` is the
    library's rms_result.walk_kernel: "persistent" is walk_seg_kernel, "one
    launch" walk_kernel)."""
    lab = "uint16" if c["labels"].dtype.itemsize == 2 or int(c["labels"].max()) >= 32 else "uint8"
    ns = int(np.asarray(c["waveform"]).reshape(-1, c["n_steps"]).shape[0])
    walker = "WalkerF64T" if fp64 else "WalkerMixedT"
    base = "walk_seg_kernel" if kind == "persistent" else "walk_kernel"
    return f"{base}<{walker}<{lab},{ns},false>> ({kind})"


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


def host_cores() -> int:
    """CPU cores this process may run on (its affinity set)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(c, sample_walkers: int, one_core_walkers: int):
    """The oracle on walkers 0..N-1 of the workload (all steps), on the host's
    cores (at most 16, the host share of one GPU), then on one core over a
    smaller sample.  Returns the bench entry and the oracle's result."""
    import oracle
    threads = min(host_cores(), 16)
    n = min(sample_walkers, c["n_walkers"])
    run = dict(seed=c["seed"], n_steps=c["n_steps"], dt=c["dt"], waveform=c["waveform"],
               dirs=c["dirs"], bvals=c["bvals"])
    t0 = time.perf_counter()
    o = oracle.run(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"], c.get("dead"),
                   n_walkers=n, n_threads=threads, **run)
    el = time.perf_counter() - t0
    n1 = min(one_core_walkers, c["n_walkers"])
    t0 = time.perf_counter()
    oracle.run(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"], c.get("dead"),
               n_walkers=n1, n_threads=1, **run)
    el1 = time.perf_counter() - t0
    entry = {"value": n * c["n_steps"] / el, "unit": "walker-steps/s", "cores": threads,
             "kind": "oracle",
             "sample": f"walkers 0..{n - 1} of the same run (all {c['n_steps']} steps), "
                       f"{el:.1f} s on {threads} threads",
             "cores_available": host_cores(),
             "value_1core": n1 * c["n_steps"] / el1,
             "sample_1core": f"walkers 0..{n1 - 1} (all steps), {el1:.1f} s on 1 thread"}
    return entry, o


def signal_error(rms, sub, c, o, prec, stream) -> dict:
    """The GPU run of the oracle's walker sample (same seed: walkers 0..N-1)
    against the oracle: max |S - S_oracle| over shapes, b values and
    directions, and the relative error of the moments."""
    n = int(o["n_walkers"])
    g = rms.rms_run(sub, seed=c["seed"], n_walkers=n, n_steps=c["n_steps"], dt=c["dt"],
                    waveform=c["waveform"], dirs=c["dirs"], bvals=c["bvals"], precision=prec,
                    stream=stream)
    rel = lambda a, b: float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
    return {"n_walkers": n,
            "max_abs_signal_err": float(np.max(np.abs(g["signal"] - o["signal"]))),
            "m2_rel_err": rel(g["m2"], o["m2"]), "m4_rel_err": rel(g["m4"], o["m4"]),
            "sum_alpha_rel_err": abs(g["sum_alpha"] - o["sum_alpha"]) / o["sum_alpha"]}


def served_substrates():
    """Sixteen resident substrates, n^3 uint16 with n = 64 ... 400 (geometric),
    alternating ellipsoid packings (cells scaled with volume) and axon bundles
    (tubes scaled with cross-section)."""
    from rms_inputs import ellipsoid_packing, axon_bundle
    out = []
    for k, n in enumerate(np.round(np.geomspace(64, 400, 16)).astype(int)):
        n = int(n)
        if k % 2 == 0:
            lab, _ = ellipsoid_packing(n=n, n_cells=max(1, round(120 * (n / 200) ** 3)),
                                       seed=100 + k)
        else:
            lab, _ = axon_bundle(n, n, n, n_axons=max(1, round(300 * (n / 400) ** 2)),
                                 seed=100 + k)
        out.append(lab)
    return out


def served_requests(n_sub, count=256, seed=5):
    """The request trace: walkers log-uniform in [1e4, 2e6], steps uniform in
    [1e3, 2e4], kappa uniform in [0, 0.05], D 2 intra / 2.5 extra, T2 80/60,
    dt 2e-4, PGSE (delta T/4, Delta 3T/4), 6-30 directions x 2-6 b values."""
    from rms_inputs import fibonacci_hemisphere, pgse
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(count):
        n_steps = int(rng.integers(1000, 20001))
        n_steps -= n_steps % 4
        dt = 2e-4
        T = n_steps * dt
        nb = int(rng.integers(2, 7))
        reqs.append(dict(sub=int(rng.integers(0, n_sub)), seed=1000 + r,
                         n_walkers=int(np.exp(rng.uniform(np.log(1e4), np.log(2e6)))),
                         n_steps=n_steps, dt=dt, kappa=float(rng.uniform(0.0, 0.05)),
                         waveform=pgse(n_steps, dt, T / 4, 3 * T / 4),
                         dirs=fibonacci_hemisphere(int(rng.integers(6, 31))),
                         bvals=np.linspace(0.0, 2.0, nb)))
    return reqs


def _tissue(n_labels, kappa):
    D = np.full(n_labels, 2.0)
    D[0] = 2.5
    T2 = np.full(n_labels, 80.0)
    T2[0] = 60.0
    k = np.zeros((n_labels, n_labels))
    k[0, 1:] = kappa
    k[1:, 0] = kappa
    return dict(D=D, kappa=k, T2=T2)


def serve(args):
    """Continuous-batching benchmark: capacity with the whole trace queued at
    once, the plain form on the same trace (each request its own rms_run, one
    after another), then Poisson arrivals at 0.7 of the capacity; latency =
    completion - arrival."""
    import torch
    import paper_2012_06478_amd as rms
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    labs = served_substrates()
    log(f"[serve] 16 substrates generated in {time.perf_counter() - t0:.1f} s "
        f"({sum(l.nbytes for l in labs) / 1e6:.0f} MB)")
    subs = []
    for lab in labs:
        L = int(lab.max()) + 1
        t = _tissue(L, 0.0)
        subs.append(rms.rms_create_substrate(lab, 0.1, t["D"], t["kappa"], t["T2"]))
    nl = [int(lab.max()) + 1 for lab in labs]
    reqs = served_requests(len(subs), args.serve_requests)
    prec = rms.RMS_MIXED if args.precision == "mixed" else rms.RMS_FP64

    def submit(srv, q):
        return rms.rms_server_submit(srv, subs[q["sub"]], seed=q["seed"],
                                     n_walkers=q["n_walkers"], n_steps=q["n_steps"], dt=q["dt"],
                                     waveform=q["waveform"], dirs=q["dirs"], bvals=q["bvals"],
                                     precision=prec, params=_tissue(nl[q["sub"]], q["kappa"]))

    rms.rms_set_option(rms.RMS_OPT_SERVER_WALKERS, int(args.serve_walkers))
    srv = rms.rms_server_create(0, 0)
    try:
        # capacity: the whole trace as one closed batch (every request queued
        # at once), so the device works on a full queue but for the drain at the end
        c0 = rms.rms_server_stats_get(srv)
        t0 = time.perf_counter()
        tk = [submit(srv, q) for q in reqs]
        for t, sh in tk:
            rms.rms_server_wait(srv, t, sh)
        cap_el = time.perf_counter() - t0
        c1 = rms.rms_server_stats_get(srv)
        cap = sum(q["n_walkers"] * q["n_steps"] for q in reqs) / cap_el
        cap_busy = (c1["busy_s"] - c0["busy_s"]) / cap_el
        log(f"[serve] capacity {cap:.3e} walker-steps/s ({len(reqs)} requests queued at once, "
            f"{cap_el:.2f} s, device busy {cap_busy:.3f})")
        # the plain form on the same trace: each request as its own rms_run, one
        # after another (what a caller without the server would do)
        t0 = time.perf_counter()
        for q in reqs:
            rms.rms_run(subs[q["sub"]], seed=q["seed"], n_walkers=q["n_walkers"],
                        n_steps=q["n_steps"], dt=q["dt"], waveform=q["waveform"], dirs=q["dirs"],
                        bvals=q["bvals"], precision=prec, params=_tissue(nl[q["sub"]], q["kappa"]))
        plain = sum(q["n_walkers"] * q["n_steps"] for q in reqs) / (time.perf_counter() - t0)
        log(f"[serve] plain rms_run, one request after another: {plain:.3e} walker-steps/s")
        work = np.array([q["n_walkers"] * q["n_steps"] for q in reqs], float)
        rate = args.serve_load * cap / work.mean()  # requests per second
        rng = np.random.default_rng(11)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(reqs)))
        log(f"[serve] {len(reqs)} requests, {work.sum():.3e} walker-steps, Poisson rate "
            f"{rate:.2f}/s over ~{arrivals[-1]:.1f} s")
        st0 = rms.rms_server_stats_get(srv)
        tickets = []
        start = time.perf_counter()
        for i, q in enumerate(reqs):
            delay = start + arrivals[i] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets.append(submit(srv, q))
            if i % 32 == 31:
                log(f"[serve] submitted {i + 1}")
        results = []
        for i, (t, sh) in enumerate(tickets):
            results.append(rms.rms_server_wait(srv, t, sh))
        end = time.perf_counter()
        st = rms.rms_server_stats_get(srv)
    finally:
        rms.rms_server_destroy(srv)
    lat = np.array([r["wall_s"] for r in results])
    queue = np.array([r["queue_s"] for r in results])
    agg = work.sum() / (end - start)
    # accuracy of the served results against the plain fp64 walk
    err = 0.0
    for i in range(0, len(reqs), max(1, len(reqs) // args.serve_check)):
        q = reqs[i]
        if q["n_walkers"] * q["n_steps"] > 4e9:
            continue
        ref = rms.rms_run(subs[q["sub"]], seed=q["seed"], n_walkers=q["n_walkers"],
                          n_steps=q["n_steps"], dt=q["dt"], waveform=q["waveform"],
                          dirs=q["dirs"], bvals=q["bvals"], precision=rms.RMS_FP64,
                          params=_tissue(nl[q["sub"]], q["kappa"]))
        err = max(err, float(np.max(np.abs(ref["signal"] - results[i]["signal"]))))
    for s_ in subs:
        s_.close()
    line = {
        "metric": "served walker-steps/s", "value": agg, "unit": "walker-steps/s",
        "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
        "dtype": "f32+i32 walk, f64 sums" if prec == rms.RMS_MIXED else "f64",
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "p50_queue_s": float(np.percentile(queue, 50)),
        "p99_queue_s": float(np.percentile(queue, 99)),
        "capacity_walker_steps_per_s": cap, "capacity_device_busy_frac": cap_busy,
        "plain_sequential_walker_steps_per_s": plain,
        "offered_load": args.serve_load,
        "device_busy_frac": (st["busy_s"] - st0["busy_s"]) / (end - start),
        "launches": st["launches"] - st0["launches"],
        "max_signal_err_vs_fp64": err,
        "config": {"workload": "16 resident substrates 64^3..400^3 u16, "
                               f"{len(reqs)} Poisson requests", "precision": args.precision,
                   "server_walkers": int(args.serve_walkers) or "auto"},
    }
    print(json.dumps(line), flush=True)


def precision_report(args):
    """The mixed-precision form against the fp64 form on the same inputs (the
    fp64 form matches the oracle walker by walker): error per b value, per
    direction and per moment, and both throughputs."""
    import torch
    import paper_2012_06478_amd as rms
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    log(f"[precision] building workload {args.workload}")
    c = workload(args.workload)
    sub = rms.rms_create_substrate(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"],
                                   c.get("dead"))
    run = dict(seed=c["seed"], n_walkers=c["n_walkers"], n_steps=c["n_steps"], dt=c["dt"],
               waveform=c["waveform"], dirs=c["dirs"], bvals=c["bvals"])
    out = {}
    for name, prec in (("fp64", rms.RMS_FP64), ("mixed", rms.RMS_MIXED)):
        r = rms.rms_run(sub, precision=prec, **run)
        out[name] = r
        log(f"[precision] {name}: {r['wall_s']:.2f} s, walk kernel {r['kernel_ms']:.0f} ms")
    sub.close()
    a, b = out["fp64"], out["mixed"]
    dS = np.abs(a["signal"] - b["signal"])  # [shape][b][dir]
    ws = c["n_walkers"] * c["n_steps"]
    line = {
        "metric": "mixed-precision error vs fp64", "workload": c["name"],
        "n_walkers": c["n_walkers"], "n_steps": c["n_steps"],
        "max_abs_signal_err": float(dS.max()),
        "max_abs_signal_err_per_b": [float(x) for x in dS.max(axis=(0, 2))],
        "max_abs_signal_err_per_dir": [float(x) for x in dS.max(axis=(0, 1))],
        "bvals": [float(x) for x in c["bvals"]],
        "m2_rel_err": [float(x) for x in np.abs(a["m2"] - b["m2"]) / np.max(np.abs(a["m2"]))],
        "m4_rel_err": [float(x) for x in np.abs(a["m4"] - b["m4"]) / np.max(np.abs(a["m4"]))],
        "D_rel_err_max": float(np.max(np.abs(a["D"] - b["D"]) / np.abs(a["D"]))),
        "K_abs_err_max": float(np.max(np.abs(a["K"] - b["K"]))),
        "sum_alpha_rel_err": abs(a["sum_alpha"] - b["sum_alpha"]) / a["sum_alpha"],
        "fp64_walker_steps_per_s": ws / a["wall_s"],
        "mixed_walker_steps_per_s": ws / b["wall_s"],
        "fp64_kernel_ms": a["kernel_ms"], "mixed_kernel_ms": b["kernel_ms"],
    }
    print(json.dumps(line), flush=True)


def record_report(args):
    """Time dependence of D and K (section 2.3): the workload with its moments
    recorded at ``--records`` equally spaced steps, against the same run without
    records (the end results are identical; the recorded run walks one launch
    per interval and reduces the moments at each record step)."""
    import torch
    import paper_2012_06478_amd as rms
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    log(f"[records] building workload {args.workload}")
    c = workload(args.workload)
    prec = rms.RMS_FP64 if args.precision == "fp64" else rms.RMS_MIXED
    sub = rms.rms_create_substrate(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"],
                                   c.get("dead"))
    n = c["n_steps"]
    steps = np.unique(np.linspace(n / args.records, n, args.records).round().astype(np.int64))
    run = dict(seed=c["seed"], n_walkers=c["n_walkers"], n_steps=n, dt=c["dt"],
               waveform=c["waveform"], dirs=c["dirs"], bvals=c["bvals"], precision=prec)
    rms.rms_run(sub, **run)  # warm-up of both paths
    rms.rms_run_record(sub, record_steps=steps, **run)
    plain = [rms.rms_run(sub, **run) for _ in range(args.steps)]
    recd = [rms.rms_run_record(sub, record_steps=steps, **run) for _ in range(args.steps)]
    sub.close()
    ws = c["n_walkers"] * n
    wall_p = min(r["wall_s"] for r in plain)
    wall_r = min(r["wall_s"] for r in recd)
    rr = recd[0]["records"]
    line = {
        "metric": "recorded walker-steps/s", "value": ws / wall_r, "unit": "walker-steps/s",
        "higher_is_better": True, "data": "synthetic", "workload": c["name"],
        "precision": args.precision, "n_records": int(steps.size),
        "plain_walker_steps_per_s": ws / wall_p,
        "kernel_ms_recorded": min(r["kernel_ms"] for r in recd),
        "kernel_ms_plain": min(r["kernel_ms"] for r in plain),
        "end_results_identical": bool(np.array_equal(recd[0]["signal"], plain[0]["signal"])
                                      and np.array_equal(recd[0]["m2"], plain[0]["m2"])),
        "t_ms": [float(x) for x in steps[:: max(1, steps.size // 10)] * c["dt"]],
        "D_dir0": [float(x) for x in rr["D"][:: max(1, steps.size // 10), 0]],
        "K_dir0": [float(x) for x in rr["K"][:: max(1, steps.size // 10), 0]],
    }
    if c["name"].startswith("axons"):
        line.update(bundle_report(rms, recd[0], steps * c["dt"], c))
    print(json.dumps(line), flush=True)


def bundle_report(rms, r, t, c):
    """Along and across the axon bundle (its axes run near z): D_par(t) =
    M2_zz / 2t, D_perp(t) = (M2_xx + M2_yy) / 4t and K_par(t) = M4_zzzz /
    M2_zz^2 - 3 from the recorded moments (section 2.3); from the end signal
    of each waveform shape, the direction average over b (the spherical mean)
    and the cumulant fit of ln S(b) over b <= 1 ms/um^2 for the directions
    nearest to and farthest from z."""
    m2, m4 = r["records"]["m2"], r["records"]["m4"]
    k = max(1, t.size // 10)
    gz = np.abs(np.asarray(c["dirs"])[:, 2])
    out = {"bundle_t_ms": [float(x) for x in t[::k]],
           "D_par": [float(x) for x in (m2[:, 5] / (2 * t))[::k]],
           "D_perp": [float(x) for x in ((m2[:, 0] + m2[:, 3]) / (4 * t))[::k]],
           "K_par": [float(x) for x in (m4[:, 14] / m2[:, 5] ** 2 - 3.0)[::k]],
           "spherical_mean": [], "fit_D_par": [], "fit_K_par": [], "fit_D_perp": [],
           "fit_K_perp": []}
    for sig in r["signal"]:
        out["spherical_mean"].append([float(x.real) for x in rms.rms_spherical_mean(sig)])
        D, K = rms.rms_cumulant_fit(sig, c["bvals"], 1.0)
        out["fit_D_par"].append(float(D[np.argmax(gz)]))
        out["fit_K_par"].append(float(K[np.argmax(gz)]))
        out["fit_D_perp"].append(float(D[np.argmin(gz)]))
        out["fit_K_perp"].append(float(K[np.argmin(gz)]))
    return out


def mt_report(args):
    """Absorbing membranes (magnetization transfer, end of section 2.1.3): the
    workload with every cell absorbing at its faces to the extracellular label
    (surface relaxivity ``--mt`` um/ms, both sides), against the same run
    without; reports both throughputs and the weight lost to saturation."""
    import torch
    import paper_2012_06478_amd as rms
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    log(f"[mt] building workload {args.workload}")
    c = workload(args.workload)
    prec = rms.RMS_FP64 if args.precision == "fp64" else rms.RMS_MIXED
    sub = rms.rms_create_substrate(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"],
                                   c.get("dead"))
    L = len(c["D"])
    rho = np.zeros((L, L))
    rho[1:, 0] = args.mt
    rho[0, 1:] = args.mt
    P = dict(D=c["D"], kappa=c["kappa"], T2=c["T2"], rho=rho)
    run = dict(seed=c["seed"], n_walkers=c["n_walkers"], n_steps=c["n_steps"], dt=c["dt"],
               waveform=c["waveform"], dirs=c["dirs"], bvals=c["bvals"], precision=prec)
    rms.rms_run(sub, **run)  # warm-up of both paths
    rms.rms_run(sub, params=P, **run)
    plain = [rms.rms_run(sub, **run) for _ in range(args.steps)]
    mt = [rms.rms_run(sub, params=P, **run) for _ in range(args.steps)]
    sub.close()
    ws = c["n_walkers"] * c["n_steps"]
    line = {
        "metric": "walker-steps/s with absorbing membranes", "unit": "walker-steps/s",
        "value": ws / min(r["wall_s"] for r in mt), "higher_is_better": True,
        "data": "synthetic", "workload": c["name"], "precision": args.precision,
        "rho_um_per_ms": args.mt,
        "plain_walker_steps_per_s": ws / min(r["wall_s"] for r in plain),
        "kernel_ms_mt": min(r["kernel_ms"] for r in mt),
        "kernel_ms_plain": min(r["kernel_ms"] for r in plain),
        "weight_kept": mt[0]["sum_alpha"] / plain[0]["sum_alpha"],
        "S_b_max_dir0_mt": [float(mt[0]["signal"][0, -1, 0].real),
                            float(mt[0]["signal"][0, -1, 0].imag)],
    }
    print(json.dumps(line), flush=True)


def conc_report(args):
    """Unequal spin concentrations (App. C, general case): the workload with
    the extracellular label at concentration ``--conc`` relative to 1 in the
    cells (printed closed-form lambda; ``--baxter`` for Baxter's rule on the
    same membranes), against the same run without; reports both throughputs
    and the walker share that starts and ends in the cells."""
    import torch
    import paper_2012_06478_amd as rms
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    log(f"[conc] building workload {args.workload}")
    c = workload(args.workload)
    prec = rms.RMS_FP64 if args.precision == "fp64" else rms.RMS_MIXED
    sub = rms.rms_create_substrate(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"],
                                   c.get("dead"))
    L = len(c["D"])
    conc = np.ones(L)
    conc[0] = args.conc
    P = dict(D=c["D"], kappa=c["kappa"], T2=c["T2"], conc=conc, lam=-1.0,
             perm_model=rms.RMS_PERM_BAXTER if args.baxter else rms.RMS_PERM_KAPPA)
    run = dict(seed=c["seed"], n_walkers=c["n_walkers"], n_steps=c["n_steps"], dt=c["dt"],
               waveform=c["waveform"], dirs=c["dirs"], bvals=c["bvals"], precision=prec)
    rms.rms_run(sub, **run)  # warm-up of both paths
    rms.rms_run(sub, params=P, **run)
    plain = [rms.rms_run(sub, **run) for _ in range(args.steps)]
    wc = [rms.rms_run(sub, params=P, **run) for _ in range(args.steps)]
    d = rms.rms_run(sub, params=P, dump=True, **run)["dump"]
    sub.close()
    lab = c["labels"]
    vin = float(np.sum(lab > 0))
    want = vin / (vin + args.conc * float(np.sum(lab == 0)))
    ws = c["n_walkers"] * c["n_steps"]
    line = {
        "metric": "walker-steps/s with spin concentrations", "unit": "walker-steps/s",
        "value": ws / min(r["wall_s"] for r in wc), "higher_is_better": True,
        "data": "synthetic", "workload": c["name"], "precision": args.precision,
        "conc_extra": args.conc, "perm_model": "baxter" if args.baxter else "kappa",
        "plain_walker_steps_per_s": ws / min(r["wall_s"] for r in plain),
        "kernel_ms_conc": min(r["kernel_ms"] for r in wc),
        "kernel_ms_plain": min(r["kernel_ms"] for r in plain),
        "share_in_cells_expected": want,
        "share_in_cells_start": float(np.mean(d[:, 11] > 0)),
        "share_in_cells_end": float(np.mean(d[:, 4] > 0)),
        "permeations": int(wc[0]["n_permeations"]),
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64")
    ap.add_argument("--workload", choices=WORKLOADS, default="axons")
    ap.add_argument("--walkers", type=int, default=0,
                    help="walker count in place of the workload's (the plain benchmark only)")
    ap.add_argument("--walk-kernel", choices=("auto", "one", "persistent"), default="auto",
                    help="walk kernel (rms_set_option RMS_OPT_WALK_KERNEL; auto is the library's "
                         "choice), for measurements of the launch paths")
    ap.add_argument("--cpu-sample-walkers", type=int, default=250_000)
    ap.add_argument("--cpu-1core-walkers", type=int, default=2_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision-report", action="store_true",
                    help="mixed vs fp64 on the same inputs: error per b, direction, moment")
    ap.add_argument("--serve", action="store_true",
                    help="continuous-batching benchmark over a Poisson request trace")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-load", type=float, default=0.7)
    ap.add_argument("--serve-walkers", type=float, default=0,
                    help="walker slots of the server (rms_set_option RMS_OPT_SERVER_WALKERS; "
                         "0: the library's automatic cap)")
    ap.add_argument("--serve-check", type=int, default=8,
                    help="requests re-run in fp64 to report the served signal error")
    ap.add_argument("--records", type=int, default=0,
                    help="time series of D and K: record the moments at this many steps and "
                         "report the recorded run's throughput against the plain one")
    ap.add_argument("--mt", type=float, default=0.0,
                    help="absorbing membranes: surface relaxivity (um/ms) of every cell face; "
                         "reports the run against the plain one")
    ap.add_argument("--conc", type=float, default=0.0,
                    help="spin concentration of the extracellular label (cells: 1); reports "
                         "the run against the plain one")
    ap.add_argument("--baxter", action="store_true",
                    help="with --conc: Baxter's permeation rule on the same membranes")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device copy (3 times), to scale the "
                         "FETCH_SIZE/WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the walk needs no communication, and each "
              "GPU would run the same kernel on its own share of walkers.", file=sys.stderr)
        sys.exit(2)

    if args.precision_report:
        precision_report(args)
        return
    if args.records > 0:
        record_report(args)
        return
    if args.mt > 0:
        mt_report(args)
        return
    if args.conc > 0:
        conc_report(args)
        return
    if args.serve:
        if args.precision == "fp64" and "--precision" not in sys.argv:
            args.precision = "mixed"  # the served form runs the mixed-precision walk
        serve(args)
        return

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
    if args.walk_kernel != "auto":
        rms.rms_set_option(rms.RMS_OPT_WALK_KERNEL, rms.RMS_WALK_ONE_LAUNCH
                           if args.walk_kernel == "one" else rms.RMS_WALK_PERSISTENT)
    c = workload(args.workload)
    default_walkers = c["n_walkers"]
    if args.walkers:
        c["n_walkers"] = args.walkers
    prec = rms.RMS_FP64 if args.precision == "fp64" else rms.RMS_MIXED
    # the process's first device allocation sets up the device's memory (about
    # 0.15 s, once): a tiny substrate takes it before the timed creation
    rms.rms_create_substrate(np.zeros((2, 2, 2), np.uint8), c["voxel_um"], [2.0]).close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sub = rms.rms_create_substrate(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"],
                                   c.get("dead"))
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    log(f"[bench] substrate resident ({c['labels'].nbytes / 1e6:.1f} MB) in {create_s:.2f} s")
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
    traffic = (traffic_from_profile(c["name"], args.precision)
               if c["n_walkers"] == default_walkers and args.walk_kernel == "auto" else None)
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
        "dtype": "f64" if prec == rms.RMS_FP64 else "f32+i32 walk, f64 sums",
        "data": "synthetic",
        "config": {"workload": c["name"], "n_walkers": c["n_walkers"], "n_steps": c["n_steps"],
                   "dt_ms": c["dt"], "voxel_um": c["voxel_um"], "n_labels": int(c["D"].size),
                   "n_signals": int(c["waveform"].shape[0] * len(c["bvals"]) * len(c["dirs"])),
                   "precision": args.precision},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS,
                     "traffic": traffic,
                     # the same launch's HBM bytes over its time, against the HBM peak
                     "hbm": (None if traffic is None else
                             {"achieved": traffic / kernel_s / 1e9, "peak": HBM_PEAK_GBPS,
                              "unit": "GB/s", "frac": traffic / kernel_s / 1e9 / HBM_PEAK_GBPS}),
                     "kernel": walk_kernel_name(prec == rms.RMS_FP64, c, r["walk_kernel"]),
                     "kernel_ms": kernel_s * 1e3, "ops_per_walker_step": OPS_TOTAL},
        # the labels come from host memory: one run together with its substrate's
        # creation (host padding, upload over PCIe) is the rate of a single job
        "substrate_create_s": create_s,
        "one_run_with_substrate_upload": ws / (create_s + el / args.steps),
        "last_signal_b_max_dir0": [float(r["signal"][0, -1, 0].real),
                                   float(r["signal"][0, -1, 0].imag)],
    }
    if not args.no_cpu_baseline:
        log(f"[bench] timing the CPU oracle on {args.cpu_sample_walkers} walkers "
            f"({min(host_cores(), 16)} threads) and {args.cpu_1core_walkers} walkers (1 thread)")
        line["cpu_baseline"], o = cpu_baseline(c, args.cpu_sample_walkers, args.cpu_1core_walkers)
        o["n_walkers"] = min(args.cpu_sample_walkers, c["n_walkers"])
        sub = rms.rms_create_substrate(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"],
                                       c.get("dead"))
        line["signal_err_vs_oracle"] = signal_error(rms, sub, c, o, prec, stream)
        sub.close()
        log(f"[bench] signal error vs oracle: {line['signal_err_vs_oracle']}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
