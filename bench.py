#!/usr/bin/env python
"""Throughput benchmark of the Hermite-4 block-step path on one MI355X.

One step = one whole integration of the workload from its initial
conditions: the O(N^2) initial force, block steps (predict, force, correct)
to t_end, and the energy at every multiple of dt_max. Default workload:
equal-mass Plummer sphere, N = 16384, eps = 1e-4, eta = 0.01, dt_max = 1/8,
t = 0 -> 1, FP64. Inputs are resident in device memory before the timed
region; the context and workspace are created once (gd_reinit restarts the
integration from the initial conditions inside each step).

Prints one JSON line: the metric is force pair interactions per second
(N_act * N per block step, plus N^2 for the initial force) over the timed
steps, with the energy drift, the roofline of the force kernel and the CPU
oracle timed on a bounded sample of the same workload.

Roofline: 60 flops per acceleration+jerk pair against the FP64 vector peak.
The force kernel's per-launch durations come from HIP events that record
each launch's own start and end (hipExtLaunchKernelGGL) during one more
integration of the same workload right after the timed steps; in that pass
the steps are launched directly rather than replayed from a graph (events
recorded by a captured graph cannot be timed). The kernels are the same, but
one launched from an idle GPU runs about a fifth longer than inside a replay
(rocprofv3), so the fraction reported is the lower reading. The same pass
splits the launches by block size (force_by_n_act), and the roofline line
also gives the fraction reached by the launches with N_act >= 4096.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOPS_PER_PAIR = 60
# Relative energy drift allowed per N-body time unit (the bound taken for the
# paper's Sec. 3.2 energy conservation): max_k |E_k - E_0| / |E_0| at the
# synchronised times, against 1e-6 * max(1, t_end).
DRIFT_TARGET_PER_TIME = 1e-6
# Goal for the force kernel: 60 % of the vector peak of its arithmetic (FP64 for
# the plain path, FP32 for the mixed one).
FRAC_TARGET = 0.60
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_FP32_VECTOR_TFLOPS = 157.3


def nact_histogram(counts):
    """Block steps by active-block size, {"lo-hi": steps} over the non-empty
    power-of-two bins of gd_nact_histogram."""
    out = {}
    for b, c in enumerate(counts):
        if c:
            out[str(1 << b) if b == 0 else f"{1 << b}-{(1 << (b + 1)) - 1}"] = c
    return out


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_force_plummer_n16384_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1702_00440_amd", "csrc", "gd_kernels.hip"),
                  os.path.join(ROOT, "paper_1702_00440_amd", "csrc", "gd_internal.h"),
                  os.path.join(ROOT, "paper_1702_00440_amd", "build.py")]


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def force_traffic(workload):
    """HBM bytes per force launch from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's reading), or None when
    there is none for this workload or the kernel sources changed since the
    counters were taken."""
    if workload != "plummer_n16384" or not os.path.exists(TRAFFIC_PROFILE):
        return None
    fields = {}
    for line in open(TRAFFIC_PROFILE):
        if ":" in line and line.startswith("- `"):
            k, v = line[3:].split("`", 1)[0].split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _oracle_rate(w, seconds, threads):
    """Pair interactions per second of the oracle over a bounded sample of the
    workload: its O(N^2) initial force, then block steps from t = 0 until about
    `seconds` of wall time (or t_end)."""
    import oracle
    from synth_inputs import plummer

    m, x, v = plummer(w["n"], w["seed"])
    t0 = time.perf_counter()
    s = oracle.State(m, x, v, w["eps"], w["eta"], w["dt_max"], w["dt_min"], threads=threads)
    pairs = w["n"] * w["n"]
    nsteps = 0
    while time.perf_counter() - t0 < seconds and s.t_now < w["t_end"]:
        act = s.block_step()
        pairs += len(act) * w["n"]
        nsteps += 1
    el = time.perf_counter() - t0
    sample = (f"initial O(N^2) force + first {nsteps} block steps (to t={s.t_now:.6g}) of the "
              f"same workload; {pairs:.3e} pairs in {el:.1f} s")
    return pairs / el, sample


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, seconds):
    """The oracle as it stands, on all the threads it is given (OpenMP over i)
    and on one thread (a third of the sample time), with the host's CPU model
    and CPU counts."""
    import oracle

    threads = oracle.max_threads()
    value, sample = _oracle_rate(w, seconds, threads)
    v1, sample1 = _oracle_rate(w, seconds / 3.0, 1)
    return {
        "value": value,
        "unit": "pair-interactions/s",
        "cores": threads,
        "kind": "oracle",
        "sample": sample,
        "single_thread": {"value": v1, "sample": sample1},
        "cpu_model": _cpu_model(),
        "host_cpus": os.cpu_count(),
        "usable_cpus": len(os.sched_getaffinity(0)),
    }


def full_force_imf(warmup, steps):
    """One O(N^2) force and jerk evaluation (N_act = N) of the mixed-precision
    workload's sphere (Plummer N = 262144, power-law IMF, eps 1e-4), in FP64
    and in mixed precision: the force launch of gd_reinit timed with its own
    HIP events (gd_profile_force), `steps` times after `warmup`; pair
    interactions per second, achieved FLOP/s at 60 flops per pair against
    the FP64 and FP32 vector peaks, and the largest per-particle relative
    difference of the mixed forces from the FP64 ones on the same state."""
    import torch

    from paper_1702_00440_amd import gravidy as g
    from synth_inputs import WORKLOADS, plummer_imf

    w = WORKLOADS["plummer_imf_n262144"]
    n = w["n"]
    dev = torch.device("cuda:0")
    m, x, v = plummer_imf(n, w["seed"])
    md, xd, vd = (torch.as_tensor(a).to(dev).contiguous() for a in (m, x, v))
    out, forces = {}, {}
    for mode, flags in (("fp64", 0), ("mixed", g.GD_FLAG_MIXED)):
        cl = g.Cluster(m, x, v, eta=w["eta"], eps=w["eps"], dt_max=w["dt_max"], dt_min=w["dt_min"],
                       device=dev, flags=flags)
        for _ in range(warmup):
            g.gd_reinit(cl.ctx, md, xd, vd)
        g.gd_profile_force(cl.ctx, True)
        for _ in range(steps):
            g.gd_reinit(cl.ctx, md, xd, vd)
        prof = g.gd_profile_get(cl.ctx)
        g.gd_profile_force(cl.ctx, False)
        forces[mode] = cl.state()[2:4]
        cl.close()
        sec = prof["force_ms"] / 1e3 / prof["launches"]
        tf = FLOPS_PER_PAIR * n * n / sec / 1e12
        frac = tf / (PEAK_FP64_VECTOR_TFLOPS if mode == "fp64" else PEAK_FP32_VECTOR_TFLOPS)
        out[mode] = {"pairs_per_s": n * n / sec, "kernel_ms": sec * 1e3, "launches": prof["launches"],
                     "achieved_tflops": tf, "frac_fp64_peak": tf / PEAK_FP64_VECTOR_TFLOPS,
                     "frac_fp32_peak": tf / PEAK_FP32_VECTOR_TFLOPS,
                     "frac_target": FRAC_TARGET, "frac_target_of": "fp64_peak" if mode == "fp64" else "fp32_peak",
                     "within_target": frac >= FRAC_TARGET}
    out["mixed_vs_fp64_max_rel_diff"] = {"acc": _rel_rows(forces["mixed"][0], forces["fp64"][0]),
                                         "jerk": _rel_rows(forces["mixed"][1], forces["fp64"][1])}
    out["workload"] = "plummer_imf_n262144 full force (N_act = N = 262144), eps 1e-4, seed 5"
    out["timing"] = "HIP events around each force launch (hipExtLaunchKernelGGL), average over launches"
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="plummer_n16384")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the force-launch event timing")
    ap.add_argument("--no-full-force", action="store_true",
                    help="skip the other workloads' figures of the default line (the N = 262144 full force in "
                         "FP64 and mixed, the 2^20 + 1 central-particle full force, 128-request serving)")
    ap.add_argument("--kernel-hash", action="store_true",
                    help="print the hash of the kernel sources that a counter summary is tied to")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES of device memory once (calibrates HBM byte counters)")
    ap.add_argument("--requests", type=int, default=512, help="serving: number of clusters")
    ap.add_argument("--rho", type=float, default=1.0,
                    help="serving: arrival rate as a multiple of the sequential solve rate")
    ap.add_argument("--max-clusters", type=int, default=256, help="serving: pool slots")
    ap.add_argument("--plan-sweep", action="store_true",
                    help="time the force kernel of the workload's sphere for a range of block sizes, with "
                         "gd_force's own decomposition and with every forced one (gd_force_plan); one JSON "
                         "line per block size")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default=None,
                    help="serving and central-particle workloads: pair arithmetic (default: fp64 for "
                         "serving, mixed for the central-particle workload)")
    args = ap.parse_args()
    if args.kernel_hash:
        print(kernel_sources_sha256())
        return
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU only; --gpus must be 1 "
              "(the multi-GPU split is described, not built).", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe:
        # One plain device-to-device copy of a known size: under rocprofv3
        # --pmc FETCH_SIZE / WRITE_SIZE its kernel reads the counter values that
        # correspond to copy_bytes read and written.
        nel = args.copy_probe // 8
        src = torch.arange(nel, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nel * 8, "check": float(dst[-1].item())}), flush=True)
        return

    from paper_1702_00440_amd import gravidy as g
    from synth_inputs import WORKLOADS, plummer

    if args.plan_sweep:
        plan_sweep(args)
        return
    if args.workload == "serving":
        serving_bench(args)
        return
    if args.workload == "plummer_imf_n262144":
        mixed_bench(args)
        return
    if args.workload == "plummer_bh_n1048576":
        central_bench(args)
        return

    w = WORKLOADS[args.workload]
    n, t_end, dt_max = w["n"], w["t_end"], w["dt_max"]
    dev = torch.device("cuda:0")
    m_h, x_h, v_h = plummer(n, w["seed"])
    m = torch.as_tensor(m_h).to(dev)
    x = torch.as_tensor(x_h).to(dev).contiguous()
    v = torch.as_tensor(v_h).to(dev).contiguous()
    cl = g.Cluster(m_h, x_h, v_h, eta=w["eta"], eps=w["eps"], dt_max=dt_max, dt_min=w["dt_min"], device=dev)
    ctx = cl.ctx
    n_chunks = int(round(t_end / dt_max))

    def one_step():
        g.gd_reinit(ctx, m, x, v)
        drift = 0.0
        st = None
        for k in range(1, n_chunks + 1):
            st = g.gd_step_to(ctx, k * dt_max)
            drift = max(drift, abs(st["e"] - st["e0"]) / abs(st["e0"]))
        return st, drift

    for _ in range(args.warmup):
        one_step()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    pairs = 0
    drift = 0.0
    stats = None
    marks = [ev0]
    for k in range(args.steps):
        stats, d = one_step()
        pairs += stats["pair_interactions"] + n * n
        drift = max(drift, d)
        if k + 1 < args.steps:
            e = torch.cuda.Event(enable_timing=True)
            e.record(stream)
            marks.append(e)
    ev1.record(stream)
    marks.append(ev1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    elapsed = max(wall, gpu_ms / 1e3)
    step_ms = [marks[k].elapsed_time(marks[k + 1]) for k in range(len(marks) - 1)]
    hist = nact_histogram(g.gd_nact_histogram(ctx))
    refills = g.gd_refills(ctx)  # of the last timed integration
    prof = {"force_ms": 0.0, "launches": 0, "pairs": 0}
    buckets = []
    if not args.no_profile:
        g.gd_profile_force(ctx, True)
        one_step()
        prof = g.gd_profile_get(ctx)
        buckets = g.gd_profile_buckets(ctx)
        g.gd_profile_force(ctx, False)
    by_nact = []
    for b in buckets:
        if b["launches"] == 0:
            continue
        sec = b["force_ms"] / 1e3
        tf = FLOPS_PER_PAIR * b["pairs"] / sec / 1e12 if sec > 0 else 0.0
        by_nact.append({"n_act_min": b["n_act_min"], "n_act_max": b["n_act_max"], "launches": b["launches"],
                        "avg_launch_us": sec / b["launches"] * 1e6, "pairs_per_s": b["pairs"] / sec if sec > 0 else 0.0,
                        "achieved_tflops": tf, "frac": tf / PEAK_FP64_VECTOR_TFLOPS})
    large = [b for b in by_nact if b["n_act_min"] >= 4096]
    launches = max(prof["launches"], 1)
    avg_s = prof["force_ms"] / 1e3 / launches
    flops_per_launch = FLOPS_PER_PAIR * prof["pairs"] / launches
    achieved = flops_per_launch / avg_s / 1e12 if avg_s > 0 else 0.0

    out = {
        "metric": "pair-interactions/s (acc+jerk)",
        "value": pairs / elapsed,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "step_ms": step_ms,
        "ms_per_step_median": sorted(step_ms)[len(step_ms) // 2],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}_fp64_t{t_end:g}",
            "n": n, "eps": w["eps"], "eta": w["eta"], "dt_max": dt_max, "dt_min": w["dt_min"],
            "t_end": t_end, "seed": w["seed"],
            "ic": "equal-mass Plummer sphere (Aarseth-Henon-Wielen sampling), Henon units",
        },
        "energy_drift": drift,
        "energy_drift_target": DRIFT_TARGET_PER_TIME * max(1.0, t_end),
        "energy_drift_within_target": drift <= DRIFT_TARGET_PER_TIME * max(1.0, t_end),
        "block_steps": stats["block_steps"],
        "particle_steps": stats["particle_steps"],
        "pairs_per_step": stats["pair_interactions"] + n * n,
        "n_act_histogram": hist,
        "refill_steps": refills,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP64_VECTOR_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_VECTOR_TFLOPS,
            "traffic": force_traffic(args.workload),
            "traffic_unit": "HBM bytes per launch",
            "kernel": "k_step_force<false,false,false,2> (FP64 acc+jerk of a replayed step, with its schedule check)",
            "launches": prof["launches"],
            "avg_launch_us": avg_s * 1e6,
            "flops_per_launch": flops_per_launch,
            "frac_n_act_ge_4096": large[0]["frac"] if large else None,
            "frac_target": FRAC_TARGET,
            "frac_within_target": achieved / PEAK_FP64_VECTOR_TFLOPS >= FRAC_TARGET,
            "frac_n_act_ge_4096_within_target": bool(large) and large[0]["frac"] >= FRAC_TARGET,
        },
        "force_by_n_act": by_nact,
    }
    cl.close()
    if not args.no_full_force:
        out["full_force_n262144"] = full_force_imf(1, 3)
        out["full_force_n1048577_central"] = central_full_force(1)
        sv = serving_result(128, 1.0, args.max_clusters, False)
        out["serving_requests128"] = {k: sv[k] for k in ("metric", "value", "unit", "latency_p50_s", "latency_p99_s",
                                                         "sequential", "pairs_per_s", "failed_requests", "config")}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


PLAN_SWEEP_SIZES = [1, 4, 16, 64, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048, 2560, 3072, 4096, 5000,
                    6144, 8192, 12288, 16384]


def plan_sweep(args):
    """Force-kernel time per launch against the decomposition: for each
    block size (lists of distinct random particles of the workload's sphere,
    on its initial state), gd_force's own decomposition and every forced
    one (16, 32 or 64 lanes per i; every slice count that gives a distinct
    decomposition), each timed over several launches with HIP events."""
    import numpy as np
    import torch

    from paper_1702_00440_amd import gravidy as g
    from synth_inputs import WORKLOADS, plummer

    w = WORKLOADS[args.workload]
    n = w["n"]
    m, x, v = plummer(n, w["seed"])
    cl = g.Cluster(m, x, v, eta=w["eta"], eps=w["eps"], dt_max=w["dt_max"], dt_min=w["dt_min"],
                   device="cuda:0")
    g.gd_predict(cl.ctx, 0.0)
    perm = np.random.default_rng(0).permutation(n).astype(np.int32)
    tiles = (n + 255) // 256
    slice_counts = sorted({-(-tiles // (-(-tiles // s))) for s in range(1, tiles + 1)})

    def timed(run, n_act):
        for _ in range(2):
            run()
        g.gd_profile_force(cl.ctx, True)
        reps = max(4, min(100, int(1e9 / (n_act * n))))
        for _ in range(reps):
            run()
        p = g.gd_profile_get(cl.ctx)
        g.gd_profile_force(cl.ctx, False)
        return p["force_ms"] * 1e3 / p["launches"]

    for n_act in [a for a in PLAN_SWEEP_SIZES if a <= n]:
        idx = torch.as_tensor(np.sort(perm[:n_act])).to("cuda:0")
        auto = timed(lambda: g.gd_force(cl.ctx, idx), n_act)
        forced = []
        for lanes in (16, 32, 64):
            for s in slice_counts:
                try:
                    g.gd_force_plan(cl.ctx, idx, lanes, s)
                except g.GdError as e:  # more partial sums than the workspace holds
                    if e.status != g.GD_EINVAL:
                        raise
                    continue
                us = timed(lambda: g.gd_force_plan(cl.ctx, idx, lanes, s), n_act)
                forced.append({"lanes_per_i": lanes, "slices": s, "us": us})
        best = min(forced, key=lambda r: r["us"])
        frac = lambda us: FLOPS_PER_PAIR * n_act * n / (us * 1e-6) / 1e12 / PEAK_FP64_VECTOR_TFLOPS
        print(json.dumps({"n": n, "n_act": n_act, "auto_us": auto, "auto_frac": frac(auto), "best": best,
                          "best_frac": frac(best["us"]), "forced": forced}), flush=True)
    cl.close()


def _rel_rows(a, b):
    import torch
    num = torch.linalg.vector_norm(a - b, dim=1)
    den = torch.linalg.vector_norm(b, dim=1).clamp_min(1e-300)
    return float((num / den).max())


def mixed_bench(args):
    """Full O(N^2) force and jerk of the mixed-precision workload (Plummer
    N = 262144, power-law IMF, eps 1e-4) in FP64 and in mixed precision on
    the same state: pair interactions per second of each, and the largest
    per-particle relative difference of the mixed result from the FP64 one
    (the tests bound both against the oracle)."""
    import torch

    from paper_1702_00440_amd import gravidy as g
    from synth_inputs import WORKLOADS, plummer_imf

    w = WORKLOADS["plummer_imf_n262144"]
    n = w["n"]
    dev = torch.device("cuda:0")
    m, x, v = plummer_imf(n, w["seed"])
    idx = torch.arange(n, dtype=torch.int32, device=dev)
    res = {}
    for mode, flags in (("fp64", 0), ("mixed", g.GD_FLAG_MIXED)):
        cl = g.Cluster(m, x, v, eta=w["eta"], eps=w["eps"], dt_max=w["dt_max"], dt_min=w["dt_min"],
                       device=dev, flags=flags)
        acc = torch.empty(n, 3, dtype=torch.float64, device=dev)
        jrk = torch.empty_like(acc)
        times = []
        for k in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.gd_predict(cl.ctx, 0.0)
            g.gd_force(cl.ctx, idx, acc, jrk)
            torch.cuda.synchronize()
            if k >= args.warmup:
                times.append(time.perf_counter() - t0)
        cl.close()
        t = sum(times) / len(times)
        res[mode] = {"value": n * n / t, "ms_per_step": t * 1e3, "acc": acc, "jerk": jrk}
    ra = _rel_rows(res["mixed"]["acc"], res["fp64"]["acc"])
    rj = _rel_rows(res["mixed"]["jerk"], res["fp64"]["jerk"])
    ach = {k: FLOPS_PER_PAIR * res[k]["value"] / 1e12 for k in res}
    out = {
        "metric": "pair-interactions/s (acc+jerk)",
        "value": res["mixed"]["value"],
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["mixed"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair arithmetic, f64 differences/state/accumulators",
        "data": "synthetic",
        "config": {"workload": "plummer_imf_n262144_full_force", "n": n, "eps": w["eps"], "seed": w["seed"],
                   "ic": "Plummer sphere, power-law IMF slope -2.35 on [0.1, 100], total mass 1",
                   "step": "one O(N^2) evaluation of all N (gd_predict + gd_force)"},
        "fp64": {"value": res["fp64"]["value"], "ms_per_step": res["fp64"]["ms_per_step"],
                 "achieved_tflops": ach["fp64"]},
        "mixed_vs_fp64_max_rel_diff": {"acc": ra, "jerk": rj},
        "roofline": {"bound": "alu", "achieved": ach["mixed"], "peak": PEAK_FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": ach["mixed"] / PEAK_FP32_VECTOR_TFLOPS, "traffic": None,
                     "frac_fp64_peak": ach["mixed"] / PEAK_FP64_VECTOR_TFLOPS,
                     "note": "the FP32 vector peak assumes packed FP32, which is disabled at compile time; "
                             "unpacked FP32 issues at the FP64 rate, so frac_fp64_peak is the reachable bound"},
    }
    print(json.dumps(out), flush=True)


def central_bench(args):
    """Plummer sphere of 2^20 stars plus a central particle (mass 0.01, at rest
    at the origin; eps 1e-4 between stars, 1e-6 with the central particle),
    mixed precision, block steps from dt_max = 1/8 down to dt_min = 2^-22,
    integrated to t = 1/8 (the library reports progress on stderr every
    30 s): pair interactions per second over the whole integration."""
    import torch

    from paper_1702_00440_amd import gravidy as g
    from synth_inputs import WORKLOADS, plummer_with_bh

    w = WORKLOADS["plummer_bh_n1048576"]
    dev = torch.device("cuda:0")
    m, x, v = plummer_with_bh(w["n_stars"], w["seed"], m_bh=w["m_bh"])
    n = m.shape[0]
    md, xd, vd = (torch.as_tensor(a).to(dev).contiguous() for a in (m, x, v))
    mixed = args.precision != "fp64"
    cl = g.Cluster(m, x, v, eta=w["eta"], eps=w["eps"], dt_max=w["dt_max"], dt_min=w["dt_min"], device=dev,
                   eps_bh=w["eps_bh"], bh_index=w["n_stars"], flags=g.GD_FLAG_MIXED if mixed else 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.gd_reinit(cl.ctx, md, xd, vd)
    g.gd_progress(cl.ctx, 30.0)
    n_chunks = int(round(w["t_end"] / w["dt_max"]))
    for k in range(1, n_chunks + 1):
        st = g.gd_step_to(cl.ctx, k * w["dt_max"])
        print(f"# t={st['t']:.6g} block_steps={st['block_steps']} elapsed={time.perf_counter() - t0:.1f}s",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    hist = nact_histogram(g.gd_nact_histogram(cl.ctx))
    cl.close()
    pairs = st["pair_interactions"] + n * n
    out = {
        "metric": "pair-interactions/s (acc+jerk)",
        "value": pairs / el,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": el * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32 pair arithmetic, f64 differences/state/accumulators; central pairs f64" if mixed
                  else "f64"),
        "data": "synthetic",
        "config": {"workload": f"plummer_bh_n1048577_{'mixed' if mixed else 'fp64'}_t0.125", "n": n, "eps": w["eps"],
                   "eps_bh": w["eps_bh"], "m_bh": w["m_bh"], "dt_min": w["dt_min"], "dt_max": w["dt_max"],
                   "t_end": w["t_end"]},
        "energy_drift": abs(st["e"] - st["e0"]) / abs(st["e0"]),
        "block_steps": st["block_steps"],
        "particle_steps": st["particle_steps"],
        "dtmin_clamps": st["dtmin_clamps"],
        "n_act_histogram": hist,
    }
    print(json.dumps(out), flush=True)


def serving_bench(args):
    """Continuous batching of independent Plummer clusters: N log-uniform in
    [256, 8192] (seeded), equal masses, eps 1e-4, eta 0.01, each integrated to
    t = 0.5; Poisson arrivals at rho times the sequential solve rate measured
    first on the same requests. Reports solves/s and latency percentiles for
    the pool and for sequential plain solves."""
    print(json.dumps(serving_result(args.requests, args.rho, args.max_clusters, args.precision == "mixed")),
          flush=True)


def serving_result(requests, rho, max_clusters, mixed):
    """The serving measurement of serving_bench as a dict."""
    import numpy as np
    import torch

    from paper_1702_00440_amd import gravidy as g
    from paper_1702_00440_amd import serving
    from synth_inputs import plummer

    rng = np.random.default_rng(2024)
    dev = "cuda:0"
    t_end = 0.5
    reqs = []
    for k in range(requests):
        n = int(round(np.exp(rng.uniform(np.log(256), np.log(8192)))))
        m, x, v = plummer(n, 1000 + k)
        reqs.append(serving.Request(k, 0.0, torch.as_tensor(m).to(dev), torch.as_tensor(x).to(dev).contiguous(),
                                    torch.as_tensor(v).to(dev).contiguous(), t_end))
    p = g.make_params(eta=0.01, eps=1e-4, dt_max=0.125, dt_min=2.0 ** -22,
                      flags=g.GD_FLAG_MIXED if mixed else 0)
    # warm-up: one small solve each way
    serving.serve_sequential(p, reqs[:1])
    # sequential baseline, all requests available at once
    t0 = time.perf_counter()
    seq = serving.serve_sequential(p, reqs)
    seq_wall = time.perf_counter() - t0
    seq_rate = len(reqs) / seq_wall
    lam = rho * seq_rate
    arr = np.cumsum(rng.exponential(1.0 / lam, len(reqs)))
    arr -= arr[0]
    for r, a in zip(reqs, arr):
        r.arrival = float(a)
    seq_lat = [r.latency for r in serving.serve_sequential(p, reqs)] if rho > 0 else []
    nmax = max(r.m.shape[0] for r in reqs)
    arena_bytes = g.gd_pool_arena_bytes(max_clusters, [nmax] * max_clusters)
    srv = serving.PoolServer(p, max_clusters, arena_bytes)
    srv.serve(reqs[:2])  # warm-up (graph capture)
    # capacity: every request available at t = 0
    burst = [serving.Request(r.rid, 0.0, r.m, r.x, r.v, r.t_end) for r in reqs]
    t0 = time.perf_counter()
    res_burst = srv.serve(burst)
    wall = time.perf_counter() - t0
    # latency under Poisson arrivals
    res = srv.serve(reqs)
    srv.close()
    lat = np.array([r.latency for r in res])
    pairs = sum(r.stats["pair_interactions"] for r in res_burst)
    out = {
        "metric": "serving solves/s",
        "value": len(res_burst) / wall,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair arithmetic, f64 state" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": f"serving_plummer_n256-8192_t0.5_{'mixed' if mixed else 'fp64'}", "requests": len(reqs), "rho": rho,
                   "arrival_rate_per_s": lam, "max_clusters": max_clusters, "eps": 1e-4, "eta": 0.01},
        "value_kind": "capacity: all requests queued at t=0",
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_kind": f"Poisson arrivals at rho={rho} x the sequential solve rate",
        "pairs_per_s": pairs / wall,
        "sequential": {
            "solves_per_s": seq_rate,
            "latency_p50_s": float(np.percentile(seq_lat, 50)) if seq_lat else None,
            "latency_p99_s": float(np.percentile(seq_lat, 99)) if seq_lat else None,
        },
        "failed_requests": sum(not r.ok for r in res_burst) + sum(not r.ok for r in res),
    }
    return out


def central_full_force(steps):
    """One O(N^2) force and jerk evaluation of the central-particle workload
    (2^20 Plummer stars plus the particle of mass 0.01 at the origin, eps 1e-4,
    eps_bh 1e-6 for its pairs), in mixed precision: the force launch of
    gd_reinit timed with its own HIP events, `steps` times; pair interactions
    per second and the fraction of the FP64 and FP32 vector peaks at 60 flops
    per pair."""
    import torch

    from paper_1702_00440_amd import gravidy as g
    from synth_inputs import WORKLOADS, plummer_with_bh

    w = WORKLOADS["plummer_bh_n1048576"]
    dev = torch.device("cuda:0")
    m, x, v = plummer_with_bh(w["n_stars"], w["seed"], m_bh=w["m_bh"])
    n = m.shape[0]
    md, xd, vd = (torch.as_tensor(a).to(dev).contiguous() for a in (m, x, v))
    cl = g.Cluster(m, x, v, eta=w["eta"], eps=w["eps"], dt_max=w["dt_max"], dt_min=w["dt_min"], device=dev,
                   eps_bh=w["eps_bh"], bh_index=w["n_stars"], flags=g.GD_FLAG_MIXED)
    g.gd_profile_force(cl.ctx, True)
    for _ in range(steps):
        g.gd_reinit(cl.ctx, md, xd, vd)
    prof = g.gd_profile_get(cl.ctx)
    cl.close()
    sec = prof["force_ms"] / 1e3 / prof["launches"]
    tf = FLOPS_PER_PAIR * n * n / sec / 1e12
    return {"workload": f"plummer_bh_n{n} full force (N_act = N), mixed, eps 1e-4, eps_bh 1e-6, seed {w['seed']}",
            "pairs_per_s": n * n / sec, "kernel_ms": sec * 1e3, "launches": prof["launches"],
            "achieved_tflops": tf, "frac_fp64_peak": tf / PEAK_FP64_VECTOR_TFLOPS,
            "frac_fp32_peak": tf / PEAK_FP32_VECTOR_TFLOPS,
            "timing": "HIP events around each force launch (hipExtLaunchKernelGGL), average over launches"}


if __name__ == "__main__":
    main()
