"""Benchmark: electron real collisions/s and secondaries/s of microscopic
avalanche transport on one MI355X, on the argon-like gas at gain ~1e3
(1000 avalanches of one primary electron each, 128 um gap, 40 kV/cm).

One step = one complete avalanche simulation of the whole batch (every
electron carried to termination, statistics reduced), primaries already
resident in HBM.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic VALU work per event, in lane operations (the minimum the
# method performs per flight / real collision / ionisation / endpoint; see the
# design notes for the derivation).  Peak: 256 CUs x 4 SIMD16 x 2.4 GHz x 16
# lanes = 3.93e13 lane-ops/s (FP64 FMA counted as one op).
OPS_PER_FLIGHT = 150
OPS_PER_REAL = 220
OPS_PER_ION = 280
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9

# Oracle samples per workload (avalanche ids divisible by the modulus, which
# replay exactly on their own): about 5-30 s on the host cores.  Electron
# capacity per workload.
# Band lookahead of the banded majorant (mean free times), headline and
# CPU baseline alike.
BAND_LOOKAHEAD = 1.0

CPU_MODULUS = {"toy": 1, "argon": 1, "batched": 64, "highgain": 16, "wire": 128, "penning": 4}
CAPACITY = {"toy": 2_000_000, "argon": 16_000_000, "batched": 200_000_000,
            "highgain": 60_000_000, "wire": 90_000_000, "penning": 40_000_000}

# HBM traffic of the transport kernel from two counter passes (FETCH_SIZE,
# WRITE_SIZE per dispatch), valid only for the kernel sources it was taken on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_persistent_argon1000_fp64_banded.json")
KERNEL_SOURCES = ("paper_2509_15377_amd/csrc/avm_kernels.hip",
                  "paper_2509_15377_amd/csrc/avm_device.hpp",
                  "paper_2509_15377_amd/csrc/avm_internal.hpp")


def kernel_source_digest():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the headline kernel, or None when the counters
    were taken on other kernel sources (or never)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_digest():
        return None
    return (t["fetch_kib_per_dispatch"] * t["fetch_scale"]
            + t["write_kib_per_dispatch"] * t["write_scale"]) * 1024.0


def copy_probe():
    """A plain device copy of known size, for scaling the HBM byte counters
    (run under rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE)."""
    import torch
    n = 1 << 28
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n}), flush=True)


def side_legs(args, make, timed, paths, gas, field, wl, capacity, stream):
    """The majorant lever on its own (same batched kernel, global majorant),
    and the headline path with primaries handed over in host memory (their
    copy to HBM then sits inside every step)."""
    from paper_2509_15377_amd import avm
    gr = make(avm.BATCHED, avm.GLOBAL, graph=not args.eager)
    gw, gk = timed(gr)
    gc = gr.counts()
    gms = gw * 1e3 / args.steps
    gfl = gc["n_real"] + gc["n_null"] + gc["n_masked"]
    paths["batched_fp64_global"] = {
        "real_collisions_per_s": gc["n_real"] / (gms * 1e-3),
        "secondaries_per_s": gc["n_ion"] / (gms * 1e-3),
        "flights_per_s": gfl / (gms * 1e-3),
        "ms_per_step": gms, "kernel_ms": sum(gk) / len(gk),
        "null_fraction": (gc["n_null"] + gc["n_masked"]) / max(gfl, 1)}
    gr.close()
    hr = avm.Run(gas, field, wl.primaries, wl.n_aval, seed=wl.seed, majorant=avm.BANDED,
                 mode=avm.BATCHED, capacity=capacity, timeout_s=300.0, stream=stream,
                 band_lookahead=BAND_LOOKAHEAD)
    hw, _ = timed(hr)
    hms = hw * 1e3 / args.steps
    paths["batched_fp64_banded_host_primaries"] = {
        "real_collisions_per_s": hr.counts()["n_real"] / (hms * 1e-3), "ms_per_step": hms}
    hr.close()
    # the headline path with the induced signal on (240 bins of 5 ps)
    sr = make(avm.BATCHED, avm.BANDED, graph=not args.eager)
    sr.set_signal(0.0, 0.005, 240)
    sw, sk = timed(sr)
    sms = sw * 1e3 / args.steps
    paths["batched_fp64_banded_signal"] = {
        "real_collisions_per_s": sr.counts()["n_real"] / (sms * 1e-3), "ms_per_step": sms,
        "kernel_ms": sum(sk) / len(sk), "signal_bins": 240}
    sr.close()


def crossover():
    """Wall time of one whole simulation against the number of avalanches
    (argon-like gas, one primary each): the GPU (batched, banded, FP64,
    primaries handed over in host memory, from execute to sync) against the
    oracle on every host core; the paper reports where the GPU overtakes the
    CPU (Sec. 4).  Prints one JSON line (not the benchmark line)."""
    import numpy as np
    import torch

    from oracle import oracle as O
    from paper_2509_15377_amd import avm, workloads as W

    full = W.argon(1024, band_bins=100)
    gas = avm.Gas(full.gas, 0)
    field = avm.Field(full.field, 0)
    og = O.Gas(full.gas, band_bins=100)
    of = O.Field(full.field)
    rows = []
    for n in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024):
        prim = full.primaries[:n]
        r = avm.Run(gas, field, prim, n, seed=full.seed, majorant=avm.BANDED, capacity=20_000_000,
                    timeout_s=120.0, band_lookahead=BAND_LOOKAHEAD)
        r.execute()
        r.sync()
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            r.execute()
            r.sync()
            ts.append(time.perf_counter() - t0)
        electrons = r.counts()["n_endpoints"]
        r.close()
        t1 = time.perf_counter()
        O.run(og, of, prim, full.seed, banded=True, band_lookahead=BAND_LOOKAHEAD)
        tc = time.perf_counter() - t1
        rows.append({"avalanches": n, "electrons": int(electrons), "gpu_s": float(np.median(ts)),
                     "oracle_s": tc})
    cross = next((r["avalanches"] for r in rows if r["gpu_s"] < r["oracle_s"]), None)
    print(json.dumps({"crossover": rows, "gpu_faster_from_avalanches": cross}), flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="argon")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-mode reference leg")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32-mixed leg")
    ap.add_argument("--eager", action="store_true",
                    help="launch the batched run eagerly instead of replaying its HIP graph")
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the headline path (for counter passes)")
    ap.add_argument("--crossover", action="store_true",
                    help="only measure the CPU/GPU crossover in the number of avalanches")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.crossover:
        crossover()
        return
    if args.headline_only:
        args.no_mixed = args.no_plain = args.no_cpu = True
    if args.workload != "argon":
        args.no_plain = True  # the generation loop on the global majorant: minutes
    import numpy as np
    import torch

    from paper_2509_15377_amd import avm, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    band_bins = 100
    wl = W.WORKLOADS[args.workload](band_bins=band_bins)
    dev = torch.device("cuda:0")
    prim_dev = torch.from_numpy(wl.primaries.view(np.uint8).copy()).to(dev)
    stream = torch.cuda.current_stream()
    gas = avm.Gas(wl.gas, 0)
    field = avm.Field(wl.field, 0)
    capacity = CAPACITY[args.workload]

    use_graph = not args.eager

    def make(mode, majorant, precision=avm.FP64, graph=False):
        return avm.Run(gas, field, prim_dev, wl.n_aval, seed=wl.seed, precision=precision,
                       majorant=majorant, mode=mode, capacity=capacity, timeout_s=300.0,
                       stream=stream, graph=graph,
                       band_lookahead=BAND_LOOKAHEAD if majorant == avm.BANDED else 0.0)

    def timed(run):
        for _ in range(args.warmup):
            run.execute()
            run.sync()
        torch.cuda.synchronize()
        kms = []
        t = time.perf_counter()
        for _ in range(args.steps):
            run.execute()
            run.sync()
            kms.append(run.timing()[0])
        torch.cuda.synchronize()
        return time.perf_counter() - t, kms

    run = make(avm.BATCHED, avm.BANDED, graph=use_graph)
    wall, kernel_ms = timed(run)
    c = run.counts()
    flights = c["n_real"] + c["n_null"] + c["n_masked"] + c["n_band"]
    ms_step = wall * 1e3 / args.steps
    value = c["n_real"] / (ms_step * 1e-3)
    k_ms = sum(kernel_ms) / len(kernel_ms)
    ops = flights * OPS_PER_FLIGHT + c["n_real"] * OPS_PER_REAL + c["n_ion"] * OPS_PER_ION
    achieved = ops / (k_ms * 1e-3)

    paths = {"batched_fp64_banded": {"real_collisions_per_s": value,
                                     "secondaries_per_s": c["n_ion"] / (ms_step * 1e-3),
                                     "flights_per_s": flights / (ms_step * 1e-3),
                                     "ms_per_step": ms_step, "kernel_ms": k_ms,
                                     "graph": use_graph}}
    if not args.no_mixed:
        # FP32 arithmetic in the flight loop, FP64 positions/times and
        # re-decided close calls (statistically equivalent, not per-trajectory)
        mr = make(avm.BATCHED, avm.BANDED, precision=avm.FP32_MIXED, graph=use_graph)
        mw, mk = timed(mr)
        mc = mr.counts()
        mms = mw * 1e3 / args.steps
        paths["batched_fp32mixed_banded"] = {
            "real_collisions_per_s": mc["n_real"] / (mms * 1e-3),
            "secondaries_per_s": mc["n_ion"] / (mms * 1e-3),
            "flights_per_s": (mc["n_real"] + mc["n_null"] + mc["n_masked"] + mc["n_band"]) / (mms * 1e-3),
            "ms_per_step": mms, "kernel_ms": sum(mk) / len(mk),
            "mean_gain": mc["n_endpoints"] / wl.n_aval, "graph": use_graph}
        mr.close()
    if not args.headline_only and args.workload == "argon":
        side_legs(args, make, timed, paths, gas, field, wl, capacity, stream)
    if not args.no_plain:
        # the paper's scheduling (one kernel per transport iteration, host
        # reads the active count back) with the global majorant, one pass
        pr = make(avm.PLAIN, avm.GLOBAL)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pr.execute()
        pr.sync()
        tp = time.perf_counter() - t1
        pc = pr.counts()
        pk, it = pr.timing()
        paths["plain_fp64_global"] = {"real_collisions_per_s": pc["n_real"] / tp,
                                      "secondaries_per_s": pc["n_ion"] / tp,
                                      "flights_per_s": (pc["n_real"] + pc["n_null"] + pc["n_masked"]) / tp,
                                      "ms_per_step": tp * 1e3, "kernel_ms": pk, "iterations": it}
        pr.close()

    cpu = None
    if not args.no_cpu:
        # the oracle on the host cores: the whole workload on every core,
        # and every 20th avalanche on one thread
        from oracle import oracle as O
        og = O.Gas(wl.gas, band_bins=band_bins)
        of = O.Field(wl.field)
        mod = CPU_MODULUS[args.workload]
        sel = W.subset_primaries(wl.primaries, mod)
        t2 = time.perf_counter()
        ep, threads = O.run(og, of, wl.primaries[sel], wl.seed, banded=True, ids=sel,
                            return_threads=True, band_lookahead=BAND_LOOKAHEAD)
        tc = time.perf_counter() - t2
        idx = W.subset_primaries(wl.primaries, 20 * mod)
        t3 = time.perf_counter()
        ep1 = O.run(og, of, wl.primaries[idx], wl.seed, banded=True, ids=idx, threads=1,
                    band_lookahead=BAND_LOOKAHEAD)
        t1c = time.perf_counter() - t3
        cpu = {"value": float(ep["n_real"].sum() / tc), "unit": "real collisions/s",
               "cores": int(threads), "kind": "oracle",
               "sample": (f"all {wl.n_aval} avalanches" if mod == 1 else
                          f"avalanches with id % {mod} == 0 ({sel.size} of {wl.n_aval})")
                         + f", banded majorant, FP64, {tc:.1f} s on {threads} threads",
               "secondaries_per_s": float(ep["n_ion"].sum() / tc),
               "single_thread": {"value": float(ep1["n_real"].sum() / t1c),
                                 "sample": f"avalanches with id % {20 * mod} == 0 ({idx.size}), {t1c:.1f} s"}}

    line = {
        "metric": "electron real collisions/s (secondaries/s alongside) at gain ~1e3",
        "value": value,
        "unit": "collisions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.description}", "avalanches": wl.n_aval,
                   "electrons_per_step": c["n_endpoints"], "mean_gain": c["n_endpoints"] / wl.n_aval,
                   "path": "batched persistent kernel, banded majorant (100 bins/band, "
                           f"lookahead {BAND_LOOKAHEAD:g} mean free time), FP64, graph replay",
                   "seed": wl.seed},
        "secondaries_per_s": c["n_ion"] / (ms_step * 1e-3),
        "flights_per_s": flights / (ms_step * 1e-3),
        "null_fraction": (c["n_null"] + c["n_masked"]) / max(flights, 1),
        "paths": paths,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_LANE_OPS,
                     "unit": "lane-ops/s", "frac": achieved / PEAK_LANE_OPS,
                     "traffic": measured_traffic() if args.workload == "argon" else None,
                     "kernel": "k_persistent<banded,%s>" % ("polar" if args.workload == "wire" else "slab"), "kernel_ms": k_ms,
                     "ops_per_launch": ops},
        "cpu_baseline": cpu,
    }
    run.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
