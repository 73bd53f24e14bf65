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

# Algorithmic VALU work per event: the minimum the method performs per
# flight / real collision / ionisation, in issue slots of one 16-lane SIMD
# (lane operations weighted by issue rate as measured on gfx950: FP64 add,
# multiply and FMA, 32-bit integer multiplies (v_mad_u64_u32 gives both
# halves of a 32 x 32-bit product) and three-input bitwise operations issue
# at one wave64 instruction per four cycles and count 1;
# FP64 reciprocal and reciprocal square root issue at a quarter of that and
# count 4).  Peak: 256 CUs x 4 SIMD16 x 2.4 GHz x 16 lanes = 3.93e13
# lane-ops/s, the FP64 vector FMA rate.
OPS_FLIGHT = {
    "Philox block: 10 rounds of 2 mad_u64_u32 (both halves of a product), 2 three-input xor; counter": 42,
    "two 53-bit uniforms": 8,
    "logarithm of the flight uniform (one reciprocal)": 28,
    "flight update: time, position, velocity": 11,
    "energy at the flight end, band test": 6,
    "decision: bin, two interpolations, comparisons": 10,
    "flight index, counters, trace": 4,
}
OPS_REAL = {
    "Philox block": 42,
    "two uniforms": 8,
    "screened scattering angle (one reciprocal)": 13,
    "energy loss": 3,
    "lab-frame cosine (one reciprocal square root)": 9,
    "direction normalisation (one reciprocal square root)": 13,
    "azimuth sin/cos (table entry, short series, addition theorem)": 25,
    "sine of the polar angle (square root)": 9,
    "rotation": 20,
    "new speed (square root) and velocity": 11,
    "channel search, band lookup, trace": 10,
}
OPS_ION = {
    "two Philox blocks": 84,
    "energy split (tangent, arc tangent)": 50,
    "two directions: sin/cos, rotation, square roots": 106,
}
# the polar map and the magnetic field add, per flight: the map gather
# (logarithm of rho^2, azimuth, bilinear weights and reads, rotation to
# Cartesian), the helical step (sin/cos of the half phase and the drift and
# gyration terms) and, with the band majorant, the helical energy bound
# (three square roots)
OPS_FLIGHT_POLAR_B = {"map gather": 90, "helical step": 70, "helical energy bound": 40}
OPS_PER_FLIGHT = sum(OPS_FLIGHT.values())
OPS_PER_REAL = sum(OPS_REAL.values())
OPS_PER_ION = sum(OPS_ION.values())
OPS_PER_FLIGHT_POLAR_B = sum(OPS_FLIGHT_POLAR_B.values())
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9


def lane_ops(c, polar_b=False):
    """Algorithmic lane operations of a run from its counts."""
    flights = c["n_real"] + c["n_null"] + c["n_masked"] + c["n_band"]
    per_flight = OPS_PER_FLIGHT + (OPS_PER_FLIGHT_POLAR_B if polar_b else 0)
    return flights * per_flight + c["n_real"] * OPS_PER_REAL + c["n_ion"] * OPS_PER_ION

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
# WRITE_SIZE per dispatch), valid only for the kernel sources, launch
# defaults (avm_internal.hpp) and compiler flags it was taken on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_persistent_argon1000_fp64_banded.json")
KERNEL_SOURCES = ("paper_2509_15377_amd/csrc/avm_kernels.hip",
                  "paper_2509_15377_amd/csrc/avm_device.hpp",
                  "paper_2509_15377_amd/csrc/avm_internal.hpp",
                  "paper_2509_15377_amd/build.py")


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


def workload_leg(name, precision, steps, warmup, stream):
    """One benchmark workload in the headline's launch configuration
    (batched, banded majorant of 100-bin bands, lookahead 1, graph replay,
    primaries in HBM): ms per step, rates and the transport kernel's own
    roofline fraction."""
    import numpy as np
    import torch

    from paper_2509_15377_amd import avm, workloads as W
    wl = W.WORKLOADS[name](band_bins=100)
    gas = avm.Gas(wl.gas, 0)
    field = avm.Field(wl.field, 0)
    prim = torch.from_numpy(wl.primaries.view(np.uint8).copy()).to("cuda:0")
    r = avm.Run(gas, field, prim, wl.n_aval, seed=wl.seed, precision=precision, majorant=avm.BANDED,
                mode=avm.BATCHED, capacity=CAPACITY[name], timeout_s=300.0, stream=stream, graph=True,
                band_lookahead=BAND_LOOKAHEAD)
    for _ in range(warmup):
        r.execute()
        r.sync()
    torch.cuda.synchronize()
    kms = []
    t = time.perf_counter()
    for _ in range(steps):
        r.execute()
        r.sync()
        r.avalanche_counts()
        kms.append(r.timing()[0])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / steps
    c = r.counts()
    r.close()
    k_ms = sum(kms) / len(kms)
    polar_b = name == "wire"
    ops = lane_ops(c, polar_b)
    flights = c["n_real"] + c["n_null"] + c["n_masked"] + c["n_band"]
    return {"workload": f"{wl.name}: {wl.description}", "avalanches": wl.n_aval,
            "precision": "fp32-mixed" if precision == avm.FP32_MIXED else "fp64",
            "real_collisions_per_s": c["n_real"] / (ms * 1e-3),
            "secondaries_per_s": c["n_ion"] / (ms * 1e-3), "flights_per_s": flights / (ms * 1e-3),
            "ms_per_step": ms, "kernel_ms": k_ms, "steps": steps, "warmup": warmup,
            "electrons_per_step": c["n_endpoints"], "mean_gain": c["n_endpoints"] / wl.n_aval,
            "roofline": {"bound": "alu", "achieved": ops / (k_ms * 1e-3), "peak": PEAK_LANE_OPS,
                         "unit": "lane-ops/s", "frac": ops / (k_ms * 1e-3) / PEAK_LANE_OPS,
                         "traffic": None, "ops_per_launch": ops,
                         "kernel": "k_persistent<%s,banded,%s>" % (
                             "float" if precision == avm.FP32_MIXED else "double",
                             "polar" if polar_b else "slab")}}


def crossover_rows(sizes):
    """Wall time of one whole simulation against the number of avalanches
    (argon-like gas, one primary each): the GPU (batched, banded, FP64,
    primaries handed over in host memory, from execute to sync) against the
    oracle on every host core (the paper's run-mode switch between CPU and
    GPU rests on where one overtakes the other, Sec. 3.2 and Sec. 4)."""
    import numpy as np
    import torch

    from oracle import oracle as O
    from paper_2509_15377_amd import avm, workloads as W

    full = W.argon(max(sizes), band_bins=100)
    gas = avm.Gas(full.gas, 0)
    field = avm.Field(full.field, 0)
    og = O.Gas(full.gas, band_bins=100)
    of = O.Field(full.field)
    rows = []
    for n in sizes:
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
            r.avalanche_counts()
            ts.append(time.perf_counter() - t0)
        electrons = r.counts()["n_endpoints"]
        r.close()
        t1 = time.perf_counter()
        _, threads = O.run(og, of, prim, full.seed, banded=True, band_lookahead=BAND_LOOKAHEAD,
                           return_threads=True)
        tc = time.perf_counter() - t1
        rows.append({"avalanches": n, "electrons": int(electrons), "gpu_s": float(np.median(ts)),
                     "oracle_s": tc, "oracle_threads": int(threads)})
    return rows


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def crossover():
    """--crossover: the crossover table alone, at more sizes (not the
    benchmark line)."""
    rows = crossover_rows((1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024))
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
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the legs of the other workloads (8192 avalanches, high gain, wire)")
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
        args.no_mixed = args.no_plain = args.no_cpu = args.no_workloads = True
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
            run.avalanche_counts()  # the per-avalanche statistics come back in the step
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
    ops = lane_ops(c, args.workload == "wire")
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
            "mean_gain": mc["n_endpoints"] / wl.n_aval, "graph": use_graph,
            "roofline_frac": lane_ops(mc, args.workload == "wire") / (sum(mk) / len(mk) * 1e-3) / PEAK_LANE_OPS}
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

    run.close()
    if not args.no_workloads and args.workload == "argon":
        # the other workloads, each in FP64 and FP32-mixed with its own
        # roofline (one warm-up and two timed steps each)
        legs = []
        for name in ("batched", "highgain", "wire"):
            for prec in (avm.FP64, avm.FP32_MIXED):
                legs.append(workload_leg(name, prec, 2, 1, stream))
                torch.cuda.empty_cache()
        paths["workloads"] = legs

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
               "cores": int(threads), "kind": "oracle", "cpu_model": cpu_model(),
               "sample": (f"all {wl.n_aval} avalanches" if mod == 1 else
                          f"avalanches with id % {mod} == 0 ({sel.size} of {wl.n_aval})")
                         + f", banded majorant, FP64, {tc:.1f} s on {threads} threads",
               "secondaries_per_s": float(ep["n_ion"].sum() / tc),
               "single_thread": {"value": float(ep1["n_real"].sum() / t1c),
                                 "sample": f"avalanches with id % {20 * mod} == 0 ({idx.size}), {t1c:.1f} s"}}
        if args.workload == "argon":
            rows = crossover_rows((1, 4, 16, 64, 256))
            cpu["crossover"] = {
                "rows": rows,
                "gpu_faster_from_avalanches": next((r["avalanches"] for r in rows
                                                    if r["gpu_s"] < r["oracle_s"]), None),
                "what": "one whole simulation of n avalanches (argon-like gas, one primary each): "
                        "GPU from execute to sync with host primaries, against the oracle on every "
                        "host core"}

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
        "timed_region": "execute to sync of the whole run replayed from its HIP graph (reset, "
                        "primary load from HBM, transport with its in-kernel statistics, totals "
                        "back to the host), then the per-avalanche statistics copied to the host; "
                        "primaries resident in HBM before the region (their PCIe copy inside "
                        "every step: paths.batched_fp64_banded_host_primaries)",
        "secondaries_per_s": c["n_ion"] / (ms_step * 1e-3),
        "flights_per_s": flights / (ms_step * 1e-3),
        "null_fraction": (c["n_null"] + c["n_masked"]) / max(flights, 1),
        "paths": paths,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_LANE_OPS,
                     "unit": "lane-ops/s", "frac": achieved / PEAK_LANE_OPS,
                     "traffic": measured_traffic() if args.workload == "argon" else None,
                     "kernel": "k_persistent<banded,%s>" % ("polar" if args.workload == "wire" else "slab"), "kernel_ms": k_ms,
                     "ops_per_launch": ops,
                     "ops_model": "minimal VALU issue slots, weighted by measured issue rate: per flight %d, "
                                  "per real collision +%d, per ionisation +%d%s" % (
                                      OPS_PER_FLIGHT, OPS_PER_REAL, OPS_PER_ION,
                                      ", per polar/B flight +%d" % OPS_PER_FLIGHT_POLAR_B if args.workload == "wire" else "")},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
