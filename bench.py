"""Benchmark of the HWENO-U hot path on one MI355X.

Workload: 2D Euler (gamma = 1.4) on a 2048 x 2048 periodic grid of [0, 10]^2,
seeded four-quadrant Riemann data (rho in [0.1, 1.5], p in [0.03, 1.5],
u, v in [-0.5, 0.5]) times an isentropic vortex of strength 5, CFL 0.6,
modified SSP-RK3.  One benchmark step = one full Runge-Kutta step: the max
wave speed / dt, and three fused stages (reconstruction, weights, moment
modification, fluxes, update), replayed from a captured HIP graph.

Reported: cell-stage updates per second of the mixed form (`value`) and of the
plain FP64 form, the mixed-vs-FP64 L1 difference after the timed run, the
stage kernel's roofline position, and the CPU oracle on a bounded sample.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--size N] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "2D Euler cell-stage updates/s, mixed vs FP64 at fixed L1 error; % HBM peak"
HBM_PEAK_GBS = 8000.0
# FP64 vector peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz;
# non-packed FP32 runs at the same instruction rate
VALU_PEAK_TFLOPS = 78.6
# dt and finish kernels of one step (rocprofv3 kernel trace: ~5 us + ~4 us)
AUX_US_PER_STEP = 9.0
KERNEL_SOURCES = ["paper_2402_03074_amd/csrc/stage2d.hip",
                  "paper_2402_03074_amd/csrc/hwenou_device.hpp",
                  "paper_2402_03074_amd/csrc/hwenou_internal.hpp"]
COUNTERS_FILE = "profiles/stage2d_euler_2048_counters.md"


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_counters():
    """Per-launch figures recorded from rocprofv3 counter runs of this
    benchmark (profiles/): algorithmic flops per cell-stage and calibrated
    HBM bytes per launch, keyed by the kernel source hash they were taken on."""
    out = {"source_sha256": None}
    try:
        with open(os.path.join(ROOT, COUNTERS_FILE)) as fh:
            for line in fh:
                if line.startswith("| ") and ":" not in line and "|" in line[2:]:
                    continue
                if line.startswith("- ") and ":" in line:
                    k, v = line[2:].split(":", 1)
                    out[k.strip()] = v.strip().strip("`")
    except OSError:
        pass
    return out

# algorithmic HBM bytes per cell and stage (state read, base read, write;
# stage 0 also writes the modified moments); 2D Euler: 4 components
def stage_bytes(precision, stage):
    mb = 8 if precision == "fp64" else 4
    state = 4 * 8 + 2 * 4 * mb  # averages FP64 + two moment directions
    moments = 2 * 4 * mb
    if stage == 0:
        return state + state + moments
    return state + (4 * 8 + moments) + state


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--size", type=int, default=2048)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--precisions", default="mixed,fp64")
    p.add_argument("--tune", action="store_true",
                   help="run the launch-shape autotuner first (default: the library's "
                        "occupancy-based launch shape)")
    return p.parse_args()


def run_precision(H, torch, u0, m0, n, precision, steps, warmup, tune):
    inst = H.make_inst(n, n, (0.0, 10.0, 0.0, 10.0), "periodic")
    S = H.Solver(2, "euler", [inst], precision=precision)
    ug = torch.tensor(u0.reshape(4, -1), device="cuda")
    mg = torch.tensor(m0.reshape(2, 4, -1), device="cuda").to(S.mom_dtype)
    launch = S.autotune(ug, mg) if tune else None
    # warm-up steps (untimed), then exactly `steps` timed steps
    if warmup > 0:
        S.advance(ug, mg, 0.6, 1e30, warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    tg, sg = S.advance(ug, mg, 0.6, 1e30, steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    assert sg == [steps], sg

    # The timed region is graph replays of whole steps: per step one dt and
    # one finish kernel (single blocks, ~9 us together by the kernel trace)
    # and three launches of the stage kernel, so the stage kernel's average
    # launch duration over the timed region is (region / steps - aux) / 3.
    stage_ms = [(ev_ms / steps - AUX_US_PER_STEP * 1e-3) / 3.0] * 3
    status = H.hwenou_status(S.h)
    out = ug.cpu().numpy(), mg.double().cpu().numpy()
    S.close()
    del ug, mg
    torch.cuda.empty_cache()
    return {"wall_s": wall, "event_ms": ev_ms, "stage_ms": stage_ms, "state": out,
            "t": tg[0], "status": status, "launch": launch}


def copy_calibration(torch, mib=1024):
    """A plain device-to-device copy of known size, outside the timed region:
    its FETCH_SIZE / WRITE_SIZE counters calibrate the HBM-traffic counters of
    the stage kernel."""
    n = mib * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    return mib


def cpu_baseline(u0, m0, n):
    """The oracle (plain C, FP64, OpenMP) on a bounded sample of the same
    workload: one Runge-Kutta step (three stages) over the full grid."""
    from oracle.driver import Problem, num_threads
    P = Problem(2, "euler", (n, n), (0.0, 10.0, 0.0, 10.0))
    alpha = P.max_wavespeed(u0)
    dt = P.dt_from(alpha, 0.6)
    t0 = time.perf_counter()
    P.step(u0, m0, dt, alpha)
    el = time.perf_counter() - t0
    cs = 3 * n * n
    return {"value": cs / el, "unit": "cell-stage/s", "cores": num_threads(),
            "kind": "oracle",
            "sample": f"one Runge-Kutta step (3 stages) of the same {n}x{n} 2D Euler data, "
                      f"{cs} cell-stages in {el:.2f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU decomposition is designed, not built)"}))
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2402_03074_amd as H
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    n = args.size
    print(f"[bench] generating {n}x{n} vortex + quadrant data", file=sys.stderr, flush=True)
    u0, m0 = W.euler_2d_vortex_quadrant(n, seed=3000, q=3)
    cells = n * n
    results = {}
    for prec in args.precisions.split(","):
        print(f"[bench] {prec}: {args.warmup} warm-up + {args.steps} timed steps",
              file=sys.stderr, flush=True)
        results[prec] = run_precision(H, torch, u0, m0, n, prec, args.steps, args.warmup,
                                      args.tune)
        r = results[prec]
        print(f"[bench] {prec}: {r['event_ms'] / args.steps:.3f} ms/step, stages "
              f"{[round(x, 3) for x in r['stage_ms']]} ms", file=sys.stderr, flush=True)

    def summary(prec):
        r = results[prec]
        ms_step = r["event_ms"] / args.steps
        rate = cells * 3 * args.steps / (r["event_ms"] * 1e-3)
        byts = [stage_bytes(prec, s) * cells for s in range(3)]
        kms = sum(r["stage_ms"])
        achieved = sum(byts) / (kms * 1e-3) / 1e9
        return ms_step, rate, achieved, kms / 3

    head = "mixed" if "mixed" in results else list(results)[0]
    ms_step, rate, achieved, kavg = summary(head)
    rec = recorded_counters()
    fresh = rec.get("source_sha256") == kernel_source_hash()
    flops_cs = float(rec.get(f"algorithmic_flops_per_cell_stage_{head}", "nan"))
    alu_tflops = flops_cs * cells / (kavg * 1e-3) / 1e12
    traffic = None
    if fresh and f"hbm_bytes_per_launch_{head}" in rec:
        traffic = float(rec[f"hbm_bytes_per_launch_{head}"])
    line = {
        "metric": METRIC,
        "value": rate,
        "unit": "cell-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"2D Euler {n}x{n} periodic on [0,10]^2, seeded four-quadrant "
                               "Riemann data x isentropic vortex (strength 5), CFL 0.6, "
                               "modified SSP-RK3, characteristic-wise HWENO-U",
                   "precision": head, "cells": cells, "seed": 3000},
        "roofline": {"bound": "alu", "achieved": alu_tflops, "peak": VALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": alu_tflops / VALU_PEAK_TFLOPS,
                     "traffic": traffic, "kernel": "stage2d_kernel", "avg_launch_ms": kavg,
                     "flops_per_cell_stage": flops_cs, "counters_current": fresh},
        "hbm": {"achieved_algorithmic": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "bytes_per_cell_stage": sum(stage_bytes(head, s) for s in range(3)) / 3},
    }
    for prec in results:
        if prec == head:
            continue
        ms2, rate2, ach2, kavg2 = summary(prec)
        fl2 = float(rec.get(f"algorithmic_flops_per_cell_stage_{prec}", "nan"))
        tf2 = fl2 * cells / (kavg2 * 1e-3) / 1e12
        line[prec] = {"value": rate2, "ms_per_step": ms2, "hbm_achieved_gbs": ach2,
                      "hbm_frac": ach2 / HBM_PEAK_GBS, "avg_stage_launch_ms": kavg2,
                      "alu_tflops": tf2, "alu_frac": tf2 / VALU_PEAK_TFLOPS}
        line["mixed_speedup_vs_fp64"] = rate / rate2 if head == "mixed" else None
    if "mixed" in results and "fp64" in results:
        a = results["mixed"]["state"][0]
        b = results["fp64"]["state"][0]
        line["mixed_vs_fp64"] = {
            "l1_rho_diff": float(np.abs(a[0] - b[0]).mean()),
            "rel_linf_rho_diff": float(np.abs(a[0] - b[0]).max() / np.abs(b[0]).max()),
            "after_steps": args.warmup + args.steps}
    line["status"] = {p: results[p]["status"] for p in results}
    line["launch"] = {p: results[p]["launch"] for p in results}
    line["kernel_source_sha256"] = kernel_source_hash()
    line["copy_calibration_mib"] = copy_calibration(torch)
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(u0, m0, n)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
