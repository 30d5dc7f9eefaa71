"""Benchmark of the HWENO-U hot path on one MI355X.

Default workload: 2D Euler (gamma = 1.4) on a 2048 x 2048 periodic grid of
[0, 10]^2, seeded four-quadrant Riemann data (rho in [0.1, 1.5], p in
[0.03, 1.5], u, v in [-0.5, 0.5]) times an isentropic vortex of strength 5,
CFL 0.6, modified SSP-RK3.  One benchmark step = one full Runge-Kutta step:
the max wave speed / dt, and three fused stages (reconstruction, weights,
moment modification, fluxes, update), replayed from a captured HIP graph.

Reported on the default workload: cell-stage updates per second of the FP64
form (`value`, the paper's precision) and, in a block of its own, of the
FP32+FP64 mixed form with its speed-up and its L1 difference from FP64 after
the timed run next to the FP64 difference between the 1024^2 and 2048^2
solutions at the same time; the same rates for component-wise
reconstruction, for one x-characteristic reconstruction per cell and for
per-interface (Roe-average) bases of the edge values; the
stage kernel's roofline position, from its average launch duration measured
with HIP events on the stream its launches run on; and the CPU oracle on a
bounded sample.

--workload names one of the other workloads (1D advection N = 200, 1D Euler
N = 65536, 512 x 1D Euler, 64 x 2D Euler); it prints one line of the same
form for it.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                  [--size N] [--no-cpu-baseline] [--no-extras]
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
# finish kernel of one step, which also sets the next dt (rocprofv3 kernel
# trace: ~4 us)
AUX_US_PER_STEP = 4.0
# the counters also depend on the work lists the host library builds (which
# wave reads which rows and columns) and on the compiler flags of each source
# (the instruction scheduler), so those sources are hashed with the kernels
COMMON_SOURCES = ["paper_2402_03074_amd/csrc/hwenou_device.hpp",
                  "paper_2402_03074_amd/csrc/hwenou_internal.hpp",
                  "paper_2402_03074_amd/csrc/hwenou_api.hip",
                  "paper_2402_03074_amd/build.py"]
KERNEL_SOURCES = ["paper_2402_03074_amd/csrc/stage2d.hip"] + COMMON_SOURCES
# rocprofv3 counter summaries (profiles/) per stage kernel and the workload
# they were taken on
COUNTERS = {
    2: ("stage2d_kernel", "profiles/stage2d_euler_2048_counters.md", "euler2d-2048",
        KERNEL_SOURCES),
    1: ("stage1d_kernel", "profiles/stage1d_euler_batch512_counters.md", "euler1d-batch512",
        ["paper_2402_03074_amd/csrc/stage1d.hip"] + COMMON_SOURCES),
}
COUNTERS_FILE = COUNTERS[2][1]
DEFAULT_WORKLOAD = "euler2d-2048"
WORKLOADS = {
    "euler2d-2048": "2D Euler {n}x{n} periodic on [0,10]^2, seeded four-quadrant Riemann data "
                    "x isentropic vortex (strength 5), CFL 0.6, modified SSP-RK3, "
                    "characteristic-wise HWENO-U",
    "advection1d-200": "1D linear advection u_t + u_x = 0, N = 200 periodic on [0,2], "
                       "u0 = sin(pi x), CFL 0.2 (1000 steps reach T = 2)",
    "euler1d-65536": "1D Euler N = 65536 transmissive on [0,1], seeded 16-interface "
                     "shock tube with a density wave, CFL 0.6, characteristic-wise",
    "euler1d-batch512": "512 independent 1D Euler shock tubes, N log-uniform in "
                        "[256, 65536], one persistent launch per stage, per-instance dt",
    "euler2d-batch64": "64 independent 2D Euler vortex+quadrant grids, sides log-uniform "
                       "in [256, 1024], one persistent launch per stage, per-instance dt",
}
DEFAULT_STEPS = {"euler2d-2048": 100, "advection1d-200": 1000, "euler1d-65536": 200,
                 "euler1d-batch512": 200, "euler2d-batch64": 50}


def kernel_source_hash(dim=2):
    """Hash of the stage kernel's code, with comments and whitespace left out,
    so that the recorded counters stay valid across changes of the comments
    only."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in COUNTERS[dim][3]:
        with open(os.path.join(ROOT, f)) as fh:
            src = fh.read()
        if f.endswith(".py"):
            src = re.sub(r'""".*?"""', "", src, flags=re.S)
            src = re.sub(r"#[^\n]*", "", src)
        else:
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            src = re.sub(r"//[^\n]*", "", src)
        h.update(re.sub(r"\s+", " ", src).strip().encode())
    return h.hexdigest()[:16]


def recorded_counters(dim=2):
    """Per-launch figures recorded from rocprofv3 counter runs of one
    workload (profiles/): algorithmic flops per cell-stage and calibrated HBM
    bytes per launch, keyed by the kernel source hash they were taken on."""
    out = {"source_sha256": None}
    try:
        with open(os.path.join(ROOT, COUNTERS[dim][1])) as fh:
            for line in fh:
                if line.startswith("- ") and ":" in line:
                    k, v = line[2:].split(":", 1)
                    out[k.strip()] = v.strip().strip("`")
    except OSError:
        pass
    return out


def stage_bytes(dim, ncomp, precision, stage):
    """Algorithmic HBM bytes per cell of one stage: the state read, the
    Runge-Kutta base read (stages 1, 2), the output written, and in stage 0
    the modified moments written.  Halo re-reads are not counted."""
    mb = 8 if precision == "fp64" else 4
    moments = dim * ncomp * mb
    state = ncomp * 8 + moments
    if stage == 0:
        return state + state + moments
    return state + (ncomp * 8 + moments) + state


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=None)
    # warm-up steps keep the GPU busy for a few tens of ms before the timed
    # region: kernel traces show the stage kernel ~20% slower in the first
    # launches after an idle host phase, while the clocks ramp up
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    p.add_argument("--size", type=int, default=2048, help="grid side of euler2d-2048")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the component-wise and mesh-difference runs")
    p.add_argument("--precisions", default=None)
    p.add_argument("--tune", action="store_true",
                   help="run the launch-shape autotuner first (default: the library's "
                        "occupancy-based launch shape; the batched workloads always tune)")
    p.add_argument("--launch", default=None,
                   help="fixed launch shape 'waves_per_cu,rows_per_item' instead of tuning")
    return p.parse_args()


class Case:
    """Problem set-up of one workload: instances, initial state, CFL."""

    def __init__(self, name, dim, eq, insts, u0, m0, cfl=0.6, kw=None, label=""):
        self.name, self.dim, self.eq, self.insts = name, dim, eq, insts
        self.u0, self.m0, self.cfl, self.kw, self.label = u0, m0, cfl, kw or {}, label
        self.ncomp = u0.shape[0]
        self.cells = u0.shape[1]


def make_case(H, W, np, name, n=2048):
    label = WORKLOADS[name].format(n=n)
    if name == "euler2d-2048":
        u0, m0 = W.euler_2d_vortex_quadrant(n, seed=3000, q=3)
        return Case(name, 2, "euler", [H.make_inst(n, n, (0.0, 10.0, 0.0, 10.0), "periodic")],
                    u0.reshape(4, -1), m0.reshape(2, 4, -1), label=label)
    if name == "advection1d-200":
        u0, m0 = W.advection_sine_1d(200)
        return Case(name, 1, "advection", [H.make_inst(200, 1, (0.0, 2.0))], u0, m0, cfl=0.2,
                    kw={"adv": (1.0, 0.0)}, label=label)
    if name == "euler1d-65536":
        u0, m0 = W.euler_1d_shocktube(65536, seed=2000)
        return Case(name, 1, "euler", [H.make_inst(65536, 1, (0.0, 1.0), "transmissive")],
                    u0, m0, label=label)
    if name == "euler1d-batch512":
        sizes, data = W.batch_1d_euler()
        insts, off = [], 0
        for s in sizes:
            insts.append(H.make_inst(int(s), 1, (0.0, 1.0), "transmissive", offset=off))
            off += int(s)
        u0 = np.concatenate([d[0] for d in data], axis=1)
        m0 = np.concatenate([d[1] for d in data], axis=2)
        return Case(name, 1, "euler", insts, u0, m0, label=label)
    if name == "euler2d-batch64":
        sides, data = W.batch_2d_euler()
        insts, off = [], 0
        for s in sides:
            insts.append(H.make_inst(int(s), int(s), (0.0, 10.0, 0.0, 10.0), "periodic",
                                     offset=off))
            off += int(s) ** 2
        u0 = np.concatenate([d[0].reshape(4, -1) for d in data], axis=1)
        m0 = np.concatenate([d[1].reshape(2, 4, -1) for d in data], axis=2)
        return Case(name, 2, "euler", insts, u0, m0, label=label)
    raise ValueError(name)


def run_case(H, torch, case, precision, steps, warmup, tune, char_decomp=True, launch=None):
    S = H.Solver(case.dim, case.eq, case.insts, precision=precision, char_decomp=char_decomp,
                 **case.kw)
    ug = torch.tensor(case.u0, device="cuda")
    mg = torch.tensor(case.m0, device="cuda").to(S.mom_dtype)
    if launch is not None:
        S.set_launch(*launch)
    elif tune:
        launch = S.autotune(ug, mg)
    # warm-up steps (untimed), then exactly `steps` timed steps
    if warmup > 0:
        S.advance(ug, mg, case.cfl, 1e30, warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    tg, sg = S.advance(ug, mg, case.cfl, 1e30, steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    assert sg == [steps] * len(case.insts), sg

    # The timed region is graph replays of whole steps: per step three
    # launches of the stage kernel and one finish kernel (a single block,
    # ~4 us by the kernel trace), so the stage kernel's average launch
    # duration implied by the timed region is (region / steps - aux) / 3.
    stage_ms_region = (ev_ms / steps - AUX_US_PER_STEP * 1e-3) / 3.0
    # right after the timed region, while the clocks are up
    stage_ms = stage_launch_ms(H, torch, S, case, ug, mg, max(3, min(steps, 20)))
    status = H.hwenou_status(S.h)
    out = ug.cpu().numpy(), mg.double().cpu().numpy()
    S.close()
    del ug, mg
    torch.cuda.empty_cache()
    return {"wall_s": wall, "event_ms": ev_ms, "stage_ms": stage_ms,
            "stage_ms_region": stage_ms_region, "state": out,
            "t": tg, "status": status, "launch": launch,
            "rate": case.cells * 3 * steps / (ev_ms * 1e-3), "ms_per_step": ev_ms / steps}


def stage_launch_ms(H, torch, S, case, ug, mg, reps):
    """Average duration of one stage-kernel launch: `reps` Runge-Kutta steps
    of explicit hwenou_stage launches (stages 0, 1, 2) on the state of the
    timed run, between two HIP events recorded on the stream those launches
    run on (the handle's stream, torch's current stream); span / (3 reps).
    The span also holds the launch gaps between the kernels, so this is an
    upper bound of the kernel's own duration (rocprofv3's figure)."""
    alpha = S.max_wavespeed(ug)
    a = alpha.cpu().numpy()  # the wave speed of the state after the timed run
    dts = []
    for k, I in enumerate(case.insts):
        dx = (I.x1 - I.x0) / I.nx
        if case.dim == 1:
            dts.append(case.cfl * dx / a[k, 0] if a[k, 0] > 0 else 0.0)
        else:
            dy = (I.y1 - I.y0) / I.ny
            den = a[k, 0] / dx + a[k, 1] / dy
            dts.append(case.cfl / den if den > 0 else 0.0)
    dt = torch.tensor(dts, dtype=torch.float64, device="cuda")
    u1, m1 = S.empty_state()
    u2, m2 = S.empty_state()
    u3, m3 = S.empty_state()
    for _ in range(3):  # warm-up
        S.stage(0, dt, alpha, ug, mg, u1, m1)
        S.stage(1, dt, alpha, u1, m1, u2, m2)
        S.stage(2, dt, alpha, u2, m2, u3, m3)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        S.stage(0, dt, alpha, ug, mg, u1, m1)
        S.stage(1, dt, alpha, u1, m1, u2, m2)
        S.stage(2, dt, alpha, u2, m2, u3, m3)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / (3 * reps)
    del u1, m1, u2, m2, u3, m3
    return ms


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


def cpu_baseline(W, u0, m0, n):
    """The oracle (plain C, FP64, OpenMP) on a bounded sample of the same
    workload: one Runge-Kutta step (three stages) over the full grid on all
    host threads, and one step of the same data generated on a 256^2 grid on
    one thread."""
    from oracle.driver import Problem, num_threads, set_num_threads
    P = Problem(2, "euler", (n, n), (0.0, 10.0, 0.0, 10.0))
    alpha = P.max_wavespeed(u0)
    dt = P.dt_from(alpha, 0.6)
    t0 = time.perf_counter()
    P.step(u0, m0, dt, alpha)
    el = time.perf_counter() - t0
    cs = 3 * n * n
    threads = num_threads()
    out = {"value": cs / el, "unit": "cell-stage/s", "cores": threads, "kind": "oracle",
           "sample": f"one Runge-Kutta step (3 stages) of the same {n}x{n} 2D Euler data, "
                     f"{cs} cell-stages in {el:.2f} s"}
    m = 256
    us, ms = W.euler_2d_vortex_quadrant(m, seed=3000, q=3)
    P1 = Problem(2, "euler", (m, m), (0.0, 10.0, 0.0, 10.0))
    a1 = P1.max_wavespeed(us)
    set_num_threads(1)
    try:
        t0 = time.perf_counter()
        P1.step(us, ms, P1.dt_from(a1, 0.6), a1)
        el1 = time.perf_counter() - t0
    finally:
        set_num_threads(threads)
    out["one_thread"] = {"value": 3 * m * m / el1, "unit": "cell-stage/s", "cores": 1,
                         "sample": f"one Runge-Kutta step of the same data on a {m}x{m} grid, "
                                   f"{3 * m * m} cell-stages in {el1:.2f} s"}
    try:
        with open("/proc/cpuinfo") as fh:
            out["cpu_model"] = next(l.split(":", 1)[1].strip() for l in fh
                                    if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return out


def mesh_difference(H, W, torch, np, n, t_final):
    """FP64 density L1 difference between the 2048^2 solution and the
    1024^2 solution of the same data at the same time: the size of the
    discretisation error against which the mixed-vs-FP64 difference is set."""
    c = n // 2
    u0, m0 = W.euler_2d_vortex_quadrant(c, seed=3000, q=3)
    S = H.Solver(2, "euler", [H.make_inst(c, c, (0.0, 10.0, 0.0, 10.0), "periodic")])
    ug = torch.tensor(u0.reshape(4, -1), device="cuda")
    mg = torch.tensor(m0.reshape(2, 4, -1), device="cuda")
    t, s = S.advance(ug, mg, 0.6, t_final, 10 ** 6)
    coarse = ug.cpu().numpy()[0].reshape(c, c)
    S.close()
    return coarse, t[0], s[0]


def summary_roofline(case, r, precision, rec):
    """Roofline position of the stage kernel: against the vector ALU peak
    when its flops per cell-stage have been counted (both stage kernels are
    limited by their vector instruction stream and its latencies, far below
    the HBM roof), with the algorithmic HBM view beside it."""
    cells = case.cells
    kavg = r["stage_ms"]
    kernel = COUNTERS[case.dim][0]
    byts = sum(stage_bytes(case.dim, case.ncomp, precision, s) for s in range(3)) / 3
    hbm = byts * cells / (kavg * 1e-3) / 1e9
    hview = {"achieved_algorithmic": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": hbm / HBM_PEAK_GBS, "bytes_per_cell_stage": byts}
    key = f"algorithmic_flops_per_cell_stage_{precision}"
    if case.eq == "euler" and key in rec:
        flops = float(rec[key])
        tf = flops * cells / (kavg * 1e-3) / 1e12
        return {"bound": "alu", "achieved": tf, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tf / VALU_PEAK_TFLOPS, "kernel": kernel,
                "avg_launch_ms": kavg, "flops_per_cell_stage": flops}, hview
    return {"bound": "hbm", "achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": hbm / HBM_PEAK_GBS, "traffic": None, "kernel": kernel,
            "avg_launch_ms": kavg, "bytes_per_cell_stage": byts}, None


def attach_traffic(roof, hbm, rec, precision, case, fresh):
    """HBM bytes per launch measured by the committed counter summary
    (calibrated FETCH_SIZE + WRITE_SIZE), when it was taken on the current
    kernel source and on this workload; null otherwise.  With it, the measured
    HBM rate over this run's launch time goes beside the algorithmic one."""
    if roof["bound"] != "alu":
        return
    key = f"hbm_bytes_per_launch_{precision}"
    roof["counters_current"] = fresh
    roof["traffic"] = (float(rec[key]) if fresh and case.name == COUNTERS[case.dim][2]
                       and key in rec else None)
    if roof["traffic"] is not None and hbm is not None:
        meas = roof["traffic"] / (roof["avg_launch_ms"] * 1e-3) / 1e9
        hbm["achieved_measured"] = meas
        hbm["frac_measured"] = meas / HBM_PEAK_GBS
        hbm["measured_over_algorithmic"] = meas / hbm["achieved_algorithmic"]


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU decomposition is designed, not built)"}))
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2402_03074_amd as H
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    name = args.workload
    n = args.size
    steps = args.steps if args.steps is not None else DEFAULT_STEPS[name]
    precs = (args.precisions or ("fp64" if name == "advection1d-200" else "fp64,mixed"))
    precs = precs.split(",")
    print(f"[bench] generating {name}", file=sys.stderr, flush=True)
    case = make_case(H, W, np, name, n)
    tune = args.tune or name.endswith(("batch512", "batch64"))
    fixed = tuple(int(v) for v in args.launch.split(",")) if args.launch else None
    results = {}
    for prec in precs:
        print(f"[bench] {prec}: {args.warmup} warm-up + {steps} timed steps",
              file=sys.stderr, flush=True)
        results[prec] = r = run_case(H, torch, case, prec, steps, args.warmup, tune,
                                     launch=fixed)
        print(f"[bench] {prec}: {r['ms_per_step']:.3f} ms/step, stage launch {r['stage_ms']:.3f}"
              f" ms (timed region: {r['stage_ms_region']:.3f} ms)", file=sys.stderr, flush=True)

    rec = recorded_counters(case.dim)
    fresh = rec.get("source_sha256") == kernel_source_hash(case.dim)
    head = precs[0]
    r = results[head]
    roof, hbm = summary_roofline(case, r, head, rec)
    attach_traffic(roof, hbm, rec, head, case, fresh)
    line = {
        "metric": METRIC if name == DEFAULT_WORKLOAD else "cell-stage updates/s",
        "value": r["rate"],
        "unit": "cell-stage/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": case.label, "precision": head, "cells": case.cells,
                   "instances": len(case.insts)},
        "roofline": roof,
    }
    if hbm is not None:
        line["hbm"] = hbm
    line["avg_stage_launch_ms"] = r["stage_ms"]
    line["stage_ms_from_timed_region"] = r["stage_ms_region"]
    for prec in precs[1:]:
        r2 = results[prec]
        roof2, hbm2 = summary_roofline(case, r2, prec, rec)
        attach_traffic(roof2, hbm2, rec, prec, case, fresh)
        line[prec] = {"value": r2["rate"], "ms_per_step": r2["ms_per_step"],
                      "dtype": "f64+f32" if prec == "mixed" else "f64",
                      "avg_stage_launch_ms": r2["stage_ms"],
                      "stage_ms_from_timed_region": r2["stage_ms_region"], "roofline": roof2}
        if hbm2 is not None:
            line[prec]["hbm"] = hbm2
        line[f"{prec}_speedup_vs_{head}"] = r2["rate"] / r["rate"]
    if "mixed" in results and "fp64" in results:
        a = results["mixed"]["state"][0]
        b = results["fp64"]["state"][0]
        line["mixed_vs_fp64"] = {
            "l1_rho_diff": float(np.abs(a[0] - b[0]).mean()),
            "rel_linf_rho_diff": float(np.abs(a[0] - b[0]).max() / np.abs(b[0]).max()),
            "after_steps": args.warmup + steps}
    if name == DEFAULT_WORKLOAD and not args.no_extras:
        cw = {}
        for prec in precs:
            print(f"[bench] component-wise {prec}", file=sys.stderr, flush=True)
            rc = run_case(H, torch, case, prec, steps, args.warmup, False, char_decomp=False)
            cw[prec] = {"value": rc["rate"], "ms_per_step": rc["ms_per_step"],
                        "status": rc["status"]}
        line["componentwise"] = cw
        sp = {}
        for prec in precs:
            print(f"[bench] single x-projection {prec}", file=sys.stderr, flush=True)
            rc = run_case(H, torch, case, prec, steps, args.warmup, False, char_decomp=2)
            sp[prec] = {"value": rc["rate"], "ms_per_step": rc["ms_per_step"],
                        "status": rc["status"]}
        line["single_projection"] = sp
        ip = {}
        for prec in precs:
            print(f"[bench] per-interface bases {prec}", file=sys.stderr, flush=True)
            rc = run_case(H, torch, case, prec, steps, args.warmup, False, char_decomp=3)
            ip[prec] = {"value": rc["rate"], "ms_per_step": rc["ms_per_step"],
                        "status": rc["status"]}
        line["interface_projection"] = ip
        if "fp64" in results and n % 2 == 0 and "mixed_vs_fp64" in line:
            print("[bench] FP64 mesh difference", file=sys.stderr, flush=True)
            tf = results["fp64"]["t"][0]
            coarse, tc, sc = mesh_difference(H, W, torch, np, n, tf)
            fine = results["fp64"]["state"][0][0].reshape(n, n)
            fine_c = fine.reshape(n // 2, 2, n // 2, 2).mean(axis=(1, 3))
            md = float(np.abs(fine_c - coarse).mean())
            line["mixed_vs_fp64"].update({
                "t": tf, "fp64_l1_rho_mesh_diff": md, "mesh_diff_coarse_steps": sc,
                "mesh_diff_t_match": abs(tc - tf),
                "mixed_diff_over_mesh_diff": line["mixed_vs_fp64"]["l1_rho_diff"] / md})
    line["status"] = {p: results[p]["status"] for p in results}
    line["launch"] = {p: results[p]["launch"] for p in results}
    line["kernel_source_sha256"] = kernel_source_hash(case.dim)
    line["copy_calibration_mib"] = copy_calibration(torch)
    if name == DEFAULT_WORKLOAD and not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(W, case.u0.reshape(4, n, n),
                                            case.m0.reshape(2, 4, n, n), n)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
