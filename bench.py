"""Benchmark: accelerated sharp-interface method on one MI355X.

Workload: 2-D shock-bubble, 1024x1024 cells, FP64 (planar water shock with
post-shock p = 1e9 Pa hitting an air bubble of radius 0.15; stiffened-gas
water, ideal-gas air; zero-gradient boundaries; reinitialisation every
level-set step), advanced with the accelerated cycle (multi_dt).  One "step"
is one accelerated cycle: the slow fluid's RK step plus the fast fluid's
sub-steps, with interpolation, interaction, extension, mixing, level-set
advection/reinitialisation and the interfacial flux correction.

Metric: cell-updates/s summed over both fluids (one cell-update = one cell
holding fluid k advanced through one complete RK step of fluid k).  The JSON
line also carries the roofline of the dominant kernel (the fused face-flux +
RK stage kernel on bulk tiles, timed with HIP events on the simulation's
stream), the time of the original single-dt method over the same simulated
interval, and the CPU oracle's rate on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VECTOR_TFLOPS = 78.6      # MI355X FP64 vector peak


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (scale reference for HBM byte counters)")
    return ap.parse_args()


def stage_bytes_per_cell(D):
    # stage 1 reads its input and writes its output (2 NV doubles), stages 2
    # and 3 also read the step's base state (3 NV doubles)
    NV = D + 2
    return {1: 2 * NV * 8, 2: 3 * NV * 8}


def cpu_baseline(case_fn, seconds):
    """The CPU oracle (single thread) on the same workload at reduced
    resolution, scaled to cell-updates/s."""
    from oracle import oracle as O
    O.build(force=False)
    n = 128
    case = case_fn(n=n, seed=0)
    o = O.OracleSim(case)
    t0 = time.perf_counter()
    cells = 0
    cycles = 0
    while time.perf_counter() - t0 < seconds:
        st = o.advance(1.0, mode=1, max_cycles=1)
        cells += sum(st["cell_updates"])
        cycles += 1
    el = time.perf_counter() - t0
    return dict(value=cells / el, unit="cell-updates/s", cores=1, kind="oracle",
                sample="shock_bubble_2d at %dx%d (same physical setup), %d accelerated cycles in %.1f s"
                       % (n, n, cycles, el))


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1905_03917_amd as P
    from paper_1905_03917_amd import workloads as WL

    torch.cuda.set_device(0)
    if a.copy_probe:
        # a device-to-device copy of exactly 256 MiB read + 256 MiB written
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    case = WL.shock_bubble_2d(n=a.n, seed=0)
    D = case["ndim"]
    print("bench: shock_bubble_2d %dx%d, warmup %d, steps %d" % (a.n, a.n, a.warmup, a.steps), flush=True)

    sim = P.Sim(case)
    if a.warmup:
        sim.advance(1.0, mode=P.SIM_MULTI_DT, max_cycles=a.warmup)
    torch.cuda.synchronize()
    t_start = sim.advance(0.0, mode=P.SIM_MULTI_DT)["t"]
    sim.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = sim.advance(1.0, mode=P.SIM_MULTI_DT, max_cycles=a.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_k, launches, bytes_k = sim.profile_read()
    sim.profile(False)
    t_end = st["t"]
    updates = sum(st["cell_updates"])
    value = updates / el
    print("bench: multi_dt %d cycles in %.3f s, t %.3e -> %.3e, steps %s, n_last %.2f"
          % (st["cycles"], el, t_start, t_end, st["steps"], st["last_n"]), flush=True)

    # the original method over the same simulated interval
    single = None
    if not a.no_single:
        s2 = P.Sim(case)
        if t_start > 0:
            s2.advance(t_start, mode=P.SIM_SINGLE_DT)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st2 = s2.advance(t_end, mode=P.SIM_SINGLE_DT)
        torch.cuda.synchronize()
        el2 = time.perf_counter() - t1
        single = dict(seconds=el2, steps=st2["cycles"], speedup=el2 / el)
        print("bench: single_dt %d steps in %.3f s (speedup of multi_dt %.2f)" % (st2["cycles"], el2, el2 / el),
              flush=True)
        s2.close()

    ach_gbs = bytes_k / (ms_k * 1e-3) / 1e9 if ms_k > 0 else 0.0
    roof = dict(bound="hbm", achieved=round(ach_gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(ach_gbs / HBM_PEAK_GBS, 4), traffic=None,
                kernel="k_stage<2,bulk>", launches=launches, avg_ms=round(ms_k / max(launches, 1), 4))
    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(WL.shock_bubble_2d, a.cpu_seconds)
    out = {
        "metric": "cell-updates/s per fluid (FP64) & %HBM roofline; multi_dt vs single_dt time @ matched L1",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": el / max(st["cycles"], 1) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "shock_bubble_2d %dx%d multi_dt" % (a.n, a.n), "cells": a.n * a.n,
                   "mode": "multi_dt", "rk": 3, "cfl": 0.6},
        "per_fluid": {"air_cell_updates_per_s": st["cell_updates"][0] / el,
                      "water_cell_updates_per_s": st["cell_updates"][1] / el,
                      "steps": st["steps"]},
        "single_dt": single,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
