"""Benchmark: accelerated sharp-interface method on one MI355X.

Headline workload: 3-D shock-droplet, 256^3 cells, FP64 (a Mach-1.5 air
shock hitting a water droplet of radius 0.2; stiffened-gas water, ideal-gas
air; zero-gradient boundaries; reinitialisation every level-set step),
advanced with the accelerated cycle (multi_dt), the water fluid sub-stepped.
One "step" is one accelerated cycle: the slow fluid's RK step plus the fast
fluid's sub-steps, with interpolation, interaction, extension, mixing,
level-set advection/reinitialisation and the interfacial flux correction.

Metric: cell-updates/s summed over both fluids (one cell-update = one cell
holding fluid k advanced through one complete RK step of fluid k), timed
without kernel profiling.  The JSON line also carries the roofline of the
dominant kernel (the fused face-flux + RK stage kernel on bulk tiles),
whose launch durations come from HIP events stamped by the dispatches on
the stream the kernel runs on, in a re-run of the same cycles; the time of
the original single-dt method over the same simulated interval; the 2-D
1024^2 shock-bubble as a second workload; and the CPU oracle's rate on a
bounded sample, on one thread and on every core of the affinity mask.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
FP64_VECTOR_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
COPY_PROBE_BYTES = 1 << 30
KERNEL_SOURCES = ["paper_1905_03917_amd/csrc/sharp_kernels.hip", "paper_1905_03917_amd/csrc/sharp_device.h"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=None, help="cells per direction (default 256 in 3-D, 1024 in 2-D)")
    ap.add_argument("--case", default="shock_droplet_3d", choices=["shock_bubble_2d", "shock_droplet_3d", "oscillating_drop", "static_drop"],
                    help="workload of the timed cycles (the headline line is shock_droplet_3d at 256^3)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-2d", action="store_true", help="skip the 1024^2 shock-bubble leg")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library choose the bulk stage's grid bound during the warm-up cycles (needs --warmup >= 5)")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--cpu-worker", nargs=3, metavar=("CASE", "N", "SECONDS"),
                    help="(internal) run the oracle on CASE at N cells per direction for SECONDS and print its rate")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timing")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-instances timing")
    ap.add_argument("--no-graph", action="store_true", help="skip the captured-steps timing")
    ap.add_argument("--no-st", action="store_true", help="skip the surface-tension (oscillating drop) timing")
    ap.add_argument("--batch-only", action="store_true", help="only the batched-instances timing")
    ap.add_argument("--batch-no-sequential", action="store_true",
                    help="with --batch-only: skip advancing the instances one at a time")
    ap.add_argument("--no-l1", action="store_true", help="skip the matched-L1 comparisons (1-D tube and 3-D droplet ladders)")
    ap.add_argument("--paper-cases", action="store_true",
                    help="only the paper's own cases in its RK2 scheme: the Sec. 4.1 tubes and the Sec. 4.2 droplet "
                         "ladder (Table 1), a few minutes")
    ap.add_argument("--paper-st", action="store_true",
                    help="only the paper's surface-tension cases (static drop, drop oscillation) in RK2")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (scale reference for HBM byte counters)")
    ap.add_argument("--reduce-valu", metavar="VALU_DIR",
                    help="reduce a pass of SQ instruction counters into the executed-work record of --case/--n")
    ap.add_argument("--reduce-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="reduce two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of "
                         "'bench.py --copy-probe' into the traffic record of --case/--n, then exit")
    ap.add_argument("--kernel-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print the measured HBM traffic and achieved bandwidth of every kernel of the same two "
                         "rocprofv3 --pmc runs (markdown table), then exit")
    a = ap.parse_args()
    if a.n is None:
        a.n = 256 if a.case == "shock_droplet_3d" else 1024
    return a


def stage_bytes(D, first):
    """Algorithmic HBM bytes of one bulk cell through one stage: the stage
    input and output (NV doubles each), plus the step's base state after the
    first stage."""
    NV = D + 2
    return (2 if first else 3) * NV * 8


def stage_flops(D, first):
    """Algorithmic FP64 operations of one bulk cell through one stage (an FMA
    counts two, a division or square root one).

    Per face and component: the split fluxes F +- aU at the six stencil cells
    (24), two WENO5-JS reconstructions (66 each: candidate stencils 15,
    smoothness indicators 33, nonlinear weights 9, weighted sum 9) and the
    combination (2).  Per face: the physical fluxes (D + 4), momenta (D) and
    wave speed (1) at the six stencil cells.  Per cell: D faces, the
    primitives and sound speed (3D + 9), and per component the flux
    difference (2D) and the Shu-Osher update (2, or 5 after the first stage).
    2-D: 1411 (first stage) / 1423."""
    NV = D + 2
    face = NV * (24 + 2 * 66 + 2) + 6 * (D + 4) + 6 * D + 6
    return D * face + (3 * D + 9) + NV * (2 * D + (2 if first else 5))


def stage_kernel(D):
    """name of the bulk-tile stage kernel as the profiler prints it"""
    return "k_stage_lds<%d, false>" % D if D <= 2 else "k_stage_lds3<false>"


def record_path(case, n, what):
    """committed per-workload record of the bulk stage's counters"""
    return os.path.join(ROOT, "profiles", "stage_bulk_%s_%d_%s.json" % (case, n, what))


def bench_args(case, n):
    return "--case %s --n %d --steps 3 --warmup 1 --no-cpu --no-2d --no-single --no-l1 --no-adjoint --no-batch --no-graph --no-st" % (case, n)


def source_digest():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def reduce_counters(fetch_dir, write_dir, case, n):
    """HBM traffic of the bulk stage kernel from FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch), each scaled by what the same counter reads for the
    1 GiB device copy of --copy-probe (the largest copy dispatch)."""
    import csv
    import glob
    D = 3 if case == "shock_droplet_3d" else 2
    kname = stage_kernel(D)

    def read(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                rows += [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]
        per = {}
        for r in rows:
            key = (r["Dispatch_Id"], r["Kernel_Name"])
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
        return per

    copy_kib = COPY_PROBE_BYTES / 1024.0
    out = {}
    for name, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        per = read(d, counter)
        copies = [v for (i, k), v in per.items() if "copybuffer" in k.lower()]
        if not copies or max(copies) < 0.25 * copy_kib:
            raise SystemExit("no 1 GiB copy dispatch found in %s" % d)
        scale = copy_kib / max(copies)
        stage = [v for (i, k), v in per.items() if kname in k]
        if not stage:
            raise SystemExit("no bulk stage dispatch found in %s" % d)
        out[name] = dict(counter=counter, copy_kib_read=max(copies), scale=scale, dispatches=len(stage),
                         kib_per_dispatch=sum(stage) / len(stage))
    traffic = (out["fetch"]["kib_per_dispatch"] * out["fetch"]["scale"]
               + out["write"]["kib_per_dispatch"] * out["write"]["scale"]) * 1024.0
    args = bench_args(case, n)
    rec = dict(kernel=kname, workload="%s %s multi_dt" % (case, "x".join([str(n)] * D)),
               source_sha256=source_digest(), sources=KERNEL_SOURCES, counters=out,
               traffic_bytes_per_launch=traffic,
               commands=["timeout -s KILL 150 rocprofv3 --pmc FETCH_SIZE --output-format csv -d <FETCH_DIR> -o run "
                         "-- python -u bench.py %s --copy-probe" % args,
                         "timeout -s KILL 150 rocprofv3 --pmc WRITE_SIZE --output-format csv -d <WRITE_DIR> -o run "
                         "-- python -u bench.py %s --copy-probe" % args,
                         "python bench.py --case %s --n %d --reduce-counters <FETCH_DIR> <WRITE_DIR>" % (case, n)])
    with open(record_path(case, n, "counters"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


VALU_COUNTERS = ["SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_TRANS_F64",
                 "SQ_INSTS_VALU_FLOPS_FP64", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES"]


def kernel_traffic(fetch_dir, write_dir, top=24):
    """Measured HBM traffic of every kernel in the FETCH_SIZE and WRITE_SIZE
    passes (each scaled by what it reads for the 1 GiB copy of --copy-probe)
    and the bandwidth it achieves over its duration under the counters (the
    profiler runs the dispatches one at a time), as a markdown table."""
    import csv
    import glob

    def read(d, counter):
        per, dur = {}, {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    if r["Counter_Name"] != counter:
                        continue
                    name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("sharp::", "")
                    key = (r["Dispatch_Id"], name)
                    per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
                    dur[key] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        return per, dur

    copy_kib = COPY_PROBE_BYTES / 1024.0
    fe, fd = read(fetch_dir, "FETCH_SIZE")
    wr, _ = read(write_dir, "WRITE_SIZE")
    sf = copy_kib / max(v for (i, k), v in fe.items() if "copybuffer" in k.lower())
    sw = copy_kib / max(v for (i, k), v in wr.items() if "copybuffer" in k.lower())
    agg = {}
    for (i, k), v in fe.items():
        if k.startswith("__amd") or k.startswith("at::"):
            continue
        a = agg.setdefault(k, [0, 0.0, 0.0, 0])
        a[0] += 1
        a[1] += v * sf * 1024.0
        a[3] += fd[(i, k)]
    for (i, k), v in wr.items():
        if k in agg:
            agg[k][2] += v * sw * 1024.0
    rows = sorted(agg.items(), key=lambda kv: -kv[1][3])
    print("| kernel | dispatches | avg us | read MB | written MB | GB/s | of 8 TB/s |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for k, (n, fb, wb, ns) in rows[:top]:
        gbs = (fb + wb) / ns if ns else 0.0
        print("| `%s` | %d | %.1f | %.2f | %.2f | %.0f | %.1f%% |" % (k, n, ns / n / 1e3, fb / n / 1e6, wb / n / 1e6,
                                                                     gbs, gbs / HBM_PEAK_GBS * 100.0))


def reduce_valu(valu_dir, case, n):
    """Executed FP64 work of the bulk stage kernel from one rocprofv3 pass of
    SQ instruction counters (wave-level counts per dispatch): executed FP64
    flops (SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes), and the VALU issue bound,
    every wave64 VALU instruction holding a 16-lane SIMD for 4 cycles on
    1024 SIMDs at 2.4 GHz, against the dispatch's duration."""
    import csv
    import glob
    D = 3 if case == "shock_droplet_3d" else 2
    kname = stage_kernel(D)
    per = {}
    for f in glob.glob(os.path.join(valu_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if kname not in r["Kernel_Name"]:
                    continue
                d = per.setdefault(r["Dispatch_Id"], {})
                d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
                d["ns"] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    if not per:
        raise SystemExit("no bulk stage dispatch found in %s" % valu_dir)
    avg = {k: sum(v.get(k, 0.0) for v in per.values()) / len(per) for k in VALU_COUNTERS + ["ns"]}
    flops = avg["SQ_INSTS_VALU_FLOPS_FP64"] * 64
    issue_s = avg["SQ_INSTS_VALU"] * 4 / (1024 * 2.4e9)
    fp64 = sum(avg[k] for k in VALU_COUNTERS[:4])
    rec = dict(kernel=kname, workload="%s %s multi_dt" % (case, "x".join([str(n)] * D)),
               source_sha256=source_digest(), sources=KERNEL_SOURCES, dispatches=len(per),
               counters_per_dispatch={k: avg[k] for k in VALU_COUNTERS},
               duration_us_under_counters=avg["ns"] / 1e3,
               executed_fp64_flops_per_launch=flops,
               fp64_share_of_valu_instructions=fp64 / avg["SQ_INSTS_VALU"],
               valu_issue_bound_us=issue_s * 1e6,
               valu_issue_frac=issue_s * 1e9 / avg["ns"],
               command="timeout -s KILL 150 rocprofv3 --pmc " + " ".join(VALU_COUNTERS) + " --output-format csv "
                       "-d <VALU_DIR> -o run -- python -u bench.py %s; python bench.py --case %s --n %d "
                       "--reduce-valu <VALU_DIR>" % (bench_args(case, n), case, n))
    with open(record_path(case, n, "valu"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def committed_record(case, n, what):
    """a committed counter record of this workload, or None when the kernel
    sources changed since the counters were taken"""
    try:
        with open(record_path(case, n, what)) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    return rec if rec.get("source_sha256") == source_digest() else None


def exact_tube_1d(case, x, t):
    """Exact solution (rho, u, p) at points x and time t of the 1-D two-fluid
    stiffened-gas Riemann problem posed by a tube_1d case (the reference of
    the matched-L1 comparison): p* from f_L(p) + f_R(p) + u_R - u_L = 0 by
    bisection on the increasing function f, then the wave pattern sampled
    at x/t."""
    import numpy as np
    g, pi = case["gamma"], case["pinf"]
    sides = [(case["prim"][0, 0, 0], case["prim"][0, 1, 0], case["prim"][0, 2, 0], g[0], pi[0]),
             (case["prim"][1, 0, -1], case["prim"][1, 1, -1], case["prim"][1, 2, -1], g[1], pi[1])]

    def f(side, p):
        r, u, pk, gm, pinf = side
        a = pk + pinf
        if p > pk:   # shock
            A, B = 2.0 / ((gm + 1.0) * r), (gm - 1.0) / (gm + 1.0) * a
            return (p - pk) * np.sqrt(A / (p + pinf + B))
        c = np.sqrt(gm * a / r)
        return 2.0 * c / (gm - 1.0) * (((p + pinf) / a) ** ((gm - 1.0) / (2.0 * gm)) - 1.0)

    L, R = sides
    du = R[1] - L[1]
    lo, hi = -min(L[4], R[4]) + 1e-12, max(L[2], R[2]) * 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(L, mid) + f(R, mid) + du > 0.0:
            hi = mid
        else:
            lo = mid
    ps = 0.5 * (lo + hi)
    us = 0.5 * (L[1] + R[1]) + 0.5 * (f(R, ps) - f(L, ps))
    out = np.empty((len(x), 3))
    for i, xx in enumerate(x):
        xi = (xx - case["x_interface"]) / t
        left = xi <= us
        r, u, pk, gm, pinf = L if left else R
        sgn = -1.0 if left else 1.0
        a = pk + pinf
        c = np.sqrt(gm * a / r)
        if ps > pk:   # shock
            m = (gm - 1.0) / (gm + 1.0)
            rs = r * ((ps + pinf) / a + m) / (m * (ps + pinf) / a + 1.0)
            shock = u + sgn * c * np.sqrt((gm + 1.0) / (2.0 * gm) * (ps + pinf) / a + (gm - 1.0) / (2.0 * gm))
            out[i] = (rs, us, ps) if sgn * (xi - shock) < 0.0 else (r, u, pk)
        else:          # rarefaction
            rs = r * ((ps + pinf) / a) ** (1.0 / gm)
            cs = np.sqrt(gm * (ps + pinf) / rs)
            head, tail = u + sgn * c, us + sgn * cs
            if sgn * (xi - head) >= 0.0:
                out[i] = (r, u, pk)
            elif sgn * (xi - tail) <= 0.0:
                out[i] = (rs, us, ps)
            else:
                uf = 2.0 / (gm + 1.0) * (-sgn * c + (gm - 1.0) / 2.0 * u + xi)
                cf = -sgn * (uf - xi)
                rf = r * (cf / c) ** (2.0 / (gm - 1.0))
                pf = a * (cf / c) ** (2.0 * gm / (gm - 1.0)) - pinf
                out[i] = (rf, uf, pf)
    return out


def matched_l1(P, WL, ladder=(400, 800, 1600, 3200, 6400)):
    """The 1-D gas-water tube over a resolution ladder in both modes: GPU time
    to t_end and the relative L1 error of the density against the exact
    solution on x in [0.25, 1]; then the time of the original method
    divided by the accelerated cycle's at equal error (log-log interpolation
    of time against error along each mode's ladder)."""
    import numpy as np
    import torch
    rows = {0: [], 1: []}
    for n in ladder:
        case = WL.tube_1d(n=n, seed=0)
        x = (np.arange(n) + 0.5) / n
        ex = exact_tube_1d(case, x, case["t_end"])
        sel = x >= 0.25
        for mode in (0, 1):
            sim = P.Sim(case)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = sim.advance(case["t_end"], mode=mode)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            _, cons, alpha = sim.state(device=False)
            a0 = alpha
            rho = np.where(a0 >= 0.5, cons[0, 0] / np.maximum(a0, 1e-300), cons[1, 0] / np.maximum(1.0 - a0, 1e-300))
            l1 = np.abs(rho - ex[:, 0])[sel].sum() / np.abs(ex[:, 0])[sel].sum()
            rows[mode].append(dict(n=n, seconds=el, l1_rho=l1, cycles=st["cycles"]))
            sim.close()
    ratios = []
    ls = np.log([r["l1_rho"] for r in rows[0]])
    ts = np.log([r["seconds"] for r in rows[0]])
    order = np.argsort(ls)
    for r in rows[1]:
        l = np.log(r["l1_rho"])
        if ls.min() <= l <= ls.max():
            ratios.append(float(np.exp(np.interp(l, ls[order], ts[order])) / r["seconds"]))
    return dict(workload="tube_1d ladder %s, t_end 2.2e-4 s" % list(ladder),
                single_dt=rows[0], multi_dt=rows[1],
                time_ratio_single_over_multi_at_matched_l1=ratios,
                geomean=float(np.exp(np.mean(np.log(ratios)))) if ratios else None)


def matched_l1_3d(P, WL, ladder=(64, 128, 256), t_end=3.0e-4):
    """The 3-D shock-droplet (slow air fills 97% of the grid) over a
    resolution ladder in both modes to t_end: GPU time and the relative L1
    error of the cell-average density against the finest single-dt run
    (restricted by averaging); the time ratio single/multi at matched error
    (log-log interpolation along the single-dt ladder) on the coarser
    levels, and at the finest level the same-grid ratio with the distance
    between the two modes (far below the coarser levels' error)."""
    import numpy as np
    import torch
    rho = {}
    rows = {0: [], 1: []}
    for n in ladder:
        for mode in (0, 1):
            case = WL.shock_droplet_3d(n=n, seed=0, t_end=t_end)
            sim = P.Sim(case)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = sim.advance(t_end, mode=mode)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            _, cons, _ = sim.state(device=False)
            rho[(n, mode)] = (cons[0, 0] + cons[1, 0]).reshape(n, n, n)
            rows[mode].append(dict(n=n, seconds=el, cycles=st["cycles"], steps=st["steps"],
                                   cell_updates=st["cell_updates"]))
            sim.close()
    nf = ladder[-1]
    ref = rho[(nf, 0)]
    for mode in (0, 1):
        for r in rows[mode]:
            n = r["n"]
            f = nf // n
            R = ref.reshape(n, f, n, f, n, f).mean(axis=(1, 3, 5))
            r["l1_rho"] = float(np.abs(rho[(n, mode)] - R).mean() / np.abs(R).mean()) if n < nf else None
    dist = float(np.abs(rho[(nf, 1)] - ref).mean() / np.abs(ref).mean())
    ls = np.log([r["l1_rho"] for r in rows[0][:-1]])
    ts = np.log([r["seconds"] for r in rows[0][:-1]])
    order = np.argsort(ls)
    ratios = []
    for r in rows[1][:-1]:
        l = np.log(r["l1_rho"])
        if ls.min() <= l <= ls.max():
            ratios.append(float(np.exp(np.interp(l, ls[order], ts[order])) / r["seconds"]))
    return dict(workload="shock_droplet_3d ladder %s, t_end %.1e s, reference: %d^3 single_dt" % (list(ladder), t_end, nf),
                single_dt=rows[0], multi_dt=rows[1],
                time_ratio_single_over_multi_at_matched_l1=ratios,
                finest_same_grid_ratio=rows[0][-1]["seconds"] / rows[1][-1]["seconds"],
                finest_l1_distance_multi_vs_single=dist)


def adjoint_timing(P, WL, n=512, steps=400, ckpt=20, probes=16, multi=False):
    """The differentiable configuration: a Gaussian acoustic pulse in air
    crossing a flat air/water interface on 512^2 (zero-gradient), 400
    single-dt steps of the CFL step of the initial state, loss = sum of
    (p - 1e5)^2 at 16 probe cells in either fluid's bulk;
    gradient with respect to the initial primitives of both fluids and the
    (gamma, p_inf) of each through sim_backward (geometry frozen at the
    recorded stage level sets, a checkpoint every 20 steps).  Reports the
    forward (taped) and backward times.  With `multi`, the same interval
    (400 steps of that length) in accelerated cycles on the fluids' own CFL
    steps, a checkpoint every 20 cycles."""
    import numpy as np
    import torch
    c = WL.smooth_2d(n=n, seed=0)
    m = 0.0
    for k in (0, 1):
        W = c["prim"][k]
        cs = np.sqrt(c["gamma"][k] * (W[3] + c["pinf"][k]) / W[0])
        m = max(m, float(((np.abs(W[1]) + cs + np.abs(W[2]) + cs) * n).max()))
    dt = 0.6 / m
    prim = torch.tensor(c["prim"], device="cuda", requires_grad=True)
    eos = torch.tensor([[c["gamma"][0], c["pinf"][0]], [c["gamma"][1], c["pinf"][1]]], dtype=torch.float64,
                       device="cuda", requires_grad=True)
    # probes at least 3 cells from the interface (which moves by far less
    # than a cell in these 400 steps): each lies in one fluid's bulk
    far = WL.probe_cells(n, 2, count=4 * probes, seed=0)
    cells = [int(q) for q in far if abs(c["phi"][q]) > 3.0 * c["h"]][:probes]
    side = [0 if c["phi"][q] < 0.0 else 1 for q in cells]
    for nst in (ckpt, steps):          # a short warm-up pass, then the timed one
        prim.grad = None
        eos.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = dict(ckpt_every=ckpt, mode=P.SIM_MULTI_DT) if multi else dict(ckpt_every=ckpt, dt_fixed=dt)
        cons = P.AdvanceFn.apply(prim, eos, c, nst * dt, o)
        J = 0.0
        for cell, k in zip(cells, side):
            U = cons[k, :, cell]
            p = (eos[k, 0] - 1.0) * (U[3] - 0.5 * (U[1] ** 2 + U[2] ** 2) / U[0]) - eos[k, 0] * eos[k, 1]
            J = J + (p - 1.0e5) ** 2
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    g = prim.grad
    what = ("accelerated cycles over the interval of %d single-dt steps" % steps) if multi else \
        ("%d single-dt steps" % steps)
    return dict(workload="smooth_2d %dx%d (air pulse at a flat air/water interface), %s, %d probes, "
                         "checkpoint every %d, geometry frozen at the recorded level sets" % (n, n, what, probes, ckpt),
                forward_s=t1 - t0, backward_s=t2 - t1, backward_over_forward=(t2 - t1) / (t1 - t0),
                cell_steps_per_s_backward=n * n * steps / (t2 - t1),
                grad_norm=[float(torch.linalg.vector_norm(g[k])) for k in (0, 1)],
                d_gamma=[float(eos.grad[k, 0]) for k in (0, 1)], d_pinf=[float(eos.grad[k, 1]) for k in (0, 1)])


def batch_timing(P, WL, cycles_multi=3, steps_single=10, one_at_a_time=True):
    """The batched configuration: 512 independent instances (384 1-D
    water-air tubes with N ~ U[200, 4000] and 128 2-D collapsing air bubbles
    in water on n^2 grids, n ~ U[64, 512], seeded density ratios 1-1e3 and
    pressure ratios 1-1e4), advanced by sim_batch_advance with launches
    fused across the instances; beside it the same instances advanced one
    at a time by sim_advance (fresh copies, the same cycles).  One warm-up
    cycle precedes each timed leg."""
    import numpy as np
    import torch
    cases = WL.batch_cases(seed=0)
    cells = sum(int(np.prod(c["n"][:c["ndim"]])) for c in cases)
    res = dict(workload="batch of %d: %d 1-D tubes N in [200, 4000], %d 2-D bubbles n^2, n in [64, 512]"
                        % (len(cases), sum(c["ndim"] == 1 for c in cases), sum(c["ndim"] == 2 for c in cases)),
               instances=len(cases), cells=cells)
    for mode, K, key in ((P.SIM_MULTI_DT, cycles_multi, "multi_dt"), (P.SIM_SINGLE_DT, steps_single, "single_dt")):
        sims = [P.Sim(c, serial=1) for c in cases]
        b = P.Batch(sims)
        b.advance(1.0, mode=mode, max_cycles=1)
        torch.cuda.synchronize()
        i0 = b.info()
        t0 = time.perf_counter()
        st = b.advance(1.0, mode=mode, max_cycles=K)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        i1 = b.info()
        ub = sum(sum(x["cell_updates"]) for x in st)
        b.close()
        for x in sims:
            x.close()
        res[key] = dict(cycles=K, batched_s=tb, cell_updates=ub, value=ub / tb,
                        passes=i1["passes"] - i0["passes"], fused_launches=i1["fused_launches"] - i0["fused_launches"],
                        launch_records=i1["records"] - i0["records"])
        if not one_at_a_time:
            continue
        sims = [P.Sim(c, serial=1) for c in cases]
        for x in sims:
            x.advance(1.0, mode=mode, max_cycles=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        us = 0
        for x in sims:
            us += sum(x.advance(1.0, mode=mode, max_cycles=K)["cell_updates"])
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        for x in sims:
            x.close()
        res[key].update(one_at_a_time_s=ts, one_at_a_time_value=us / ts, speedup=(ub / tb) / (us / ts))
    return res


def graph_timing(P, WL, steps=200):
    """Captured single-dt steps (opts graph=2: captured at any size) against
    the same steps issued launch by launch (default schedule), at a fixed
    step (half the first CFL step): 1-D water-air tubes of 400 and 4000 cells
    and the 2-D shock-bubble case at 128^2 to 1024^2, which brackets the
    largest grid graph=1 captures.  Reports ms per step of each and checks
    that both reach the same state bit for bit."""
    import torch
    res = []
    for name, case in (("tube_1d 400", WL.tube_1d(n=400, seed=0)),
                       ("tube_1d 4000", WL.tube_1d(n=4000, seed=0)),
                       ("shock_bubble_2d 128x128", WL.shock_bubble_2d(n=128, seed=0)),
                       ("shock_bubble_2d 256x256", WL.shock_bubble_2d(n=256, seed=0)),
                       ("shock_bubble_2d 512x512", WL.shock_bubble_2d(n=512, seed=0)),
                       ("shock_bubble_2d 1024x1024", WL.shock_bubble_2d(n=1024, seed=0))):
        s0 = P.Sim(case)
        dt = 0.5 * min(s0.advance(1.0, P.SIM_SINGLE_DT, max_cycles=1)["last_dt"])
        s0.close()
        row = dict(workload=name, dt=dt, steps=steps)
        states = []
        for key, g in (("launches", 0), ("graph", 2)):
            sim = P.Sim(case, dt_fixed=dt, graph=g)
            sim.advance(1.0, P.SIM_SINGLE_DT, max_cycles=4)     # warm-up (and the captures)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = sim.advance(1.0, P.SIM_SINGLE_DT, max_cycles=steps)
            torch.cuda.synchronize()
            row[key + "_ms_per_step"] = (time.perf_counter() - t0) / st["cycles"] * 1e3
            if g:
                row["captures"], row["replays"], _ = sim.graph_info()
            states.append(sim.state())
            sim.close()
        row["speedup"] = row["launches_ms_per_step"] / row["graph_ms_per_step"]
        row["identical"] = all(torch.equal(x, y) for x, y in zip(states[0], states[1]))
        res.append(row)
    return res


def graph_cycle_timing(P, WL, cycles=40):
    """Captured accelerated cycles (opts dt_fixed_fluid: both fluids' steps
    prescribed, half their first CFL steps; graph=2) against the same cycles
    issued launch by launch: the 1-D water-air tube at 400 and 4000 cells and
    the 2-D shock-bubble at 128^2, 256^2 and 512^2.  Reports ms per cycle of each,
    the fast sub-steps per cycle, and whether both reach the same state bit
    for bit."""
    import torch
    res = []
    for name, case in (("tube_1d 400", WL.tube_1d(n=400, seed=0)),
                       ("tube_1d 4000", WL.tube_1d(n=4000, seed=0)),
                       ("shock_bubble_2d 128x128", WL.shock_bubble_2d(n=128, seed=0)),
                       ("shock_bubble_2d 256x256", WL.shock_bubble_2d(n=256, seed=0)),
                       ("shock_bubble_2d 512x512", WL.shock_bubble_2d(n=512, seed=0))):
        s0 = P.Sim(case)
        dts = [0.5 * x for x in s0.advance(1.0, P.SIM_MULTI_DT, max_cycles=1)["last_dt"]]
        s0.close()
        row = dict(workload=name + " accelerated cycles", dt_fixed_fluid=dts, cycles=cycles)
        states = []
        for key, g in (("launches", 0), ("graph", 2)):
            sim = P.Sim(case, dt_fixed_fluid=dts, graph=g)
            sim.advance(1.0, P.SIM_MULTI_DT, max_cycles=4)     # warm-up (and the captures)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = sim.advance(1.0, P.SIM_MULTI_DT, max_cycles=cycles)
            torch.cuda.synchronize()
            row[key + "_ms_per_cycle"] = (time.perf_counter() - t0) / st["cycles"] * 1e3
            row["steps_per_fluid"] = st["steps"]
            if g:
                row["captures"], row["replays"], _ = sim.graph_info()
            states.append(sim.state())
            sim.close()
        row["speedup"] = row["launches_ms_per_cycle"] / row["graph_ms_per_cycle"]
        row["identical"] = all(torch.equal(x, y) for x, y in zip(states[0], states[1]))
        res.append(row)
    return res


def surface_tension_timing(P, WL, steps=20, warmup=1):
    """The Sec. 4.5 oscillating drop (surface tension: the Laplace jump in
    every interaction).  At the paper's 128^2, one period (t = 0.0878) in
    each mode from t = 0, after a warm-up run: r_s = original time /
    accelerated time (the paper's 2.196 on its CPU is context only).  At
    1024^2, `steps` accelerated cycles after `warmup` against the original
    method over the same interval: cell-updates/s summed over both fluids."""
    import torch
    c = WL.oscillating_drop(128)
    res = {"workload": "oscillating_drop 128x128, one period", "t_end": c["period"]}
    w = P.Sim(c)
    w.advance(1.0, mode=P.SIM_MULTI_DT, max_cycles=2)
    w.advance(1.0, mode=P.SIM_SINGLE_DT, max_cycles=2)
    w.close()
    for mode, key in ((P.SIM_SINGLE_DT, "single_dt"), (P.SIM_MULTI_DT, "multi_dt")):
        sim = P.Sim(c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = sim.advance(c["period"], mode=mode)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        sim.close()
        res[key] = dict(seconds=el, cycles=st["cycles"], steps=st["steps"], value=sum(st["cell_updates"]) / el)
    res["r_s"] = res["single_dt"]["seconds"] / res["multi_dt"]["seconds"]
    c2 = WL.oscillating_drop(1024)
    h = time_workload(P, c2, steps, warmup)
    res["oscillating_drop_1024"] = dict(workload="oscillating_drop 1024x1024 multi_dt", value=h["value"],
                                        unit="cell-updates/s",
                                        ms_per_cycle=h["seconds"] / max(h["st"]["cycles"], 1) * 1e3,
                                        steps_per_fluid=h["st"]["steps"], single_dt=h.get("single"))
    return res


def paper_cases(P, WL, ladder=(32, 64, 128, 256), n3=128, frac3=0.1, skip3=False):
    """The paper's compressible cases in its TVD-RK2 scheme (Tait water as the
    stiffened gas of its isentrope): the two 1-D tubes of Sec. 4.1 at 200
    cells in both modes (relative L1 of the density against the exact
    solution), and the Sec. 4.2 droplet over one period on 32^2 .. 256^2
    and a tenth of a period on 128^3, timed in both modes (r_s = original
    time / accelerated time, beside Table 1 as context), with the droplet's
    area error E(area) = |S - 0.01 pi| / (0.01 pi) after the period and its
    relative mass."""
    import math
    import numpy as np
    import torch
    out = dict(tubes=[], droplet=[])
    for name in ("e1_gas_water_tube", "e2_shock_air_water"):
        c = getattr(WL, name)(n=200)
        x = (np.arange(200) + 0.5) / 200
        ex = exact_tube_1d(c, x, c["t_end"])[:, 0]
        row = dict(case=name)
        for mode in (0, 1):
            s = P.Sim(c, rk=2)
            st = s.advance(c["t_end"], mode=mode)
            _, cons, alpha = s.state(device=False)
            s.close()
            rho = np.where(alpha >= 0.5, cons[0, 0] / np.maximum(alpha, 1e-300),
                           cons[1, 0] / np.maximum(1 - alpha, 1e-300))
            row["l1_rho_%s" % ("multi" if mode else "single")] = float(np.abs(rho - ex).mean() / np.abs(ex).mean())
            row["steps_%s" % ("multi" if mode else "single")] = st["steps"]
        out["tubes"].append(row)
    table1 = {32: 1.539, 64: 1.923, 128: 2.322, 256: 2.873, "128^3": 2.862}
    for ndim, n in [(2, m) for m in ladder] + ([] if skip3 else [(3, n3)]):
        c = WL.e3_droplet(n=n, ndim=ndim)
        t_end = c["t_end"] * (1.0 if ndim == 2 else frac3)
        row = dict(grid="x".join([str(n)] * ndim), t_end=t_end)
        for mode in (0, 1):
            s = P.Sim(c, rk=2)
            m0 = s.totals()[0, 0]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = s.advance(t_end, mode=mode)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            key = "multi" if mode else "single"
            row["seconds_" + key] = el
            row["cycles_" + key] = st["cycles"]
            row["steps_" + key] = st["steps"]
            row["relative_mass_" + key] = float(s.totals()[0, 0] / m0)
            print("bench: paper droplet %s %s: %.2f s, %d cycles" % (row["grid"], key, el, st["cycles"]), flush=True)
            if ndim == 2:
                _, _, alpha = s.state(device=False)
                area = float(alpha.sum()) / n ** 2
                row["area_error_" + key] = abs(area - 0.01 * math.pi) / (0.01 * math.pi)
            s.close()
        row["r_s"] = row["seconds_single"] / row["seconds_multi"]
        row["paper_r_s"] = table1[n if ndim == 2 else "128^3"]
        out["droplet"].append(row)
        print("bench: paper droplet %s: single %.2f s, multi %.2f s, r_s %.2f (paper, CPU: %.3f)"
              % (row["grid"], row["seconds_single"], row["seconds_multi"], row["r_s"], row["paper_r_s"]), flush=True)
    return out


def _drop_jump(case, cons, alpha):
    """mean pressure of the drop's pure cells (more than 2 cells inside)
    minus that of the pure gas cells from 2 cells outside to 3 radii"""
    import numpy as np
    D, n = case["ndim"], case["n"][0]
    h = case["h"]
    x = (np.arange(n) + 0.5) * h
    grids = np.meshgrid(*([x] * D), indexing="ij")
    r = np.sqrt(sum((grids[D - 1 - d] - case["centre"][d]) ** 2 for d in range(D))).reshape(-1)
    R = case["radius"]
    p = []
    for k in range(2):
        a = alpha if k == 0 else 1.0 - alpha
        m = a > 0.5
        U = cons[k][:, m] / a[m]
        ke = 0.5 * sum(U[1 + d] ** 2 for d in range(D)) / U[0]
        pk = np.full(alpha.shape, np.nan)
        pk[m] = (case["gamma"][k] - 1.0) * (U[D + 1] - ke) - case["gamma"][k] * case["pinf"][k]
        p.append(pk)
    inner = (alpha > 1.0 - 1e-9) & (r < R - 2.0 * h)
    outer = (alpha < 1e-9) & (r > R + 2.0 * h) & (r < 3.0 * R)
    return float(p[0][inner].mean() - p[1][outer].mean())


def paper_st_cases(P, WL, ladder=(32, 64, 128, 256), t_drop=0.05):
    """The paper's surface-tension cases in its TVD-RK2 scheme: the Sec. 4.3
    static drop (started at its Laplace equilibrium; the inviscid run from
    the paper's uniform start does not settle) to t = t_drop on 32^2 ..
    256^2, timed in both modes (r_s beside Table 2 as context), with the
    relative error of the mean pressure jump against sigma/R = 360; and the
    Sec. 4.5 drop oscillation at 128^2: its period (the extent along x
    through the centre, first minimum, twice its time) against the 0.0878
    of Eq. (oscillation), and r_s over one period."""
    import numpy as np
    import torch
    out = dict(static_drop=[], oscillating_drop=None)
    table2 = {32: 1.595, 64: 2.153, 128: 2.531, 256: 3.1048}
    for n in ladder:
        c = WL.static_drop(n, 2)
        row = dict(grid="%dx%d" % (n, n), t_end=t_drop)
        for mode in (0, 1):
            s = P.Sim(c, rk=2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = s.advance(t_drop, mode=mode)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            _, cons, alpha = s.state(device=False)
            s.close()
            key = "multi" if mode else "single"
            row["seconds_" + key] = el
            row["steps_" + key] = st["steps"]
            row["jump_error_" + key] = abs(_drop_jump(c, cons, alpha) - 360.0) / 360.0
        row["r_s"] = row["seconds_single"] / row["seconds_multi"]
        row["paper_r_s"] = table2[n]
        out["static_drop"].append(row)
        print("bench: paper static drop %s: single %.2f s, multi %.2f s, r_s %.2f (paper, CPU: %.3f), "
              "E(dp) %.2e / %.2e" % (row["grid"], row["seconds_single"], row["seconds_multi"], row["r_s"],
                                     row["paper_r_s"], row["jump_error_single"], row["jump_error_multi"]), flush=True)
    c = WL.oscillating_drop(128)
    h = c["h"]
    j0 = int(round(c["centre"][1] / h - 0.5))
    row = dict(grid="128x128", paper_period=c["period"], paper_r_s=2.196)
    for mode in (0, 1):
        key = "multi" if mode else "single"
        s = P.Sim(c, rk=2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance(c["period"], mode=mode)
        torch.cuda.synchronize()
        row["seconds_" + key] = time.perf_counter() - t0
        s.close()
        s = P.Sim(c, rk=2)
        ts, ext = [], []
        while True:
            st = s.advance(1e30, mode=mode, max_cycles=1)
            rw = s.state(device=False)[0].reshape(128, 128)[j0]
            i = np.where((rw[:-1] >= 0) != (rw[1:] >= 0))[0]
            i = i[i >= 64][0]
            ts.append(st["t"])
            ext.append((i + 0.5 + rw[i] / (rw[i] - rw[i + 1])) * h - c["centre"][0])
            if st["t"] > 0.055:
                break
        s.close()
        k = int(np.argmin(ext))
        A = np.polyfit(np.array(ts[k - 1:k + 2]) - ts[k], ext[k - 1:k + 2], 2)
        row["period_" + key] = 2.0 * (ts[k] - A[1] / (2.0 * A[0]))
    row["r_s"] = row["seconds_single"] / row["seconds_multi"]
    out["oscillating_drop"] = row
    print("bench: paper oscillating drop 128^2: period %.5f / %.5f (0.0878), single %.2f s, multi %.2f s, r_s %.2f "
          "(paper, CPU: 2.196)" % (row["period_single"], row["period_multi"], row["seconds_single"],
                                   row["seconds_multi"], row["r_s"]), flush=True)
    return out


def cpu_worker(case_name, n, seconds):
    """(child process) the oracle as it is, on one thread: accelerated cycles
    of the workload at n cells per direction for about `seconds`"""
    from oracle import oracle as O
    from paper_1905_03917_amd import workloads as WL
    case = getattr(WL, case_name)(n=n, seed=0)
    o = O.OracleSim(case)
    t0 = time.perf_counter()
    cells = cycles = 0
    while time.perf_counter() - t0 < seconds:
        st = o.advance(1.0, mode=1, max_cycles=1)
        cells += sum(st["cell_updates"])
        cycles += 1
    print(json.dumps(dict(cells=cells, cycles=cycles, seconds=time.perf_counter() - t0)), flush=True)


def cpu_baseline(case_name, n, seconds):
    """The CPU oracle (plain C, one thread per process) on a bounded sample of
    the headline workload: the same physical setup at n cells per direction,
    accelerated cycles for about `seconds`, first alone, then in one process
    per core of the affinity mask (at most 16, one GPU's share of the host) at once;
    the aggregate of the second is the all-core rate."""
    import subprocess
    from oracle import oracle as O
    O.build(force=False)
    cores = min(len(os.sched_getaffinity(0)), 16)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-worker", case_name, str(n), str(seconds)]

    def run(k):
        procs = [subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True, env=env) for _ in range(k)]
        outs = [json.loads(p.communicate()[0].strip().splitlines()[-1]) for p in procs]
        if any(p.returncode for p in procs):
            raise RuntimeError("oracle worker failed")
        return outs

    one = run(1)[0]
    many = run(cores)
    agg = sum(r["cells"] / r["seconds"] for r in many)
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    dims = {"shock_droplet_3d": 3, "shock_bubble_2d": 2}[case_name]
    grid = "x".join([str(n)] * dims)
    return dict(value=agg, unit="cell-updates/s", cores=cores, kind="oracle",
                sample="%s at %s (same physical setup as the timed workload), accelerated cycles for %.0f s: "
                       "one oracle process per core of the affinity mask (%d), summed; alone on one core: %.4g "
                       "cell-updates/s (%d cycles)" % (case_name, grid, seconds, cores, one["cells"] / one["seconds"],
                                                         one["cycles"]),
                single_thread=one["cells"] / one["seconds"], cpu_model=cpu_model)


def time_workload(P, case, steps, warmup, want_single=True):
    """The accelerated cycle on `case`: `steps` timed cycles after `warmup`
    (no kernel profiling), the original method over the same simulated
    interval, and a re-run of the same cycles with the bulk stage's launches
    bracketed by dispatch-stamped events (its roofline)."""
    import torch
    D = case["ndim"]
    res = {}
    sim = P.Sim(case)
    if warmup:
        sim.advance(1.0, mode=P.SIM_MULTI_DT, max_cycles=warmup)
    torch.cuda.synchronize()
    t_start = sim.advance(0.0, mode=P.SIM_MULTI_DT)["t"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = sim.advance(1.0, mode=P.SIM_MULTI_DT, max_cycles=steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    bulk_bound, _, serial_sched = sim.tuned()
    sim.close()
    res.update(seconds=el, st=st, t_start=t_start, t_end=st["t"], bulk_bound=bulk_bound, serial=serial_sched,
               value=sum(st["cell_updates"]) / el)
    # the original method over the same simulated interval
    if want_single:
        s2 = P.Sim(case)
        if t_start > 0:
            s2.advance(t_start, mode=P.SIM_SINGLE_DT)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st2 = s2.advance(st["t"], mode=P.SIM_SINGLE_DT)
        torch.cuda.synchronize()
        el2 = time.perf_counter() - t1
        s2.close()
        res["single"] = dict(seconds=el2, steps=st2["cycles"], speedup=el2 / el,
                             cell_updates=st2["cell_updates"])
    # the same cycles again, with the bulk stage's launches timed
    sim = P.Sim(case)
    if warmup:
        sim.advance(1.0, mode=P.SIM_MULTI_DT, max_cycles=warmup)
    sim.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stp = sim.advance(1.0, mode=P.SIM_MULTI_DT, max_cycles=steps)
    torch.cuda.synchronize()
    res["profiled_seconds"] = time.perf_counter() - t0
    ms_k, launches, cells_k, first_k = sim.profile_read()
    sim.profile(False)
    sim.close()
    assert stp["steps"] == st["steps"], (stp["steps"], st["steps"])
    flops_k = first_k * stage_flops(D, True) + (cells_k - first_k) * stage_flops(D, False)
    bytes_k = first_k * stage_bytes(D, True) + (cells_k - first_k) * stage_bytes(D, False)
    sec_k = ms_k * 1e-3
    res["kernel"] = dict(ms=ms_k, launches=launches, flops=flops_k, bytes=bytes_k, seconds=sec_k)
    return res


def roofline(case_name, n, D, k):
    """roofline object of the bulk stage kernel from its timed launches"""
    sec_k, launches = k["seconds"], max(k["launches"], 1)
    ach_tf = k["flops"] / sec_k / 1e12 if sec_k > 0 else 0.0
    ach_gbs = k["bytes"] / sec_k / 1e9 if sec_k > 0 else 0.0
    cnt = committed_record(case_name, n, "counters")
    roof = dict(bound="alu", achieved=round(ach_tf, 2), peak=round(FP64_VECTOR_TFLOPS, 1), unit="TFLOP/s",
                frac=round(ach_tf / FP64_VECTOR_TFLOPS, 4),
                traffic=round(cnt["traffic_bytes_per_launch"]) if cnt else None,
                kernel=stage_kernel(D), launches=k["launches"], avg_ms=round(k["ms"] / launches, 4),
                flops_per_launch=round(k["flops"] / launches),
                algorithmic_bytes_per_launch=round(k["bytes"] / launches),
                hbm=dict(achieved=round(ach_gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                         frac=round(ach_gbs / HBM_PEAK_GBS, 4)))
    valu = committed_record(case_name, n, "valu")
    if valu and sec_k > 0:
        ex_tf = valu["executed_fp64_flops_per_launch"] * k["launches"] / sec_k / 1e12
        roof["executed"] = dict(fp64_flops_per_launch=round(valu["executed_fp64_flops_per_launch"]),
                                achieved=round(ex_tf, 2), frac=round(ex_tf / FP64_VECTOR_TFLOPS, 4),
                                valu_issue_bound_us=round(valu["valu_issue_bound_us"], 1),
                                valu_issue_frac=round(valu["valu_issue_bound_us"] / (k["ms"] * 1e3 / launches), 4))
    return roof


def speedup_model(st, single):
    """Eq. (speedup_ratio) of Sec. 3.1 with the measured step ratio and the
    slow fluid's share m of the original method's work (cell-updates as the
    proxy of work), beside the measured ratio"""
    import math
    S = 0 if st["steps"][0] < st["steps"][1] else 1
    F = 1 - S
    n = st["steps"][F] / max(st["steps"][S], 1)
    cu = single["cell_updates"]
    m = cu[S] / max(cu[0] + cu[1], 1)
    nc = math.ceil(n - 1e-9)
    pred = n / (nc - (nc - 1) * m) if nc > 0 else None
    return dict(fast_substeps_per_cycle=n, slow_share_m=m, predicted=pred, measured=single["speedup"])


def main():
    a = parse()
    if a.cpu_worker:
        cpu_worker(a.cpu_worker[0], int(a.cpu_worker[1]), float(a.cpu_worker[2]))
        return
    if a.kernel_traffic:
        kernel_traffic(*a.kernel_traffic)
        return
    if a.reduce_counters:
        reduce_counters(*a.reduce_counters, a.case, a.n)
        return
    if a.reduce_valu:
        reduce_valu(a.reduce_valu, a.case, a.n)
        return
    if a.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1905_03917_amd as P
    from paper_1905_03917_amd import workloads as WL

    torch.cuda.set_device(0)
    if a.batch_only:
        print(json.dumps({"batch": batch_timing(P, WL, one_at_a_time=not a.batch_no_sequential)}), flush=True)
        return
    if a.paper_cases:
        print(json.dumps({"paper_cases": paper_cases(P, WL)}), flush=True)
        return
    if a.paper_st:
        print(json.dumps({"paper_st_cases": paper_st_cases(P, WL)}), flush=True)
        return
    if a.copy_probe:
        # a device-to-device copy of exactly 1 GiB read + 1 GiB written; a
        # 1 GiB fill in between evicts the source from the 256 MB last-level
        # cache, so the copy's reads come from HBM
        src = torch.ones(COPY_PROBE_BYTES // 8, dtype=torch.float64, device="cuda")
        flush = torch.zeros_like(src)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, flush, dst
    case = getattr(WL, a.case)(n=a.n, seed=0)
    D = case["ndim"]
    grid_name = "x".join([str(a.n)] * D)
    print("bench: %s %s, warmup %d, steps %d" % (a.case, grid_name, a.warmup, a.steps), flush=True)
    h = time_workload(P, case, a.steps, a.warmup, want_single=not a.no_single)
    st, el = h["st"], h["seconds"]
    print("bench: multi_dt %d cycles in %.3f s, t %.3e -> %.3e, steps %s, cells %s (profiled re-run %.3f s)"
          % (st["cycles"], el, h["t_start"], h["t_end"], st["steps"], st["active_cells"], h["profiled_seconds"]),
          flush=True)
    single = h.get("single")
    if single:
        single = dict(single, speedup_model=speedup_model(st, single))
        print("bench: single_dt %d steps in %.3f s (speedup of multi_dt %.2f)"
              % (single["steps"], single["seconds"], single["speedup"]), flush=True)
    roof = roofline(a.case, a.n, D, h["kernel"])
    # the 1024^2 shock-bubble: the second workload (its own roofline)
    w2d = None
    if not a.no_2d and a.case != "shock_bubble_2d":
        c2 = WL.shock_bubble_2d(n=1024, seed=0)
        h2 = time_workload(P, c2, a.steps, a.warmup, want_single=not a.no_single)
        w2d = dict(workload="shock_bubble_2d 1024x1024 multi_dt", value=h2["value"], unit="cell-updates/s",
                   ms_per_step=h2["seconds"] / max(h2["st"]["cycles"], 1) * 1e3, steps_per_fluid=h2["st"]["steps"],
                   single_dt=h2.get("single"), roofline=roofline("shock_bubble_2d", 1024, 2, h2["kernel"]))
        print("bench: shock_bubble_2d 1024^2: %.3e cell-updates/s, %.3f ms per cycle, single_dt speedup %s"
              % (w2d["value"], w2d["ms_per_step"], h2.get("single", {}).get("speedup")), flush=True)
    bat = None
    if not a.no_batch:
        bat = batch_timing(P, WL)
        print("bench: batch of %d: multi_dt %.3e cell-updates/s (%.1fx one at a time), single_dt %.3e (%.1fx)"
              % (bat["instances"], bat["multi_dt"]["value"], bat["multi_dt"]["speedup"], bat["single_dt"]["value"],
                 bat["single_dt"]["speedup"]), flush=True)
    gph = None
    if not a.no_graph:
        gph = graph_timing(P, WL)
        print("bench: captured steps: %s" % ", ".join("%s %.3f -> %.3f ms (%.2fx, identical %s)"
              % (r["workload"], r["launches_ms_per_step"], r["graph_ms_per_step"], r["speedup"], r["identical"])
              for r in gph), flush=True)
        gph_c = graph_cycle_timing(P, WL)
        print("bench: captured cycles: %s" % ", ".join("%s %.3f -> %.3f ms (%.2fx, identical %s)"
              % (r["workload"], r["launches_ms_per_cycle"], r["graph_ms_per_cycle"], r["speedup"], r["identical"])
              for r in gph_c), flush=True)
        gph = dict(steps=gph, cycles=gph_c)
    stt = None
    if not a.no_st:
        stt = surface_tension_timing(P, WL)
        print("bench: oscillating drop (surface tension) 128^2 one period: single %.3f s, multi %.3f s (r_s %.2f); "
              "1024^2: %.3e cell-updates/s, %.2f ms per cycle, single_dt speedup %.2f"
              % (stt["single_dt"]["seconds"], stt["multi_dt"]["seconds"], stt["r_s"],
                 stt["oscillating_drop_1024"]["value"], stt["oscillating_drop_1024"]["ms_per_cycle"],
                 stt["oscillating_drop_1024"]["single_dt"]["speedup"]), flush=True)
    ml1 = None
    if not a.no_l1:
        ml1 = matched_l1(P, WL)
        print("bench: matched L1 (1-D tube ladder): single/multi time ratios %s"
              % ml1["time_ratio_single_over_multi_at_matched_l1"], flush=True)
        ml1_3d = matched_l1_3d(P, WL)
        ml1["droplet_3d"] = ml1_3d
        print("bench: matched L1 (3-D droplet ladder): single/multi time ratios %s, same grid %d^3 %.2f"
              % (ml1_3d["time_ratio_single_over_multi_at_matched_l1"], ml1_3d["single_dt"][-1]["n"],
                 ml1_3d["finest_same_grid_ratio"]), flush=True)
    adj = None
    if not a.no_adjoint:
        adj = adjoint_timing(P, WL)
        print("bench: adjoint (512^2 air/water, 400 steps): forward %.3f s, backward %.3f s"
              % (adj["forward_s"], adj["backward_s"]), flush=True)
        adj["multi_dt"] = adjoint_timing(P, WL, multi=True)
        print("bench: adjoint (512^2 air/water, accelerated cycles over the same interval): forward %.3f s, "
              "backward %.3f s" % (adj["multi_dt"]["forward_s"], adj["multi_dt"]["backward_s"]), flush=True)
    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(a.case, 48 if D == 3 else 128, a.cpu_seconds)
        print("bench: oracle %.3e cell-updates/s on %d cores (%.3e on one)" % (cpu["value"], cpu["cores"],
              cpu["single_thread"]), flush=True)
    out = {
        "metric": "cell-updates/s per fluid (FP64) & %HBM roofline; multi_dt vs single_dt time @ matched L1",
        "value": h["value"],
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
        "config": {"workload": "%s %s multi_dt" % (a.case, grid_name), "cells": a.n ** D,
                   "mode": "multi_dt", "rk": 3, "cfl": 0.6, "bulk_grid_bound": h["bulk_bound"],
                   "schedule": "serial" if h["serial"] else "overlapped"},
        "per_fluid": {("%s_cell_updates_per_s" % ("air" if case["gamma"][k] == 1.4 else "water")):
                      st["cell_updates"][k] / el for k in range(2)},
        "cells_per_fluid": st["active_cells"],
        "steps_per_fluid": st["steps"],
        "single_dt": single,
        "shock_bubble_2d_1024": w2d,
        "matched_l1": ml1,
        "adjoint": adj,
        "batch": bat,
        "graph": gph,
        "surface_tension": stt,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
