"""Benchmark of the kinetic IMEX stage (coupled ES-BGK / Euler, 2D2V) on one GPU.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--precision fp32|bf16|fp64]
                    [--workload riemann4|blast|shear] [--no-cpu-baseline]

Workload (default): four-quadrant Riemann problem on a periodic 256 x 256 grid
with a 32 x 32 velocity grid on [-10, 10]^2, Knudsen number varying smoothly
from 1e-4 to 1, ARS(2,3,3), minmod reconstruction, FP32, regime indicator on
every step (domain decomposition active).  A step is one pass of Algorithm 1:
regime update + compaction, two implicit kinetic stages, the final
combination, and the Euler stages on fluid cells.

Prints ONE JSON line.  `value` is phase-space point-updates per second per
implicit IMEX stage: sum over timed steps of (kinetic cells x nv^2 x 2) / time.
The roofline entry is for the kernel with the largest share of the step,
timed with HIP events on its stream during the timed region; its algorithmic
bytes per point are the f-array passes it must make.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")

WORKLOADS = {
    # name: (generator, kwargs, nx, nv, vmax, steps in the configuration)
    "riemann4": dict(gen="riemann4", nx=256, nv=32, vmax=10.0, kw=dict(seed=0), steps=200),
    # the learned indicator's evaluation size (trained on 256^2 runs of the same generator)
    "riemann4_1024": dict(gen="riemann4", nx=1024, nv=32, vmax=10.0, kw=dict(seed=1000), steps=300),
    "shear": dict(gen="shear_modes", nx=512, nv=48, vmax=8.0, kw=dict(seed=0), steps=100),
    "blast": dict(gen="blast", nx=1024, nv=64, vmax=20.0, kw=dict(), steps=200),
}

# f-array passes (reads + writes) per point of each kinetic kernel class:
# (state arrays f^n / f^{n+1}, stage arrays f^(2), f^(3), partial sum P).  The
# last implicit stage writes P, the final combination reads P and f^(3).
PASSES = {"stage2": (1, 1, 0), "stage3": (1, 2, 1), "final": (1, 1, 1)}
# bytes per value of (state, stage, partial) arrays.  The mixed form stores
# f^(2) - f^n in BF16, f^(3) in FP32 and P - f^(3) in BF16: per kernel the same
# byte counts as (4, 2, 4) with f^(3) and P exchanged.
ELEM = {"fp64": (8, 8, 8), "fp32": (4, 4, 4), "bf16": (2, 2, 4), "mixed": (4, 2, 4)}


def kernel_source_digest():
    """sha256 of the sources the kinetic stage kernels are built from: a
    recorded traffic figure holds only for the kernels it was measured on."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2512_03586_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name in ("device.h", "kernels.h", "kinetic_impl.h") or (name.startswith("kinetic_") and name.endswith(".hip")):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def recorded_traffic(kernel, workload, precision, steps):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary of this same command, or None when the kernel sources,
    the workload or the step count differ from the profiled run."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_digest():
        return None
    e = rec.get("kernels", {}).get(kernel)
    if not e or rec.get("workload") != workload or rec.get("precision") != precision or rec.get("steps") != steps:
        return None
    return e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0, help="timed steps (default: the workload's, 200 or 300)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp64", "mixed"])
    ap.add_argument("--workload", default="riemann4", choices=sorted(WORKLOADS))
    ap.add_argument("--indicator", default="plain", choices=["plain", "learned", "dilated"],
                    help="plain: the criterion every step; learned: the trained network between plain checks "
                         "every --learned-k steps (trained first, untimed, on other seeds of the generator); "
                         "dilated: the plain check every K steps with its mask dilated")
    ap.add_argument("--learned-k", type=int, default=10)
    ap.add_argument("--train-seeds", type=int, default=8)
    ap.add_argument("--learned-miss", type=float, default=2e-3,
                    help="threshold: the fraction of held-out positive cells allowed below it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--error-vs-fp64", action="store_true",
                    help="after the timed run, run the FP64 form with the plain indicator (the path the "
                         "parity tests hold to the oracle at 1e-10) over the same steps and report the "
                         "relative L1 density error of the timed run against it")
    ap.add_argument("--cpu-steps", type=int, default=16)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device tensor copy of MIB MiB (a kernel of "
                         "known traffic, to scale HBM byte counters)")
    ap.add_argument("--record-traffic", nargs=3, metavar=("STATS_CSV", "FETCH_CSV", "WRITE_CSV"),
                    help="no GPU: summarize rocprofv3 output of this same bench command (--kernel-trace "
                         "--stats, then --pmc FETCH_SIZE, then --pmc WRITE_SIZE, each with "
                         "--calibrate-copy) as a markdown table, and for the default FP32 workload write "
                         "the per-launch HBM bytes of the stage kernels to profiles/traffic.json")
    return ap.parse_args()


def stage_class(name):
    """stage2 / stage3 / final for a stage_kernel<SN, SS, NV, L, C, NL, NQ, FINAL, RECON, SIDE>
    dispatch name, else None."""
    if "stage_kernel<" not in name:
        return None
    t = [x.strip() for x in name.split("stage_kernel<", 1)[1].split(">", 1)[0].split(",")]
    nl, final = int(t[5]), t[7] == "true"
    return "final" if final else ("stage3" if nl == 2 else "stage2")


def record_traffic(args):
    """Per-launch HBM bytes from rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch), scaled by what the same counters read for the calibration copy,
    over the timed dispatches of each stage kernel (the last `steps` ones)."""
    import csv
    stats_csv, fetch_csv, write_csv = args.record_traffic
    wl = WORKLOADS[args.workload]
    steps = args.steps if args.steps > 0 else wl["steps"]
    mib = args.calibrate_copy
    if mib <= 0:
        sys.exit("--record-traffic needs the --calibrate-copy MIB of the profiled command")

    def counters(path):
        rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Dispatch_Id"]))
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        factor = mib * 1024.0 / max(copies)  # KiB the copy must move / KiB counted
        per = {}
        for r in rows:
            per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0 * factor)
        return factor, per

    ff, fetch = counters(fetch_csv)
    wf, write = counters(write_csv)
    stats = list(csv.DictReader(open(stats_csv)))
    print(f"Calibration: FETCH_SIZE x {ff:.3f}, WRITE_SIZE x {wf:.3f} (the {mib} MiB device copy)\n")
    print("| Kernel | Calls | Avg us | Min us | Max us | Share | FETCH MB/launch | WRITE MB/launch |")
    print("|---|---|---|---|---|---|---|---|")
    for r in stats:
        n = r["Name"]
        short = n.replace("void ", "").replace("esbgk::", "").split("(")[0]
        fm = sum(fetch.get(n, [0])) / max(len(fetch.get(n, [1])), 1) / 1e6
        wm = sum(write.get(n, [0])) / max(len(write.get(n, [1])), 1) / 1e6
        print(f"| `{short[:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} "
              f"| {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.1f}% | {fm:.1f} | {wm:.1f} |")
    rec = {"command": "python -u bench.py --no-cpu-baseline"
                      + (f" --precision {args.precision}" if args.precision != "fp32" else "")
                      + (f" --workload {args.workload}" if args.workload != "riemann4" else "")
                      + f" --calibrate-copy {mib}",
           "workload": args.workload, "precision": args.precision, "steps": steps,
           "source_sha256": kernel_source_digest(), "fetch_factor": ff, "write_factor": wf, "kernels": {},
           "sources": "device.h, kernels.h, kinetic_impl.h, kinetic_*.hip"}
    # durations of the timed dispatches from the kernel trace beside the stats file
    trace_csv = os.path.join(os.path.dirname(stats_csv), os.path.basename(stats_csv).replace("kernel_stats",
                                                                                            "kernel_trace"))
    dur = {}
    for r in sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Dispatch_Id"])):
        c = stage_class(r["Kernel_Name"])
        if c:
            dur.setdefault(c, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    print(f"\nTimed dispatches (the last {steps} of each stage kernel): average duration and HBM MB per launch\n")
    print("| Kernel | avg us (trace) | FETCH MB | WRITE MB | total MB |")
    print("|---|---|---|---|---|")
    for cls in ("stage2", "stage3", "final"):
        fs = [v for n, vs in fetch.items() if stage_class(n) == cls for v in vs][-steps:]
        ws = [v for n, vs in write.items() if stage_class(n) == cls for v in vs][-steps:]
        ds = dur.get(cls, [])[-steps:]
        if not fs or not ws:
            continue
        f, w = sum(fs) / len(fs), sum(ws) / len(ws)
        rec["kernels"][cls] = {"fetch_bytes_per_launch": f, "write_bytes_per_launch": w}
        print(f"| {cls} | {sum(ds) / max(len(ds), 1):.1f} | {f / 1e6:.1f} | {w / 1e6:.1f} | {(f + w) / 1e6:.1f} |")
    if args.precision == "fp32" and args.workload == "riemann4":
        with open(TRAFFIC_FILE, "w") as fh:
            json.dump(rec, fh, indent=1)
            fh.write("\n")


def cpu_baseline(wl, nsteps):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload:
    the same generator, grid and physics, the first `nsteps` steps after one
    warm-up step (the kinetic region is still small then, so the sample holds
    fewer kinetic cells per step than the timed GPU run)."""
    import numpy as np

    import oracle
    from paper_2512_03586_amd import inputs
    oracle.build(force=False)
    nx = min(wl["nx"], 256)                  # larger grids: a 256^2 slice, same velocity grid
    if wl["nv"] > 32:
        nsteps = max(3, nsteps // 4)
    d = getattr(inputs, wl["gen"])(nx=nx, ny=nx, nv=wl["nv"], vmax=wl["vmax"], **wl["kw"])
    p = oracle.Problem(nx=nx, ny=nx, nv=wl["nv"], vmax=wl["vmax"], scheme=1, recon=1, eta=1e-2, delta=1e-3)
    st = oracle.State.from_primitives(p, d["rho"], d["ux"], d["uy"], d["T"], d["eps"])
    st.run(1, update_regime=True)          # warm-up step (also makes cells kinetic)
    kin = 0
    t = time.perf_counter()
    for _ in range(nsteps):
        st.run(1, update_regime=True)
        kin += int(st.mask.sum())
    el = time.perf_counter() - t
    pu = kin * wl["nv"] ** 2 * 2
    return {"value": pu / el, "unit": "point-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{wl['gen']} {nx}x{nx} cells x {wl['nv']}x{wl['nv']} velocities, FP64, "
                      f"{nsteps} steps after 1 warm-up step, regime update on "
                      f"({kin / nsteps:.0f} kinetic cells/step), {el:.1f} s"}


def main():
    args = parse()
    if args.record_traffic:
        record_traffic(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU path is a "
              f"design, not built in this project", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2512_03586_amd import esbgk as E
    from paper_2512_03586_amd import inputs

    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    wl = WORKLOADS[args.workload]
    if args.steps <= 0:
        args.steps = wl["steps"]
    prec = {"fp32": E.FP32, "bf16": E.BF16, "fp64": E.FP64, "mixed": E.MIXED}[args.precision]
    es = ELEM[args.precision]
    nx, nv, vmax = wl["nx"], wl["nv"], wl["vmax"]
    d = getattr(inputs, wl["gen"])(nx=nx, ny=nx, nv=nv, vmax=vmax, **wl["kw"])
    learned_info = None
    ind = {"plain": E.IND_PLAIN, "learned": E.IND_LEARNED, "dilated": E.IND_LEARNED}[args.indicator]
    cfg = E.make_config(nx, nx, nv, vmax, precision=prec, indicator=ind, scheme=E.ARS233,
                        recon=E.MINMOD2, eta=1e-2, delta=1e-3, learned_k=args.learned_k)
    eng = E.Engine(cfg)
    if args.indicator != "plain":
        from paper_2512_03586_amd import learned as LR
        K = args.learned_k
        if args.indicator == "learned":
            t0 = time.perf_counter()
            # training data: plain runs of the four-quadrant generator at 256^2 x 32^2
            kw = dict(nx=256, nv=32, vmax=10.0, steps=100, K=K, precision=prec)
            train = LR.collect(range(1, 1 + args.train_seeds), **kw)
            val = LR.collect(range(100, 102), **kw)
            net, res = LR.train(train, val, iters=1500, batch=16384, lr=3e-3, w_pos=4.0, miss=args.learned_miss)
            torch.cuda.synchronize()
            eng.set_learned(net, res.threshold)
            learned_info = {"K": K, "train_seeds": args.train_seeds, "miss_quantile": args.learned_miss,
                            "train_seconds_incl_data": round(time.perf_counter() - t0, 2),
                            "threshold": res.threshold, "val_recall": res.val_recall}
        else:
            eng.set_learned(None, 0.0, LR.dilation_radius(K))
            learned_info = {"K": K, "dilation": LR.dilation_radius(K)}
    dev = {k: torch.as_tensor(d[k]).cuda() for k in ("rho", "ux", "uy", "T", "eps")}

    def reset():
        E.esbgk_set_state(eng.ctx, dev["rho"], dev["ux"], dev["uy"], dev["T"], dev["eps"])

    reset()
    eng.step(args.warmup)
    torch.cuda.synchronize()
    reset()                                   # time the configuration from t = 0
    torch.cuda.synchronize()
    E.esbgk_set_timing(eng.ctx, True)
    E.esbgk_kernel_times(eng.ctx, reset=True)
    t0 = time.perf_counter()
    eng.step(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    E.esbgk_set_timing(eng.ctx, False)
    ms, launches = E.esbgk_kernel_times(eng.ctx, reset=True)
    stats = eng.stats()
    kin_steps = stats.kinetic_cell_steps
    pu = kin_steps * nv * nv * 2
    value = pu / el
    names = ["stage2", "stage3", "final"]
    dom = max(range(3), key=lambda k: ms[k])
    kin_avg = kin_steps / max(args.steps, 1)
    t_launch = ms[dom] / max(launches[dom], 1) * 1e-3
    bytes_launch = sum(n * b for n, b in zip(PASSES[names[dom]], es)) * kin_avg * nv * nv
    achieved = bytes_launch / t_launch / 1e9
    breakdown = {names[k]: round(ms[k] / max(launches[k], 1), 4) for k in range(3)}
    breakdown["fill"] = round(ms[3] / max(launches[3], 1), 4)
    print(f"# kernel ms/launch {breakdown}; kinetic cells/step {kin_avg:.0f} of {nx * nx}; "
          f"step {el / args.steps * 1e3:.3f} ms", file=sys.stderr)
    out = {
        "metric": "phase-space point-updates/s per IMEX stage",
        "value": value,
        "unit": "point-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16-storage/f32", "fp64": "f64",
                  "mixed": "f32-state/bf16-increments/f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{wl['gen']} {nx}x{nx} cells x {nv}x{nv} velocities on [-{vmax:g},{vmax:g}]^2, "
                               f"ARS(2,3,3), minmod, "
                               + ("regime update every step" if args.indicator == "plain" else
                                  f"{args.indicator} indicator, plain check every {args.learned_k} steps")
                               + f", {args.steps} steps from t=0",
                   "nx": nx, "ny": nx, "nv": nv, "precision": args.precision,
                   "kinetic_cells_per_step": round(kin_avg, 1),
                   "kernel_ms_per_launch": breakdown},
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": recorded_traffic(names[dom], args.workload, args.precision, args.steps),
                     "algorithmic_bytes_per_launch": bytes_launch},
    }
    if stats.error_flags:
        out["error_flags"] = stats.error_flags
    if learned_info is not None:
        checks, missed, extra, plain_kin = eng.learned_stats()
        learned_info.update(checks=checks, missed_cell_rate=missed / max(checks * nx * nx, 1),
                            extra_cell_rate=extra / max(checks * nx * nx, 1))
        out["config"]["indicator"] = learned_info
    if args.error_vs_fp64:
        rho = eng.moments()[0].double()
        del eng
        torch.cuda.empty_cache()
        ref = E.Engine(E.make_config(nx, nx, nv, vmax, precision=E.FP64, indicator=E.IND_PLAIN, scheme=E.ARS233,
                                     recon=E.MINMOD2, eta=1e-2, delta=1e-3))
        ref.set_state(d["rho"], d["ux"], d["uy"], d["T"], d["eps"])
        ref.step(args.steps)
        rref = ref.moments()[0].double()
        out["error_vs_fp64"] = {"rel_l1_rho": float((rho - rref).abs().sum() / rref.abs().sum()),
                                "reference": "FP64 form, plain indicator every step, same steps from t=0"}
        del ref
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
