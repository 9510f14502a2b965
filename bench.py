"""Benchmark: reaction firings per second of the random-time SSA ensemble on
one MI355X, with a roofline figure and the CPU oracle timed beside it.

Default workload: Lotka-Volterra (c = 10, 0.01, 10; x0 = (1000, 1000);
t_end = 5; 101-point grid; 2^20 trajectories), thread-per-trajectory mapping.
A step is one full ensemble simulation (every trajectory to t_end) with all
outputs written to HBM.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Issue-slot count of one firing of the method for a 3-channel, 2-species
# network on CDNA (full-rate VALU op = 1 slot; 32-bit integer multiplies,
# 32x32->64 products and v_rcp_f64 = 4 slots).  Derivation per item:
#   gaps 3x(sub, mul, max, cmp, 2 sel) 18; argmin with second minimum 15;
#   near-tie 3; time/termination/sample checks 3; internal-time update 3x3 9;
#   jump with overflow check 10; firing counts 6; Philox4x32-10 10x(2 products
#   x4 + 2 xor3) 100; 53-bit uniform 8; correctly rounded log fast phase 55;
#   P refresh 8; three propensities with reciprocals 51.
ALG_SLOTS_PER_FIRING_LV = 286
PEAK_LANE_SLOTS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock = 3.93e13 /s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--trajectories", type=int, default=1 << 20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="after the timed steps, run one device copy of this size so that "
                         "profiler byte counters can be scaled against known traffic")
    return ap.parse_args()


def cpu_baseline(w, target_s):
    import numpy as np

    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    probe_R = 2 * threads
    t0 = time.perf_counter()
    o = oracle.simulate(w.net, w.x0, w.t_end, w.sample_t, w.seed, probe_R, threads=threads)
    dt = time.perf_counter() - t0
    per_traj = dt / probe_R
    R = int(max(threads, min(w.R, target_s / max(per_traj, 1e-9))))
    R = (R // threads) * threads or threads
    t0 = time.perf_counter()
    o = oracle.simulate(w.net, w.x0, w.t_end, w.sample_t, w.seed, R, threads=threads)
    dt = time.perf_counter() - t0
    fir = int(o["stats"]["firings"])
    return {"value": fir / dt, "unit": "firings/s", "cores": oracle.threads_used(threads, R),
            "kind": "oracle",
            "sample": "first %d of the %d trajectories (%d firings, %.1f s)" % (R, w.R, fir, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported (trajectory "
              "sharding across GPUs is described in DESIGN.md, not run)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2103_00405_amd import api, workloads as W

    w = W.lv_ensemble(args.trajectories)
    dev = torch.device("cuda:0")
    net = api.Network(w.net, device=dev)
    R, G, N, M = w.R, len(w.sample_t), w.net.N, w.net.M
    out = {
        "samples": torch.empty((R, G, N), dtype=torch.int32, device=dev),
        "n": torch.empty((R, M), dtype=torch.int32, device=dev),
        "T": torch.empty((R, M), dtype=torch.float64, device=dev),
        "x_final": torch.empty((R, N), dtype=torch.int32, device=dev),
        "status": torch.empty((R,), dtype=torch.uint8, device=dev),
    }
    x0 = torch.tensor(w.x0, dtype=torch.int32, device=dev)
    s = torch.tensor(w.sample_t, dtype=torch.float64, device=dev)

    def step():
        return api.simulate(net, x0, w.t_end, s, R, seed=w.seed, out=out, want=tuple(out),
                            block=args.block, grid=args.grid)["stats"]

    for i in range(args.warmup):
        st = step()
        print("warmup %d: %.1f ms, %d firings" % (i, st["kernel_ms"], st["firings"]),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    firings, kms = 0, []
    for i in range(args.steps):
        st = step()
        firings += st["firings"]
        kms.append(st["kernel_ms"])
        print("step %d: %.1f ms, %d firings" % (i, st["kernel_ms"], st["firings"]),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = firings / wall
    k_avg_s = sum(kms) / len(kms) / 1e3
    fir_per_launch = firings / args.steps
    achieved = ALG_SLOTS_PER_FIRING_LV * fir_per_launch / k_avg_s
    res = {
        "metric": "reaction firings/sec per GPU (ensemble)",
        "value": value,
        "unit": "firings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "lotka_volterra_ensemble", "N": N, "M": M, "trajectories": R,
                   "t_end": w.t_end, "grid_points": G, "x0": [int(v) for v in w.x0],
                   "c": [float(v) for v in w.net.c], "mapping": "thread", "block": st["block"],
                   "grid": st["grid"], "parallelism": "trajectories"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_SLOTS / 1e12,
                     "unit": "Tslot/s", "frac": achieved / PEAK_LANE_SLOTS, "traffic": None,
                     "kernel": "rt_thread_kernel<3,2>", "kernel_ms": k_avg_s * 1e3,
                     "slots_per_firing": ALG_SLOTS_PER_FIRING_LV},
        "firings_per_step": fir_per_launch,
        "near_ties": st["near_ties"],
        "slow_logs": st["slow_logs"],
    }
    if args.calibrate_copy_mib:
        nb = args.calibrate_copy_mib << 20
        src = torch.ones(nb // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        res["calibration_copy_bytes"] = nb
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
