"""Benchmark: reaction firings per second of the random-time SSA ensemble on
one MI355X, with a roofline figure and the CPU oracle timed beside it.

Headline workload: Lotka-Volterra (c = 10, 0.01, 10; x0 = (1000, 1000);
t_end = 5; 101-point grid; 2^20 trajectories), thread-per-trajectory mapping.
A step is one full ensemble simulation (every trajectory to t_end) with all
outputs written to HBM; inputs are resident before the timed region.

Secondary measurements (attached to the same JSON line, or alone with
--workload): the small parity case; Gillespie's direct method on the headline
ensemble (direct); the large random network (N = 1000, M = 4000, 512
trajectories: eager workgroup kernel, lazy form, direct method on a sum tree;
large_random); piecewise-constant rates on the Lotka-Volterra model
(schedule); the gradient form (score-function gradient evals/s against plain
expectation evals/s and against coupled finite differences at equal standard
error, birth-death and Lotka-Volterra, 2^18 trajectories; gradient); the
batched form (4096 networks in one captured graph; batched).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--workload all|lv_ensemble|direct|large_random|schedule|gradient|batched]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic issue slots of one firing of a 3-channel, 2-species network
# (full-rate VALU op = 1 slot; 32-bit integer products and v_rcp_f64 = 4):
# per channel sub, mul, fma and about three compares or selects; the fired
# channel's propensities with one division each (~13); one Philox4x32-10
# block (~100 instructions, 20 multi-pass products), the 53-bit uniform (~6),
# the correctly rounded log's fast path (~30) and bookkeeping (~15): about
# 200 instructions = 240-270 slots, taken as 255.  This is the figure the
# roofline fraction uses.
ALG_SLOTS_PER_FIRING_LV = 255
# The same firing itemised for this kernel's own code (reported beside it):
# gaps 3x(sub, mul, max, cmp, 2 sel) 18; argmin with second minimum 15;
# near-tie, time, termination and sample checks 6; internal-time update 9;
# jump with overflow check 10; firing counts 6; Philox4x32-10 10x(2 products
# x4 + 2 xor3) 100; 53-bit uniform 8; correctly rounded log fast phase 55; P
# refresh 8; three propensities with reciprocals 51.
ITEMISED_SLOTS_PER_FIRING_LV = 286
# Instructions the profiler counts per firing of the headline kernel
# (SQ_INSTS_VALU x 64 / firings; profiles/rt_thread_kernel_lv_ensemble_sq_counters.md).
ISSUED_VALU_PER_FIRING_LV = 307


# Algorithmic lane-ops of one firing of an M-channel network in the eager
# form: per channel about 3 FP64 operations (T update, P - T, times 1/a) and 3
# compares or selects (clamp, dead-channel test, argmin), the wavefront and
# workgroup argmin (~600), about 20 dependent propensities (~13 each) and the
# draw with its log (~150): 25k at M = 4000.  The roofline fraction uses it.
def alg_lane_ops_eager(M, deps=20):
    return 6 * M + 600 + 13 * deps + 150


# The same firing itemised for the workgroup kernel's code (reported beside
# it): per channel T update (1), gap (sub, mul, max, cmp, 2 sel = 6), argmin
# with second minimum (5); the draw (~163) and the dependents (~17 each).
def itemised_slots_group(M, deps=20):
    return 12 * M + 163 + 17 * deps


CLOCK_HZ = 2.4e9
PEAK_LANE_SLOTS = 256 * 4 * 16 * CLOCK_HZ   # CUs x SIMDs x lanes x clock = 3.93e13 /s

# HBM bytes per launch of rt_thread_kernel<3,2> on the Lotka-Volterra ensemble,
# from two rocprofv3 counter passes (FETCH_SIZE, WRITE_SIZE) scaled by the same
# counters on a 1 GiB copy (factors 2.0 and 1.0).  Valid for the kernel as
# profiled; set to None when the kernel changes until it is measured again.
LV_TRAFFIC_BYTES_PER_LAUNCH = 1.331e+09

# VALU instructions (wave64) of one step of the batched workload: SQ_INSTS_VALU
# summed over the timed replay's ten class kernels in one rocprofv3 counter
# pass.  At 4 cycles per instruction on 256 x 4 SIMDs the step cannot take
# less than this many cycles' worth of issue; valid for the kernels and the
# autotuner's plan as profiled, None when they change until measured again.
BATCH_VALU_INSTR_PER_STEP = 6.217e+11
SIMD_ISSUE_HZ = 256 * 4 * CLOCK_HZ / 4        # wave64 VALU instructions per second


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--trajectories", type=int, default=1 << 20)
    ap.add_argument("--workload", default="all",
                    choices=["all", "lv_ensemble", "large_random", "gradient", "batched",
                             "direct", "schedule"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="after the timed steps, run one device copy of this size so that "
                         "profiler byte counters can be scaled against known traffic")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(w, target_s):
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    probe_R = threads
    t0 = time.perf_counter()
    oracle.simulate(w.net, w.x0, w.t_end, w.sample_t, w.seed, probe_R, threads=threads)
    per_traj = (time.perf_counter() - t0) / probe_R
    R = int(max(threads, min(w.R, target_s / max(per_traj, 1e-9))))
    R = (R // threads) * threads or threads
    t0 = time.perf_counter()
    o = oracle.simulate(w.net, w.x0, w.t_end, w.sample_t, w.seed, R, threads=threads)
    dt = time.perf_counter() - t0
    fir = int(o["stats"]["firings"])
    # cores = the threads the oracle used (one std::thread each, at most the
    # 16-core CPU share of the GPU host); host_cores = what the host reports
    return {"value": fir / dt, "unit": "firings/s", "cores": oracle.threads_used(threads, R),
            "host_cores": os.cpu_count(), "kind": "oracle",
            "sample": "first %d of the %d trajectories (%d firings, %.1f s)" % (R, w.R, fir, dt)}


def run_ensemble(api, w, steps, warmup, block=0, grid=0, mapping=0, method=0, schedule=None):
    import torch
    dev = torch.device("cuda:0")
    net = api.Network(w.net, device=dev)
    if schedule is not None:
        net.set_schedule(*schedule)
    R, G, N, M = w.R, len(w.sample_t), w.net.N, w.net.M
    out = {
        "samples": torch.empty((R, G, N), dtype=torch.int32, device=dev),
        "n": torch.empty((R, M), dtype=torch.int32, device=dev),
        "T": torch.empty((R, M), dtype=torch.float64, device=dev),
        "x_final": torch.empty((R, N), dtype=torch.int32, device=dev),
        "status": torch.empty((R,), dtype=torch.uint8, device=dev),
    }
    if method in (api.METHOD_DIRECT, api.METHOD_DIRECT_TREE):
        del out["T"]                      # the direct method has no internal times
    x0 = torch.tensor(w.x0, dtype=torch.int32, device=dev)
    s = torch.tensor(w.sample_t, dtype=torch.float64, device=dev)

    def step():
        return api.simulate(net, x0, w.t_end, s, R, seed=w.seed, out=out, want=tuple(out),
                            block=block, grid=grid, mapping=mapping, method=method)["stats"]

    for i in range(warmup):
        st = step()
        log("%s warmup %d: %.1f ms, %d firings" % (w.name, i, st["kernel_ms"], st["firings"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    firings, kms = 0, []
    for i in range(steps):
        st = step()
        firings += st["firings"]
        kms.append(st["kernel_ms"])
        log("%s step %d: %.1f ms, %d firings" % (w.name, i, st["kernel_ms"], st["firings"]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return dict(firings=firings, wall=wall, kernel_s=sum(kms) / len(kms) / 1e3, stats=st,
                firings_per_step=firings / steps, out=out)


def oracle_rate(jobs, threads, target_s):
    """Oracle firings/s on a bounded sample: jobs = [(net, x0, t_end, grid, R,
    net_id, max_firings)], run in order until about target_s seconds."""
    import oracle
    fir, dt, runs = 0, 0.0, 0
    for net, x0, t_end, grid, R, net_id, maxf in jobs:
        t0 = time.perf_counter()
        o = oracle.simulate(net, x0, t_end, grid, 1, R, net_id=net_id, max_firings=maxf,
                            threads=threads)
        dt += time.perf_counter() - t0
        fir += int(o["stats"]["firings"])
        runs += 1
        if dt > target_s:
            break
    return fir, dt, runs


def ensemble_moments(out, sample_t):
    """Mean and sample variance (n - 1) of every species at every sample
    point over the trajectories of the last step that ended OK or absorbed
    (computed after the timed region; a report, not part of a step)."""
    import torch
    ok = out["status"] <= 1
    x = out["samples"][ok].to(torch.float64)            # [trajectories, G, N]
    mean, var = x.mean(dim=0).cpu().numpy(), x.var(dim=0).cpu().numpy()
    res = {"trajectories": int(ok.sum()), "t": [float(v) for v in sample_t]}
    for j in range(mean.shape[1]):
        res["mean_X%d" % (j + 1)] = [float("%.7g" % v) for v in mean[:, j]]
        res["var_X%d" % (j + 1)] = [float("%.7g" % v) for v in var[:, j]]
    return res


def bench_lv_small(api, W, reps=5):
    """The small parity case (256 trajectories, about 1.5e6 firings): too few
    trajectories to fill the device, so it is reported as time per launch."""
    import torch
    w = W.lv_small()
    net = api.Network(w.net)
    x0 = torch.tensor(w.x0, dtype=torch.int32, device="cuda")
    s = torch.tensor(w.sample_t, dtype=torch.float64, device="cuda")
    api.simulate(net, x0, w.t_end, s, w.R, seed=w.seed)
    kms, fir = [], 0
    for _ in range(reps):
        st = api.simulate(net, x0, w.t_end, s, w.R, seed=w.seed)["stats"]
        kms.append(st["kernel_ms"])
        fir = st["firings"]
    return {"workload": "lotka_volterra_small", "trajectories": w.R, "t_end": w.t_end,
            "grid_points": len(w.sample_t), "firings_per_launch": fir,
            "kernel_ms": min(kms), "mapping": "thread"}


def bench_schedule(api, W, R=1 << 18, reps=2):
    """Piecewise-constant rates (Eq. 28 solved piece by piece) on the
    Lotka-Volterra ensemble's model (2^18 trajectories, t_end 5): the rates
    switch at t = 1, 2, 3, 4, each piece scaling all three by one factor
    (1.2, 0.8, 1.1, 0.9: a time warp that keeps the fixed point, so the
    firing counts stay comparable and the ratio shows the cost of the
    breakpoints themselves); firings/s with the schedule and without it,
    thread mapping both."""
    import numpy as np
    import torch
    w = W.lv_ensemble(R)
    x0 = torch.tensor(w.x0, dtype=torch.int32, device="cuda")
    s = torch.tensor(w.sample_t, dtype=torch.float64, device="cuda")
    times = np.array([1.0, 2.0, 3.0, 4.0])
    scale = np.array([[1.2] * 3, [0.8] * 3, [1.1] * 3, [0.9] * 3])
    res = {}
    for tag in ("constant", "schedule"):
        net = api.Network(w.net)
        if tag == "schedule":
            net.set_schedule(times, scale * np.asarray(w.net.c)[None, :])
        out = {"samples": torch.empty((R, len(w.sample_t), 2), dtype=torch.int32, device="cuda"),
               "n": torch.empty((R, 3), dtype=torch.int32, device="cuda"),
               "T": torch.empty((R, 3), dtype=torch.float64, device="cuda")}
        api.simulate(net, x0, w.t_end, s, R, seed=w.seed, out=out, want=tuple(out))
        fir, ms = 0, 0.0
        for _ in range(reps):
            st = api.simulate(net, x0, w.t_end, s, R, seed=w.seed, out=out, want=tuple(out))["stats"]
            fir += st["firings"]
            ms += st["kernel_ms"]
        res[tag] = {"value": fir / (ms / 1e3), "unit": "firings/s (kernel time)",
                    "kernel_ms": ms / reps, "firings_per_launch": fir / reps}
    res["workload"] = "lotka_volterra_rate_schedule"
    res["trajectories"] = R
    res["breakpoints"] = [float(v) for v in times]
    res["schedule_vs_constant"] = res["schedule"]["value"] / res["constant"]["value"]
    return res


def bench_direct(api, W, steps=2, warmup=1, R=1 << 20):
    """Gillespie's direct method (the paper's comparison method, section 3) on
    the headline Lotka-Volterra ensemble, same outputs except the internal
    times, thread mapping: firings/s to set beside the random-time method's."""
    import torch
    w = W.lv_ensemble(R)
    dev = torch.device("cuda:0")
    net = api.Network(w.net, device=dev)
    N, M, G = w.net.N, w.net.M, len(w.sample_t)
    out = {"samples": torch.empty((R, G, N), dtype=torch.int32, device=dev),
           "n": torch.empty((R, M), dtype=torch.int32, device=dev),
           "x_final": torch.empty((R, N), dtype=torch.int32, device=dev),
           "status": torch.empty((R,), dtype=torch.uint8, device=dev)}
    x0 = torch.tensor(w.x0, dtype=torch.int32, device=dev)
    s = torch.tensor(w.sample_t, dtype=torch.float64, device=dev)

    def step():
        return api.simulate(net, x0, w.t_end, s, R, seed=w.seed, out=out, want=tuple(out),
                            method=api.METHOD_DIRECT)["stats"]

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fir, kms = 0, []
    for i in range(steps):
        st = step()
        fir += st["firings"]
        kms.append(st["kernel_ms"])
        log("direct method step %d: %.1f ms, %d firings" % (i, st["kernel_ms"], st["firings"]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"workload": "lotka_volterra_ensemble", "method": "direct", "trajectories": R,
            "value": fir / wall, "unit": "firings/s", "ms_per_step": wall / steps * 1e3,
            "kernel_ms": sum(kms) / len(kms), "firings_per_step": fir / steps}


def bench_large(api, W, steps, warmup, cpu_s=0.0):
    w = W.large_random()
    r = run_ensemble(api, w, steps, warmup)
    slots = alg_lane_ops_eager(w.net.M)
    ach = slots * r["firings_per_step"] / r["kernel_s"]
    cpu = None
    if cpu_s > 0:
        threads = max(1, min(16, os.cpu_count() or 1))
        fir, dt, _ = oracle_rate([(w.net, w.x0, w.t_end, w.sample_t, threads, 0, 20000)],
                                 threads, cpu_s)
        cpu = {"value": fir / dt, "unit": "firings/s", "cores": threads, "kind": "oracle",
               "sample": "%d trajectories, first 20000 firings each (%d firings, %.1f s)" % (
                   threads, fir, dt)}
    return {"workload": "large_random_network", "N": w.net.N, "M": w.net.M, "trajectories": w.R,
            "cpu_baseline": cpu,
            "t_end": w.t_end, "value": r["firings"] / r["wall"], "unit": "firings/s",
            "ms_per_step": r["wall"] / steps * 1e3, "firings_per_step": r["firings_per_step"],
            "mapping": "workgroup", "block": r["stats"]["block"], "grid": r["stats"]["grid"],
            "roofline": {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_LANE_SLOTS / 1e12,
                         "unit": "Tslot/s", "frac": ach / PEAK_LANE_SLOTS,
                         "slots_per_firing": slots,
                         "itemised_slots_per_firing": itemised_slots_group(w.net.M),
                         "kernel_ms": r["kernel_s"] * 1e3}}


def bench_large_lazy(api, W, steps, warmup, eager_value=None):
    """The large random network with the lazy form (dependency-graph updates,
    minimum tree in LDS, one wavefront per trajectory).  With 512 trajectories
    at most one wavefront runs per SIMD, so a firing costs its full latency:
    cycles_per_firing is that latency per wavefront (kernel time x clock x
    resident wavefronts / firings)."""
    w = W.large_random()
    r = run_ensemble(api, w, steps, warmup, method=api.METHOD_LAZY)
    grid = r["stats"]["grid"]
    out = {"workload": "large_random_network", "method": "lazy", "N": w.net.N, "M": w.net.M,
           "trajectories": w.R, "t_end": w.t_end, "value": r["firings"] / r["wall"],
           "unit": "firings/s", "ms_per_step": r["wall"] / steps * 1e3,
           "firings_per_step": r["firings_per_step"], "mapping": "wave", "block": 64,
           "grid": grid, "kernel_ms": r["kernel_s"] * 1e3,
           "cycles_per_firing": r["kernel_s"] * CLOCK_HZ * min(grid, w.R) /
           r["firings_per_step"]}
    if eager_value:
        out["vs_eager"] = out["value"] / eager_value
    # Gillespie's direct method in the same mapping (sum tree of fan-out 8):
    # the paper's comparison of one reduction against a sum and a search
    d = run_ensemble(api, w, steps, warmup, method=api.METHOD_DIRECT_TREE)
    out["direct_tree"] = {"value": d["firings"] / d["wall"], "unit": "firings/s",
                          "kernel_ms": d["kernel_s"] * 1e3,
                          "firings_per_step": d["firings_per_step"]}
    out["random_time_vs_direct"] = out["value"] / out["direct_tree"]["value"]
    # the same network with piecewise-constant rates: breakpoints at 0.2, 0.4,
    # 0.6 and 0.8 of t_end, each piece scaling every rate by one factor (1.2,
    # 0.8, 1.1, 0.9; a time warp with the same integral, so the firing counts
    # match and the ratio is the cost of the breakpoints: every clock run to
    # each, every leaf and the whole tree rebuilt)
    import numpy as np
    times = np.array([0.2, 0.4, 0.6, 0.8]) * w.t_end
    rates = np.array([1.2, 0.8, 1.1, 0.9])[:, None] * np.asarray(w.net.c)[None, :]
    s = run_ensemble(api, w, steps, warmup, method=api.METHOD_LAZY, schedule=(times, rates))
    out["with_schedule"] = {"value": s["firings"] / s["wall"], "unit": "firings/s",
                            "kernel_ms": s["kernel_s"] * 1e3,
                            "firings_per_step": s["firings_per_step"],
                            "breakpoints": [float(v) for v in times]}
    out["schedule_vs_constant"] = out["with_schedule"]["value"] / out["value"]
    return out


def bench_gradient(api, W, reps=3):
    """Gradient evals/s (forward + f + backward kernel) vs plain evals/s
    (forward + f), and vs central finite differences in log c (2M extra
    forwards with common random numbers) at equal standard error."""
    import numpy as np
    import torch
    res = {}
    for w in (W.bd_gradient(), W.lv_gradient()):
        net = api.Network(w.net)
        R, M = w.R, w.net.M
        x0 = torch.tensor(w.x0, dtype=torch.int32, device="cuda")
        grid = torch.tensor([w.t_end], dtype=torch.float64, device="cuda")
        out = {"x_final": torch.empty((R, w.net.N), dtype=torch.int32, device="cuda"),
               "n": torch.empty((R, M), dtype=torch.int32, device="cuda"),
               "T": torch.empty((R, M), dtype=torch.float64, device="cuda")}

        def forward(seed, c=None):
            if c is not None:
                net.set_rates(c)
            o = api.simulate(net, x0, w.t_end, grid, R, seed=seed, out=out,
                             want=("x_final", "n", "T"), stats=False)
            return o["x_final"][:, 0].to(torch.float64)

        def plain(seed):
            f = forward(seed)
            return float(f.mean())

        def grad(seed):
            f = forward(seed)
            g, se = api.score_grad(f, out["n"], out["T"])
            return g, se

        def fd(seed):
            c0 = np.array(w.net.c)
            ds = []
            for k in range(M):
                vals = []
                for sgn in (1, -1):
                    c = c0.copy()
                    c[k] *= math.exp(sgn * 1e-3)
                    vals.append(forward(seed, c))
                ds.append((vals[0] - vals[1]) / 2e-3)
            net.set_rates(c0)
            return ds

        timings = {}
        for name, fn in (("plain", plain), ("gradient", grad), ("fd", fd)):
            fn(100)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(reps):
                last = fn(101 + i)
            torch.cuda.synchronize()
            timings[name] = (time.perf_counter() - t0) / reps
            if name == "gradient":
                g_last, se_last = last
            if name == "fd":
                fd_last = last
        se_score = se_last.cpu().numpy()
        se_fd = np.array([float(d.std() / math.sqrt(R)) for d in fd_last])
        # cost to reach a common standard error scales with time x variance
        eq = [(timings["fd"] * se_fd[k] ** 2) / (timings["gradient"] * se_score[k] ** 2)
              for k in range(M)]
        res[w.name] = {"trajectories": R, "M": M,
                       "plain_evals_per_s": 1.0 / timings["plain"],
                       "gradient_evals_per_s": 1.0 / timings["gradient"],
                       "gradient_vs_plain": timings["plain"] / timings["gradient"],
                       "fd_evals_per_s": 1.0 / timings["fd"],
                       "gradient": [float(v) for v in g_last.cpu().numpy()],
                       "se_score": [float(v) for v in se_score],
                       "se_fd": [float(v) for v in se_fd],
                       "score_vs_fd_at_equal_se": [float(v) for v in eq]}
        log("%s: plain %.1f/s, gradient %.1f/s, fd %.2f/s" % (
            w.name, 1 / timings["plain"], 1 / timings["gradient"], 1 / timings["fd"]))
    return res


BATCH_MAX_FIRINGS = 100_000     # per trajectory; 5x the 2e4 the t_end is set for
LAZY_ABOVE_M = 256              # batched networks above this many channels run the lazy form


def batch_jobs(api, wl):
    """Jobs of the batched workload: networks above LAZY_ABOVE_M channels run
    the lazy form (a class of its own, launched first), the others the eager
    mappings; the per-network launches use the same method per network."""
    return [dict(net=api.Network(w.net), x0=w.x0, t_end=w.t_end, sample_t=w.sample_t, R=w.R,
                 net_id=w.net_id,
                 method=api.METHOD_LAZY if w.net.M > LAZY_ABOVE_M else api.METHOD_RANDOM_TIME)
            for w in wl]


def bench_batched(api, W, steps=2, n_nets=4096, solo_sample=32, tune_samples=16, cpu_s=0.0):
    """4096 random networks (M log-uniform in [3, 2048], N = M/4, 64
    trajectories each, t_end for about 2e4 firings) in one captured launch per
    size class -- the networks above LAZY_ABOVE_M channels in the lazy form, the others
    with lane counts chosen by the autotuner, each class's networks queued by
    the firings of a pilot run with another seed -- against one rtssa_simulate
    launch per network with the same method.  Networks whose rates grow with the state can run far
    past 2e4 firings; every trajectory is capped at 1e5 firings (status
    MAX_FIRINGS, counted), in the batch and in the per-network launches alike.
    The per-network time is measured on a stratified sample (every
    n_nets/solo_sample-th network in order of M) and scaled to the batch."""
    import tempfile

    import numpy as np
    import torch
    t0 = time.perf_counter()
    wl = W.batch_networks(n_nets)
    jobs = batch_jobs(api, wl)
    log("batched: %d networks generated in %.1f s" % (n_nets, time.perf_counter() - t0))
    want = ("samples", "n", "T", "x_final", "status")
    b0 = api.Batch(jobs, want=want, max_firings=BATCH_MAX_FIRINGS)
    with tempfile.TemporaryDirectory() as d:
        plan = os.path.join(d, "plan.txt")
        t0 = time.perf_counter()
        api.autotune(b0, plan, samples=tune_samples)
        tune_s = time.perf_counter() - t0
        plan_text = open(plan).read().strip().splitlines()
        del b0
        b = api.Batch(jobs, want=want, max_firings=BATCH_MAX_FIRINGS, plan_path=plan)
        log("batched: autotuned in %.1f s: %s" % (tune_s, "; ".join(plan_text)))
        # a run with another seed gives each network's work; the batch is then
        # rebuilt with those weights so that every class queue starts its
        # longest networks first (the timed runs draw seed 1)
        st = b.run(seed=2)
        log("batched pilot (seed 2): %.1f ms, %d firings" % (st["kernel_ms"], st["firings"]))
        for j, o in zip(jobs, b.outputs):
            j["weight"] = float(o["n"].to(torch.int64).sum())
        del b
        b = api.Batch(jobs, want=want, max_firings=BATCH_MAX_FIRINGS, plan_path=plan)
    st = b.run(seed=1)                                   # captures the graph
    log("batched warmup: %.1f ms, %d firings" % (st["kernel_ms"], st["firings"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fir, kms = 0, []
    for i in range(steps):
        st = b.run(seed=1)
        fir += st["firings"]
        kms.append(st["kernel_ms"])
        log("batched step %d: %.1f ms, %d firings" % (i, st["kernel_ms"], st["firings"]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    capped = int((torch.cat([o["status"] for o in b.outputs]) == api.TRAJ_MAX_FIRINGS).sum())
    # one launch per network, on a stratified sample of networks
    order = sorted(range(n_nets), key=lambda i: wl[i].net.M)
    stride = max(1, n_nets // solo_sample)
    idx = order[stride // 2::stride][:solo_sample]
    solo_ms, solo_fir = 0.0, 0
    for i in idx:
        j = jobs[i]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        o = api.simulate(j["net"], j["x0"], j["t_end"], j["sample_t"], j["R"], seed=1,
                         net_id=j["net_id"], want=want, stats=False,
                         max_firings=BATCH_MAX_FIRINGS, method=j["method"])
        torch.cuda.synchronize()
        solo_ms += (time.perf_counter() - t1) * 1e3
        solo_fir += int(o["n"].to(torch.int64).sum())
    est_ms = solo_ms * n_nets / len(idx)
    per_step = fir / steps
    cpu = None
    if cpu_s > 0:
        threads = max(1, min(16, os.cpu_count() or 1))
        mix = [idx[q] for q in np.random.default_rng(1).permutation(len(idx))]
        cfir, cdt, cruns = oracle_rate(
            [(wl[i].net, wl[i].x0, wl[i].t_end, wl[i].sample_t, threads, wl[i].net_id,
              BATCH_MAX_FIRINGS) for i in mix], threads, cpu_s)
        cpu = {"value": cfir / cdt, "unit": "firings/s", "cores": threads, "kind": "oracle",
               "sample": "%d of the sampled networks, %d trajectories each (%d firings, %.1f s)"
               % (cruns, threads, cfir, cdt)}
    ms_step = wall / steps * 1e3
    log("batched: per-network launches, %d sampled: %.1f ms -> %.0f ms for all" %
        (len(idx), solo_ms, est_ms))
    return {"workload": "batched_random_networks", "networks": n_nets, "trajectories_each": 64,
            "value": fir / wall, "unit": "firings/s", "ms_per_step": ms_step,
            "firings_per_step": per_step, "graph": True,
            "max_firings_per_trajectory": BATCH_MAX_FIRINGS,
            "trajectories_capped": capped, "autotune_s": tune_s, "plan": plan_text,
            "classes": b.classes(),
            "lazy_above_M": LAZY_ABOVE_M,
            "lazy_networks": sum(1 for j in jobs if j["method"] == api.METHOD_LAZY),
            "per_network_launches": {"networks_timed": len(idx), "sample_ms": solo_ms,
                                     "sample_firings": solo_fir,
                                     "estimated_ms_for_all": est_ms,
                                     "value": per_step / (est_ms / 1e3), "unit": "firings/s"},
            "speedup_vs_per_network": est_ms / ms_step, "cpu_baseline": cpu,
            "valu_issue": None if BATCH_VALU_INSTR_PER_STEP is None else {
                "bound": "alu", "valu_instr_per_step_profiled": BATCH_VALU_INSTR_PER_STEP,
                "floor_ms": BATCH_VALU_INSTR_PER_STEP / SIMD_ISSUE_HZ * 1e3,
                "frac": BATCH_VALU_INSTR_PER_STEP / SIMD_ISSUE_HZ / (ms_step / 1e3)}}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported (trajectory "
              "sharding across GPUs is described in DESIGN.md, not run)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2103_00405_amd import api, workloads as W

    if args.workload in ("large_random", "gradient", "batched", "direct", "schedule"):
        if args.workload == "schedule":
            out = bench_schedule(api, W)
        elif args.workload == "direct":
            out = bench_direct(api, W, args.steps, args.warmup)
        elif args.workload == "large_random":
            out = bench_large(api, W, args.steps, args.warmup)
            out["lazy"] = bench_large_lazy(api, W, args.steps, args.warmup, out["value"])
        elif args.workload == "gradient":
            out = bench_gradient(api, W)
        else:
            out = bench_batched(api, W, args.steps)
        print(json.dumps(out), flush=True)
        return

    w = W.lv_ensemble(args.trajectories)
    r = run_ensemble(api, w, args.steps, args.warmup, args.block, args.grid)
    st = r["stats"]
    value = r["firings"] / r["wall"]
    achieved = ALG_SLOTS_PER_FIRING_LV * r["firings_per_step"] / r["kernel_s"]
    N, M, G = w.net.N, w.net.M, len(w.sample_t)
    res = {
        "metric": "reaction firings/sec per GPU (ensemble)",
        "value": value,
        "unit": "firings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "lotka_volterra_ensemble", "N": N, "M": M, "trajectories": w.R,
                   "t_end": w.t_end, "grid_points": G, "x0": [int(v) for v in w.x0],
                   "c": [float(v) for v in w.net.c], "mapping": "thread", "block": st["block"],
                   "grid": st["grid"], "parallelism": "trajectories"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                     "peak": PEAK_LANE_SLOTS / 1e12, "unit": "Tslot/s",
                     "frac": achieved / PEAK_LANE_SLOTS, "traffic": LV_TRAFFIC_BYTES_PER_LAUNCH,
                     "traffic_unit": "B per launch",
                     "kernel": "rt_thread_kernel<3,2>", "kernel_ms": r["kernel_s"] * 1e3,
                     "slots_per_firing": ALG_SLOTS_PER_FIRING_LV,
                     "itemised_slots_per_firing": ITEMISED_SLOTS_PER_FIRING_LV,
                     "frac_itemised": ITEMISED_SLOTS_PER_FIRING_LV * r["firings_per_step"] /
                     r["kernel_s"] / PEAK_LANE_SLOTS,
                     "issued_valu_per_firing_profiled": ISSUED_VALU_PER_FIRING_LV},
        "firings_per_step": r["firings_per_step"],
        "near_ties": st["near_ties"],
        "slow_logs": st["slow_logs"],
        # the measured HBM traffic of one launch over its kernel time
        "hbm_GBps": LV_TRAFFIC_BYTES_PER_LAUNCH / r["kernel_s"] / 1e9,
        "ensemble": ensemble_moments(r["out"], w.sample_t),
    }
    if args.calibrate_copy_mib:
        nb = args.calibrate_copy_mib << 20
        src = torch.ones(nb // 4, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        res["calibration_copy_bytes"] = nb
    if args.workload == "all":
        cs = 0.0 if args.no_cpu_baseline else 5.0
        direct = bench_direct(api, W)
        direct["vs_random_time"] = direct["value"] / value
        large = bench_large(api, W, 2, 1, cpu_s=cs)
        res["secondary"] = {"lv_small": bench_lv_small(api, W),
                            "direct_method": direct,
                            "large_random": large,
                            "large_random_lazy": bench_large_lazy(api, W, 2, 1, large["value"]),
                            "rate_schedule": bench_schedule(api, W),
                            "gradient": bench_gradient(api, W),
                            "batched": bench_batched(api, W, 2, cpu_s=cs)}
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
