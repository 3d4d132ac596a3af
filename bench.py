#!/usr/bin/env python3
"""Benchmark of the EMT nodal-analysis time loop on one MI355X.

One bench step = one full simulation of the workload: emt_factor (every
topology) + emt_step over the whole horizon, recording the outputs, with the
inputs already resident on the device. Default workload: a 1000-bus
three-phase grid (3000 nodes, 15,903 branches), 50,000 steps at 20 us, one
three-phase fault at step 25,000, every node recorded.

value = node-steps/s = nodes * steps * K / (timed seconds for K bench steps).

Prints one JSON line. Secondary figures (batched N-1, adjoint/forward ratio,
uneven batched gradients) ride along as extra keys unless --no-extras.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "node-steps/s (plain vs batched N-1) and adjoint/forward time ratio, FP64"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector, published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes_per_step(info, n_rec_total, component_sizes=None):
    """Bytes one time step touches if nothing stayed on chip: branch
    coefficients, terminals and state (g, beta, gamma, k, m, i, u read;
    i, u written: 64 B per branch) and the recorded outputs (8 B each),
    plus the solve: for the sweeps the L factor read twice with its index
    (24 B per strictly-lower nonzero) and D^-1 (8 B per node); for the dense
    inverse (component_sizes given) the whole inverse of every component
    (8 n^2 B)."""
    b = 64 * info["total_branches"] + 8 * n_rec_total
    if component_sizes is None:
        return b + 24 * info["nnz_L"] + 8 * info["total_nodes"]
    return b + 8 * sum(int(n) ** 2 for n in component_sizes)


def algorithmic_flops_per_step(info, component_sizes=None):
    """FP64 operations of one time step: companion history, injection and
    branch update (10 per branch), plus the solve: for the sweeps 4 per
    strictly-lower nonzero of L and 1 per node; for the dense inverse a
    multiply-add per inverse entry (2 n^2 per component)."""
    f = 10 * info["total_branches"]
    if component_sizes is None:
        return f + 4 * info["nnz_L"] + info["total_nodes"]
    return f + 2 * sum(int(n) ** 2 for n in component_sizes)


def latency_object(sim, kernel, us_per_step, info):
    """The step kernel's time per step against its latency floor: the same
    launch shape running only its barrier-separated phases (and, for the
    split path, its exchange), measured by emt_latency_floor after the timed
    region."""
    kind = "split" if kernel == "k_split" else "one_workgroup"
    floor = sim.latency_floor(kind, 20000)
    return {"us_per_time_step": us_per_step, "block_size": info["block_size"],
            "floor_us_per_time_step": floor, "floor_kind": kind,
            "floor_over_step": floor / us_per_step}


def component_sizes(net):
    """Node counts of the connected components of a network's branch graph."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    ok = (net.k >= 0) & (net.m >= 0)
    g = sp.coo_matrix((np.ones(int(ok.sum())), (net.k[ok], net.m[ok])), shape=(net.n_nodes, net.n_nodes))
    _, lab = connected_components(g, directed=False)
    return np.bincount(lab)


# Per step kernel: its sources and the committed rocprofv3 summary of the
# grid1000 workload that holds its measured HBM traffic.
KERNELS = {
    "k_forward": (("paper_1903_01081_amd/csrc/step.h", "paper_1903_01081_amd/csrc/step.hip",
                   "paper_1903_01081_amd/csrc/device.h"), "profiles/k_forward_grid1000.md"),
    "k_split": (("paper_1903_01081_amd/csrc/split.hip", "paper_1903_01081_amd/csrc/step.h",
                 "paper_1903_01081_amd/csrc/device.h"), "profiles/k_split_grid1000.md"),
}
KERNEL_SOURCES, TRAFFIC_PROFILE = KERNELS["k_forward"]


def kernel_source_digest(sources=None):
    h = hashlib.sha256()
    for f in (KERNEL_SOURCES if sources is None else sources):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel=None):
    """HBM bytes per launch of a step kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (scaled by a plain copy's counters), or
    None when the kernel sources have changed since it was taken."""
    sources, profile = (KERNEL_SOURCES, TRAFFIC_PROFILE) if kernel is None else KERNELS[kernel]
    try:
        with open(os.path.join(ROOT, profile)) as fh:
            for line in fh:
                if line.startswith("traffic-record:"):
                    rec = json.loads(line.split(":", 1)[1])
                    if rec.get("source_digest") == kernel_source_digest(sources):
                        return float(rec["bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        pass
    return None


def time_simulation(torch, sim, rec, steps, warmup):
    """Warmup, then `steps` full runs (reset + factor + all steps). Returns
    (wall seconds, forward-kernel seconds per run from HIP events on the
    launch stream)."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        sim.reset()
        sim.factor()
        sim.step(sim.n_steps, rec=rec)
        torch.cuda.synchronize()
        log(f"  warmup run done")
    evs = []
    t0 = time.perf_counter()
    for k in range(steps):
        sim.reset()
        sim.factor()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        sim.step(sim.n_steps, rec=rec)
        b.record(stream)
        evs.append((a, b))
        if k == 0:
            torch.cuda.synchronize()
            log(f"  first timed run: {a.elapsed_time(b) / 1e3:.3f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = float(np.mean([a.elapsed_time(b) for a, b in evs])) / 1e3
    return wall, kern


def cpu_baseline_config1(nets, cfg):
    """The oracle (dense LU, one thread) on a bounded sample of the workload:
    two short runs (50 and 2550 steps) give the factorisation and per-step
    costs, extrapolated to the full horizon with its two factorisations."""
    from oracle import oracle as O
    net = nets[0]
    dt = cfg["dt"]
    t0 = time.perf_counter()
    O.run(net, dt, 50)
    t50 = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.run(net, dt, 2550)
    t_long = time.perf_counter() - t0
    per_step = max((t_long - t50) / 2500.0, 1e-12)
    factor = max(t50 - 50 * per_step, 0.0)
    T = cfg["n_steps"]
    total = 2 * factor + T * per_step
    return {"value": net.n_nodes * T / total, "unit": "node-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle runs of 50 and 2550 steps of the same 3000-node grid "
                      f"({t50 + t_long:.1f} s of CPU); per-step {per_step * 1e3:.2f} ms and "
                      f"factorisation {factor:.2f} s extrapolated to 50,000 steps and 2 factorisations"}


def solver_comparison(torch, nets, cfg, tuned, shape, best_run_s):
    """grid1000 over the whole horizon with the other solver family than the
    tuned one (one-workgroup sparse sweeps + dense tail vs the column-split
    dense inverse), plus the tuner's prefix timings of every shape."""
    from paper_1903_01081_amd.sim import Simulator
    N, T = nets[0].n_nodes, cfg["n_steps"]
    other = dict(solver="auto") if shape.get("solver") == "dense" else dict(solver="dense")
    sim = Simulator(nets, cfg["dt"], T, **other)
    rec = torch.empty((1, T, sim.R), dtype=torch.float64, device=sim.device)
    wall, kern = time_simulation(torch, sim, rec, 1, 1)
    floor = sim.latency_floor("split" if sim.info()["split_tiles"] > 0 else "one_workgroup", 20000)
    sim.close()
    return {"tuned_shape": shape, "tuned_node_steps_per_s": N * T / best_run_s,
            "other_shape": other, "other_node_steps_per_s": N * T / wall,
            "other_us_per_time_step": kern / T * 1e6, "other_floor_us_per_time_step": floor,
            "tuner_trials": [
                {"shape": t["shape"], "us_per_step": t["s_per_step"] * 1e6, "factor_ms": t["factor_s"] * 1e3}
                if "s_per_step" in t else {"shape": t["shape"], "rejected": t["rejected"]}
                for t in tuned["trials"]]}


def batched_n1(torch):
    """The 400-scenario N-1 batch in one launch with its tuned shape: returns
    (networks, settings, shape, wall s, kernel s)."""
    from paper_1903_01081_amd import netgen
    from paper_1903_01081_amd.sim import Simulator
    from paper_1903_01081_amd.tune import tune
    nets, cfg = netgen.config2()
    shape_b = tune(nets, cfg["dt"], cfg["n_steps"], probe_steps=300)["shape"]
    sim = Simulator(nets, cfg["dt"], cfg["n_steps"], **shape_b)
    rec = torch.empty((sim.S, sim.n_steps, sim.R), dtype=torch.float64, device=sim.device)
    wall, kern = time_simulation(torch, sim, rec, 1, 1)
    sim.close()
    del rec
    return nets, cfg, shape_b, wall, kern


def extras(torch, args):
    """Batched N-1 vs the per-scenario loop, adjoint/forward ratio, and
    uneven batched gradients; each measured once after a warmup."""
    from paper_1903_01081_amd import netgen
    from paper_1903_01081_amd.sim import Simulator, theta_matrix
    from paper_1903_01081_amd.tune import tune
    out = {}
    # Batched N-1 contingencies: 400 scenarios x 600 nodes, 15,000 steps;
    # each side with its own tuned launch shape.
    nets, cfg, shape_b, wall, kern = batched_n1(torch)
    N = nets[0].n_nodes
    batched = len(nets) * N * cfg["n_steps"] / wall
    # plain per-scenario loop: a sample of scenarios run one at a time
    shape_1 = tune(nets[:1], cfg["dt"], cfg["n_steps"], probe_steps=300)["shape"]
    n_plain = 8
    plain_t = []
    for s in range(n_plain):
        one = Simulator([nets[s]], cfg["dt"], cfg["n_steps"], **shape_1)
        r1 = torch.empty((1, one.n_steps, one.R), dtype=torch.float64, device=one.device)
        w1, _ = time_simulation(torch, one, r1, 1, 1 if s == 0 else 0)
        plain_t.append(w1)
        one.close()
    plain = N * cfg["n_steps"] / float(np.mean(plain_t))
    out["batched_n1"] = {"workload": "grid200 N-1: 400 scenarios x 600 nodes, 15,000 steps at 20 us",
                         "value": batched, "unit": "node-steps/s", "seconds": wall, "launch_shape": shape_b,
                         "plain_loop_value": plain, "plain_loop_sample": f"{n_plain} scenarios run one at a time",
                         "plain_launch_shape": shape_1, "speedup_vs_plain_loop": batched / plain}
    # Adjoint: 300 nodes, 10,000 steps, checkpoint every 500 (tuned shape).
    nets, cfg = netgen.config3()
    shape_a = tune(nets, cfg["dt"], cfg["n_steps"], checkpoint_every=cfg["checkpoint_every"],
                   probe_steps=300)["shape"]
    sim = Simulator(nets, cfg["dt"], cfg["n_steps"], checkpoint_every=cfg["checkpoint_every"], **shape_a)
    rec = torch.empty((1, sim.n_steps, sim.R), dtype=torch.float64, device=sim.device)
    cot = torch.randn((1, sim.n_steps, sim.R), dtype=torch.float64, device=sim.device)
    for _ in range(2):
        sim.reset()
        sim.factor()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(sim.n_steps, rec=rec)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        t0 = time.perf_counter()
        sim.adjoint(cot)
        torch.cuda.synchronize()
        t_adj = time.perf_counter() - t0
    out["adjoint"] = {"workload": "grid100: 300 nodes, 10,000 steps at 50 us, 450 parameters, checkpoint every 500",
                      "launch_shape": shape_a, "pipelined": bool(sim.info()["adjoint_pipelined"]),
                      "forward_s": t_fwd, "adjoint_s": t_adj, "adjoint_over_forward": t_adj / t_fwd}
    sim.close()
    # Uneven batch: 256 networks of 90-900 nodes, forward + adjoint (tuned
    # shape for the batch; the per-instance loop keeps the library default).
    nets, cfg = netgen.config4()
    shape_u = tune(nets, cfg["dt"], cfg["n_steps"], checkpoint_every=cfg["checkpoint_every"],
                   probe_steps=300)["shape"]
    sim = Simulator(nets, cfg["dt"], cfg["n_steps"], checkpoint_every=cfg["checkpoint_every"], **shape_u)
    theta = theta_matrix(nets, device=sim.device)
    rec = torch.empty((sim.S, sim.n_steps, sim.R), dtype=torch.float64, device=sim.device)
    cot = torch.randn_like(rec)
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.set_params(theta)
        sim.factor()
        sim.step(sim.n_steps, rec=rec)
        sim.adjoint(cot)
        torch.cuda.synchronize()
        t_b = time.perf_counter() - t0
    n_loop = 8
    loop_t = []
    for j in range(n_loop):
        one = Simulator([nets[j]], cfg["dt"], cfg["n_steps"], checkpoint_every=cfg["checkpoint_every"])
        th1 = theta_matrix([nets[j]], device=one.device)
        r1 = torch.empty((1, one.n_steps, one.R), dtype=torch.float64, device=one.device)
        c1 = torch.randn_like(r1)
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            one.set_params(th1)
            one.factor()
            one.step(one.n_steps, rec=r1)
            one.adjoint(c1)
            torch.cuda.synchronize()
            tj = time.perf_counter() - t0
        loop_t.append(tj)
        one.close()
    out["uneven_gradients"] = {"workload": "256 grids of 90-900 nodes, 5000 steps at 50 us, forward + adjoint",
                               "launch_shape": shape_u, "pipelined": bool(sim.info()["adjoint_pipelined"]),
                               "gradients_per_s": len(nets) / t_b, "seconds": t_b,
                               "per_instance_loop_gradients_per_s": 1.0 / float(np.mean(loop_t)),
                               "loop_sample": f"{n_loop} instances run one at a time"}
    sim.close()
    return out


def calibrate_copy(torch, gib=1):
    """A plain device-to-device copy of a known size, run under the same
    rocprofv3 --pmc counters as the step kernel: FETCH_SIZE and WRITE_SIZE
    of this copy, against its true bytes, give the counters' scale."""
    n = gib * (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only-n1", action="store_true",
                    help="run only the batched N-1 workload (one line; for profiling its kernel)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (counter scale for rocprofv3 --pmc)")
    ap.add_argument("--solver", choices=["tuned", "auto", "dense", "sparse"], default="tuned",
                    help="headline launch shape: tuned (default) or a fixed solver with library defaults")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the EMT time loop runs each scenario on one device "
              "and this build has no multi-GPU path (scenarios would shard across GPUs with "
              "no exchange during the loop). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        calibrate_copy(torch)
        return
    if args.only_n1:
        nets, cfg, shape, wall, kern = batched_n1(torch)
        nsteps = len(nets) * nets[0].n_nodes * cfg["n_steps"]
        print(json.dumps({"metric": "node-steps/s, batched N-1", "value": nsteps / wall, "unit": "node-steps/s",
                          "workload": "grid200 N-1: 400 scenarios x 600 nodes, 15,000 steps at 20 us",
                          "launch_shape": shape, "seconds": wall, "kernel_s": kern}), flush=True)
        return
    from paper_1903_01081_amd import netgen
    from paper_1903_01081_amd.sim import Simulator
    from paper_1903_01081_amd.tune import tune

    nets, cfg = netgen.config1()
    net = nets[0]
    N, T = net.n_nodes, cfg["n_steps"]
    # launch shape: the tuner times every feasible shape on a 400-step prefix
    # (outside the timed region, like building the context)
    t0 = time.perf_counter()
    if args.solver == "tuned":
        tuned = tune(nets, cfg["dt"], T, probe_steps=400)
        shape = tuned["shape"]
        log(f"tuned: {shape}; trials "
            f"{[(t['shape'], t.get('s_per_step'), t.get('rejected')) for t in tuned['trials']]}")
    else:
        tuned = {"shape": dict(solver=args.solver), "trials": []}
        shape = tuned["shape"]
    tune_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    sim = Simulator(nets, cfg["dt"], T, **shape)
    build_s = time.perf_counter() - t0
    info = sim.info()
    rec = torch.empty((1, sim.n_steps, sim.R), dtype=torch.float64, device=sim.device)
    log(f"built grid1000 in {build_s:.2f} s: {info}")
    wall, kern = time_simulation(torch, sim, rec, args.steps, args.warmup)
    # split components whose workgroups exchanged through one XCD's L2
    split_local = sim.info()["split_local"]
    value = N * T * args.steps / wall
    kernel = "k_split" if info["split_tiles"] > 0 else "k_forward"
    sizes = component_sizes(net) if kernel == "k_split" else None
    per_step_bytes = algorithmic_bytes_per_step(info, net.n_rec, sizes)
    achieved = per_step_bytes * T / kern / 1e9
    per_step_flops = algorithmic_flops_per_step(info, sizes)
    tflops = per_step_flops * T / kern / 1e12
    line = {
        "metric": METRIC, "value": value, "unit": "node-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "grid1000: 1000-bus three-phase grid, 3000 nodes, 15903 branches, "
                               "50000 steps at 20 us, three-phase fault at step 25000, all nodes recorded",
                   "nodes": N, "branches": int(net.n_branches), "time_steps": T,
                   "bench_step": "emt_factor + emt_step over the whole horizon",
                   "launch_shape": shape, "split_tiles": info["split_tiles"],
                   "split_cols": info["split_cols"], "split_components_xcd_local": split_local},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kernel),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "kernel": kernel, "kernel_s": kern,
                     "algorithmic_bytes_per_time_step": per_step_bytes,
                     # the same kernel against the FP64 vector peak: both
                     # paths keep their solve data on chip (LDS, VGPRs), so
                     # the per-step latency chain binds, not HBM or FP64
                     "fp64_flops_per_time_step": per_step_flops, "fp64_tflops": tflops,
                     "fp64_peak_tflops": FP64_PEAK_TFLOPS, "fp64_frac": tflops / FP64_PEAK_TFLOPS},
        "latency": latency_object(sim, kernel, kern / T * 1e6, info),
        "build_s": build_s, "tune_s": tune_s,
    }
    sim.close()
    del rec
    if not args.no_extras:
        line["solver_comparison"] = solver_comparison(torch, nets, cfg, tuned, shape, wall / args.steps)
        line.update(extras(torch, args))
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_config1(nets, cfg)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
