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


def roofline_object(info, n_rec_total, time_steps, kernel, kernel_s, traffic=None, passes=1.0,
                    extra_bytes_per_step=0):
    """The method's roofline for one launch of a step kernel: the bytes the
    sparse method touches per time step (the figure above without a dense
    inverse, whichever solver ran: the dense inverse is extra work this
    library chooses, not work the method needs) times the time steps of
    the launch (times `passes` for launches that step each time step more
    than once, e.g. an adjoint's recompute + reverse), over the kernel's
    time from HIP events on its stream, against the 8 TB/s HBM peak. The
    step kernels keep their per-step data on chip, so the binding limit is
    the chain of dependent phases per step (the `latency` object), not
    HBM; `traffic` is the counter-measured HBM bytes per launch when a
    profile of the current sources exists."""
    per_step = algorithmic_bytes_per_step(info, n_rec_total) + extra_bytes_per_step
    achieved = per_step * time_steps * passes / kernel_s / 1e9
    flops = algorithmic_flops_per_step(info) * time_steps * passes / kernel_s / 1e12
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
           "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
           "limiter": "latency (see the latency object)",
           "kernel": kernel, "kernel_s": kernel_s, "time_steps": time_steps, "passes": passes,
           "algorithmic_bytes_per_time_step": per_step,
           "fp64_flops_per_time_step": algorithmic_flops_per_step(info), "fp64_tflops": flops,
           "fp64_peak_tflops": FP64_PEAK_TFLOPS, "fp64_frac": flops / FP64_PEAK_TFLOPS}
    if traffic is not None:
        out["traffic_gbs"] = traffic / kernel_s / 1e9
        out["traffic_frac"] = traffic / kernel_s / 1e9 / HBM_PEAK_GBS
    return out


def latency_object(sim, kernel, us_per_step, info):
    """The step kernel's time per step against its latency floor: the same
    launch shape running only its barrier-separated phases (and, for the
    split path, its exchange), measured by emt_latency_floor after the timed
    region. floor_over_step is the efficiency figure of a latency-bound
    loop (1 = the step costs no more than its empty phases)."""
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
    "k_comp": (("paper_1903_01081_amd/csrc/comp.hip", "paper_1903_01081_amd/csrc/comp.h",
                "paper_1903_01081_amd/csrc/step.h", "paper_1903_01081_amd/csrc/device.h"),
               "profiles/k_comp_n1_grid200.md"),
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
    launch stream). Every run's device-side status is checked (emt_sync)."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        sim.reset()
        sim.factor()
        sim.step(sim.n_steps, rec=rec)
        sim.sync()
        log(f"  warmup run done")
    evs = []
    t0 = time.perf_counter()
    for k in range(steps):
        sim.reset()
        sim.factor()   # synchronises: also reports the previous run's device status
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        sim.step(sim.n_steps, rec=rec)
        b.record(stream)
        evs.append((a, b))
        if k == 0:
            sim.sync()
            log(f"  first timed run: {a.elapsed_time(b) / 1e3:.3f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.sync()
    kern = float(np.mean([a.elapsed_time(b) for a, b in evs])) / 1e3
    return wall, kern


def median_time(fn, repeats=3):
    ts = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), ts


# --------------------------------------------------------------------------
# CPU baselines: the oracle (plain dense LU, test infrastructure) compiled
# with -O3 -march=native on the host that runs the bench, timed on bounded
# samples of the same workloads.
# --------------------------------------------------------------------------

CPU_THREADS = 8


def cpu_baselines(O):
    """Returns (headline cpu_baseline, {"n1": ..., "uneven": ...})."""
    import concurrent.futures as cf
    from paper_1903_01081_amd import netgen
    O.use_native_build()
    log("cpu baseline: grid1000 prefix, 1 thread")
    out = {}
    # grid1000, one thread: median of 3 runs of a 500-step prefix (one
    # factorisation each)
    nets, cfg = netgen.config1()
    net, k = nets[0], 500
    med, ts = median_time(lambda: O.run(net, cfg["dt"], k))
    head = {"value": net.n_nodes * k / med, "unit": "node-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle (g++ -O3 -march=native, 1 thread) on the first {k} of the 50,000 steps of the "
                      f"same 3000-node grid, factorisation included; median of 3 runs "
                      f"({', '.join(f'{t:.2f}' for t in ts)} s)"}
    log("cpu baseline: grid200 N-1 sample, 8 threads")
    # grid200 N-1, 8 threads over scenarios: 16 of the 400 scenarios (every
    # 25th) over a 3000-step prefix that includes the event at step 2500
    nets, cfg = netgen.config2()
    sample = nets[::25]
    k = 3000
    med, ts = median_time(lambda: O.run_batch(sample, cfg["dt"], k, n_threads=CPU_THREADS))
    out["n1"] = {"value": len(sample) * nets[0].n_nodes * k / med, "unit": "node-steps/s",
                 "cores": CPU_THREADS, "kind": "oracle",
                 "sample": f"{len(sample)} of the 400 scenarios (every 25th), first {k} of 15,000 steps "
                           f"(the event at step 2500 included), OpenMP over scenarios on {CPU_THREADS} threads; "
                           f"median of 3 runs ({', '.join(f'{t:.2f}' for t in ts)} s)"}
    log("cpu baseline: uneven forward + adjoint sample, 8 threads")
    # uneven batch, 8 threads over instances: forward + adjoint of 8
    # instances spread over the size range; the full batch's time is
    # predicted from a fit t = a + b n^2 (dense LU work per step) over the
    # sample
    nets, cfg = netgen.config4()
    sizes = np.array([n.n_nodes for n in nets])
    order = np.argsort(sizes, kind="stable")
    pick = [int(order[int(round(q * (len(nets) - 1)))]) for q in np.linspace(0, 1, CPU_THREADS)]

    def one(j):
        net = nets[j]
        cot = np.random.default_rng(100 + j).standard_normal((cfg["n_steps"], len(net.rec_nodes)))
        t0 = time.perf_counter()
        O.adjoint(net, cfg["dt"], cfg["n_steps"], cot)
        return time.perf_counter() - t0

    with cf.ThreadPoolExecutor(CPU_THREADS) as ex:
        t_one = np.array(list(ex.map(one, pick)))
    n2 = sizes[pick].astype(float) ** 2
    A = np.stack([np.ones_like(n2), n2], 1)
    coef, *_ = np.linalg.lstsq(A, t_one, rcond=None)
    total_1thread = float(np.sum(coef[0] + coef[1] * sizes.astype(float) ** 2))
    out["uneven"] = {"value": len(nets) / (total_1thread / CPU_THREADS), "unit": "gradients/s",
                     "cores": CPU_THREADS, "kind": "oracle",
                     "sample": f"forward + adjoint (oracle_adjoint, 5000 steps) of {len(pick)} instances spread "
                               f"over the size range ({', '.join(str(int(sizes[j])) for j in pick)} nodes), one per "
                               f"thread on {CPU_THREADS} threads ({', '.join(f'{t:.1f}' for t in t_one)} s); "
                               f"all 256 predicted by a fit t = a + b n^2, spread over {CPU_THREADS} threads"}
    return head, out


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


N1_WORKLOAD = "grid200 N-1: 400 scenarios x 600 nodes, 15,000 steps at 20 us"


def comp_roofline_object(info, nets, time_steps, kernel_s):
    """Roofline of the compensation kernel (k_comp): its solve is a dense
    product, Z rhs for every component of every scenario and step (2 n^2
    FP64 operations, fused multiply-adds on the vector units), plus 10 per
    branch for the branch phase (the Woodbury correction, 4 n per switched
    branch, is left out); bound by the FP64 rate, 78.6 TF/s. Each workgroup
    reads its family's Z (8 n^2 B) from L2 once per step: l2_gbs."""
    sizes = [int(c) for n in nets for c in component_sizes(n)]
    fam = [int(c) for c in component_sizes(nets[0])]
    flops = 2 * sum(c * c for c in sizes) + 10 * info["total_branches"]
    tflops = flops * time_steps / kernel_s / 1e12
    z_bytes = info["comp_blocks"] * 8 * float(np.mean([c * c for c in fam]))
    traffic = measured_traffic("k_comp")
    return {"bound": "alu", "achieved": tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": tflops / FP64_PEAK_TFLOPS, "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "kernel": "k_comp", "kernel_s": kernel_s, "time_steps": time_steps,
            "fp64_flops_per_time_step": flops, "l2_z_bytes_per_time_step": z_bytes,
            "l2_gbs": z_bytes * time_steps / kernel_s / 1e9,
            "comp_items": info["comp_items"], "comp_blocks": info["comp_blocks"],
            "limiter": "L2 throughput of the Z stream (see l2_gbs)"}


def batched_n1(torch, exclude_solvers=()):
    """The 400-scenario N-1 batch in one launch with its tuned shape:
    returns (networks, settings, shape, wall s, kernel s, roofline, latency)."""
    from paper_1903_01081_amd import netgen
    from paper_1903_01081_amd.sim import Simulator
    from paper_1903_01081_amd.tune import tune
    nets, cfg = netgen.config2()
    shape_b = tune(nets, cfg["dt"], cfg["n_steps"], probe_steps=300, exclude_solvers=exclude_solvers)["shape"]
    sim = Simulator(nets, cfg["dt"], cfg["n_steps"], **shape_b)
    info = sim.info()
    rec = torch.empty((sim.S, sim.n_steps, sim.R), dtype=torch.float64, device=sim.device)
    wall, kern = time_simulation(torch, sim, rec, 1, 1)
    T = cfg["n_steps"]
    if shape_b.get("solver") == "compensation":
        kernel = "k_comp"
        roof = comp_roofline_object(info, nets, T, kern)
    else:
        kernel = "k_split" if info["split_tiles"] > 0 else "k_forward"
        roof = roofline_object(info, sum(n.n_rec for n in nets), T, kernel, kern)
    lat = latency_object(sim, kernel, kern / T * 1e6, info)
    sim.close()
    del rec
    return nets, cfg, shape_b, wall, kern, roof, lat


def extras(torch, args):
    """Batched N-1 vs the per-scenario loop, adjoint/forward ratio, uneven
    batched gradients vs the per-instance loop, and the grid with
    travelling-wave lines; every side with its own tuned launch shape,
    medians of repeated timings."""
    out = extras_n1(torch)
    out.update(extras_adjoint(torch))
    out.update(extras_lines(torch, with_cpu=not args.no_cpu))
    out.update(extras_coupled(torch, with_cpu=not args.no_cpu))
    out.update(extras_rectifiers(torch, with_cpu=not args.no_cpu))
    out.update(extras_choppers(torch, with_cpu=not args.no_cpu))
    return out


RECTIFIER_WORKLOAD = ("grid200-rect20: a 200-bus grid whose first 20 loads also feed six-pulse diode bridges "
                      "(120 ideal diodes refactorised inside the loop), 640 nodes, 15000 steps at 20 us, "
                      "three-phase fault at step 7500, all nodes recorded")


def extras_rectifiers(torch, with_cpu=True):
    """The 200-bus grid with diode-bridge loads: forward node-steps/s in its
    tuned launch shape (every diode change refactorises its component inside
    the loop), latency, and the oracle's rate."""
    from paper_1903_01081_amd import netgen
    from paper_1903_01081_amd.sim import Simulator
    from paper_1903_01081_amd.tune import tune
    log("extras: diode-bridge loads")
    nets, cfg = netgen.config1(n_bus=200, n_steps=15000, rectifiers=20)
    net = nets[0]
    N, T = net.n_nodes, cfg["n_steps"]
    shape = tune(nets, cfg["dt"], T, probe_steps=400)["shape"]
    sim = Simulator(nets, cfg["dt"], T, **shape)
    info = sim.info()
    rec = torch.empty((1, sim.n_steps, sim.R), dtype=torch.float64, device=sim.device)
    runs = [time_simulation(torch, sim, rec, 1, 1 if k == 0 else 0) for k in range(3)]
    wall, kern = sorted(runs)[1]
    roof = roofline_object(info, net.n_rec, T, "k_forward", kern)
    lat = latency_object(sim, "k_forward", kern / T * 1e6, info)
    sim.close()
    del rec
    out = {"workload": RECTIFIER_WORKLOAD, "value": N * T / wall, "unit": "node-steps/s", "seconds": wall,
           "kernel_s": kern, "launch_shape": shape, "diodes": int(np.sum(net.kind == netgen.DIODE)),
           "roofline": roof, "latency": lat,
           "note": "roofline bytes exclude the factorisations inside the loop (their count depends on the run)"}
    if with_cpu:
        from oracle import oracle as O
        O.use_native_build()
        k = 1000
        med, ts = median_time(lambda: O.run(net, cfg["dt"], k))
        out["cpu_baseline"] = {
            "value": N * k / med, "unit": "node-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle (g++ -O3 -march=native, 1 thread) on the first {k} of the 15,000 steps of the "
                      f"same grid (a dense refactorisation at every diode change); median of 3 runs "
                      f"({', '.join(f'{t:.2f}' for t in ts)} s)"}
    return {"diode_rectifiers": out}


CHOPPER_WORKLOAD = ("grid200-chop20: a 200-bus grid whose first 20 loads also feed controlled choppers (20 "
                    "switches each set by a hysteresis comparator of its DC voltage, refactorised inside the loop), "
                    "620 nodes, 15000 steps at 20 us, three-phase fault at step 7500, all nodes recorded")


def extras_choppers(torch, with_cpu=True):
    """The 200-bus grid with controlled-chopper loads: forward node-steps/s in
    its tuned launch shape (every switch change refactorises its component
    inside the loop), the changes per step, latency, and the oracle's rate."""
    from paper_1903_01081_amd import netgen
    from paper_1903_01081_amd.sim import Simulator
    from paper_1903_01081_amd.tune import tune
    log("extras: controlled choppers")
    nets, cfg = netgen.config1(n_bus=200, n_steps=15000, choppers=20)
    net = nets[0]
    N, T = net.n_nodes, cfg["n_steps"]
    shape = tune(nets, cfg["dt"], T, probe_steps=400)["shape"]
    sim = Simulator(nets, cfg["dt"], T, **shape)
    info = sim.info()
    rec = torch.empty((1, sim.n_steps, sim.R), dtype=torch.float64, device=sim.device)
    runs = [time_simulation(torch, sim, rec, 1, 1 if k == 0 else 0) for k in range(3)]
    wall, kern = sorted(runs)[1]
    roof = roofline_object(info, net.n_rec, T, "k_forward", kern)
    lat = latency_object(sim, "k_forward", kern / T * 1e6, info)
    sim.close()
    del rec
    out = {"workload": CHOPPER_WORKLOAD, "value": N * T / wall, "unit": "node-steps/s", "seconds": wall,
           "kernel_s": kern, "launch_shape": shape, "controlled_switches": int(np.sum(net.kind == netgen.CSWITCH)),
           "roofline": roof, "latency": lat,
           "note": "roofline bytes exclude the factorisations inside the loop (their count depends on the run)"}
    if with_cpu:
        from oracle import oracle as O
        O.use_native_build()
        k = 3000
        med, ts = median_time(lambda: O.run(net, cfg["dt"], k))
        out["cpu_baseline"] = {
            "value": N * k / med, "unit": "node-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle (g++ -O3 -march=native, 1 thread) on the first {k} of the 15,000 steps of the "
                      f"same grid (a dense refactorisation at every switch change); median of 3 runs "
                      f"({', '.join(f'{t:.2f}' for t in ts)} s)"}
    return {"controlled_choppers": out}


COUPLED_WORKLOAD = ("grid200-coupled: a 200-bus grid with coupled three-phase lines (300 series R-L and 600 "
                    "shunt C circulant groups), 600 nodes in one component, 15000 steps at 20 us, three-phase "
                    "fault at step 7500, all nodes recorded")


def extras_coupled(torch, with_cpu=True):
    """The 200-bus grid with coupled three-phase lines: forward node-steps/s
    in its tuned launch shape, roofline, latency and the oracle's rate."""
    from paper_1903_01081_amd import netgen
    from paper_1903_01081_amd.sim import Simulator
    from paper_1903_01081_amd.tune import tune
    log("extras: coupled three-phase lines")
    nets, cfg = netgen.config1(n_bus=200, n_steps=15000, coupled=True)
    net = nets[0]
    N, T = net.n_nodes, cfg["n_steps"]
    n_groups = int(np.max(net.group)) + 1
    shape = tune(nets, cfg["dt"], T, probe_steps=400)["shape"]
    sim = Simulator(nets, cfg["dt"], T, **shape)
    info = sim.info()
    rec = torch.empty((1, sim.n_steps, sim.R), dtype=torch.float64, device=sim.device)
    runs = [time_simulation(torch, sim, rec, 1, 1 if k == 0 else 0) for k in range(3)]
    wall, kern = sorted(runs)[1]
    # per group and step: the four mutual coefficients and the members'
    # descriptor read (the members' own bytes are in the per-branch figure)
    roof = roofline_object(info, net.n_rec, T, "k_forward", kern, extra_bytes_per_step=(32 + 40) * n_groups)
    lat = latency_object(sim, "k_forward", kern / T * 1e6, info)
    sim.close()
    del rec
    out = {"workload": COUPLED_WORKLOAD, "value": N * T / wall, "unit": "node-steps/s", "seconds": wall,
           "kernel_s": kern, "launch_shape": shape, "groups": n_groups, "nnz_L": info["nnz_L"],
           "roofline": roof, "latency": lat}
    if with_cpu:
        from oracle import oracle as O
        O.use_native_build()
        k = 3000
        med, ts = median_time(lambda: O.run(net, cfg["dt"], k))
        out["cpu_baseline"] = {
            "value": N * k / med, "unit": "node-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle (g++ -O3 -march=native, 1 thread) on the first {k} of the 15,000 steps of the "
                      f"same grid, factorisation included; median of 3 runs "
                      f"({', '.join(f'{t:.2f}' for t in ts)} s)"}
    return {"coupled_three_phase_lines": out}


# per distributed-parameter line and time step: the two new waves written,
# the four delayed ones read (the interpolation's two per end)
LINE_BYTES_PER_STEP = 48
LINES_WORKLOAD = ("grid1000-tw: the grid1000 draw with its 1354 lines of travel time >= one step as "
                  "distributed-parameter lines (4062 line phases), 3000 nodes, 50000 steps at 20 us, "
                  "three-phase fault at step 25000, all nodes recorded")


def extras_lines(torch, with_cpu=True):
    """The 1000-bus grid with travelling-wave lines: forward node-steps/s in
    its tuned launch shape, roofline, latency and the oracle's rate."""
    from paper_1903_01081_amd import netgen
    from paper_1903_01081_amd.sim import Simulator
    from paper_1903_01081_amd.tune import tune
    log("extras: travelling-wave lines")
    nets, cfg = netgen.config1(travelling_wave=True)
    net = nets[0]
    N, T = net.n_nodes, cfg["n_steps"]
    n_line = int(np.sum(net.kind == netgen.LINE))
    shape = tune(nets, cfg["dt"], T, probe_steps=400)["shape"]
    sim = Simulator(nets, cfg["dt"], T, **shape)
    info = sim.info()
    rec = torch.empty((1, sim.n_steps, sim.R), dtype=torch.float64, device=sim.device)
    runs = [time_simulation(torch, sim, rec, 1, 1 if k == 0 else 0) for k in range(3)]
    wall, kern = sorted(runs)[1]
    kernel = "k_split" if info["split_tiles"] > 0 else "k_forward"
    roof = roofline_object(info, net.n_rec, T, kernel, kern,
                           extra_bytes_per_step=LINE_BYTES_PER_STEP * n_line)
    lat = latency_object(sim, kernel, kern / T * 1e6, info)
    sim.close()
    del rec
    out = {"workload": LINES_WORKLOAD, "value": N * T / wall, "unit": "node-steps/s", "seconds": wall,
           "kernel_s": kern, "launch_shape": shape, "line_phases": n_line, "components": info["n_items"],
           "nnz_L": info["nnz_L"], "roofline": roof, "latency": lat}
    if with_cpu:
        from oracle import oracle as O
        O.use_native_build()
        k = 500
        med, ts = median_time(lambda: O.run(net, cfg["dt"], k))
        out["cpu_baseline"] = {
            "value": N * k / med, "unit": "node-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle (g++ -O3 -march=native, 1 thread) on the first {k} of the 50,000 steps of the "
                      f"same grid, factorisation included; median of 3 runs "
                      f"({', '.join(f'{t:.2f}' for t in ts)} s)"}
    return {"travelling_wave_lines": out}


def extras_n1(torch):
    from paper_1903_01081_amd.sim import Simulator
    from paper_1903_01081_amd.tune import tune
    out = {}
    # Batched N-1 contingencies: 400 scenarios x 600 nodes, 15,000 steps.
    log("extras: batched N-1")
    nets, cfg, shape_b, wall, kern, roof, lat = batched_n1(torch)
    N, T = nets[0].n_nodes, cfg["n_steps"]
    batched = len(nets) * N * T / wall
    # plain per-scenario loop: every 50th scenario run alone (all scenarios
    # have the same size), median of 3 runs each, its own tuned shape
    log("extras: per-scenario loop")
    shape_1 = tune(nets[:1], cfg["dt"], T, probe_steps=300)["shape"]
    plain_t = []
    for s in range(0, len(nets), 50):
        one = Simulator([nets[s]], cfg["dt"], T, **shape_1)
        r1 = torch.empty((1, one.n_steps, one.R), dtype=torch.float64, device=one.device)
        ts = [time_simulation(torch, one, r1, 1, 1 if k == 0 else 0)[0] for k in range(3)]
        plain_t.append(float(np.median(ts)))
        one.close()
        del r1
    plain = N * T / float(np.mean(plain_t))
    out["batched_n1"] = {"workload": N1_WORKLOAD, "value": batched, "unit": "node-steps/s", "seconds": wall,
                         "launch_shape": shape_b, "roofline": roof, "latency": lat,
                         "plain_loop_value": plain,
                         "plain_loop_sample": f"{len(plain_t)} scenarios (every 50th) run one at a time, "
                                              f"median of 3 runs each",
                         "plain_launch_shape": shape_1, "speedup_vs_plain_loop": batched / plain}
    if shape_b.get("solver") == "compensation":
        # the same batch with the per-scenario factors (sweeps), tuned without
        # the compensation solver
        log("extras: batched N-1, sweep solvers")
        _, _, shape_s, wall_s, _, roof_s, lat_s = batched_n1(torch, exclude_solvers=("compensation",))
        sweeps = len(nets) * N * T / wall_s
        out["batched_n1"]["per_scenario_factors"] = {
            "value": sweeps, "seconds": wall_s, "launch_shape": shape_s, "roofline": roof_s, "latency": lat_s}
        out["batched_n1"]["speedup_vs_per_scenario_factors"] = batched / sweeps
    return out


def extras_adjoint(torch):
    from paper_1903_01081_amd import netgen
    from paper_1903_01081_amd.sim import Simulator, theta_matrix
    from paper_1903_01081_amd.tune import tune
    out = {}
    # Adjoint: 300 nodes, 10,000 steps, checkpoint every 500 (tuned shape),
    # for the pipelined kernel and the serial one; medians of 5.
    log("extras: adjoint")
    nets, cfg = netgen.config3()
    T, K = cfg["n_steps"], cfg["checkpoint_every"]
    shape_a = tune(nets, cfg["dt"], T, checkpoint_every=K, probe_steps=300)["shape"]
    adj = {"workload": "grid100: 300 nodes, 10,000 steps at 50 us, 450 parameters, checkpoint every 500",
           "launch_shape": shape_a}
    for serial in (False, True):
        sim = Simulator(nets, cfg["dt"], T, checkpoint_every=K, **dict(shape_a, serial_adjoint=serial))
        info = sim.info()
        rec = torch.empty((1, T, sim.R), dtype=torch.float64, device=sim.device)
        cot = torch.randn((1, T, sim.R), dtype=torch.float64, device=sim.device,
                          generator=torch.Generator(device=sim.device).manual_seed(3))
        stream = torch.cuda.current_stream()
        t_f, t_a, k_a = [], [], []
        for _ in range(6):
            sim.reset()
            sim.factor()
            t0 = time.perf_counter()
            sim.step(T, rec=rec)
            sim.sync()
            t1 = time.perf_counter()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            sim.adjoint(cot)
            b.record(stream)
            sim.sync()
            t_f.append(t1 - t0)
            t_a.append(time.perf_counter() - t1)
            k_a.append(a.elapsed_time(b) / 1e3)
        t_f, t_a, k_a = t_f[1:], t_a[1:], k_a[1:]   # the first is a warmup
        kname = "k_adjoint" if serial else ("k_adjoint_pipe" if info["adjoint_pipelined"] else "k_adjoint")
        n_br = info["total_branches"]
        # recompute + reverse each step; segment buffer written and read
        # (i, u per branch: 16 B per branch, twice)
        roof = roofline_object(info, 0, T, kname, float(np.median(k_a)), passes=2.0,
                               extra_bytes_per_step=32 * n_br)
        lat = latency_object(sim, "k_forward", float(np.median(k_a)) / T * 1e6, info)
        key = "serial" if serial else "default"
        adj[key] = {"pipelined": bool(info["adjoint_pipelined"]), "kernel": kname,
                    "forward_s": float(np.median(t_f)), "adjoint_s": float(np.median(t_a)),
                    "adjoint_over_forward": float(np.median(t_a)) / float(np.median(t_f)),
                    "timings": "median of 5 after one warmup", "roofline": roof, "latency": lat}
        sim.close()
        del rec, cot
    adj["adjoint_over_forward"] = adj["default"]["adjoint_over_forward"]
    out["adjoint"] = adj
    # Uneven batch: 256 networks of 90-900 nodes, forward + adjoint, tuned
    # shape; median of 3.
    log("extras: uneven batch")
    nets, cfg = netgen.config4()
    T, K = cfg["n_steps"], cfg["checkpoint_every"]
    shape_u = tune(nets, cfg["dt"], T, checkpoint_every=K, probe_steps=300)["shape"]
    sim = Simulator(nets, cfg["dt"], T, checkpoint_every=K, **shape_u)
    info = sim.info()
    theta = theta_matrix(nets, device=sim.device)
    rec = torch.empty((sim.S, T, sim.R), dtype=torch.float64, device=sim.device)
    cot = torch.randn((sim.S, T, sim.R), dtype=torch.float64, device=sim.device,
                      generator=torch.Generator(device=sim.device).manual_seed(4))

    def run_batch():
        sim.set_params(theta)
        sim.factor()
        sim.step(T, rec=rec)
        sim.adjoint(cot)
        sim.sync()

    run_batch()
    t_b, ts_b = median_time(run_batch)
    # the same iteration (set_params, factorisation, forward, mismatch
    # against a target, adjoint) captured once as a HIP graph and replayed
    from paper_1903_01081_amd.sim import IdentificationGraph
    log("  uneven batch: captured iteration")
    graph = IdentificationGraph(sim, torch.zeros_like(rec), theta)
    graph.replay()
    t_g, ts_g = median_time(graph.replay)
    del graph
    kname = "k_adjoint_pipe" if info["adjoint_pipelined"] else "k_adjoint"
    roof = roofline_object(info, sum(n.n_rec for n in nets), T, f"k_forward + {kname}", t_b, passes=3.0,
                           extra_bytes_per_step=32 * info["total_branches"])
    lat = latency_object(sim, "k_forward", t_b / (3 * T) * 1e6, info)
    sim.close()
    del rec, cot, theta
    # per-instance loop: 8 instances spread over the size range, each with
    # its own tuned shape, median of 3; the loop over all 256 is predicted
    # from a fit t = a + b n over the sample
    sizes = np.array([n.n_nodes for n in nets])
    order = np.argsort(sizes, kind="stable")
    pick = [int(order[int(round(q * (len(nets) - 1)))]) for q in np.linspace(0, 1, 8)]
    loop_t, loop_shapes = [], []
    log("extras: per-instance loop")
    for j in pick:
        log(f"  instance {j} ({sizes[j]} nodes): tuning")
        sh = tune([nets[j]], cfg["dt"], T, checkpoint_every=K, probe_steps=300)["shape"]
        one = Simulator([nets[j]], cfg["dt"], T, checkpoint_every=K, **sh)
        th1 = theta_matrix([nets[j]], device=one.device)
        r1 = torch.empty((1, T, one.R), dtype=torch.float64, device=one.device)
        c1 = torch.randn((1, T, one.R), dtype=torch.float64, device=one.device,
                         generator=torch.Generator(device=one.device).manual_seed(j))

        def run_one():
            one.set_params(th1)
            one.factor()
            one.step(T, rec=r1)
            one.adjoint(c1)
            one.sync()

        run_one()
        loop_t.append(median_time(run_one)[0])
        loop_shapes.append(sh)
        one.close()
        del r1, c1, th1
    A = np.stack([np.ones(len(pick)), sizes[pick].astype(float)], 1)
    coef, *_ = np.linalg.lstsq(A, np.array(loop_t), rcond=None)
    loop_total = float(np.sum(coef[0] + coef[1] * sizes.astype(float)))
    out["uneven_gradients"] = {
        "workload": "256 grids of 90-900 nodes, 5000 steps at 50 us, forward + adjoint",
        "launch_shape": shape_u, "pipelined": bool(info["adjoint_pipelined"]), "adjoint_kernel": kname,
        "gradients_per_s": len(nets) / t_b, "seconds": t_b, "timings": ts_b, "roofline": roof, "latency": lat,
        "graph_gradients_per_s": len(nets) / t_g, "graph_seconds": t_g, "graph_timings": ts_g,
        "graph": "one identification iteration (set_params, factorisation, forward, mismatch, adjoint) "
                 "captured as one HIP graph, replayed; median of 3",
        "per_instance_loop_gradients_per_s": len(nets) / loop_total,
        "loop_sample": f"{len(pick)} instances spread over the size range "
                       f"({', '.join(str(int(sizes[j])) for j in pick)} nodes), each with its own tuned shape, "
                       f"median of 3 runs each ({', '.join(f'{t * 1e3:.1f}' for t in loop_t)} ms); the loop "
                       f"over all 256 predicted by a fit t = a + b n",
        "loop_shapes": loop_shapes, "speedup_vs_per_instance_loop": loop_total / t_b}
    return out


def profile_adjoint(torch, which):
    """The adjoint workloads in the launch shapes the tuner picks for them on
    MI355X, without the tuner, two runs each, for a rocprofv3 kernel trace:
    "pipelined": grid100 forward + pipelined adjoint (k_adjoint_pipe);
    "serial": grid100 forward + one-workgroup adjoint and the uneven batch
    forward + adjoint (k_adjoint)."""
    from paper_1903_01081_amd import netgen
    from paper_1903_01081_amd.sim import Simulator, theta_matrix
    out = {}
    if which == "pipelined":
        runs = [("grid100_pipelined", netgen.config3, dict(solver="auto", block_size=512))]
    else:
        runs = [("grid100_serial", netgen.config3, dict(solver="auto", block_size=512, serial_adjoint=True)),
                ("uneven_serial", netgen.config4, dict(solver="auto", block_size=256, dense_tail=64))]
    for name, make, shape in runs:
        nets, cfg = make()
        T, K = cfg["n_steps"], cfg["checkpoint_every"]
        sim = Simulator(nets, cfg["dt"], T, checkpoint_every=K, **shape)
        theta = theta_matrix(nets, device=sim.device)
        rec = torch.empty((sim.S, T, sim.R), dtype=torch.float64, device=sim.device)
        cot = torch.randn((sim.S, T, sim.R), dtype=torch.float64, device=sim.device,
                          generator=torch.Generator(device=sim.device).manual_seed(5))
        ts = []
        for _ in range(2):
            sim.set_params(theta)
            sim.factor()
            t0 = time.perf_counter()
            sim.step(T, rec=rec)
            sim.sync()
            t1 = time.perf_counter()
            sim.adjoint(cot)
            sim.sync()
            ts.append((t1 - t0, time.perf_counter() - t1))
        out[name] = {"shape": shape, "pipelined": bool(sim.info()["adjoint_pipelined"]),
                     "forward_s": ts[-1][0], "adjoint_s": ts[-1][1]}
        log(name, out[name])
        sim.close()
        del rec, cot, theta
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
    ap.add_argument("--n1-solver", choices=["tuned", "sweeps"], default="tuned",
                    help="with --only-n1: the tuned shape (any solver) or the best shape without the "
                         "compensation solver (per-scenario factors)")
    ap.add_argument("--only-adjoint", action="store_true",
                    help="run only the adjoint workloads (one line; for profiling the adjoint kernels)")
    ap.add_argument("--profile-adjoint", choices=["serial", "pipelined"],
                    help="only the adjoint kernels in fixed launch shapes, two runs each (for rocprofv3): "
                         "the one-workgroup adjoint (grid100 and the uneven batch) or the pipelined one (grid100)")
    ap.add_argument("--only-lines", action="store_true",
                    help="run only the grids with travelling-wave lines, coupled three-phase lines, "
                         "diode-bridge loads and controlled-chopper loads (one line)")
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

    import gc
    import torch
    try:
        if args.calibrate_copy:
            calibrate_copy(torch)
        elif args.only_n1:
            excl = ("compensation",) if args.n1_solver == "sweeps" else ()
            nets, cfg, shape, wall, kern, roof, lat = batched_n1(torch, exclude_solvers=excl)
            nsteps = len(nets) * nets[0].n_nodes * cfg["n_steps"]
            print(json.dumps({"metric": "node-steps/s, batched N-1", "value": nsteps / wall, "unit": "node-steps/s",
                              "workload": N1_WORKLOAD, "launch_shape": shape, "seconds": wall, "kernel_s": kern,
                              "roofline": roof, "latency": lat}), flush=True)
        elif args.only_lines:
            out = extras_lines(torch, with_cpu=not args.no_cpu)
            out.update(extras_coupled(torch, with_cpu=not args.no_cpu))
            out.update(extras_rectifiers(torch, with_cpu=not args.no_cpu))
            out.update(extras_choppers(torch, with_cpu=not args.no_cpu))
            print(json.dumps(out), flush=True)
        elif args.only_adjoint:
            print(json.dumps(extras_adjoint(torch)), flush=True)
        elif args.profile_adjoint is not None:
            print(json.dumps(profile_adjoint(torch, args.profile_adjoint)), flush=True)
        else:
            headline(torch, args)
    finally:
        # every context is closed by now; leave no device work or library
        # object for the interpreter's (or a profiler's) exit handlers
        gc.collect()
        if torch.cuda.is_available():
            torch.cuda.synchronize()


def headline(torch, args):
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
    lat = latency_object(sim, kernel, kern / T * 1e6, info)
    roof = roofline_object(info, net.n_rec, T, kernel, kern, traffic=measured_traffic(kernel))
    # the work the launch actually does with the dense inverse (8 n^2 B and
    # 2 n^2 flops per component per step, on chip)
    roof["dense_inverse_bytes_per_time_step"] = algorithmic_bytes_per_step(info, net.n_rec, sizes) \
        if sizes is not None else None
    roof["dense_inverse_fp64_tflops"] = (algorithmic_flops_per_step(info, sizes) * T / kern / 1e12
                                         if sizes is not None else None)
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
        "roofline": roof,
        "latency": lat,
        "efficiency": {"figure": "latency.floor_over_step", "value": lat["floor_over_step"]},
        "build_s": build_s, "tune_s": tune_s,
    }
    sim.close()
    del rec
    if not args.no_extras:
        line["solver_comparison"] = solver_comparison(torch, nets, cfg, tuned, shape, wall / args.steps)
        line.update(extras(torch, args))
    if not args.no_cpu:
        from oracle import oracle as O
        head, others = cpu_baselines(O)
        line["cpu_baseline"] = head
        line["cpu_baseline_other"] = others
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
