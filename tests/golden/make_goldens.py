"""Writes the sampled expected values that the full-size GPU parity tests
compare against. Calls only the CPU oracle (oracle/) on the seeded inputs of
paper_1903_01081_amd.netgen (which draws networks and holds none of the
method's arithmetic); nothing here runs or reads the HIP library.

    python tests/golden/make_goldens.py grid1000   # ~10 min, one core
    python tests/golden/make_goldens.py grid100fd  # ~1 min, one core
    python tests/golden/make_goldens.py grid1000tw # ~10 min, one core

grid1000_samples.npz: the 1000-bus grid (3000 nodes, 50,000 steps at 20 us,
three-phase fault at step 25,000, every node recorded) over its whole
horizon, sampled: every 100th step at 64 seeded nodes, every node at steps
24,999-25,003 (the fault) and at step 50,000, plus max |v| over all steps
and nodes (the scale of the relative tolerance).

grid1000_tw_samples.npz: the same grid and samples with every line whose
travel time is at least one step entered as a distributed-parameter
(travelling-wave) line.

grid100_fd.npz: central differences of the loss J = sum (v - v_target)^2 of
the 100-bus adjoint workload (300 nodes, 10,000 steps at 50 us, 30 monitored
nodes, target from the perturbed parameters theta*) at the nominal
parameters, for the 20 seeded parameter indices the workload draws, with a
relative step of 1e-6.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1903_01081_amd import netgen  # noqa: E402


def grid1000(travelling_wave=False):
    nets, cfg = netgen.config1(travelling_wave=travelling_wave)
    net = nets[0]
    T = cfg["n_steps"]
    rng = np.random.default_rng(12345)
    nodes = np.sort(rng.choice(net.n_nodes, size=64, replace=False)).astype(np.int64)
    steps = np.arange(100, T + 1, 100, dtype=np.int64)      # 1-based step numbers
    fault = np.arange(24999, 25004, dtype=np.int64)
    t0 = time.time()
    rec = O.run(net, cfg["dt"], T)                          # [T][n_nodes], row j = step j+1
    print(f"oracle run {time.time() - t0:.0f} s", flush=True)
    name = "grid1000_tw_samples.npz" if travelling_wave else "grid1000_samples.npz"
    np.savez_compressed(
        os.path.join(HERE, name),
        nodes=nodes, steps=steps, v_steps_nodes=rec[np.ix_(steps - 1, nodes)],
        fault_steps=fault, v_fault=rec[fault - 1], v_last=rec[T - 1],
        vmax=np.array(np.max(np.abs(rec))), dt=np.array(cfg["dt"]), n_steps=np.array(T))


def grid100fd(h=1e-6):
    nets, cfg = netgen.config3()
    net = nets[0]
    dt, T = cfg["dt"], cfg["n_steps"]
    th0 = net.theta0()
    target = O.run(net, dt, T, theta=cfg["theta_true"][0])
    idx = np.asarray(cfg["fd_idx"], np.int64)

    def loss(th):
        v = O.run(net, dt, T, theta=th)
        return float(np.sum((v - target) ** 2))

    g = np.empty(idx.shape[0])
    t0 = time.time()
    for a, j in enumerate(idx):
        step = h * th0[j]
        tp, tm = th0.copy(), th0.copy()
        tp[j] += step
        tm[j] -= step
        g[a] = (loss(tp) - loss(tm)) / (2 * step)
    print(f"{2 * idx.shape[0]} oracle runs {time.time() - t0:.0f} s", flush=True)
    np.savez(os.path.join(HERE, "grid100_fd.npz"), fd_idx=idx, g_fd=g, h=np.array(h),
             theta0=th0, loss0=np.array(loss(th0)))


if __name__ == "__main__":
    which = sys.argv[1:] or ["grid1000", "grid100fd", "grid1000tw"]
    for w in which:
        {"grid1000": grid1000, "grid100fd": grid100fd,
         "grid1000tw": lambda: grid1000(travelling_wave=True)}[w]()
