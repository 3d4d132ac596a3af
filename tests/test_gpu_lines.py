"""Distributed-parameter (travelling-wave) lines on the HIP path against the
CPU oracle: grids whose longer lines are lossless Bergeron lines (each end a
Norton equivalent 1/Z to ground fed by the wave that left the other end one
travel time earlier, interpolated between steps), with the remaining lines as
pi-sections; both solvers; a fault switching during the run; stepping in
chunks; a batch of grids with and without lines; reset; and the cases the
library refuses (checkpoints, the split dense solver, set_state)."""
import sys

import numpy as np
import pytest

from paper_1903_01081_amd import netgen
from paper_1903_01081_amd.netgen import LINE

pytestmark = pytest.mark.gpu

TOL = 1e-9


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def rel(a, b):
    s = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (s if s > 0 else 1.0))


def grid(seed, n_bus, dt, fault_step=None):
    net = netgen.small_grid(seed, n_bus, fault_step=fault_step, travelling_wave_dt=dt)
    n_line = int(np.sum(net.kind == LINE))
    assert n_line > 0 and n_line < net.n_branches
    return net


@pytest.mark.parametrize("solver", ["auto", "sparse", "dense"])
@pytest.mark.parametrize("dt", [20e-6, 5e-6])
def test_lines_vs_oracle(torch_cuda, oracle_mod, solver, dt):
    # dt = 20 us: travel times of 1-5 steps; 5 us: up to 20 steps (longer
    # rings); the fault closes mid-run (a refactorisation with lines present)
    from paper_1903_01081_amd.sim import Simulator
    T = 600
    net = grid(3, 12, dt, fault_step=250)
    D = net.L[net.kind == LINE] / dt
    say(f"lines: 12 buses, dt={dt}, solver={solver}, {len(D)} line phases, tau/dt {D.min():.2f}-{D.max():.2f}")
    sim = Simulator([net], dt, T, solver=solver)
    sim.factor()
    got = sim.step(T).cpu().numpy()[0]
    ref = oracle_mod.run(net, dt, T)
    err = rel(got, ref)
    say("rel err", err)
    assert err < TOL


def test_lines_branch_state_vs_oracle(torch_cuda, oracle_mod):
    # a line's branch current is the current into it at its k end, its
    # voltage that of the k end
    from paper_1903_01081_amd.sim import Simulator
    dt, T = 20e-6, 400
    net = grid(5, 10, dt)
    say("lines: branch state after 400 steps")
    sim = Simulator([net], dt, T)
    sim.factor()
    sim.step(T, record=False)
    v, i = sim.get_state(0)
    _, vt, it, _ = oracle_mod.run(net, dt, T, trajectories=True)
    assert rel(v, vt[T]) < TOL
    assert rel(i, it[T]) < TOL


def test_lines_chunked_and_reset(torch_cuda, oracle_mod):
    # the wave rings carry over between emt_step calls (chunks shorter and
    # longer than the travel times) and return to rest at reset
    from paper_1903_01081_amd.sim import Simulator
    dt, T = 5e-6, 500
    net = grid(7, 10, dt, fault_step=123)
    say("lines: chunked stepping 1 + 2 + 17 + 180 + 300, then reset")
    sim = Simulator([net], dt, T)
    sim.factor()
    parts = [sim.step(k).cpu().numpy()[0] for k in (1, 2, 17, 180, 300)]
    got = np.concatenate(parts, axis=0)
    ref = oracle_mod.run(net, dt, T)
    assert rel(got, ref) < TOL
    sim.reset()
    again = sim.step(T).cpu().numpy()[0]
    assert rel(again, ref) < TOL


def test_lines_batch_mixed(torch_cuda, oracle_mod):
    # grids with and without lines, of different sizes, in one launch
    from paper_1903_01081_amd.sim import Simulator
    dt, T = 20e-6, 300
    nets = [grid(11, 8, dt), netgen.small_grid(12, 9), grid(13, 20, dt, fault_step=100),
            grid(14, 5, dt)]
    say("lines: mixed batch of 4 grids")
    sim = Simulator(nets, dt, T)
    sim.factor()
    rec = sim.step(T).cpu().numpy()
    for s, net in enumerate(nets):
        ref = oracle_mod.run(net, dt, T)
        err = rel(rec[s][:, :net.n_rec], ref)
        say("grid", s, "rel err", err)
        assert err < TOL


def test_lines_refused(torch_cuda):
    from paper_1903_01081_amd.sim import Simulator
    dt, T = 20e-6, 50
    net = grid(3, 12, dt)
    say("lines: refused configurations")
    with pytest.raises(Exception, match="forward only"):
        Simulator([net], dt, T, checkpoint_every=10)
    # 150 nodes per (uncoupled) phase: the dense solver would split such a
    # component over workgroups
    with pytest.raises(Exception, match="one workgroup"):
        Simulator([grid(3, 150, dt)], dt, T, solver="dense")
    sim = Simulator([net], dt, T)
    with pytest.raises(Exception, match="rest"):
        sim.set_state(0, np.zeros(net.n_nodes), np.zeros(net.n_branches))
    # a travel time shorter than the step
    with pytest.raises(Exception, match="travel time"):
        Simulator([net], 1e-3, T)


# ---------------------------------------------------------------------------
# Full size: the 1000-bus grid with its long lines as travelling-wave lines
# (3000 nodes, 4062 line phases, 50,000 steps), in the launch bench.py times.
# ---------------------------------------------------------------------------

# the two shapes the tuner picks between on MI355X (within 1 % of each other)
@pytest.fixture(scope="module", params=["auto", "sparse"])
def grid1000_tw_run(request, torch_cuda):
    from paper_1903_01081_amd.sim import Simulator
    nets, cfg = netgen.config1(travelling_wave=True)
    say(f"grid1000-tw full horizon: 3000 nodes, 4062 line phases, 50000 steps, {request.param}")
    sim = Simulator(nets, cfg["dt"], cfg["n_steps"], solver=request.param)
    sim.factor()
    rec = sim.step(cfg["n_steps"])
    sim.sync()
    return nets, cfg, sim, rec


def test_grid1000_tw_prefix_vs_oracle(grid1000_tw_run, oracle_mod):
    nets, cfg, _, rec = grid1000_tw_run
    T0 = 300
    ref = oracle_mod.run(nets[0], cfg["dt"], T0)
    err = rel(rec[0, :T0].cpu().numpy(), ref)
    say("grid1000-tw prefix rel err", err)
    assert err < TOL


def test_grid1000_tw_zero_sequence_whole_horizon(grid1000_tw_run):
    # identical phases (each line's three phases share Z and tau), balanced
    # sources, symmetric fault: every bus's phase voltages sum to zero
    _, _, _, rec = grid1000_tw_run
    r = rec[0]
    zs = r.view(r.shape[0], -1, 3).sum(dim=2).abs().max().item()
    assert zs / r.abs().max().item() < 1e-11


def test_grid1000_tw_whole_horizon_vs_oracle_samples(grid1000_tw_run):
    """All 50,000 steps checked at the samples the oracle wrote over its own
    full run (tests/golden/make_goldens.py grid1000tw): every 100th step at
    64 nodes, every node at steps 24,999-25,003 (the fault) and at step
    50,000; error relative to the largest |v| of the oracle trajectory."""
    import os
    import torch
    nets, cfg, _, rec = grid1000_tw_run
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "grid1000_tw_samples.npz"))
    assert int(g["n_steps"]) == cfg["n_steps"] and float(g["dt"]) == cfg["dt"]
    r = rec[0]
    steps = torch.as_tensor(g["steps"] - 1, device=r.device)
    nodes = torch.as_tensor(g["nodes"], device=r.device)
    got = r.index_select(0, steps).index_select(1, nodes).cpu().numpy()
    fault = r.index_select(0, torch.as_tensor(g["fault_steps"] - 1, device=r.device)).cpu().numpy()
    last = r[-1].cpu().numpy()
    vmax = float(g["vmax"])
    errs = [float(np.max(np.abs(got - g["v_steps_nodes"]))) / vmax,
            float(np.max(np.abs(fault - g["v_fault"]))) / vmax,
            float(np.max(np.abs(last - g["v_last"]))) / vmax]
    say("grid1000-tw whole-horizon sampled rel errs", errs)
    assert max(errs) < TOL
