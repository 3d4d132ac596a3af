"""Coupled three-phase lines (circulant 3 x 3 series R-L and shunt C groups)
on the HIP path against the CPU oracle: both one-workgroup solvers and the
dense tail, a fault during the run, a batch mixing coupled, uncoupled and
travelling-wave grids, stepping in chunks and reset, an arbitrary initial
state, the steady-state start, the refusals, and at full size a 200-bus
grid (600 nodes, one coupled component) over its whole 15,000-step
horizon."""
import sys

import numpy as np
import pytest

from paper_1903_01081_amd import netgen

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


@pytest.mark.parametrize("solver", ["auto", "sparse", "dense"])
def test_coupled_vs_oracle(torch_cuda, oracle_mod, solver):
    from paper_1903_01081_amd.sim import Simulator
    net = netgen.small_grid(7, 12, coupled=True, fault_step=250)
    dt, T = 50e-6, 600
    say(f"coupled 12-bus grid, {solver}")
    sim = Simulator([net], dt, T, solver=solver)
    assert sim.info()["n_items"] == 1
    sim.factor()
    got = sim.step(T).cpu().numpy()[0]
    err = rel(got, oracle_mod.run(net, dt, T))
    say("rel err", err)
    assert err < TOL


def test_coupled_single_phase_fault_vs_oracle(torch_cuda, oracle_mod):
    # an unbalanced event: only phase a of one bus faults (no sequence
    # decoupling), and a branch of an uncoupled load switched out
    from paper_1903_01081_amd.sim import Simulator
    from paper_1903_01081_amd.netgen import SWITCH
    net = netgen.small_grid(9, 16, coupled=True, fault_step=200)
    sw = np.where(net.kind == SWITCH)[0]
    keep = net.ev_branch != sw[1]
    keep &= net.ev_branch != sw[2]
    net.ev_step, net.ev_branch, net.ev_in_service = net.ev_step[keep], net.ev_branch[keep], net.ev_in_service[keep]
    dt, T = 20e-6, 500
    say("coupled grid, single-phase fault")
    sim = Simulator([net], dt, T)
    sim.factor()
    got = sim.step(T).cpu().numpy()[0]
    assert rel(got, oracle_mod.run(net, dt, T)) < TOL


def test_coupled_mixed_batch_chunks_and_reset(torch_cuda, oracle_mod):
    from paper_1903_01081_amd.sim import Simulator
    dt, T = 20e-6, 400
    nets = [netgen.small_grid(11, 10, coupled=True, fault_step=90), netgen.small_grid(12, 9),
            netgen.small_grid(13, 8, travelling_wave_dt=dt), netgen.small_grid(14, 6, coupled=True)]
    say("mixed batch: coupled, uncoupled, travelling-wave, coupled")
    sim = Simulator(nets, dt, T)
    sim.factor()
    parts = [sim.step(k).cpu().numpy() for k in (1, 37, 162, 200)]
    got = np.concatenate(parts, axis=1)
    for s, net in enumerate(nets):
        err = rel(got[s][:, :net.n_rec], oracle_mod.run(net, dt, T))
        say("grid", s, "rel err", err)
        assert err < TOL
    sim.reset()
    again = sim.step(T).cpu().numpy()
    assert rel(again[0][:, :nets[0].n_rec], oracle_mod.run(nets[0], dt, T)) < TOL


def test_coupled_from_a_given_state(torch_cuda, oracle_mod):
    # the group pass forms the first history from the stored state
    from paper_1903_01081_amd.sim import Simulator
    net = netgen.small_grid(15, 10, coupled=True)
    dt, T = 50e-6, 300
    rng = np.random.default_rng(5)
    v0 = rng.standard_normal(net.n_nodes)
    i0 = rng.standard_normal(net.n_branches) * 0.01
    i0[net.in_service0 == 0] = 0.0
    say("coupled grid from a random state")
    sim = Simulator([net], dt, T)
    sim.factor()
    sim.set_state(0, v0, i0)
    got = sim.step(T).cpu().numpy()[0]
    assert rel(got, oracle_mod.run(net, dt, T, v0=v0, i0=i0)) < TOL


def test_coupled_steady_state(torch_cuda, oracle_mod):
    from paper_1903_01081_amd.sim import Simulator
    net = netgen.small_grid(23, 15, coupled=True, fault_step=150)
    dt, T = 50e-6, 300
    say("coupled grid, steady-state start")
    sim = Simulator([net], dt, T)
    sim.factor()
    sim.steady_state()
    v, i = sim.get_state(0)
    v0, i0, _ = oracle_mod.steady_state(net, dt)
    assert rel(v, v0) < 1e-10 and rel(i, i0) < 1e-10
    got = sim.step(T).cpu().numpy()[0]
    assert rel(got, oracle_mod.run(net, dt, T, v0=v0, i0=i0)) < TOL


def test_coupled_refusals(torch_cuda):
    from paper_1903_01081_amd.sim import Simulator
    net = netgen.small_grid(7, 12, coupled=True)
    with pytest.raises(Exception, match="forward only"):
        Simulator([net], 50e-6, 50, checkpoint_every=10)
    # 50 buses: one 150-node coupled component, which the dense solver would split
    with pytest.raises(Exception, match="one workgroup"):
        Simulator([netgen.small_grid(7, 50, coupled=True)], 50e-6, 50, solver="dense")
    ev = netgen.small_grid(7, 12, coupled=True, remove_series=0, remove_step=20)
    with pytest.raises(Exception, match="no switching events"):
        Simulator([ev], 50e-6, 50)


@pytest.fixture(scope="module")
def grid200_coupled_run(torch_cuda):
    from paper_1903_01081_amd.sim import Simulator
    nets, cfg = netgen.config1(n_bus=200, n_steps=15000, coupled=True)
    say("grid200-coupled full horizon: 600 nodes, 15000 steps")
    sim = Simulator(nets, cfg["dt"], cfg["n_steps"])
    sim.factor()
    rec = sim.step(cfg["n_steps"]).cpu().numpy()[0]
    sim.sync()
    sim.close()
    return nets, cfg, rec


def test_grid200_coupled_whole_horizon_vs_oracle(grid200_coupled_run, oracle_mod):
    """All 15,000 steps and 600 nodes element by element (the fault at step
    7500 included)."""
    nets, cfg, rec = grid200_coupled_run
    ref = oracle_mod.run(nets[0], cfg["dt"], cfg["n_steps"])
    err = rel(rec, ref)
    say("grid200-coupled whole-horizon rel err", err)
    assert err < TOL
