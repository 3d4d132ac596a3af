"""The compensation solver (a shared base inverse per component, applied to
several scenarios' right-hand sides at once, plus a Sherman-Morrison-Woodbury
correction for each scenario's switched branches) on the HIP path against
the CPU oracle: N-1 batches with a removed branch and a fault per scenario
at every items-per-workgroup count (ragged last workgroups included), a
component larger than one product chunk, a scenario that recloses its branch
(three topologies), stepping in chunks and reset, a given initial state and
the steady-state start, new line parameters, the refusals, and the full N-1
workload (400 scenarios x 600 nodes, 15,000 steps) in the launch bench.py
times: sampled scenarios against the oracle over the whole horizon and every
scenario against the sweep solver."""
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


def small_n1(n_bus=20, n_scen=12, n_steps=600, event_step=200):
    return netgen.config2(n_bus=n_bus, n_scen=n_scen, n_steps=n_steps, event_step=event_step)


def check_all(oracle_mod, nets, cfg, rec, T, **kw):
    refs = oracle_mod.run_batch(nets, cfg["dt"], T, n_threads=4, **kw)
    errs = [rel(rec[s][:, :nets[s].n_rec], refs[s]) for s in range(len(nets))]
    say("max rel err", max(errs))
    assert max(errs) < TOL


@pytest.mark.parametrize("q", [0, 1, 5, 6])
def test_comp_n1_vs_oracle(torch_cuda, oracle_mod, q):
    from paper_1903_01081_amd.sim import Simulator
    nets, cfg = small_n1()
    T = cfg["n_steps"]
    say(f"N-1 20 buses x 12 scenarios, comp_items {q}")
    sim = Simulator(nets, cfg["dt"], T, solver="compensation", comp_items=q)
    info = sim.info()
    assert info["comp_families"] == 3 and info["comp_max_rank"] == 2
    if q:
        assert info["comp_items"] == q
        assert info["comp_blocks"] == 3 * -(-12 // q)
    sim.factor()
    rec = sim.step(T).cpu().numpy()
    sim.sync()
    check_all(oracle_mod, nets, cfg, rec, T)


def test_comp_larger_component_vs_oracle(torch_cuda, oracle_mod):
    # 60-node phases: several product chunks and a tail, two branch slots per lane
    from paper_1903_01081_amd.sim import Simulator
    nets, cfg = small_n1(n_bus=60, n_scen=10, n_steps=400, event_step=150)
    T = cfg["n_steps"]
    say("N-1 60 buses x 10 scenarios")
    sim = Simulator(nets, cfg["dt"], T, solver="compensation", comp_items=4)
    assert sim.info()["lanes_per_block"] >= 2
    sim.factor()
    rec = sim.step(T).cpu().numpy()
    sim.sync()
    check_all(oracle_mod, nets, cfg, rec, T)


def test_comp_reclose_three_topologies(torch_cuda, oracle_mod):
    # scenario 3 recloses its removed branch later: its third topology
    # differs from the base by the fault only
    from paper_1903_01081_amd.sim import Simulator
    nets, cfg = small_n1()
    T = cfg["n_steps"]
    n = nets[3]
    br = n.meta["removed_branch"]
    n.ev_step = np.append(n.ev_step, 420).astype(n.ev_step.dtype)
    n.ev_branch = np.append(n.ev_branch, br).astype(n.ev_branch.dtype)
    n.ev_in_service = np.append(n.ev_in_service, 1).astype(n.ev_in_service.dtype)
    sim = Simulator(nets, cfg["dt"], T, solver="compensation")
    assert sim.info()["max_topologies"] == 3
    sim.factor()
    rec = sim.step(T).cpu().numpy()
    sim.sync()
    check_all(oracle_mod, nets, cfg, rec, T)


def test_comp_chunks_reset_and_given_state(torch_cuda, oracle_mod):
    from paper_1903_01081_amd.sim import Simulator
    nets, cfg = small_n1()
    T, dt = cfg["n_steps"], cfg["dt"]
    sim = Simulator(nets, dt, T, solver="compensation", comp_items=5)
    sim.factor()
    say("chunks 1 + 199 + 400")
    rec = np.concatenate([sim.step(k).cpu().numpy() for k in (1, 199, 400)], axis=1)
    sim.sync()
    check_all(oracle_mod, nets, cfg, rec, T)
    sim.reset()
    again = sim.step(T).cpu().numpy()
    sim.sync()
    assert np.array_equal(again, rec)
    # from a given state
    sim.reset()
    rng = np.random.default_rng(7)
    v0, i0 = [], []
    for s, net in enumerate(nets):
        v = rng.standard_normal(net.n_nodes)
        i = rng.standard_normal(net.n_branches) * 0.01
        i[net.in_service0 == 0] = 0.0
        sim.set_state(s, v, i)
        v0.append(v)
        i0.append(i)
    got = sim.step(T).cpu().numpy()
    sim.sync()
    for s in (0, 5, 11):
        ref = oracle_mod.run(nets[s], dt, T, v0=v0[s], i0=i0[s])
        assert rel(got[s][:, :nets[s].n_rec], ref) < TOL


def test_comp_steady_state_start(torch_cuda, oracle_mod):
    from paper_1903_01081_amd.sim import Simulator
    nets, cfg = small_n1()
    T, dt = cfg["n_steps"], cfg["dt"]
    sim = Simulator(nets, dt, T, solver="compensation")
    sim.factor()
    sim.steady_state()
    got = sim.step(T).cpu().numpy()
    sim.sync()
    for s in (0, 4, 9):
        v0, i0, _ = oracle_mod.steady_state(nets[s], dt)
        ref = oracle_mod.run(nets[s], dt, T, v0=v0, i0=i0)
        assert rel(got[s][:, :nets[s].n_rec], ref) < TOL


def test_comp_set_params(torch_cuda, oracle_mod):
    from paper_1903_01081_amd.sim import EMTError, Simulator, theta_matrix
    nets, cfg = small_n1()
    T, dt = cfg["n_steps"], cfg["dt"]
    sim = Simulator(nets, dt, T, solver="compensation")
    rng = np.random.default_rng(3)
    th = netgen.perturbed_theta(rng, nets[0].theta0())
    thetas = [th.copy() for _ in nets]
    sim.set_params(theta_matrix(nets, thetas, device=sim.device))
    sim.factor()
    rec = sim.step(T).cpu().numpy()
    sim.sync()
    check_all(oracle_mod, nets, cfg, rec, T, thetas=thetas)
    # one scenario's line parameters no longer match the base's
    thetas[5] = thetas[5] * 1.01
    sim.set_params(theta_matrix(nets, thetas, device=sim.device))
    with pytest.raises(EMTError, match="pi-section"):
        sim.factor()


def test_comp_refusals(torch_cuda):
    from paper_1903_01081_amd.sim import EMTError, Simulator
    nets, cfg = small_n1()
    dt, T = cfg["dt"], cfg["n_steps"]
    with pytest.raises(EMTError, match="lanes per component"):
        Simulator(nets, dt, T, solver="compensation", block_size=512)
    with pytest.raises(EMTError, match="forward only"):
        Simulator(nets, dt, T, solver="compensation", checkpoint_every=100)
    with pytest.raises(EMTError, match="more than 4"):
        Simulator(nets[:2] + [netgen.small_grid(3, 20)], dt, T, solver="compensation")
    with pytest.raises(EMTError, match="not a component|does not have"):
        Simulator(nets[:2] + [netgen.small_grid(3, 21)], dt, T, solver="compensation")


@pytest.fixture(scope="module")
def n1_full(torch_cuda):
    from paper_1903_01081_amd.sim import Simulator
    nets, cfg = netgen.config2()
    T = cfg["n_steps"]
    say("grid200 N-1 full: 400 scenarios x 600 nodes, 15000 steps, compensation")
    sim = Simulator(nets, cfg["dt"], T, solver="compensation")
    info = sim.info()
    say("comp_items", info["comp_items"], "blocks", info["comp_blocks"])
    sim.factor()
    rec = sim.step(T)
    sim.sync()
    sim.close()
    return nets, cfg, rec


def test_comp_n1_full_size_sampled_scenarios(n1_full, oracle_mod):
    nets, cfg, rec = n1_full
    pick = [0, 137, 399]
    got = rec[pick].cpu().numpy()
    refs = oracle_mod.run_batch([nets[s] for s in pick], cfg["dt"], cfg["n_steps"], n_threads=3)
    errs = [rel(got[q], refs[q]) for q in range(len(pick))]
    say("grid200 N-1 compensation sampled rel errs", errs)
    assert max(errs) < TOL


def test_comp_n1_full_size_every_scenario_vs_sweeps(n1_full, torch_cuda):
    from paper_1903_01081_amd.sim import Simulator
    nets, cfg, rec = n1_full
    say("grid200 N-1 full, sweep solver for comparison")
    sim = Simulator(nets, cfg["dt"], cfg["n_steps"], solver="auto", block_size=256)
    sim.factor()
    ref = sim.step(cfg["n_steps"])
    sim.sync()
    sim.close()
    err = ((rec - ref).abs().amax(dim=(1, 2)) / ref.abs().amax(dim=(1, 2))).max().item()
    say("every scenario, max rel difference", err)
    assert err < TOL
