"""Packed work items (pack_nodes > 0: several connected components of one
scenario share a workgroup, their G block-diagonal within the item) against
the CPU oracle: forward waveforms and adjoint gradients of uneven batches,
an N-1 batch with each scenario's three phases in one item, and with
events, checkpoints and both solvers."""
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


def grad_err(g, ref, theta):
    a, b = theta * g, theta * ref
    floor = 1e-12 * np.max(np.abs(b))
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), floor)))


@pytest.mark.parametrize("pack,solver", [(96, "auto"), (256, "auto"), (512, "sparse"), (128, "dense")])
def test_packed_uneven_forward(torch_cuda, oracle_mod, pack, solver):
    from paper_1903_01081_amd.sim import Simulator
    nets, cfg = netgen.config4(n_inst=10, n_steps=400)
    dt, T = cfg["dt"], cfg["n_steps"]
    sim = Simulator(nets, dt, T, solver=solver, pack_nodes=pack)
    plain = Simulator(nets, dt, T, solver=solver)
    assert sim.info()["n_items"] < plain.info()["n_items"]
    plain.close()
    say(f"packed uneven forward: pack {pack}, {solver}, {sim.info()['n_items']} items")
    sim.factor()
    rec = sim.step(T).cpu().numpy()
    refs = oracle_mod.run_batch(nets, dt, T, n_threads=4)
    errs = [rel(rec[s][:, :n.n_rec], refs[s]) for s, n in enumerate(nets)]
    say("rel errs", max(errs))
    assert max(errs) < TOL


@pytest.mark.parametrize("serial", [False, True])
def test_packed_uneven_adjoint(torch_cuda, oracle_mod, serial):
    from paper_1903_01081_amd.sim import Simulator, theta_matrix
    torch = torch_cuda
    nets, cfg = netgen.config4(n_inst=8, n_steps=500)
    dt, T, K = cfg["dt"], cfg["n_steps"], 100
    sim = Simulator(nets, dt, T, checkpoint_every=K, pack_nodes=256, serial_adjoint=serial)
    say(f"packed uneven adjoint: {sim.info()['n_items']} items, serial={serial}")
    sim.set_params(theta_matrix(nets, device=sim.device))
    sim.factor()
    sim.step(T)
    rng = np.random.default_rng(9)
    cot = rng.standard_normal((len(nets), T, sim.R))
    g = sim.adjoint(torch.tensor(cot, dtype=torch.float64, device=sim.device)).cpu().numpy()
    for s, net in enumerate(nets):
        ref = oracle_mod.adjoint(net, dt, T, cot[s, :, :net.n_rec])
        err = grad_err(g[s, :net.n_params], ref, net.theta0())
        assert err < 1e-6, (s, err)


def test_packed_n1_three_phases_per_item(torch_cuda, oracle_mod):
    # each scenario's three phase components in one item: one workgroup per
    # scenario; scenarios with a branch out and a fault at step 120
    from paper_1903_01081_amd.sim import Simulator
    nets, cfg = netgen.config2(n_bus=30, n_scen=12, n_steps=300, event_step=120)
    dt, T = cfg["dt"], cfg["n_steps"]
    sim = Simulator(nets, dt, T, pack_nodes=90)
    assert sim.info()["n_items"] == len(nets)
    say("packed N-1: 12 scenarios, one item each")
    sim.factor()
    rec = sim.step(T).cpu().numpy()
    refs = oracle_mod.run_batch(nets, dt, T, n_threads=4)
    errs = [rel(rec[s][:, :n.n_rec], refs[s]) for s, n in enumerate(nets)]
    assert max(errs) < TOL

