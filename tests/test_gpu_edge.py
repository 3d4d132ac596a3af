"""Degenerate and boundary cases of the HIP path, each against the CPU
oracle: a one-node network, a single step, a chain (the deepest
elimination), events at the first and the last step, several events in
one step, a branch removed and restored (three topologies), a batch of
networks with different event schedules, nothing recorded, one-node dense
components, and emt_step(0)."""
import math
import sys

import numpy as np
import pytest

from paper_1903_01081_amd import netgen
from paper_1903_01081_amd.netgen import CAP, RES, RL, SRC, SWITCH

pytestmark = pytest.mark.gpu

TOL = 1e-9
W60 = 2 * math.pi * 60


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


def run(nets, dt, T, **shape):
    from paper_1903_01081_amd.sim import Simulator
    sim = Simulator(nets, dt, T, **shape)
    sim.factor()
    return sim, sim.step(T).cpu().numpy()


def one_node():
    return netgen.circuit(1, [
        dict(k=0, m=-1, kind=SRC, R=0.5, L=10e-3, E=1.0, omega=W60, phase=0.3),
        dict(k=0, m=-1, kind=CAP, C=1e-6),
        dict(k=0, m=-1, kind=RL, R=100.0, L=0.2),
    ])


@pytest.mark.parametrize("T", [1, 300])
@pytest.mark.parametrize("solver", ["auto", "sparse", "dense"])
def test_one_node(torch_cuda, oracle_mod, T, solver):
    net = one_node()
    say(f"one node, T={T}, solver={solver}")
    _, rec = run([net], 20e-6, T, solver=solver)
    assert rec.shape == (1, T, 1)
    assert rel(rec[0], oracle_mod.run(net, 20e-6, T)) < TOL


def three_bus(events):
    # bus 0 - line a - bus 1 - line b - bus 2, capacitors at every bus, a
    # source at bus 0, a load at bus 2 and an open switch from bus 2 to ground
    br = [
        dict(k=0, m=-1, kind=SRC, R=0.5, L=10e-3, E=1.0, omega=W60, phase=0.1),
        dict(k=0, m=1, kind=RL, R=1.0, L=5e-3, line=0),
        dict(k=1, m=2, kind=RL, R=2.0, L=8e-3, line=1),
        dict(k=0, m=-1, kind=CAP, C=2e-7, line=0),
        dict(k=1, m=-1, kind=CAP, C=2e-7, line=0),
        dict(k=1, m=-1, kind=CAP, C=3e-7, line=1),
        dict(k=2, m=-1, kind=CAP, C=3e-7, line=1),
        dict(k=2, m=-1, kind=RL, R=80.0, L=0.1),
        dict(k=2, m=-1, kind=SWITCH, R=1e-3, ins=0),
        dict(k=1, m=-1, kind=RES, R=500.0),
    ]
    return netgen.circuit(3, br, events=events)


def test_events_first_last_same_step_and_toggle(torch_cuda, oracle_mod):
    T = 240
    events = [(1, 8, 1),            # switch closes at the first step
              (60, 2, 0), (60, 9, 0),  # two branches out in one step
              (150, 2, 1),          # line b restored: a third topology
              (T, 8, 0)]            # switch opens at the last step
    net = three_bus(events)
    say("three buses: events at steps 1, 60 (two), 150 and T")
    sim, rec = run([net], 20e-6, T)
    assert sim.info()["max_topologies"] == 5
    assert rel(rec[0], oracle_mod.run(net, 20e-6, T)) < TOL


def test_batch_with_different_event_schedules(torch_cuda, oracle_mod):
    nets = [three_bus([]), three_bus([(30, 8, 1)]), three_bus([(10, 2, 0), (20, 2, 1), (90, 8, 1)])]
    say("three buses x 3 event schedules in one batch")
    _, rec = run(nets, 20e-6, 120)
    for s, net in enumerate(nets):
        assert rel(rec[s], oracle_mod.run(net, 20e-6, 120)) < TOL


@pytest.mark.parametrize("solver", ["auto", "sparse"])
def test_chain(torch_cuda, oracle_mod, solver):
    # a 250-node chain: series R-L between neighbours, a capacitor at every
    # node, a source at one end; the elimination's deepest level structure
    n = 250
    br = [dict(k=0, m=-1, kind=SRC, R=0.5, L=10e-3, E=1.0, omega=W60, phase=0.0)]
    for a in range(n - 1):
        br.append(dict(k=a, m=a + 1, kind=RL, R=0.05, L=1e-4, line=a))
    for a in range(n):
        br.append(dict(k=a, m=-1, kind=CAP, C=1e-7))
    br.append(dict(k=n - 1, m=-1, kind=RL, R=50.0, L=0.05))
    net = netgen.circuit(n, br, rec_nodes=list(range(0, n, 7)))
    say(f"chain of {n} nodes, solver={solver}")
    _, rec = run([net], 20e-6, 200, solver=solver)
    assert rel(rec[0], oracle_mod.run(net, 20e-6, 200)) < TOL


def test_nothing_recorded(torch_cuda, oracle_mod):
    # no recorded node: the output is empty, the state still evolves and a
    # gradient of an empty waveform is zero
    import torch
    from paper_1903_01081_amd.sim import Simulator
    net = three_bus([(40, 8, 1)])
    net.rec_nodes = np.zeros(0, np.int32)
    sim = Simulator([net], 20e-6, 100, checkpoint_every=25)
    assert sim.R == 0
    sim.factor()
    rec = sim.step(100)
    assert tuple(rec.shape) == (1, 100, 0)
    v, _ = sim.get_state(0)
    _, vt, _, _ = oracle_mod.run(net, 20e-6, 100, trajectories=True)
    assert rel(v, vt[100]) < TOL
    g = sim.adjoint(torch.zeros((1, 100, 0), dtype=torch.float64, device=sim.device))
    assert torch.count_nonzero(g).item() == 0


def test_step_zero_is_a_no_op(torch_cuda):
    from paper_1903_01081_amd.sim import Simulator
    net = three_bus([])
    sim = Simulator([net], 20e-6, 50)
    sim.factor()
    a = sim.step(20).cpu().numpy()
    sim.step(0, record=False)
    assert sim.info()["step"] == 20
    b = sim.step(30).cpu().numpy()
    sim.reset()
    c = sim.step(50).cpu().numpy()
    assert np.array_equal(np.concatenate([a, b], axis=1), c)
