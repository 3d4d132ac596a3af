"""One parameter-identification iteration of an uneven batch (set_params,
emt_factor_async, forward, emt_mismatch, adjoint) recorded into a HIP graph
and replayed: every replay is checked against the same calls run eagerly
(bitwise: same kernels, same order) with eager work and synchronisations
between replays, the parameters are changed in place between replays, and
one replay's gradient is compared with the oracle's adjoint."""
import sys

import numpy as np
import pytest

from paper_1903_01081_amd import netgen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def eager(torch, sim, theta, target):
    rec = torch.zeros((sim.S, sim.n_steps, sim.R), dtype=torch.float64, device=sim.device)
    dJ = torch.zeros_like(rec)
    loss = torch.zeros((sim.S,), dtype=torch.float64, device=sim.device)
    sim.set_params(theta)
    sim.factor()
    sim.step(sim.n_steps, rec=rec)
    sim.mismatch(rec, target, dJ, loss)
    grad = sim.adjoint(dJ)
    sim.sync()
    return loss.cpu().numpy(), grad.cpu().numpy()


def test_identification_graph_replays(torch_cuda, oracle_mod):
    torch = torch_cuda
    from paper_1903_01081_amd.sim import IdentificationGraph, Simulator, theta_matrix
    nets, cfg = netgen.config4(n_inst=6, n_steps=600)
    dt, T = cfg["dt"], cfg["n_steps"]
    say("identification graph: 6 uneven grids, 600 steps, K=100")
    # target waveforms from the perturbed parameters (device forward)
    sim = Simulator(nets, dt, T, checkpoint_every=100)
    th_true = theta_matrix(nets, cfg["theta_true"], device=sim.device)
    th0 = theta_matrix(nets, device=sim.device)
    sim.set_params(th_true)
    sim.factor()
    target = sim.step(T).clone()
    sim.sync()
    ref0 = eager(torch, sim, th0, target)
    ref1 = eager(torch, sim, th_true, target)
    g = IdentificationGraph(sim, target, th0)
    for k, (th, ref) in enumerate([(th0, ref0), (th_true, ref1), (th0, ref0), (th0, ref0)]):
        g.theta.copy_(th)
        loss, grad = g.replay()
        l_np, g_np = loss.cpu().numpy(), grad.cpu().numpy()
        say(f"replay {k}: loss {l_np[:3]}")
        assert np.array_equal(l_np, ref[0]), f"replay {k}: loss differs from the eager run"
        assert np.array_equal(g_np, ref[1]), f"replay {k}: gradient differs from the eager run"
        # eager work between replays
        eager(torch, sim, th_true if k % 2 == 0 else th0, target)
    # at the true parameters the mismatch is zero
    assert np.all(ref1[0] == 0.0)
    # one replay against the oracle: loss and adjoint of scenario 0
    net = nets[0]
    tgt = oracle_mod.run(net, dt, T, theta=cfg["theta_true"][0])
    v = oracle_mod.run(net, dt, T)
    loss_ref = float(np.sum((v - tgt) ** 2))
    g_ref = oracle_mod.adjoint(net, dt, T, 2.0 * (v - tgt))
    assert abs(ref0[0][0] - loss_ref) <= 1e-9 * loss_ref
    th = net.theta0()
    a, b = th * ref0[1][0, :net.n_params], th * g_ref
    err = float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-12 * np.max(np.abs(b)))))
    say("graph gradient vs oracle adjoint", err)
    assert err < 1e-6
    sim.close()


def test_factor_async_reports_pivots_at_sync(torch_cuda):
    """A parameter vector with a negative capacitance makes a pivot
    non-positive: emt_factor_async queues without error and emt_sync
    reports EMT_ESINGULAR; afterwards the context needs a new factorisation."""
    torch = torch_cuda
    from paper_1903_01081_amd import _lib
    from paper_1903_01081_amd.sim import Simulator, theta_matrix
    net = netgen.small_grid(81, 6, n_mon=6)
    sim = Simulator([net], 50e-6, 20, checkpoint_every=10)
    th = net.theta0().copy()
    th[2::3] = -1e-3     # every line's C: the node diagonals turn negative
    sim.set_params(theta_matrix([net], [th], device=sim.device))
    sim.factor_async()
    with pytest.raises(_lib.EMTError) as e:
        sim.sync()
    assert e.value.status == _lib.EMT_ESINGULAR
    with pytest.raises(_lib.EMTError) as e:
        sim.step(5)
    assert e.value.status == _lib.EMT_ESTATE
    sim.set_params(theta_matrix([net], device=sim.device))
    sim.factor_async()
    sim.step(20)
    sim.sync()
    sim.close()
