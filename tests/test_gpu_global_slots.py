"""Regression: the step kernels whose sweep data stay in global memory exist
for 4, 8 and 16 branches per lane; a batch whose LDS variant would hold 1,
2, 6 or 12 per lane is padded to the global variant's count. Forward and
adjoint in those shapes against the CPU oracle, and the padding reported."""
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


def rel(a, b):
    s = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (s if s > 0 else 1.0))


def grad_err(g, ref, theta):
    a, b = theta * g, theta * ref
    floor = 1e-12 * np.max(np.abs(b))
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), floor)))


# (buses, block size, branches per lane the LDS variant would use)
CASES = [(10, 64, 1), (64, 64, 6), (64, 256, 2), (120, 64, 12)]


@pytest.mark.parametrize("n_bus,bs,lds_bpt", CASES, ids=[f"bus{c[0]}-bs{c[1]}" for c in CASES])
def test_global_sweep_variant_padding(torch_cuda, oracle_mod, n_bus, bs, lds_bpt):
    from paper_1903_01081_amd.sim import Simulator, theta_matrix
    torch = torch_cuda
    net = netgen.small_grid(21, n_bus, fault_step=40, n_mon=10)
    dt, T, K = 20e-6, 200, 50
    say(f"global sweep data: {n_bus} buses, block {bs}")
    sim = Simulator([net], dt, T, checkpoint_every=K, block_size=bs, sweep_from_global=True)
    info = sim.info()
    assert info["lds_staged"] == 0
    want = 4 if lds_bpt <= 4 else (8 if lds_bpt <= 8 else 16)
    assert info["lanes_per_block"] == want
    sim.set_params(theta_matrix([net], device=sim.device))
    sim.factor()
    rec = sim.step(T).cpu().numpy()[0]
    assert rel(rec, oracle_mod.run(net, dt, T)) < 1e-9
    rng = np.random.default_rng(n_bus)
    cot = rng.standard_normal((1, T, net.n_rec))
    g = sim.adjoint(torch.tensor(cot, dtype=torch.float64, device=sim.device)).cpu().numpy()[0]
    ref = oracle_mod.adjoint(net, dt, T, cot[0])
    assert grad_err(g[:net.n_params], ref, net.theta0()) < 1e-6
