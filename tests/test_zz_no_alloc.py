"""emt_step_noalloc (the entry point for callers that cannot allocate)
against emt_step: two calls in a row through the C ABI, the second on a
smaller network, each compared bitwise with emt_step on a twin context and
with the oracle to the forward tolerance (1e-9 relative to the largest
|v|); plus the host-side rejection of a batch whose exchange exceeds the
static space."""
import ctypes as C
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


def run_pair(torch, net, dt, T, cols):
    """Returns (emt_step rec, emt_step_noalloc rec) of twin contexts."""
    from paper_1903_01081_amd import _lib
    from paper_1903_01081_amd.sim import Simulator, _dev_ptr, _stream
    out = []
    for noalloc in (False, True):
        sim = Simulator([net], dt, T, solver="dense", split_cols=cols)
        assert sim.info()["split_tiles"] > 0
        sim.factor()
        rec = torch.full((1, T, sim.R), float("nan"), dtype=torch.float64, device=sim.device)
        fn = sim.lib.emt_step_noalloc if noalloc else sim.lib.emt_step
        # two chunks, as a caller stepping in a loop would
        h = T // 2
        for a, b in ((0, h), (h, T)):
            _lib.check(fn(sim._ctx, b - a, _dev_ptr(rec[:, a:b], (1, b - a, sim.R), "rec"), _stream()))
        sim.sync()
        out.append(rec.cpu().numpy()[0])
        sim.close()
    return out


def test_noalloc_matches_emt_step_twice_second_smaller(torch_cuda, oracle_mod):
    cases = [(netgen.small_grid(71, 300, fault_step=700, n_mon=40), 1400, 32),
             (netgen.small_grid(72, 150, fault_step=300, remove_series=4, remove_step=450, n_mon=30), 600, 16)]
    for net, T, cols in cases:
        say(f"noalloc vs emt_step: {net.n_nodes} nodes, {T} steps, {cols}-column tiles")
        ref_gpu, got = run_pair(torch_cuda, net, 20e-6, T, cols)
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref_gpu), "emt_step_noalloc differs from emt_step"
        ref = oracle_mod.run(net, 20e-6, T)
        err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        say("rel err vs oracle", err)
        assert err < TOL


def test_noalloc_rejects_exchange_beyond_static_space(torch_cuda):
    from paper_1903_01081_amd import _lib
    from paper_1903_01081_amd.sim import Simulator, _stream
    # 3 x 1000 nodes in 16-column tiles: 63 tiles per component, 3 MB of
    # partials (host-side check; nothing is launched)
    nets, cfg = netgen.config1(n_steps=10, fault_step=5)
    say("noalloc rejection: grid1000 in 16-column tiles")
    sim = Simulator(nets, cfg["dt"], 10, solver="dense", split_cols=16)
    sim.factor()
    st = sim.lib.emt_step_noalloc(sim._ctx, 10, None, _stream())
    assert st == _lib.EMT_EINVAL
    assert b"static exchange space" in sim.lib.emt_last_error()
    # the context is untouched: emt_step still runs it
    sim.step(10, record=False)
    sim.sync()
    sim.close()
