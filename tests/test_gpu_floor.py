"""The latency floors of the step kernels (emt_latency_floor): positive,
below the step kernel's own time per step in the same launch shape, and
without effect on the simulation (the run after a floor measurement equals
a run without one, bitwise)."""
import sys
import time

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


def step_us(torch, sim, T):
    sim.reset()
    sim.factor()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(T, record=False)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / T * 1e6


@pytest.mark.parametrize("shape,kind", [(dict(solver="dense", split_cols=32), "split"),
                                        (dict(solver="auto"), "one_workgroup")])
def test_floor_below_step_time_and_state_untouched(torch_cuda, shape, kind):
    from paper_1903_01081_amd.sim import Simulator
    nets, cfg = netgen.config1(n_steps=2000, fault_step=1000)
    T = cfg["n_steps"]
    sim = Simulator(nets, cfg["dt"], T, **shape)
    sim.factor()
    ref = sim.step(T).cpu().numpy()
    step = step_us(torch_cuda, sim, T)
    sim.reset()
    sim.factor()
    first = sim.step(T // 2).cpu().numpy()
    floor = sim.latency_floor(kind, 2000)
    rest = sim.step(T - T // 2).cpu().numpy()
    say(f"{kind}: step {step:.2f} us, floor {floor:.2f} us")
    assert 0.0 < floor < step
    assert np.array_equal(np.concatenate([first, rest], axis=1), ref)


def test_floor_rejects_missing_kind_and_bad_steps(torch_cuda):
    from paper_1903_01081_amd._lib import EMTError
    from paper_1903_01081_amd.sim import Simulator
    nets, cfg = netgen.config0(n_steps=50)
    sim = Simulator(nets, cfg["dt"], 50)
    assert sim.latency_floor("one_workgroup", 10) > 0.0
    with pytest.raises(EMTError, match="EMT_EINVAL"):
        sim.latency_floor("split", 10)
    with pytest.raises(EMTError, match="EMT_EINVAL"):
        sim.latency_floor("one_workgroup", 0)
