"""Controlled switches (one hysteresis comparator per switch, a control
vertex that measures a node voltage of a step and sets the switch for the
next step, refactorised inside the time loop) on the HIP path against the
CPU oracle: the open-loop chopper whose schedule is the reference's alone,
bang-bang control of a capacitor voltage, a grid whose loads include
controlled choppers, with a fault, stepped in chunks and reset, both sweep
solvers, and the refusals. Every comparator decision in these runs clears
its threshold by a wide margin (checked on the oracle run), so rounding
differences between the two sides cannot flip one."""
import dataclasses
import math
import sys

import numpy as np
import pytest

from paper_1903_01081_amd import netgen
from paper_1903_01081_amd.netgen import CAP, CSWITCH, RES, SRC

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


def chopper(ref_E=0.0, ref_w=0.0, ref_ph=0.0, ref_C=5.0, h=0.2, meas=(1, -1), E=10.0, w=0.0, on=1):
    return netgen.circuit(2, [
        dict(k=0, m=-1, kind=SRC, R=1.0, L=1e-4, E=E, omega=w, phase=0.0),
        dict(k=0, m=1, kind=CSWITCH, R=1e-2, E=ref_E, omega=ref_w, phase=ref_ph, C=ref_C, L=h, meas=meas, ins=on),
        dict(k=1, m=-1, kind=CAP, C=1e-3),
        dict(k=1, m=-1, kind=RES, R=20.0),
    ])


def grid_with_choppers(seed, n_bus, buses, fault_step=None, V_ref=0.4, h=0.05):
    """A grid whose listed buses (phase a) also feed a controlled chopper:
    switch -> a capacitor and load resistor to ground, its comparator holding
    the capacitor voltage near V_ref."""
    net = netgen.small_grid(seed, n_bus, fault_step=fault_step)
    n = net.n_nodes
    cols = {f: [] for f in ("k", "m", "kind", "R", "L", "C", "E", "omega", "phase", "line", "in_service0")}
    meas = [(-1, -1)] * net.n_branches
    for q, bus in enumerate(buses):
        d = n + q
        for br in (dict(k=3 * bus, m=d, kind=CSWITCH, R=1e-2, L=h, C=V_ref, meas=(d, -1)),
                   dict(k=d, m=-1, kind=CAP, C=2e-4), dict(k=d, m=-1, kind=RES, R=40.0)):
            cols["k"].append(br["k"]); cols["m"].append(br["m"]); cols["kind"].append(br["kind"])
            cols["R"].append(br.get("R", 0.0)); cols["L"].append(br.get("L", 0.0)); cols["C"].append(br.get("C", 0.0))
            cols["E"].append(0.0); cols["omega"].append(0.0); cols["phase"].append(0.0)
            cols["line"].append(-1); cols["in_service0"].append(1)
            meas.append(br.get("meas", (-1, -1)))
    out = dataclasses.replace(net, n_nodes=n + len(buses), rec_nodes=None)
    for f, vals in cols.items():
        setattr(out, f, np.concatenate([getattr(net, f), np.asarray(vals, getattr(net, f).dtype)]))
    out.meas = np.asarray(meas, np.int32)
    return out


def decision_margin(oracle_mod, net, dt, T):
    """Smallest distance of a comparator's error e = r - s from its
    thresholds +h and -h over the oracle's run, relative to the largest
    |reference|, |measured voltage| and half-width involved."""
    _, vt, _, _ = oracle_mod.run(net, dt, T, trajectories=True)
    cs = np.where(net.kind == CSWITCH)[0]
    best, scale = np.inf, 0.0
    for b in cs:
        a0, a1 = net.meas[b]
        s = (vt[:, a0] if a0 >= 0 else 0.0) - (vt[:, a1] if a1 >= 0 else 0.0)
        t = dt * np.arange(T + 1)
        r = net.E[b] * np.cos(net.omega[b] * t + net.phase[b]) + net.C[b]
        e = (r - s)[1:T]
        h = net.L[b]
        best = min(best, float(np.min(np.minimum(np.abs(e - h), np.abs(e + h)))))
        scale = max(scale, float(np.max(np.abs(r))), float(np.max(np.abs(s))), h)
    return best / scale


@pytest.mark.parametrize("solver", ["auto", "sparse"])
def test_open_loop_chopper_vs_oracle(torch_cuda, oracle_mod, solver):
    from paper_1903_01081_amd.sim import Simulator
    net = chopper(ref_E=1.0, ref_w=2 * math.pi * 50, ref_ph=0.3, ref_C=0.1, h=0.3, meas=(-1, -1),
                  E=10.0, w=2 * math.pi * 60)
    dt, T = 20e-6, 3000
    assert decision_margin(oracle_mod, net, dt, T) > 1e-10
    say(f"open-loop chopper, {solver}")
    sim = Simulator([net], dt, T, solver=solver)
    sim.factor()
    got = sim.step(T).cpu().numpy()[0]
    sim.sync()
    assert rel(got, oracle_mod.run(net, dt, T)) < TOL


def test_bang_bang_band_vs_oracle(torch_cuda, oracle_mod):
    from paper_1903_01081_amd.sim import Simulator
    net = chopper()
    dt, T = 20e-6, 6000
    assert decision_margin(oracle_mod, net, dt, T) > 1e-10
    say("bang-bang capacitor voltage control")
    sim = Simulator([net], dt, T)
    sim.factor()
    got = sim.step(T).cpu().numpy()[0]
    sim.sync()
    ref = oracle_mod.run(net, dt, T)
    assert rel(got, ref) < TOL
    v = got[:, 1]
    assert np.count_nonzero(np.diff((v > 5.0).astype(int))) > 10


def test_grid_with_choppers_chunks_and_reset(torch_cuda, oracle_mod):
    from paper_1903_01081_amd.sim import Simulator
    net = grid_with_choppers(46, 10, [1, 4, 8], fault_step=600)
    dt, T = 20e-6, 1200
    assert decision_margin(oracle_mod, net, dt, T) > 1e-10
    say("grid with three controlled choppers and a fault, chunks 1 + 399 + 800")
    sim = Simulator([net], dt, T)
    sim.factor()
    parts = [sim.step(k).cpu().numpy()[0] for k in (1, 399, 800)]
    sim.sync()
    ref = oracle_mod.run(net, dt, T)
    assert rel(np.concatenate(parts, axis=0), ref) < TOL
    sim.reset()
    again = sim.step(T).cpu().numpy()[0]
    sim.sync()
    assert rel(again, ref) < TOL


def test_cswitch_batch_vs_oracle(torch_cuda, oracle_mod):
    from paper_1903_01081_amd.sim import Simulator
    dt, T = 20e-6, 1500
    nets = [chopper(), chopper(ref_C=3.0, h=0.1), netgen.small_grid(5, 8),
            grid_with_choppers(48, 8, [2, 5], fault_step=700)]
    for net in nets:
        if np.any(net.kind == CSWITCH):
            assert decision_margin(oracle_mod, net, dt, T) > 1e-10
    say("batch: two choppers, a plain grid, a grid with choppers")
    sim = Simulator(nets, dt, T)
    sim.factor()
    rec = sim.step(T).cpu().numpy()
    sim.sync()
    for s, net in enumerate(nets):
        err = rel(rec[s][:, :net.n_rec], oracle_mod.run(net, dt, T))
        say("net", s, "rel err", err)
        assert err < TOL


def test_cswitch_refusals(torch_cuda):
    from paper_1903_01081_amd.sim import EMTError, Simulator
    net = chopper()
    with pytest.raises(EMTError, match="forward only"):
        Simulator([net], 20e-6, 50, checkpoint_every=10)
    with pytest.raises(EMTError, match="sweep solvers"):
        Simulator([net], 20e-6, 50, solver="dense")
    sim = Simulator([net], 20e-6, 50)
    with pytest.raises(EMTError, match="controlled switches"):
        sim.steady_state()
    sim.close()
    ev = chopper()
    ev.ev_step, ev.ev_branch, ev.ev_in_service = np.array([5]), np.array([1], np.int32), np.array([0], np.uint8)
    with pytest.raises(EMTError, match="controller"):
        Simulator([ev], 20e-6, 50)
    other = netgen.circuit(4, [
        dict(k=0, m=-1, kind=SRC, R=1.0, L=1e-4, E=10.0),
        dict(k=0, m=1, kind=CSWITCH, R=1e-2, C=5.0, L=0.2, meas=(3, -1)),
        dict(k=1, m=-1, kind=RES, R=20.0),
        dict(k=2, m=-1, kind=SRC, R=1.0, L=1e-4, E=1.0),
        dict(k=2, m=3, kind=RES, R=1.0), dict(k=3, m=-1, kind=RES, R=1.0)])
    with pytest.raises(EMTError, match="outside its connected component"):
        Simulator([other], 20e-6, 50)


def test_grid200_choppers_full_size(torch_cuda, oracle_mod):
    """The benchmarked grid with controlled-chopper loads (200 buses, 20
    controlled switches, 620 nodes, 15,000 steps) in the launch bench.py
    times: the first 3000 steps element by element (every comparator
    decision there clears its threshold by more than 1e-10 of the
    quantities involved), and at the last step KCL at every node."""
    from paper_1903_01081_amd.sim import Simulator
    nets, cfg = netgen.config1(n_bus=200, n_steps=15000, choppers=20)
    net, dt, T = nets[0], cfg["dt"], cfg["n_steps"]
    say("grid200 with 20 controlled choppers, 15000 steps")
    sim = Simulator(nets, dt, T)
    sim.factor()
    rec = sim.step(T).cpu().numpy()[0]
    sim.sync()
    T0 = 3000
    assert decision_margin(oracle_mod, net, dt, T0) > 1e-10
    err = rel(rec[:T0], oracle_mod.run(net, dt, T0))
    say("prefix rel err", err)
    assert err < TOL
    v, i = sim.get_state(0)
    inj = np.zeros(net.n_nodes)
    mag = np.zeros(net.n_nodes)
    for arr, sgn in ((net.k, 1.0), (net.m, -1.0)):
        ok = arr >= 0
        np.add.at(inj, arr[ok], sgn * i[ok])
        np.add.at(mag, arr[ok], np.abs(i[ok]))
    assert np.max(np.abs(inj)) <= 1e-9 * np.max(mag)
    assert np.allclose(rec[-1], v, rtol=0, atol=0)
    sim.close()
