"""Host side of the compensation solver (no device): the plan that groups
work items into families around the first scenario's components and finds
each scenario's switched branches, and the batches it refuses."""
import numpy as np
import pytest

from paper_1903_01081_amd import _lib, netgen
from paper_1903_01081_amd.sim import SOLVERS

COMP = SOLVERS["compensation"]


def analyze(nets, cfg, **kw):
    return _lib.analyze(nets, cfg["dt"], cfg["n_steps"], solver=COMP, **kw)


def test_n1_families_and_rank():
    # every scenario: one series branch out (one phase) and a three-phase
    # fault: two switched branches in one phase, one in the others
    nets, cfg = netgen.config2(n_bus=20, n_scen=12, n_steps=600, event_step=200)
    info = analyze(nets, cfg)
    assert info["n_items"] == 36
    assert info["comp_families"] == 3
    assert info["comp_max_rank"] == 2


def test_full_n1_batch_plans():
    nets, cfg = netgen.config2()
    info = analyze(nets, cfg)
    assert info["n_items"] == 1200 and info["comp_families"] == 3 and info["comp_max_rank"] == 2


def test_same_network_has_rank_zero():
    net = netgen.small_grid(5, 12)
    net.ev_step = net.ev_step[:0]
    net.ev_branch = net.ev_branch[:0]
    net.ev_in_service = net.ev_in_service[:0]
    info = _lib.analyze([net, net], 50e-6, 100, solver=COMP)
    assert info["comp_max_rank"] == 0


def test_reordered_branches_match():
    # the same network with its branch list permuted: every branch matches
    nets, cfg = netgen.config2(n_bus=12, n_scen=2, n_steps=100, event_step=50)
    import dataclasses
    a = nets[0]
    p = np.random.default_rng(1).permutation(a.n_branches)
    inv = np.argsort(p)
    b = dataclasses.replace(a, k=a.k[p], m=a.m[p], kind=a.kind[p], R=a.R[p], L=a.L[p], C=a.C[p], E=a.E[p],
                            omega=a.omega[p], phase=a.phase[p], line=a.line[p], in_service0=a.in_service0[p],
                            ev_branch=inv[a.ev_branch].astype(np.int32))
    info = analyze([a, b], cfg)
    assert info["comp_max_rank"] == 2  # the base's own event: branch out + fault


def test_refusals():
    nets, cfg = netgen.config2(n_bus=20, n_scen=4, n_steps=100, event_step=50)
    with pytest.raises(_lib.EMTError, match="forward only"):
        _lib.analyze(nets, cfg["dt"], cfg["n_steps"], checkpoint_every=10, solver=COMP)
    with pytest.raises(_lib.EMTError, match="more than 4"):
        analyze(nets[:2] + [netgen.small_grid(3, 20)], cfg)
    with pytest.raises(_lib.EMTError, match="not a component|does not have"):
        analyze(nets[:2] + [netgen.small_grid(3, 21)], cfg)
    with pytest.raises(_lib.EMTError, match="distributed-parameter"):
        tw = netgen.small_grid(4, 10, travelling_wave_dt=cfg["dt"])
        analyze([tw, tw], cfg)
    with pytest.raises(_lib.EMTError, match="coupled"):
        cp = netgen.small_grid(4, 10, coupled=True)
        analyze([cp, cp], cfg)
    with pytest.raises(_lib.EMTError, match="at most 256"):
        big, bcfg = netgen.config2(n_bus=300, n_scen=2, n_steps=100, event_step=50)
        analyze(big, bcfg)
    with pytest.raises(_lib.EMTError, match="comp_items"):
        sim = _lib.make_sim(cfg["dt"], cfg["n_steps"], solver=COMP, comp_items=7)
        import ctypes as C
        P = _lib.PackedNets(nets)
        info = _lib.EmtInfo()
        _lib.check(_lib.load().emt_analyze(P.ref, P.n, C.addressof(sim), C.addressof(info)))


def test_five_switched_branches_refused():
    nets, cfg = netgen.config2(n_bus=20, n_scen=3, n_steps=100, event_step=50)
    n = nets[1]
    series = [b for b in range(n.n_branches) if n.line[b] >= 0 and n.kind[b] == netgen.RL]
    # five more series branches of phase 0 out at step 60 (they may island
    # nodes: the rank check comes first only if the topology is valid, so
    # take branches whose removal keeps every node grounded through shunts)
    ph0 = [b for b in series if n.k[b] % 3 == 0][:5]
    n.ev_step = np.concatenate([n.ev_step, np.full(5, 60)]).astype(np.int64)
    n.ev_branch = np.concatenate([n.ev_branch, ph0]).astype(np.int32)
    n.ev_in_service = np.concatenate([n.ev_in_service, np.zeros(5)]).astype(np.uint8)
    with pytest.raises(_lib.EMTError, match="more than 4"):
        analyze(nets, cfg)
