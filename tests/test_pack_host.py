"""Host-side analysis of packed work items (no GPU): how a scenario's
components are packed into items and what the library refuses."""
import pytest

from paper_1903_01081_amd import _lib, netgen


def test_packing_counts():
    nets, cfg = netgen.config4(n_inst=10, n_steps=100)
    dt = cfg["dt"]
    base = _lib.analyze(nets, dt, 100)
    assert base["n_items"] == 30  # three uncoupled phases per grid
    prev = base["n_items"]
    for p in (96, 256, 512, 4000):
        a = _lib.analyze(nets, dt, 100, pack_nodes=p)
        # same nodes, branches and factor sizes, fewer items
        assert a["total_nodes"] == base["total_nodes"] and a["total_branches"] == base["total_branches"]
        assert a["nnz_L"] == base["nnz_L"]
        assert a["n_items"] <= prev and a["max_item_nodes"] <= max(p, base["max_item_nodes"])
        prev = a["n_items"]
    # a budget above every grid's size: one item per grid
    assert prev == len(nets)


def test_packing_keeps_scenarios_apart():
    nets, cfg = netgen.config2(n_bus=30, n_scen=12, n_steps=100, event_step=50)
    a = _lib.analyze(nets, cfg["dt"], 100, pack_nodes=10000)
    assert a["n_items"] == 12


def test_pack_refusals():
    nets, cfg = netgen.config4(n_inst=2, n_steps=10)
    with pytest.raises(Exception, match="at most 128"):
        _lib.analyze(nets, cfg["dt"], 10, solver=1, pack_nodes=256)
    with pytest.raises(Exception, match="pack_nodes"):
        _lib.analyze(nets, cfg["dt"], 10, pack_nodes=-1)
