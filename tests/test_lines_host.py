"""Host-side analysis of networks with distributed-parameter lines (no GPU):
what the library accepts, how it lays the lines out, and what it refuses."""
import numpy as np
import pytest

from paper_1903_01081_amd import _lib, netgen
from paper_1903_01081_amd.netgen import LINE, RL, SRC


def line_pair(tau=50e-6, Z=300.0, events=()):
    return netgen.circuit(2, [
        dict(k=0, m=-1, kind=SRC, R=1.0, L=1e-3, E=1.0, omega=377.0, phase=0.0),
        dict(k=0, m=1, kind=LINE, R=Z, L=tau),
        dict(k=1, m=-1, kind=RL, R=200.0, L=0.1),
    ], events=events)


def test_line_is_two_local_branches():
    info = _lib.analyze([line_pair()], 20e-6, 10)
    # each line becomes two Norton ends to ground: 3 network branches -> 4
    assert info["total_branches"] == 4
    # the ends share one component (one workgroup carries both)
    assert info["n_items"] == 1 and info["max_item_nodes"] == 2
    # no off-diagonal conductance between the two ends
    assert info["nnz_L"] == 0


def test_lines_decouple_the_grid():
    nets, cfg = netgen.config1(n_bus=60, n_steps=100, travelling_wave=True)
    pi, _ = netgen.config1(n_bus=60, n_steps=100)
    a = _lib.analyze(nets, cfg["dt"], 100)
    b = _lib.analyze(pi, cfg["dt"], 100)
    assert a["nnz_L"] < b["nnz_L"] and a["max_levels"] <= b["max_levels"]


@pytest.mark.parametrize("what", ["short", "checkpoints", "event", "ground", "lossy", "param"])
def test_line_refusals(what):
    dt = 20e-6
    kw = {}
    if what == "short":
        net = line_pair(tau=10e-6)
        match = "travel time"
    elif what == "checkpoints":
        net = line_pair()
        kw = dict(checkpoint_every=5)
        match = "forward only"
    elif what == "event":
        net = line_pair(events=[(3, 1, 0)])
        match = "no switching events"
    elif what == "ground":
        net = line_pair()
        net.m[1] = -1
        match = "two nodes"
    elif what == "lossy":
        net = line_pair()
        net.C[1] = 1e-9
        match = "lossless"
    else:
        net = line_pair()
        net.line = np.array([-1, 0, -1], np.int32)
        net.n_lines = 1
        match = "only R-L and C"
    with pytest.raises(Exception, match=match):
        _lib.analyze([net], dt, 10, **kw)
