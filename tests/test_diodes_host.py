"""Host-side analysis of ideal diodes (no GPU): a diode belongs to its
component whatever its initial state, and the forward-only and solver
restrictions are enforced."""
import math

import pytest

from paper_1903_01081_amd import _lib, netgen
from paper_1903_01081_amd.netgen import DIODE, RES, SRC


def rectifier(on):
    return netgen.circuit(2, [
        dict(k=0, m=-1, kind=SRC, R=1.0, L=20e-3, E=1.0, omega=2 * math.pi * 60, phase=0.0),
        dict(k=0, m=1, kind=DIODE, R=1e-2, ins=on),
        dict(k=1, m=-1, kind=RES, R=5.0)])


@pytest.mark.parametrize("on", [0, 1])
def test_diode_joins_its_component(on):
    info = _lib.analyze([rectifier(on)], 20e-6, 10)
    assert info["n_items"] == 1 and info["nnz_L"] == 1


def test_diode_refusals():
    with pytest.raises(Exception, match="forward only"):
        _lib.analyze([rectifier(1)], 20e-6, 10, checkpoint_every=5)
    with pytest.raises(Exception, match="sweep solvers"):
        _lib.analyze([rectifier(1)], 20e-6, 10, solver=1)
    bad = rectifier(1)
    bad.R = bad.R.copy()
    bad.R[1] = 0.0
    with pytest.raises(Exception, match="on-resistance"):
        _lib.analyze([bad], 20e-6, 10)
