"""Host validation of controlled switches (no device): the analysis accepts
them with their measured nodes and refuses what the time loop cannot run."""
import numpy as np
import pytest

from paper_1903_01081_amd import _lib, netgen
from paper_1903_01081_amd.netgen import CSWITCH, RES, SRC


def net_with(**kw):
    sw = dict(k=0, m=1, kind=CSWITCH, R=1e-2, C=5.0, L=0.2, meas=(1, -1))
    sw.update(kw)
    return netgen.circuit(2, [dict(k=0, m=-1, kind=SRC, R=1.0, L=1e-4, E=10.0), sw,
                              dict(k=1, m=-1, kind=RES, R=20.0)])


def test_accepted_and_one_component():
    info = _lib.analyze([net_with()], 20e-6, 100)
    assert info["n_items"] == 1


@pytest.mark.parametrize("kw,msg", [
    (dict(R=0.0), "on-resistance"),
    (dict(L=-1.0), "half-width"),
    (dict(C=np.inf), "offset"),
    (dict(meas=(5, -1)), "out of range"),
])
def test_refused(kw, msg):
    with pytest.raises(_lib.EMTError, match=msg):
        _lib.analyze([net_with(**kw)], 20e-6, 100)


def test_missing_meas_refused():
    n = net_with()
    n.meas = None
    with pytest.raises(_lib.EMTError, match="meas"):
        _lib.analyze([n], 20e-6, 100)


def test_forward_only_and_no_events():
    with pytest.raises(_lib.EMTError, match="forward only"):
        _lib.analyze([net_with()], 20e-6, 100, checkpoint_every=10)
    n = net_with()
    n.ev_step, n.ev_branch, n.ev_in_service = np.array([5]), np.array([1], np.int32), np.array([0], np.uint8)
    with pytest.raises(_lib.EMTError, match="controller"):
        _lib.analyze([n], 20e-6, 100)
