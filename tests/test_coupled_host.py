"""Host-side analysis of coupled three-phase groups (no GPU): the phases a
group couples form one component, with the mutual entries in its factor
pattern; malformed groups are refused."""
import copy

import numpy as np
import pytest

from paper_1903_01081_amd import _lib, netgen


def test_coupled_phases_form_one_component():
    plain = netgen.small_grid(7, 12)
    coupled = netgen.small_grid(7, 12, coupled=True)
    a = _lib.analyze([plain], 50e-6, 10)
    b = _lib.analyze([coupled], 50e-6, 10)
    assert a["n_items"] == 3 and b["n_items"] == 1
    assert b["total_nodes"] == a["total_nodes"] and b["total_branches"] == a["total_branches"]
    # the mutual couplings add off-diagonal entries between phases
    assert b["nnz_L"] > a["nnz_L"]


def _broken(what):
    net = netgen.small_grid(7, 8, coupled=True)
    n = copy.deepcopy(net)
    n.group, n.Rm, n.Lm, n.Cm = net.group.copy(), net.Rm.copy(), net.Lm.copy(), net.Cm.copy()
    if what == "pair":
        n.group[2] = -1
    elif what == "unequal":
        n.Lm[1] *= 1.01
    elif what == "indefinite":
        n.Lm[:3] = -0.6 * n.L[:3]  # zero-sequence L + 2 Lm < 0
    elif what == "mixed":
        n.kind[0] = netgen.CAP
        n.C[0] = 1e-6
    return n


@pytest.mark.parametrize("what,match", [("pair", "exactly three"), ("unequal", "equal R, L"),
                                        ("indefinite", "positive definite"), ("mixed", "three R-L or three C")])
def test_malformed_groups_refused(what, match):
    with pytest.raises(Exception, match=match):
        _lib.analyze([_broken(what)], 50e-6, 10)


def test_coupled_forward_only():
    net = netgen.small_grid(7, 8, coupled=True)
    with pytest.raises(Exception, match="forward only"):
        _lib.analyze([net], 50e-6, 10, checkpoint_every=5)
