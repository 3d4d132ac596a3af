"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/emt.h, and the host-side validation and analysis behave
(error codes, singular detection, shared symbolic analysis)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1903_01081_amd import netgen
from paper_1903_01081_amd.netgen import CAP, RL, SRC

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1903_01081_amd import _lib
    return _lib


def header_functions():
    text = open(os.path.join(ROOT, "include", "emt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(emt_[a-z_]+)\s*\(", text)))


def test_header_lists_the_boundary():
    names = header_functions()
    for required in ("emt_build", "emt_factor", "emt_step", "emt_adjoint", "emt_set_params",
                     "emt_get_state", "emt_set_state", "emt_destroy", "emt_last_error"):
        assert required in names


def test_library_exports_every_header_symbol(lib):
    so = lib.load()
    for name in header_functions():
        assert hasattr(so, name), name
    assert set(lib.EXPORTS) == set(header_functions())


def test_every_declaration_names_its_source():
    """Each function of the boundary carries, in the comment just above it,
    the passage of the paper it follows ("Source: Sec. ...") or says that it
    is not in the paper."""
    text = open(os.path.join(ROOT, "include", "emt.h")).read()
    body = text[text.index("#ifdef __cplusplus"):]
    for name in header_functions():
        m = re.search(r"/\*((?:(?!\*/).)*)\*/\s*(?:typedef[^;]*;\s*)?(?:#define[^\n]*\n\s*)?[a-z_ *]+\b" + name + r"\s*\(", body, flags=re.S)
        assert m is not None, f"{name} has no comment"
        comment = m.group(1)
        assert re.search(r"Source: Sec\. [IV]+", comment) or "Not in the paper" in comment, name


def test_destroy_null_is_safe(lib):
    lib.load().emt_destroy(None)


def _status(lib, nets, dt=50e-6, T=10, K=0):
    try:
        lib.analyze(nets, dt, T, K)
        return lib.EMT_OK
    except lib.EMTError as e:
        return e.status


def test_invalid_inputs(lib):
    good = netgen.small_grid(1, 4, fault_step=5)
    assert _status(lib, [good]) == lib.EMT_OK
    assert _status(lib, [good], dt=0.0) == lib.EMT_EINVAL
    assert _status(lib, [good], dt=float("nan")) == lib.EMT_EINVAL
    assert _status(lib, [good], T=0) == lib.EMT_EINVAL
    assert _status(lib, [good], K=-1) == lib.EMT_EINVAL

    def mutate(**kw):
        d = dict(good.__dict__)
        for key, fn in kw.items():
            d[key] = fn(np.array(d[key], copy=True))
        return netgen.Network(**d)

    def at(arr, idx, val):
        arr[idx] = val
        return arr

    b_rl = int(np.where(good.kind == RL)[0][0])
    b_c = int(np.where(good.kind == CAP)[0][0])
    assert _status(lib, [mutate(k=lambda a: at(a, 0, good.n_nodes))]) == lib.EMT_EINVAL
    assert _status(lib, [mutate(m=lambda a: at(a, b_c, int(good.k[b_c])))]) == lib.EMT_EINVAL
    assert _status(lib, [mutate(L=lambda a: at(a, b_rl, 0.0))]) == lib.EMT_EINVAL
    assert _status(lib, [mutate(R=lambda a: at(a, b_rl, -1.0))]) == lib.EMT_EINVAL
    assert _status(lib, [mutate(C=lambda a: at(a, b_c, float("nan")))]) == lib.EMT_EINVAL
    assert _status(lib, [mutate(kind=lambda a: at(a, 0, 9))]) == lib.EMT_EINVAL
    assert _status(lib, [mutate(ev_step=lambda a: at(a, 0, 0))]) == lib.EMT_EINVAL
    assert _status(lib, [mutate(ev_branch=lambda a: at(a, 0, 10**6))]) == lib.EMT_EINVAL
    assert _status(lib, [mutate(line=lambda a: at(a, b_rl, 10**6))]) == lib.EMT_EINVAL
    bad_rec = netgen.Network(**{**good.__dict__, "rec_nodes": np.array([0, good.n_nodes], np.int32)})
    assert _status(lib, [bad_rec]) == lib.EMT_EINVAL
    # a bad scenario anywhere in a batch rejects the batch
    assert _status(lib, [good, mutate(L=lambda a: at(a, b_rl, -2.0))]) == lib.EMT_EINVAL


def test_singular_island_detected(lib):
    net = netgen.circuit(3, [dict(k=0, m=-1, kind=CAP, C=1e-6),
                             dict(k=1, m=2, kind=RL, R=1.0, L=1e-3)])
    assert _status(lib, [net]) == lib.EMT_ESINGULAR
    # a node that is grounded only through a switch that opens later
    net2 = netgen.circuit(2, [
        dict(k=0, m=-1, kind=CAP, C=1e-6),
        dict(k=1, m=-1, kind=3, R=1.0, ins=1),
    ], events=[(5, 1, 0)])
    assert _status(lib, [net2], T=4) == lib.EMT_OK        # event beyond the horizon
    assert _status(lib, [net2], T=10) == lib.EMT_ESINGULAR
    msg = lib.load().emt_last_error().decode()
    assert "ground" in msg


def test_analysis_shapes(lib):
    nets, sim = netgen.config0()
    info = lib.analyze(nets, sim["dt"], sim["n_steps"])
    assert info["n_items"] == 3                      # uncoupled phases
    assert info["max_item_nodes"] == 9
    assert info["rec_stride"] == 27
    assert info["param_stride"] == 27
    assert info["max_topologies"] == 2
    assert info["total_branches"] == nets[0].n_branches


def test_isomorphic_scenarios_share_symbolic(lib):
    nets, sim = netgen.config2(n_bus=20, n_scen=12, n_steps=100, event_step=50)
    info = lib.analyze(nets, sim["dt"], sim["n_steps"])
    assert info["n_items"] == 36
    assert info["n_symbolic"] == 3                   # one per phase, shared by all scenarios
    nets4, sim4 = netgen.config4(n_inst=4, n_steps=100)
    info4 = lib.analyze(nets4, sim4["dt"], sim4["n_steps"])
    assert info4["n_symbolic"] == 12                 # uneven networks share nothing


def test_levels_bound_and_fill(lib):
    # a path graph (radial feeder) ordered by minimum degree has no fill and
    # logarithmic-ish depth; a tree can never need more levels than nodes
    n = 64
    br = [dict(k=i, m=i + 1, kind=RL, R=0.1, L=1e-3) for i in range(n - 1)]
    br += [dict(k=i, m=-1, kind=CAP, C=1e-6) for i in range(n)]
    br += [dict(k=0, m=-1, kind=SRC, R=0.5, L=1e-2, E=1.0, omega=377.0)]
    info = lib.analyze([netgen.circuit(n, br)], 50e-6, 10)
    assert info["nnz_L"] == n - 1
    assert info["max_levels"] <= n


def _analyze_sim(lib, nets, **fields):
    so = lib.load()
    P = lib.PackedNets(nets)
    sim = lib.make_sim(50e-6, 10, **fields)
    info = lib.EmtInfo()
    return so.emt_analyze(P.ref, P.n, C.addressof(sim), C.addressof(info)), info


def test_empty_batch_and_null_arguments(lib):
    so = lib.load()
    sim = lib.make_sim(50e-6, 10)
    info = lib.EmtInfo()
    assert so.emt_analyze(None, 0, C.addressof(sim), C.addressof(info)) == lib.EMT_EINVAL
    good = lib.PackedNets([netgen.small_grid(2, 4)])
    assert so.emt_analyze(good.ref, good.n, None, C.addressof(info)) == lib.EMT_EINVAL
    assert so.emt_analyze(good.ref, good.n, C.addressof(sim), None) == lib.EMT_EINVAL
    assert so.emt_last_error()  # a message for the last failure


def test_launch_shape_fields_validated(lib):
    net = netgen.small_grid(3, 5)
    assert _analyze_sim(lib, [net])[0] == lib.EMT_OK
    for bad in (dict(block_size=128), dict(block_size=-1), dict(split_cols=8), dict(dense_tail=-2),
                dict(sweep_from_global=2), dict(serial_adjoint=-1), dict(split_device_scope=2),
                dict(solver=7)):
        st, _ = _analyze_sim(lib, [net], **bad)
        assert st == lib.EMT_EINVAL, bad


def test_network_without_branches_is_singular(lib):
    # nodes with no branch at all have no path to ground
    net = netgen.circuit(2, [dict(k=0, m=-1, kind=CAP, C=1e-6)])
    assert _status(lib, [net]) == lib.EMT_ESINGULAR


def test_one_node_and_empty_recording_analyse(lib):
    net = netgen.circuit(1, [dict(k=0, m=-1, kind=SRC, R=0.5, L=1e-2, E=1.0, omega=377.0),
                             dict(k=0, m=-1, kind=CAP, C=1e-6)], rec_nodes=[])
    info = lib.analyze([net], 50e-6, 10)
    assert info["n_items"] == 1 and info["max_item_nodes"] == 1 and info["rec_stride"] == 0
