"""ctypes binding of libemt.so (include/emt.h). Argument marshalling only.

The HIP library is required: importing this module raises if libemt.so has
not been built (``python -m paper_1903_01081_amd.build``). There is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libemt.so")

EMT_OK, EMT_EINVAL, EMT_ESINGULAR, EMT_ENOMEM, EMT_EDEVICE, EMT_ESTATE = range(6)
STATUS_NAMES = {0: "EMT_OK", 1: "EMT_EINVAL", 2: "EMT_ESINGULAR", 3: "EMT_ENOMEM",
                4: "EMT_EDEVICE", 5: "EMT_ESTATE"}

# Exported functions of include/emt.h.
EXPORTS = ("emt_build", "emt_analyze", "emt_info_get", "emt_set_params", "emt_factor", "emt_factor_async",
           "emt_mismatch",
           "emt_step", "emt_step_noalloc", "emt_sync", "emt_reset", "emt_steady_state", "emt_adjoint",
           "emt_branch_adjoints", "emt_get_state",
           "emt_set_state", "emt_latency_floor", "emt_destroy", "emt_last_error")

# emt_floor_kernel
FLOOR_KERNELS = {"one_workgroup": 0, "split": 1}


class EMTError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class EmtNet(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int32), ("n_branches", C.c_int32),
        ("k", C.c_void_p), ("m", C.c_void_p), ("kind", C.c_void_p),
        ("R", C.c_void_p), ("L", C.c_void_p), ("C", C.c_void_p),
        ("E", C.c_void_p), ("omega", C.c_void_p), ("phase", C.c_void_p),
        ("line", C.c_void_p), ("n_params", C.c_int32),
        ("in_service0", C.c_void_p),
        ("n_events", C.c_int32), ("ev_step", C.c_void_p), ("ev_branch", C.c_void_p),
        ("ev_in_service", C.c_void_p),
        ("n_rec", C.c_int32), ("rec_nodes", C.c_void_p),
        ("group", C.c_void_p), ("Rm", C.c_void_p), ("Lm", C.c_void_p), ("Cm", C.c_void_p),
        ("meas", C.c_void_p),
    ]


class EmtSim(C.Structure):
    _fields_ = [("dt", C.c_double), ("n_steps", C.c_int64),
                ("checkpoint_every", C.c_int32), ("solver", C.c_int32),
                ("block_size", C.c_int32), ("split_cols", C.c_int32),
                ("dense_tail", C.c_int32), ("sweep_from_global", C.c_int32),
                ("serial_adjoint", C.c_int32), ("split_device_scope", C.c_int32),
                ("pack_nodes", C.c_int32), ("comp_items", C.c_int32)]


class EmtInfo(C.Structure):
    _fields_ = [
        ("n_scen", C.c_int32), ("rec_stride", C.c_int32), ("param_stride", C.c_int32),
        ("n_items", C.c_int32), ("n_symbolic", C.c_int32),
        ("max_item_nodes", C.c_int32), ("max_item_branches", C.c_int32),
        ("total_nodes", C.c_int64), ("total_branches", C.c_int64), ("nnz_L", C.c_int64),
        ("max_levels", C.c_int32), ("max_topologies", C.c_int32),
        ("step", C.c_int64), ("device_bytes", C.c_int64),
        ("dense_items", C.c_int32), ("block_size", C.c_int32),
        ("sweep_levels", C.c_int32), ("max_tail", C.c_int32), ("lds_bytes", C.c_int32),
        ("lds_limit", C.c_int32), ("lds_staged", C.c_int32), ("lanes_per_block", C.c_int32),
        ("split_tiles", C.c_int32), ("split_cols", C.c_int32), ("adjoint_pipelined", C.c_int32),
        ("split_local", C.c_int32),
        ("comp_families", C.c_int32), ("comp_max_rank", C.c_int32), ("comp_items", C.c_int32),
        ("comp_blocks", C.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load():
    """Loads libemt.so; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1903_01081_amd.build` (needs hipcc)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    sigs = {
        "emt_build": [vp, i32, vp, vp],
        "emt_analyze": [vp, i32, vp, vp],
        "emt_info_get": [vp, vp],
        "emt_set_params": [vp, vp, vp],
        "emt_factor": [vp, vp],
        "emt_factor_async": [vp, vp],
        "emt_mismatch": [vp, vp, vp, vp, vp, vp],
        "emt_step": [vp, i64, vp, vp],
        "emt_sync": [vp, vp],
        "emt_steady_state": [vp, vp],
        "emt_step_noalloc": [vp, i64, vp, vp],
        "emt_reset": [vp, vp],
        "emt_adjoint": [vp, vp, vp, vp],
        "emt_branch_adjoints": [vp, i32, vp, vp, vp],
        "emt_get_state": [vp, i32, vp, vp],
        "emt_set_state": [vp, i32, vp, vp],
        "emt_latency_floor": [vp, i32, i64, vp, vp],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.emt_destroy.argtypes = [vp]
    lib.emt_destroy.restype = None
    lib.emt_last_error.argtypes = []
    lib.emt_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def check(status: int):
    if status != EMT_OK:
        msg = load().emt_last_error().decode(errors="replace")
        raise EMTError(status, msg)


def _ptr(a):
    return None if a is None else a.ctypes.data


class PackedNets:
    """Contiguous copies of networks' arrays and the emt_net array pointing at
    them (alive as long as this object)."""

    def __init__(self, nets):
        self.keep = []
        structs = []
        for net in nets:
            n_ev = int(len(net.ev_step))
            a = dict(
                k=np.ascontiguousarray(net.k, np.int32), m=np.ascontiguousarray(net.m, np.int32),
                kind=np.ascontiguousarray(net.kind, np.int32),
                R=np.ascontiguousarray(net.R, np.float64), L=np.ascontiguousarray(net.L, np.float64),
                C=np.ascontiguousarray(net.C, np.float64), E=np.ascontiguousarray(net.E, np.float64),
                omega=np.ascontiguousarray(net.omega, np.float64),
                phase=np.ascontiguousarray(net.phase, np.float64),
                line=np.ascontiguousarray(net.line, np.int32),
                ins=None if net.in_service0 is None else np.ascontiguousarray(net.in_service0, np.uint8),
                ev_step=np.ascontiguousarray(net.ev_step, np.int64).reshape(n_ev),
                ev_branch=np.ascontiguousarray(net.ev_branch, np.int32).reshape(n_ev),
                ev_ins=np.ascontiguousarray(net.ev_in_service, np.uint8).reshape(n_ev),
                rec=None if net.rec_nodes is None else np.ascontiguousarray(net.rec_nodes, np.int32),
            )
            grp = getattr(net, "group", None)
            for f, t in (("group", np.int32), ("Rm", np.float64), ("Lm", np.float64), ("Cm", np.float64)):
                a[f] = None if grp is None else np.ascontiguousarray(getattr(net, f), t)
            meas = getattr(net, "meas", None)
            a["meas"] = None if meas is None else np.ascontiguousarray(meas, np.int32).reshape(-1)
            self.keep.append(a)
            n_rec = int(net.n_nodes) if a["rec"] is None else int(a["rec"].shape[0])
            structs.append(EmtNet(
                int(net.n_nodes), int(a["k"].shape[0]), _ptr(a["k"]), _ptr(a["m"]), _ptr(a["kind"]),
                _ptr(a["R"]), _ptr(a["L"]), _ptr(a["C"]), _ptr(a["E"]), _ptr(a["omega"]),
                _ptr(a["phase"]), _ptr(a["line"]), 3 * int(net.n_lines), _ptr(a["ins"]), n_ev,
                _ptr(a["ev_step"]), _ptr(a["ev_branch"]), _ptr(a["ev_ins"]), n_rec, _ptr(a["rec"]),
                _ptr(a["group"]), _ptr(a["Rm"]), _ptr(a["Lm"]), _ptr(a["Cm"]), _ptr(a["meas"])))
        self.array = (EmtNet * len(structs))(*structs)
        self.n = len(structs)

    @property
    def ref(self):
        return C.addressof(self.array)


def make_sim(dt, n_steps, checkpoint_every=0, solver=0, block_size=0, split_cols=0, dense_tail=-1,
             sweep_from_global=0, serial_adjoint=0, split_device_scope=0, pack_nodes=0,
             comp_items=0) -> EmtSim:
    return EmtSim(float(dt), int(n_steps), int(checkpoint_every), int(solver), int(block_size),
                  int(split_cols), int(dense_tail), int(sweep_from_global), int(serial_adjoint),
                  int(split_device_scope), int(pack_nodes), int(comp_items))


def analyze(nets, dt, n_steps, checkpoint_every=0, solver=0, pack_nodes=0) -> dict:
    """Host-only validation and analysis (no device needed)."""
    lib = load()
    P = PackedNets(nets)
    sim = make_sim(dt, n_steps, checkpoint_every, solver, pack_nodes=pack_nodes)
    info = EmtInfo()
    check(lib.emt_analyze(P.ref, P.n, C.addressof(sim), C.addressof(info)))
    return info.as_dict()
