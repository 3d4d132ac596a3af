"""ctypes binding of the C++ oracle (oracle.cpp). Test infrastructure only.

Networks are read by attribute (n_nodes, k, m, kind, R, L, C, E, omega,
phase, line, n_lines, in_service0, ev_step, ev_branch, ev_in_service,
rec_nodes), so any object with that shape works; this module imports nothing
from the GPU package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (plain -O2, OpenMP over scenarios)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-march=x86-64-v2", "-std=c++17", "-fopenmp",
                               "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Net(C.Structure):
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


_lib = None
_native = False


def use_native_build() -> str:
    """For timing the oracle on the machine it runs on: compile the same
    source with -O3 -march=native into liboracle_native.so and route every
    later call of this process through it. The compiler may fuse
    multiply-adds there, so results can differ from the test build in the
    last bits: timing only. Must come before the first oracle call (a
    second call once the native build is loaded does nothing)."""
    global _lib, _native
    path = os.path.join(_HERE, "liboracle_native.so")
    if _lib is not None:
        if _native:
            return path
        raise RuntimeError("use_native_build() must come before the first oracle call")
    tmp = path + ".tmp"
    subprocess.check_call(["g++", "-O3", "-march=native", "-std=c++17", "-fopenmp",
                           "-shared", "-fPIC", "-o", tmp, _SRC])
    os.replace(tmp, path)
    _load(path)
    _native = True
    return path


def _load(path=None):
    global _lib
    if _lib is None:
        if path is None:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        lib = C.CDLL(path)
        vp, i64, f64, i32 = C.c_void_p, C.c_int64, C.c_double, C.c_int32
        lib.oracle_run.argtypes = [vp, vp, f64, i64, vp, vp, vp, vp, vp, vp]
        lib.oracle_loss_complex.argtypes = [vp, vp, vp, f64, i64, vp, vp, vp]
        lib.oracle_adjoint.argtypes = [vp, vp, f64, i64, vp, vp, vp, vp, vp]
        lib.oracle_run_batch.argtypes = [vp, i32, vp, f64, i64, vp, i32]
        lib.oracle_assemble.argtypes = [vp, vp, f64, vp, vp]
        lib.oracle_companions.argtypes = [vp, vp, f64, vp, vp, vp, vp]
        lib.oracle_lu_solve.argtypes = [i32, vp, vp, vp, i32]
        lib.oracle_steady_state.argtypes = [vp, vp, f64, vp, vp, vp, vp]
        for f in ("oracle_run", "oracle_loss_complex", "oracle_adjoint", "oracle_run_batch",
                  "oracle_assemble", "oracle_companions", "oracle_lu_solve",
                  "oracle_max_threads", "oracle_steady_state"):
            getattr(lib, f).restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class _Packed:
    """Holds contiguous copies of a network's arrays plus the C struct."""

    def __init__(self, net):
        n_ev = int(len(net.ev_step))
        self.arrs = dict(
            k=np.ascontiguousarray(net.k, np.int32), m=np.ascontiguousarray(net.m, np.int32),
            kind=np.ascontiguousarray(net.kind, np.int32),
            R=np.ascontiguousarray(net.R, np.float64), L=np.ascontiguousarray(net.L, np.float64),
            C=np.ascontiguousarray(net.C, np.float64), E=np.ascontiguousarray(net.E, np.float64),
            omega=np.ascontiguousarray(net.omega, np.float64),
            phase=np.ascontiguousarray(net.phase, np.float64),
            line=np.ascontiguousarray(net.line, np.int32),
            ins=np.ascontiguousarray(net.in_service0, np.uint8),
            ev_step=np.ascontiguousarray(net.ev_step, np.int64).reshape(n_ev),
            ev_branch=np.ascontiguousarray(net.ev_branch, np.int32).reshape(n_ev),
            ev_ins=np.ascontiguousarray(net.ev_in_service, np.uint8).reshape(n_ev),
            rec=None if net.rec_nodes is None else np.ascontiguousarray(net.rec_nodes, np.int32),
        )
        grp = getattr(net, "group", None)
        for f, dt_ in (("group", np.int32), ("Rm", np.float64), ("Lm", np.float64), ("Cm", np.float64)):
            self.arrs[f] = None if grp is None else np.ascontiguousarray(getattr(net, f), dt_)
        meas = getattr(net, "meas", None)
        self.arrs["meas"] = None if meas is None else np.ascontiguousarray(meas, np.int32).reshape(-1)
        a = self.arrs
        self.n_rec = net.n_nodes if a["rec"] is None else int(a["rec"].shape[0])
        self.n_params = 3 * int(net.n_lines)
        self.n_nodes = int(net.n_nodes)
        self.n_branches = int(a["k"].shape[0])
        self.s = _Net(self.n_nodes, self.n_branches, _ptr(a["k"]), _ptr(a["m"]),
                      _ptr(a["kind"]), _ptr(a["R"]), _ptr(a["L"]), _ptr(a["C"]), _ptr(a["E"]),
                      _ptr(a["omega"]), _ptr(a["phase"]), _ptr(a["line"]), self.n_params,
                      _ptr(a["ins"]), n_ev, _ptr(a["ev_step"]), _ptr(a["ev_branch"]),
                      _ptr(a["ev_ins"]), self.n_rec, _ptr(a["rec"]), _ptr(a["group"]), _ptr(a["Rm"]),
                      _ptr(a["Lm"]), _ptr(a["Cm"]), _ptr(a["meas"]))

    @property
    def ref(self):
        return C.addressof(self.s)


def _check(st, what):
    if st == 1:
        raise ValueError(f"{what}: invalid network or arguments")
    if st == 2:
        raise np.linalg.LinAlgError(f"{what}: singular conductance matrix")
    if st != 0:
        raise RuntimeError(f"{what}: status {st}")


def _theta(theta, n_params):
    if theta is None:
        return None
    th = np.ascontiguousarray(theta, np.float64)
    if th.shape != (n_params,):
        raise ValueError("theta must have shape (3 * n_lines,)")
    return th


def run(net, dt: float, n_steps: int, theta=None, v0=None, i0=None, trajectories=False):
    """Forward run. Returns rec [T][n_rec]; with trajectories=True also
    (v [T+1][N], i [T+1][B], u [T+1][B])."""
    lib = _load()
    P = _Packed(net)
    th = _theta(theta, P.n_params)
    T = int(n_steps)
    rec = np.empty((T, P.n_rec))
    v0a = None if v0 is None else np.ascontiguousarray(v0, np.float64)
    i0a = None if i0 is None else np.ascontiguousarray(i0, np.float64)
    vt = it = ut = None
    if trajectories:
        vt = np.empty((T + 1, P.n_nodes))
        it = np.empty((T + 1, P.n_branches))
        ut = np.empty((T + 1, P.n_branches))
    st = lib.oracle_run(P.ref, _ptr(th), float(dt), T, _ptr(v0a), _ptr(i0a), _ptr(rec),
                        _ptr(vt), _ptr(it), _ptr(ut))
    _check(st, "oracle_run")
    return (rec, vt, it, ut) if trajectories else rec


def steady_state(net, dt: float, theta=None):
    """Sinusoidal steady state of the initial topology under the sources'
    common frequency (the trapezoidal recursion's own periodic solution).
    Returns (v0 [N], i0 [B], V [N] complex node phasors): run(net, dt, T,
    v0=v0, i0=i0) then gives v_n = Re(V exp(j w n dt)) until the first
    event."""
    lib = _load()
    P = _Packed(net)
    th = _theta(theta, P.n_params)
    v0 = np.empty(P.n_nodes)
    i0 = np.empty(P.n_branches)
    vr = np.empty(P.n_nodes)
    vi = np.empty(P.n_nodes)
    st = lib.oracle_steady_state(P.ref, _ptr(th), float(dt), _ptr(v0), _ptr(i0), _ptr(vr), _ptr(vi))
    _check(st, "oracle_steady_state")
    return v0, i0, vr + 1j * vi


def run_batch(nets, dt: float, n_steps: int, thetas=None, n_threads: int = 0):
    """Independent forward runs, OpenMP over scenarios. Returns a list of rec."""
    lib = _load()
    packs = [_Packed(n) for n in nets]
    arr = (_Net * len(packs))(*[p.s for p in packs])
    T = int(n_steps)
    recs = [np.empty((T, p.n_rec)) for p in packs]
    rec_ptrs = (C.c_void_p * len(packs))(*[r.ctypes.data for r in recs])
    th_keep = None
    th_ptrs = None
    if thetas is not None:
        th_keep = [_theta(t, p.n_params) for t, p in zip(thetas, packs)]
        th_ptrs = (C.c_void_p * len(packs))(*[_ptr(t) for t in th_keep])
    st = lib.oracle_run_batch(C.addressof(arr), len(packs),
                              None if th_ptrs is None else C.addressof(th_ptrs), float(dt), T,
                              C.addressof(rec_ptrs), int(n_threads))
    _check(st, "oracle_run_batch")
    return recs


def adjoint(net, dt: float, n_steps: int, dJ_drec, theta=None, branch_adjoints=False):
    """dJ/dtheta for a cotangent dJ/drec [T][n_rec]. With branch_adjoints,
    also returns (gbar, betabar, gammabar) per branch."""
    lib = _load()
    P = _Packed(net)
    th = _theta(theta, P.n_params)
    T = int(n_steps)
    d = np.ascontiguousarray(dJ_drec, np.float64)
    if d.shape != (T, P.n_rec):
        raise ValueError("dJ_drec must have shape (T, n_rec)")
    grad = np.empty(P.n_params)
    gb = np.empty(P.n_branches)
    bb = np.empty(P.n_branches)
    cb = np.empty(P.n_branches)
    st = lib.oracle_adjoint(P.ref, _ptr(th), float(dt), T, _ptr(d), _ptr(grad), _ptr(gb),
                            _ptr(bb), _ptr(cb))
    _check(st, "oracle_adjoint")
    return (grad, gb, bb, cb) if branch_adjoints else grad


def loss_complex(net, dt: float, n_steps: int, theta_re, theta_im, target):
    """J(theta_re + i theta_im) = sum (v - target)^2 in complex arithmetic."""
    lib = _load()
    P = _Packed(net)
    T = int(n_steps)
    tr = _theta(theta_re, P.n_params)
    ti = _theta(theta_im, P.n_params)
    tg = np.ascontiguousarray(target, np.float64)
    if tg.shape != (T, P.n_rec):
        raise ValueError("target must have shape (T, n_rec)")
    jr, ji = C.c_double(), C.c_double()
    st = lib.oracle_loss_complex(P.ref, _ptr(tr), _ptr(ti), float(dt), T, _ptr(tg),
                                 C.addressof(jr), C.addressof(ji))
    _check(st, "oracle_loss_complex")
    return complex(jr.value, ji.value)


def assemble(net, dt: float, in_service, theta=None):
    lib = _load()
    P = _Packed(net)
    ins = np.ascontiguousarray(in_service, np.uint8)
    G = np.empty((P.n_nodes, P.n_nodes))
    lib.oracle_assemble(P.ref, _ptr(_theta(theta, P.n_params)), float(dt), _ptr(ins), _ptr(G))
    return G


def companions(net, dt: float, in_service, theta=None):
    lib = _load()
    P = _Packed(net)
    ins = np.ascontiguousarray(in_service, np.uint8)
    g, b, c = (np.empty(P.n_branches) for _ in range(3))
    lib.oracle_companions(P.ref, _ptr(_theta(theta, P.n_params)), float(dt), _ptr(ins),
                          _ptr(g), _ptr(b), _ptr(c))
    return g, b, c


def lu_solve(G, b, transposed=False):
    lib = _load()
    G = np.ascontiguousarray(G, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    x = np.empty_like(b)
    st = lib.oracle_lu_solve(int(b.shape[0]), _ptr(G), _ptr(b), _ptr(x), int(bool(transposed)))
    _check(st, "oracle_lu_solve")
    return x


def max_threads() -> int:
    return int(_load().oracle_max_threads())
