"""Python front end of the EMT library: a Simulator over libemt.so.

Torch tensors only carry device memory and the current stream; every step of
the time loop runs in the HIP kernels behind include/emt.h.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import EMTError, check

SOLVERS = {"auto": 0, "dense": 1, "sparse": 2, "compensation": 3}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t: torch.Tensor, shape, name: str):
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


class Simulator:
    """A batch of networks (scenarios) stepped together on the current HIP device.

    rec layout: [S, n, R] with R = max n_rec; theta / grad layout: [S, P] with
    P = max n_params (3 per line: R_l, L_l, C_l).
    """

    def __init__(self, nets: Sequence, dt: float, n_steps: int, checkpoint_every: int = 0,
                 solver: str = "auto", device: Optional[torch.device] = None, block_size: int = 0,
                 split_cols: int = 0, dense_tail: int = -1, sweep_from_global: bool = False,
                 serial_adjoint: bool = False, split_device_scope: bool = False, pack_nodes: int = 0,
                 comp_items: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("the EMT library needs a HIP device")
        self.lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.nets = list(nets)
        self.dt = float(dt)
        self.n_steps = int(n_steps)
        self.checkpoint_every = int(checkpoint_every)
        packed = _lib.PackedNets(self.nets)
        self.shape = dict(solver=solver, block_size=int(block_size), split_cols=int(split_cols),
                          dense_tail=int(dense_tail), sweep_from_global=bool(sweep_from_global),
                          serial_adjoint=bool(serial_adjoint), split_device_scope=bool(split_device_scope),
                          pack_nodes=int(pack_nodes), comp_items=int(comp_items))
        sim = _lib.make_sim(dt, n_steps, checkpoint_every, SOLVERS[solver], block_size, split_cols, dense_tail,
                            int(bool(sweep_from_global)), int(bool(serial_adjoint)),
                            int(bool(split_device_scope)), int(pack_nodes), int(comp_items))
        self._ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            check(self.lib.emt_build(packed.ref, packed.n, C.addressof(sim), C.byref(self._ctx)))
        info = self.info()
        self.S = info["n_scen"]
        self.R = info["rec_stride"]
        self.P = info["param_stride"]
        self.n_nodes = [int(n.n_nodes) for n in self.nets]
        self.n_branches = [int(n.n_branches) for n in self.nets]

    # -- lifecycle --------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self.lib.emt_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = _lib.EmtInfo()
        check(self.lib.emt_info_get(self._ctx, C.addressof(inf)))
        return inf.as_dict()

    @property
    def step_index(self) -> int:
        return int(self.info()["step"])

    # -- the loop ---------------------------------------------------------
    def set_params(self, theta: torch.Tensor):
        """theta: [S, P] float64 device tensor of line parameters."""
        check(self.lib.emt_set_params(self._ctx, _dev_ptr(theta, (self.S, self.P), "theta"), _stream()))

    def factor(self):
        check(self.lib.emt_factor(self._ctx, _stream()))

    def factor_async(self):
        """emt_factor without waiting: pivots are checked by sync()."""
        check(self.lib.emt_factor_async(self._ctx, _stream()))

    def reset(self):
        check(self.lib.emt_reset(self._ctx, _stream()))

    def steady_state(self):
        """Every scenario back to step 0 in the sinusoidal steady state of its
        initial topology (emt_steady_state); forward only afterwards."""
        check(self.lib.emt_steady_state(self._ctx, _stream()))

    def mismatch(self, rec: torch.Tensor, target: torch.Tensor, dJ: torch.Tensor, loss: torch.Tensor):
        """dJ = 2 (rec - target) on the recorded columns, loss[s] = sum of
        squares (emt_mismatch); all device tensors, queued."""
        T = self.n_steps
        check(self.lib.emt_mismatch(self._ctx, _dev_ptr(rec, (self.S, T, self.R), "rec"),
                                    _dev_ptr(target, (self.S, T, self.R), "target"),
                                    _dev_ptr(dJ, (self.S, T, self.R), "dJ"),
                                    _dev_ptr(loss, (self.S,), "loss"), _stream()))

    def latency_floor(self, kernel: str, n_steps: int) -> float:
        """Microseconds per step of the no-arithmetic floor of a step kernel
        ("one_workgroup" or "split"), same launch shape; state untouched."""
        us = C.c_double(0.0)
        check(self.lib.emt_latency_floor(self._ctx, _lib.FLOOR_KERNELS[kernel], int(n_steps), C.byref(us),
                                         _stream()))
        return us.value

    def sync(self):
        """Wait for the queued work of this run and raise EMTError if the
        device reported a failure (a split launch that gave up)."""
        check(self.lib.emt_sync(self._ctx, _stream()))

    def step(self, n: int, rec: Optional[torch.Tensor] = None, record: bool = True):
        """Advance n steps; returns rec [S, n, R] (allocated if not given).
        Queues the work and returns; sync() waits and reports device errors."""
        if record and rec is None:
            rec = torch.zeros((self.S, n, self.R), dtype=torch.float64, device=self.device)
        ptr = _dev_ptr(rec, (self.S, n, self.R), "rec") if record else None
        check(self.lib.emt_step(self._ctx, int(n), ptr, _stream()))
        return rec

    def run(self, record: bool = True):
        """factor (if needed by the caller) then all n_steps from step 0."""
        return self.step(self.n_steps, record=record)

    def adjoint(self, dJ_drec: torch.Tensor, grad: Optional[torch.Tensor] = None) -> torch.Tensor:
        """dJ/dtheta [S, P] for a cotangent dJ/drec [S, T, R]."""
        if grad is None:
            grad = torch.empty((self.S, self.P), dtype=torch.float64, device=self.device)
        d = _dev_ptr(dJ_drec, (self.S, self.n_steps, self.R), "dJ_drec")
        g = _dev_ptr(grad, (self.S, self.P), "grad")
        check(self.lib.emt_adjoint(self._ctx, d, g, _stream()))
        return grad

    def branch_adjoints(self, scen: int):
        nb = self.n_branches[scen]
        out = [np.empty(nb) for _ in range(3)]
        check(self.lib.emt_branch_adjoints(self._ctx, int(scen), *[o.ctypes.data for o in out]))
        return tuple(out)

    # -- state ------------------------------------------------------------
    def get_state(self, scen: int):
        v = np.empty(self.n_nodes[scen])
        i = np.empty(self.n_branches[scen])
        check(self.lib.emt_get_state(self._ctx, int(scen), v.ctypes.data, i.ctypes.data))
        return v, i

    def set_state(self, scen: int, v, i):
        v = np.ascontiguousarray(v, np.float64)
        i = np.ascontiguousarray(i, np.float64)
        if v.shape != (self.n_nodes[scen],) or i.shape != (self.n_branches[scen],):
            raise ValueError("state shapes do not match the scenario")
        check(self.lib.emt_set_state(self._ctx, int(scen), v.ctypes.data, i.ctypes.data))


class IdentificationGraph:
    """One parameter-identification iteration of a batch recorded into a HIP
    graph: set the line parameters, factorise (pivots checked at sync()),
    run forward over the horizon, form the waveform mismatch against the
    target and run the adjoint. replay() launches the whole iteration as one
    graph; `theta` (input), `loss` [S] and `grad` [S, P] are fixed device
    tensors the caller writes and reads between replays.

    Every call in the iteration only queues kernels (no host wait, no
    allocation, no memset nodes), which is what lets the stream be captured;
    the pipelined adjoint is a cooperative launch and is replaced by the
    one-workgroup adjoint inside the graph (bitwise the same gradient).
    """

    def __init__(self, sim: Simulator, target: torch.Tensor, theta: Optional[torch.Tensor] = None):
        if sim.checkpoint_every <= 0:
            raise ValueError("the simulator needs checkpoints for the adjoint")
        dev = sim.device
        T = sim.n_steps
        self.sim = sim
        self.theta = (theta_matrix(sim.nets, device=dev) if theta is None else theta).clone()
        self.target = target.contiguous().clone()
        # untouched rec columns (past a scenario's n_rec) stay zero
        self.rec = torch.zeros((sim.S, T, sim.R), dtype=torch.float64, device=dev)
        self.dJ = torch.zeros_like(self.rec)
        self.loss = torch.zeros((sim.S,), dtype=torch.float64, device=dev)
        self.grad = torch.zeros((sim.S, sim.P), dtype=torch.float64, device=dev)
        self.graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            self._iteration()          # eager, once: kernels loaded, attributes set
            sim.sync()
        torch.cuda.current_stream(dev).wait_stream(side)
        with torch.cuda.graph(self.graph, capture_error_mode="relaxed"):
            self._iteration()
        torch.cuda.current_stream(dev).synchronize()

    def _iteration(self):
        sim = self.sim
        sim.set_params(self.theta)
        sim.factor_async()
        sim.step(sim.n_steps, rec=self.rec)
        sim.mismatch(self.rec, self.target, self.dJ, self.loss)
        sim.adjoint(self.dJ, grad=self.grad)

    def replay(self, check_status: bool = True):
        """Runs the iteration; with check_status, waits and raises EMTError
        on a device-side failure (e.g. EMT_ESINGULAR)."""
        self.graph.replay()
        if check_status:
            self.sim.sync()
        return self.loss, self.grad


def theta_matrix(nets, thetas=None, device=None) -> torch.Tensor:
    """Stacks per-scenario parameter vectors (default: nominal) into [S, P]."""
    P = max(3 * int(n.n_lines) for n in nets)
    out = np.zeros((len(nets), P))
    for s, n in enumerate(nets):
        th = n.theta0() if thetas is None else np.asarray(thetas[s], np.float64)
        out[s, :th.shape[0]] = th
    return torch.tensor(out, dtype=torch.float64, device=device)


__all__ = ["Simulator", "IdentificationGraph", "EMTError", "theta_matrix", "SOLVERS"]
