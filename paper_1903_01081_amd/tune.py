"""Launch-shape autotuner: times the feasible solver and shape choices of a
batch on a short prefix of its own run and returns the fastest.

The choices (all fields of emt_sim, see include/emt.h):
  * solver "auto" (sparse sweeps + dense tail in one workgroup) at each
    feasible block size, with the largest dense tail of the 256- and
    512-lane blocks, and with the sweep data read from global memory;
  * solver "sparse" (sweeps only);
  * solver "dense": components up to 128 nodes with their inverse in one
    workgroup, larger ones split by columns over 16- or 32-column
    workgroups (forward only, so skipped when checkpoints are asked for);
  * "auto" with a scenario's small components packed into shared
    workgroups (pack_nodes 256 or 512), where that changes the work items;
  * solver "compensation" (scenarios that differ from the first one by a
    few switched branches share its components' inverses; forward only).
Every candidate factorises and runs the same prefix of `probe_steps` steps
(recorded like the real run) twice; the second run's factorisation time
plus n_steps times its time per step ranks it, so a long horizon is not
judged by the factorisation of a short prefix. With checkpoints (a
gradient workload) each candidate instead runs forward and adjoint over a
horizon of at least two checkpoint segments, and the per-step time counts
both.
Candidates the library rejects for this batch (EMT_EINVAL: shapes that do
not fit) are skipped and listed with the reason.
"""
from __future__ import annotations

import time
from typing import List, Optional, Sequence

import torch

from ._lib import EMTError
from .sim import Simulator


def candidates(checkpoint_every: int = 0) -> List[dict]:
    c = [dict(solver="auto", block_size=b) for b in (0, 64, 256, 512)]
    # the largest dense tail a block size holds (fewer sweep passes, more
    # tail work per lane)
    c += [dict(solver="auto", block_size=b, dense_tail=d) for b, d in ((256, 64), (512, 128))]
    c.append(dict(solver="auto", sweep_from_global=True))
    c.append(dict(solver="sparse"))
    if checkpoint_every == 0:
        c += [dict(solver="dense", split_cols=k) for k in (16, 32)]
    else:
        c.append(dict(solver="dense"))
    # small components packed into shared workgroups (kept only where the
    # packing changes the batch's work items)
    c += [dict(solver="auto", pack_nodes=p) for p in PACK_BUDGETS]
    c += [dict(solver="auto", block_size=256, dense_tail=64, pack_nodes=p) for p in PACK_BUDGETS]
    if checkpoint_every == 0:
        c.append(dict(solver="compensation"))
    return c


PACK_BUDGETS = (256, 512)


def _packing_changes_items(nets, dt, n_steps, checkpoint_every, shape) -> bool:
    from . import _lib
    p = shape.get("pack_nodes", 0)
    if p <= 0:
        return True
    a = _lib.analyze(nets, dt, n_steps, checkpoint_every, pack_nodes=p)
    b = _lib.analyze(nets, dt, n_steps, checkpoint_every)
    return a["n_items"] != b["n_items"]


def _time_one(nets, dt, n_steps, checkpoint_every, shape, probe_steps, device):
    if checkpoint_every > 0:
        # forward + adjoint over a short horizon of its own
        k = min(n_steps, max(probe_steps, 2 * checkpoint_every))
        sim = Simulator(nets, dt, k, checkpoint_every=checkpoint_every, device=device, **shape)
    else:
        k = min(probe_steps, n_steps)
        sim = Simulator(nets, dt, n_steps, device=device, **shape)
    try:
        rec = torch.empty((sim.S, k, sim.R), dtype=torch.float64, device=sim.device)
        cot = torch.ones_like(rec) if checkpoint_every > 0 else None
        t_fac = t_step = 0.0
        for _ in range(2):
            sim.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.factor()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sim.step(k, rec=rec)
            if cot is not None:
                sim.adjoint(cot)
            torch.cuda.synchronize()
            t_fac, t_step = t1 - t0, (time.perf_counter() - t1) / k
        return t_fac, t_step, sim.info()
    finally:
        sim.close()


def tune(nets: Sequence, dt: float, n_steps: int, checkpoint_every: int = 0, probe_steps: int = 400,
         shapes: Optional[List[dict]] = None, device=None, exclude_solvers: Sequence[str] = ()) -> dict:
    """Returns {"shape": best shape (Simulator keyword arguments),
    "s_per_step": its time per step on the probe (forward, plus adjoint
    with checkpoints), "run_s": its estimated factorisation + n_steps time,
    "trials": [...]}. Solvers named in exclude_solvers are not tried."""
    trials = []
    for shape in (shapes if shapes is not None else candidates(checkpoint_every)):
        if shape.get("solver") in exclude_solvers:
            continue
        if shapes is None and not _packing_changes_items(nets, dt, n_steps, checkpoint_every, shape):
            continue
        try:
            t_fac, t_step, info = _time_one(nets, dt, n_steps, checkpoint_every, shape, probe_steps, device)
            trials.append(dict(shape=shape, s_per_step=t_step, factor_s=t_fac,
                               run_s=t_fac + n_steps * t_step, block_size=info["block_size"],
                               split_tiles=info["split_tiles"], split_cols=info["split_cols"],
                               max_tail=info["max_tail"]))
        except EMTError as e:
            trials.append(dict(shape=shape, rejected=str(e)))
    ok = [t for t in trials if "s_per_step" in t]
    if not ok:
        raise RuntimeError("no launch shape fits this batch: " + "; ".join(t["rejected"] for t in trials))
    best = min(ok, key=lambda t: t["run_s"])
    return dict(shape=best["shape"], s_per_step=best["s_per_step"], run_s=best["run_s"], trials=trials)


def tuned_simulator(nets: Sequence, dt: float, n_steps: int, checkpoint_every: int = 0, probe_steps: int = 400,
                    device=None) -> Simulator:
    """A Simulator built with the fastest shape for this batch."""
    r = tune(nets, dt, n_steps, checkpoint_every, probe_steps, device=device)
    return Simulator(nets, dt, n_steps, checkpoint_every=checkpoint_every, device=device, **r["shape"])


__all__ = ["candidates", "tune", "tuned_simulator"]
