"""Seeded synthetic three-phase networks: the inputs of the EMT time loop.

This module only *draws* networks (topology, component parameters, events,
monitored nodes). It contains none of the simulation method's arithmetic: no
companion models, no matrix assembly, no solves. Both the GPU library and the
CPU oracle read the `Network` objects it returns, so it is the one piece of
code they share.

The paper's own test network (a 33-node distribution feeder with PV
subsystems, Sec. IV-A, Fig. 5) is not published in usable form, so these
transmission-style networks stand in for it. Their shapes follow the five
benchmark workloads (27, 3000, 600x400, 300 and 90-900 nodes); the recipe is:

* buses are joined by a random spanning tree (random attachment over a random
  permutation) plus uniformly drawn extra lines up to round(1.5 * n_bus) lines
  (mean degree 3);
* every line is a per-phase pi-section: a series R-L branch between the same
  phase of its two buses and C/2 from each end to ground, with
  R ~ U(0.01, 0.05) ohm/km, L ~ U(0.05, 0.2) mH/km, C ~ U(8, 12) nF/km, all
  times a length ~ U(10, 100) km; the three phases share one (R, L, C);
* generators are Thevenin sources (0.5 ohm, 10 mH per phase, a 60 Hz EMF of
  magnitude U(0.95, 1.05) and random phase, phases shifted by 2*pi/3);
* loads are wye-grounded series R-L, R ~ U(50, 200) ohm, L ~ U(0.1, 0.5) H;
* a solid three-phase fault is three 1e-3 ohm switches to ground that close
  at the event step.

Node numbering: node = 3 * bus + phase, ground = -1.
Line parameters theta[3l + 0..2] = (R_l [ohm], L_l [H], C_l [F]).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# Branch kinds; the integer codes are part of the C interface. LINE is a
# distributed-parameter (travelling-wave) line: R = surge impedance Z,
# L = travel time tau. DIODE is an ideal diode (state-dependent switch):
# R = on-resistance, conducting from k to m while its current is positive,
# blocking while its voltage v_k - v_m is not. CSWITCH is a switch set by a
# hysteresis comparator: R = on-resistance, reference E cos(omega t + phase)
# + C, half-width L, measuring the voltage between the node pair meas.
RL, CAP, RES, SWITCH, SRC, LINE, DIODE, CSWITCH = 0, 1, 2, 3, 4, 5, 6, 7

F_HZ = 60.0
R_SRC = 0.5          # Thevenin source resistance per phase [ohm]
L_SRC = 10e-3        # Thevenin source inductance per phase [H]
R_FAULT = 1e-3       # closed fault switch resistance [ohm]
# diode-bridge loads: diode on-resistance, DC capacitor, DC-side reference
R_DIODE_ON, C_DC, R_DC_REF = 1e-2, 100e-6, 1e6
CHOP_V_REF, CHOP_H, CHOP_C, CHOP_R = 0.08, 0.01, 200e-6, 40.0
# coupled three-phase lines: mutual / self ratios of the circulant series R,
# L and (negative) shunt C matrices
COUPLING_R, COUPLING_L, COUPLING_C = 0.25, 0.4, 0.2


@dataclasses.dataclass
class Network:
    """One network: a branch list plus its switching events and outputs.

    Arrays are per branch unless noted. ``kind`` uses the codes above. For a
    source branch the EMF is E*cos(omega*t + phase) and R, L are its internal
    impedance. ``line`` is the line index of a pi-section branch, -1 otherwise.
    ``in_service0`` is the state at t = 0 (switches start open).
    Events: at step ``ev_step[j]`` branch ``ev_branch[j]`` is put in service
    (``ev_in_service[j] == 1``) or taken out (0).
    ``rec_nodes`` lists recorded nodes; None records every node.
    """
    n_nodes: int
    k: np.ndarray
    m: np.ndarray
    kind: np.ndarray
    R: np.ndarray
    L: np.ndarray
    C: np.ndarray
    E: np.ndarray
    omega: np.ndarray
    phase: np.ndarray
    line: np.ndarray
    in_service0: np.ndarray
    ev_step: np.ndarray
    ev_branch: np.ndarray
    ev_in_service: np.ndarray
    rec_nodes: Optional[np.ndarray] = None
    n_lines: int = 0
    # coupled three-phase groups: group[b] = group id (three branches of one
    # kind, RL or CAP, with equal self values), -1 otherwise; Rm, Lm, Cm are
    # the mutual (off-diagonal) entries of the group's circulant 3 x 3 R, L
    # or C matrix. None when the network has no coupled groups.
    group: Optional[np.ndarray] = None
    Rm: Optional[np.ndarray] = None
    Lm: Optional[np.ndarray] = None
    Cm: Optional[np.ndarray] = None
    # controlled switches: meas[b] = (a, b) the node pair whose voltage the
    # switch's controller measures; None when the network has none
    meas: Optional[np.ndarray] = None
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_branches(self) -> int:
        return int(self.k.shape[0])

    @property
    def n_params(self) -> int:
        return 3 * self.n_lines

    @property
    def n_rec(self) -> int:
        return self.n_nodes if self.rec_nodes is None else int(self.rec_nodes.shape[0])

    def theta0(self) -> np.ndarray:
        """Nominal per-line totals (R_l, L_l, C_l) read back from the branches."""
        th = np.zeros(self.n_params)
        for b in range(self.n_branches):
            l = int(self.line[b])
            if l < 0:
                continue
            if self.kind[b] == RL:
                th[3 * l] = self.R[b]
                th[3 * l + 1] = self.L[b]
            elif self.kind[b] == CAP:
                th[3 * l + 2] = 2.0 * self.C[b]
        return th


class _Builder:
    """Accumulates branches in a fixed order."""

    def __init__(self, n_nodes: int):
        self.n_nodes = n_nodes
        self.cols = {c: [] for c in ("k", "m", "kind", "R", "L", "C", "E",
                                     "omega", "phase", "line", "ins", "group", "Rm", "Lm", "Cm", "meas")}
        self.n_groups = 0
        self.n_cswitch = 0

    def add(self, k, m, kind, R=0.0, L=0.0, C=0.0, E=0.0, omega=0.0,
            phase=0.0, line=-1, ins=1, group=-1, Rm=0.0, Lm=0.0, Cm=0.0, meas=(-1, -1)) -> int:
        c = self.cols
        c["k"].append(k); c["m"].append(m); c["kind"].append(kind)
        c["R"].append(R); c["L"].append(L); c["C"].append(C)
        c["E"].append(E); c["omega"].append(omega); c["phase"].append(phase)
        c["line"].append(line); c["ins"].append(ins)
        c["group"].append(group); c["Rm"].append(Rm); c["Lm"].append(Lm); c["Cm"].append(Cm)
        c["meas"].append(tuple(meas))
        if kind == CSWITCH:
            self.n_cswitch += 1
        return len(c["k"]) - 1

    def new_group(self) -> int:
        self.n_groups += 1
        return self.n_groups - 1

    def network(self, events, rec_nodes, n_lines, meta) -> Network:
        c = self.cols
        ev = sorted(events)
        return Network(
            n_nodes=self.n_nodes,
            k=np.asarray(c["k"], np.int32), m=np.asarray(c["m"], np.int32),
            kind=np.asarray(c["kind"], np.int32),
            R=np.asarray(c["R"], np.float64), L=np.asarray(c["L"], np.float64),
            C=np.asarray(c["C"], np.float64), E=np.asarray(c["E"], np.float64),
            omega=np.asarray(c["omega"], np.float64),
            phase=np.asarray(c["phase"], np.float64),
            line=np.asarray(c["line"], np.int32),
            in_service0=np.asarray(c["ins"], np.uint8),
            ev_step=np.asarray([e[0] for e in ev], np.int64),
            ev_branch=np.asarray([e[1] for e in ev], np.int32),
            ev_in_service=np.asarray([e[2] for e in ev], np.uint8),
            rec_nodes=None if rec_nodes is None else np.asarray(rec_nodes, np.int32),
            n_lines=n_lines, meta=meta,
            meas=None if self.n_cswitch == 0 else np.asarray(c["meas"], np.int32).reshape(-1, 2),
            **({} if self.n_groups == 0 else dict(
                group=np.asarray(c["group"], np.int32), Rm=np.asarray(c["Rm"], np.float64),
                Lm=np.asarray(c["Lm"], np.float64), Cm=np.asarray(c["Cm"], np.float64))))


def random_lines(rng: np.random.Generator, n_bus: int, n_lines: int) -> np.ndarray:
    """Spanning tree by random attachment over a random permutation, then
    uniformly drawn extra edges (no duplicates, no self loops)."""
    if n_lines < n_bus - 1:
        raise ValueError("need at least n_bus - 1 lines for a connected grid")
    if n_lines > n_bus * (n_bus - 1) // 2:
        raise ValueError("too many lines for a simple graph")
    perm = rng.permutation(n_bus)
    edges = []
    seen = set()
    for i in range(1, n_bus):
        a = int(perm[i])
        b = int(perm[rng.integers(0, i)])
        e = (min(a, b), max(a, b))
        seen.add(e)
        edges.append(e)
    while len(edges) < n_lines:
        a, b = (int(x) for x in rng.integers(0, n_bus, size=2))
        if a == b:
            continue
        e = (min(a, b), max(a, b))
        if e in seen:
            continue
        seen.add(e)
        edges.append(e)
    return np.asarray(edges, np.int64)


def three_phase_grid(rng: np.random.Generator, n_bus: int, n_lines: int,
                     n_gen: int, n_load: int, *, fault_bus: Optional[int] = None,
                     fault_step: int = 0, rec_nodes=None, with_fault_switch=True,
                     travelling_wave_dt: Optional[float] = None, coupled: bool = False,
                     rectifiers: int = 0, choppers: int = 0):
    """Draw one grid. Returns (builder, bookkeeping) so callers can add events.

    Branch order: for each line its 3 series R-L branches, then the 3 shunt
    capacitors at its first bus, then the 3 at its second bus; then 3 source
    branches per generator, 3 load branches per load, 3 fault switches.

    rectifiers: the first this many loads also feed a six-pulse diode
    bridge (ideal diodes, 10 mOhm on, starting blocked) whose DC side is a
    resistor of twice the load's R in parallel with 100 uF, referenced to
    ground through 1 MOhm at its negative node; each bridge adds two DC
    nodes after the 3 n_bus AC nodes. No extra random draws.

    choppers: the first this many loads also feed, from their phase a, a
    controlled switch (10 mOhm on, starting on) into a DC node with 200 uF
    and 40 ohm to ground, its hysteresis comparator holding the DC voltage
    at 0.08 +- 0.01 (CHOP_V_REF, CHOP_H); one DC node each after the bridges'.
    No extra random draws.

    coupled: every line's three phases are coupled: its series R-L
    branches form one group with mutual Rm = 0.25 R, Lm = 0.4 L, and the
    C/2 shunts at each end one group with mutual Cm = -0.2 C/2 (a
    transposed line's circulant matrices; positive sequence R - Rm, L - Lm,
    C/2 - Cm, zero sequence R + 2 Rm, L + 2 Lm, C/2 + 2 Cm). Coupled lines
    are not part of the parameter vector. The same random draws as the
    uncoupled grid.

    travelling_wave_dt: if given, every line whose travel time
    tau = sqrt(L C) is at least this time step is drawn the same way but
    entered as three lossless distributed-parameter lines (one per phase,
    kind LINE, Z = sqrt(L / C), series resistance dropped) instead of
    pi-sections; it is then not part of the parameter vector.
    """
    edges = random_lines(rng, n_bus, n_lines)
    n_nodes = 3 * n_bus + 2 * rectifiers + choppers
    bld = _Builder(n_nodes)
    series = np.zeros((n_lines, 3), np.int32)
    for l, (a, b) in enumerate(edges):
        km = rng.uniform(10.0, 100.0)
        R = rng.uniform(0.01, 0.05) * km              # ohm
        L = rng.uniform(0.05, 0.2) * 1e-3 * km        # H
        C = rng.uniform(8.0, 12.0) * 1e-9 * km        # F
        tau = math.sqrt(L * C)
        if travelling_wave_dt is not None and tau >= travelling_wave_dt:
            for p in range(3):
                series[l, p] = bld.add(3 * a + p, 3 * b + p, LINE, R=math.sqrt(L / C), L=tau)
            continue
        if coupled:
            g = bld.new_group()
            for p in range(3):
                series[l, p] = bld.add(3 * a + p, 3 * b + p, RL, R=R, L=L, group=g,
                                       Rm=COUPLING_R * R, Lm=COUPLING_L * L)
            for bus in (a, b):
                g = bld.new_group()
                for p in range(3):
                    bld.add(3 * bus + p, -1, CAP, C=C / 2.0, group=g, Cm=-COUPLING_C * C / 2.0)
            continue
        for p in range(3):
            series[l, p] = bld.add(3 * a + p, 3 * b + p, RL, R=R, L=L, line=l)
        for p in range(3):
            bld.add(3 * a + p, -1, CAP, C=C / 2.0, line=l)
        for p in range(3):
            bld.add(3 * b + p, -1, CAP, C=C / 2.0, line=l)
    bus_perm = rng.permutation(n_bus)
    gens = bus_perm[:n_gen]
    loads = bus_perm[n_gen:n_gen + n_load]
    w = 2.0 * math.pi * F_HZ
    for g in gens:
        mag = rng.uniform(0.95, 1.05)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        for p in range(3):
            bld.add(3 * int(g) + p, -1, SRC, R=R_SRC, L=L_SRC, E=mag, omega=w,
                    phase=phi - p * 2.0 * math.pi / 3.0)
    for q, ld in enumerate(loads):
        R = rng.uniform(50.0, 200.0)
        L = rng.uniform(0.1, 0.5)
        for p in range(3):
            bld.add(3 * int(ld) + p, -1, RL, R=R, L=L)
        if q < rectifiers:
            P, N = 3 * n_bus + 2 * q, 3 * n_bus + 2 * q + 1
            for p in range(3):
                bld.add(3 * int(ld) + p, P, DIODE, R=R_DIODE_ON, ins=0)
                bld.add(N, 3 * int(ld) + p, DIODE, R=R_DIODE_ON, ins=0)
            bld.add(P, N, RES, R=2.0 * R)
            bld.add(P, N, CAP, C=C_DC)
            bld.add(N, -1, RES, R=R_DC_REF)
        if q < choppers:
            d = 3 * n_bus + 2 * rectifiers + q
            bld.add(3 * int(ld), d, CSWITCH, R=R_DIODE_ON, C=CHOP_V_REF, L=CHOP_H, meas=(d, -1), ins=1)
            bld.add(d, -1, CAP, C=CHOP_C)
            bld.add(d, -1, RES, R=CHOP_R)
    fault_sw = []
    if with_fault_switch:
        if fault_bus is None:
            fault_bus = int(rng.integers(0, n_bus))
        for p in range(3):
            fault_sw.append(bld.add(3 * fault_bus + p, -1, SWITCH, R=R_FAULT, ins=0))
    info = dict(edges=edges, series=series, gens=gens, loads=loads,
                fault_bus=fault_bus, fault_sw=fault_sw, n_bus=n_bus)
    return bld, info


def _fault_events(info, step):
    return [(int(step), int(b), 1) for b in info["fault_sw"]]


def _monitored(rng, n_nodes, n_mon=30):
    return np.sort(rng.choice(n_nodes, size=min(n_mon, n_nodes), replace=False))


# --------------------------------------------------------------------------
# The five benchmark workloads. Each returns (list of Network, sim dict);
# keyword arguments shrink a workload for tests without changing its recipe.
# --------------------------------------------------------------------------

def config0(seed: int = 0, n_steps: int = 4000):
    """9-bus grid (27 nodes), 9 lines, 3 sources, 3 RL loads, dt = 50 us,
    0.2 s, solid three-phase fault closing at t = 0.1 s, all nodes recorded."""
    rng = np.random.default_rng(seed)
    dt = 50e-6
    ev = int(round(0.1 / dt))
    bld, info = three_phase_grid(rng, 9, 9, 3, 3)
    net = bld.network(_fault_events(info, ev), None, 9, dict(info, name="grid9"))
    return [net], dict(dt=dt, n_steps=n_steps)


def config1(seed: int = 1, n_bus: int = 1000, n_steps: int = 50000,
            fault_step: Optional[int] = None, travelling_wave: bool = False,
            coupled: bool = False, rectifiers: int = 0, choppers: int = 0):
    """1000-bus grid (3000 nodes), 1500 lines, 200 sources, 600 loads,
    dt = 20 us, 1 s, one fault at mid-horizon, all nodes recorded.
    travelling_wave: the same draw with every line whose travel time is at
    least one step entered as distributed-parameter lines (see
    three_phase_grid). coupled: the same draw with coupled three-phase
    lines (one component of 3 n_bus nodes). rectifiers: the same draw with
    that many loads also feeding diode bridges; choppers: with that many
    loads also feeding controlled choppers."""
    rng = np.random.default_rng(seed)
    dt = 20e-6
    n_lines = int(round(1.5 * n_bus))
    ev = n_steps // 2 if fault_step is None else fault_step
    bld, info = three_phase_grid(rng, n_bus, n_lines, int(round(0.2 * n_bus)),
                                 int(round(0.6 * n_bus)),
                                 travelling_wave_dt=dt if travelling_wave else None, coupled=coupled,
                                 rectifiers=rectifiers, choppers=choppers)
    name = (f"grid{n_bus}" + ("-tw" if travelling_wave else "") + ("-coupled" if coupled else "")
            + (f"-rect{rectifiers}" if rectifiers else "") + (f"-chop{choppers}" if choppers else ""))
    net = bld.network(_fault_events(info, ev), None, n_lines, dict(info, name=name))
    return [net], dict(dt=dt, n_steps=n_steps)


def config2(seed: int = 2, n_bus: int = 200, n_scen: int = 400,
            n_steps: int = 15000, event_step: int = 2500):
    """N-1 contingencies on one 200-bus grid (600 nodes): scenario s removes
    one distinct series branch (one phase of one line) and closes a solid
    fault on a random bus, both at t = 0.05 s (step 2500 at dt = 20 us).
    30 monitored nodes."""
    rng = np.random.default_rng(seed)
    dt = 20e-6
    n_lines = int(round(1.5 * n_bus))
    n_gen, n_load = int(round(0.2 * n_bus)), int(round(0.6 * n_bus))
    # One base grid drawn once; scenarios differ in the removed branch and the
    # fault bus only, so each scenario is rebuilt from the same sub-seed.
    base_seed = int(rng.integers(0, 2**31 - 1))
    rec = _monitored(rng, 3 * n_bus)
    n_cand = 3 * n_lines
    if n_scen > n_cand:
        raise ValueError("more scenarios than candidate branches")
    removed = rng.choice(n_cand, size=n_scen, replace=False)
    fault_buses = rng.integers(0, n_bus, size=n_scen)
    nets = []
    for s in range(n_scen):
        brng = np.random.default_rng(base_seed)
        bld, info = three_phase_grid(brng, n_bus, n_lines, n_gen, n_load,
                                     fault_bus=int(fault_buses[s]))
        l, p = divmod(int(removed[s]), 3)
        br = int(info["series"][l, p])
        events = _fault_events(info, event_step) + [(event_step, br, 0)]
        nets.append(bld.network(events, rec, n_lines,
                                dict(info, name=f"grid{n_bus}_n1_{s}",
                                     removed_branch=br)))
    return nets, dict(dt=dt, n_steps=n_steps)


def perturbed_theta(rng: np.random.Generator, theta0: np.ndarray, sigma=0.1):
    """theta* = theta0 * exp(sigma * z), z ~ N(0, I): the 'true' parameters
    of an identification problem."""
    return theta0 * np.exp(sigma * rng.standard_normal(theta0.shape[0]))


def config3(seed: int = 3, n_bus: int = 100, n_steps: int = 10000):
    """Adjoint workload: 100-bus grid (300 nodes), no events, 30 monitored
    nodes, dt = 50 us, 10,000 steps, checkpoint every 500 steps. Returns the
    network, sim, and the perturbed 'true' parameters theta* whose waveform
    is the identification target."""
    rng = np.random.default_rng(seed)
    dt = 50e-6
    n_lines = int(round(1.5 * n_bus))
    bld, info = three_phase_grid(rng, n_bus, n_lines, int(round(0.2 * n_bus)),
                                 int(round(0.6 * n_bus)), with_fault_switch=False)
    rec = _monitored(rng, 3 * n_bus)
    net = bld.network([], rec, n_lines, dict(info, name=f"grid{n_bus}_adj"))
    theta_true = perturbed_theta(rng, net.theta0())
    fd_idx = np.sort(rng.choice(net.n_params, size=min(20, net.n_params), replace=False))
    return [net], dict(dt=dt, n_steps=n_steps, checkpoint_every=500,
                       theta_true=[theta_true], fd_idx=fd_idx)


def config4(seed: int = 4, n_inst: int = 256, n_steps: int = 5000,
            bus_range=(30, 300)):
    """Uneven batch: instance j is a grid with log-uniform bus count in
    [30, 300] drawn from seed 4000 + j, its own perturbed parameters, one
    fault at mid-horizon, 30 monitored nodes, dt = 50 us, 5000 steps."""
    dt = 50e-6
    nets, thetas = [], []
    lo, hi = bus_range
    for j in range(n_inst):
        rng = np.random.default_rng(4000 + j + (seed - 4) * 100000)
        n_bus = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        n_lines = int(round(1.5 * n_bus))
        bld, info = three_phase_grid(rng, n_bus, n_lines, max(1, int(round(0.2 * n_bus))),
                                     int(round(0.6 * n_bus)))
        rec = _monitored(rng, 3 * n_bus)
        net = bld.network(_fault_events(info, n_steps // 2), rec, n_lines,
                          dict(info, name=f"inst{j}_grid{n_bus}"))
        nets.append(net)
        thetas.append(perturbed_theta(rng, net.theta0()))
    return nets, dict(dt=dt, n_steps=n_steps, checkpoint_every=500,
                      theta_true=thetas)


def small_grid(seed: int, n_bus: int, *, n_lines=None, n_gen=None, n_load=None,
               fault_step: Optional[int] = None, n_mon: Optional[int] = None,
               remove_series: Optional[int] = None, remove_step: Optional[int] = None,
               travelling_wave_dt: Optional[float] = None, coupled: bool = False):
    """A grid of the same recipe at an arbitrary size, for tests."""
    rng = np.random.default_rng(seed)
    if n_lines is None:
        n_lines = min(int(round(1.5 * n_bus)), n_bus * (n_bus - 1) // 2)
    n_gen = max(1, int(round(0.2 * n_bus))) if n_gen is None else n_gen
    n_load = int(round(0.6 * n_bus)) if n_load is None else n_load
    bld, info = three_phase_grid(rng, n_bus, n_lines, n_gen, n_load,
                                 with_fault_switch=fault_step is not None,
                                 travelling_wave_dt=travelling_wave_dt, coupled=coupled)
    events = [] if fault_step is None else _fault_events(info, fault_step)
    if remove_series is not None:
        l, p = divmod(int(remove_series), 3)
        events.append((int(remove_step), int(info["series"][l, p]), 0))
    rec = None if n_mon is None else _monitored(rng, 3 * n_bus, n_mon)
    return bld.network(events, rec, n_lines, dict(info, name=f"small{n_bus}"))


def make_config(index: int, **kw):
    return [config0, config1, config2, config3, config4][index](**kw)


# --------------------------------------------------------------------------
# Tiny hand-built circuits used by the closed-form checks.
# --------------------------------------------------------------------------

def circuit(n_nodes: int, branches: Sequence[dict], events=(), rec_nodes=None) -> Network:
    """Build a network from explicit branch dicts, e.g.
    dict(k=0, m=-1, kind=CAP, C=1e-6)."""
    bld = _Builder(n_nodes)
    n_lines = 0
    for b in branches:
        b = dict(b)
        n_lines = max(n_lines, int(b.get("line", -1)) + 1)
        bld.add(**b)
    return bld.network(list(events), rec_nodes, n_lines, dict(name="circuit"))
