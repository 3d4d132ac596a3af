/*
 * emt.h — C ABI of the MI355X EMT nodal-analysis time loop (FP64).
 *
 * The library runs the fixed-step nodal-analysis loop of an EMTP-type
 * simulator: the paper (Sec. III-A) splits each step into four basic
 * processes — update each component's Norton equivalent (history current and
 * conductance), update the nodal injected currents, factorise the nodal
 * conductance matrix, and forward/back substitute for the node voltages —
 * and (Sec. III-B) runs many scenarios of one topology as one vectorised
 * computation. The companion models are the trapezoidal-rule ones of the
 * EMTP method (the paper's reference [2]):
 *
 *   series R-L (also a source's internal impedance):
 *       g = 1/(R + 2L/dt), beta = (2L/dt - R) g, gamma = g
 *   capacitor:                 g = 2C/dt, beta = -1, gamma = -g
 *   resistor / closed switch:  g = 1/R,   beta = gamma = 0
 *   out of service:            g = beta = gamma = 0 and u = i = 0
 *
 *   step n (t_n = n dt):  h = beta*i + gamma*u           (history, n-1 state)
 *                         e = E cos(omega t_n + phase)    (source branches)
 *                         rhs = A (g*e - h)               (nodal injection)
 *                         v = G^{-1} rhs,  G = A diag(g) A^T
 *                         u = A^T v - e,   i = g*u + h    (branch update)
 *
 * A is the node-by-branch incidence (+1 at k, -1 at m; ground = -1 is
 * dropped), u is the voltage across a branch's passive part, i flows k -> m.
 * The initial state is v = 0, i = 0, u = A^T v - e(0). Switching events
 * apply at a step index: the new topology produces v at that step. The
 * conductance matrix is factorised once per topology (LDL^T on a symbolic
 * pattern shared by all topologies and by isomorphic scenarios); no
 * factorisation happens inside the time loop.
 *
 * Conventions: FP64 values, int32 indices, node ids 0..n_nodes-1, ground -1,
 * row-major arrays. Host arrays passed to a call are borrowed for that call
 * only and copied. Device buffers (`*_dev`) belong to the caller, must be
 * device memory of the current HIP device, and must stay valid until the
 * work queued on `stream` has finished. `stream` is a hipStream_t (NULL =
 * the default stream); the calls of one run go to one stream. Calls are
 * stream-ordered: emt_set_params, emt_factor_async, emt_reset, emt_step,
 * emt_adjoint and emt_mismatch only queue work and return without waiting
 * for the device (so a caller can record them into a HIP graph); the calls
 * documented as synchronising (emt_factor, emt_sync, emt_get_state,
 * emt_set_state, emt_branch_adjoints, emt_latency_floor, emt_destroy,
 * emt_build, emt_info_get with split components) wait. Errors found by the
 * device during queued work (non-positive pivots of emt_factor_async, a
 * split launch or the pipelined adjoint whose workgroups gave up waiting for
 * each other) are reported by emt_sync. A context is not thread-safe. Every call returns a
 * status; on a non-OK status returned before any work was queued, nothing
 * was queued, and emt_last_error() describes the cause. No C++ exception
 * crosses this interface.
 *
 * Sources: each declaration below names the passage of the paper that
 * defines what it computes ("Sec." = a section of arXiv 1903.01081); calls
 * that are not in the paper say so.
 */
#ifndef EMT_H
#define EMT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct emt_ctx emt_ctx;

typedef enum {
  EMT_OK = 0,
  EMT_EINVAL = 1,     /* bad argument: sizes, indices, NaN or non-positive parameters */
  EMT_ESINGULAR = 2,  /* a node has no conductive path to ground, or a non-positive pivot */
  EMT_ENOMEM = 3,     /* host or device allocation failed */
  EMT_EDEVICE = 4,    /* HIP runtime error or no device */
  EMT_ESTATE = 5      /* call out of order (see each call) */
} emt_status;

typedef enum {
  EMT_RL = 0, EMT_C = 1, EMT_R = 2, EMT_SWITCH = 3, EMT_SRC = 4, EMT_LINE = 5, EMT_DIODE = 6,
  EMT_CSWITCH = 7
} emt_kind;

typedef enum {
  EMT_SOLVER_AUTO = 0, EMT_SOLVER_DENSE = 1, EMT_SOLVER_SPARSE = 2, EMT_SOLVER_COMPENSATION = 3
} emt_solver;

/* One network (scenario): a branch list, its switching events and outputs.
 * Per-branch arrays have n_branches entries.
 *   k, m       terminals (-1 = ground; not both -1), kind = emt_kind.
 *   R, L, C    RL: R >= 0, L > 0 (source: internal R, L); C: C > 0;
 *              R and SWITCH: R > 0 (SWITCH: closed resistance).
 *              LINE (a lossless distributed-parameter line between two
 *              nodes, the travelling-wave line model of the EMTP method the
 *              paper cites as its reference [2]): R = surge impedance Z > 0,
 *              L = travel time tau >= dt, C = 0. Each end is a Norton
 *              equivalent 1/Z to ground whose history current is the wave
 *              that left the other end tau earlier (linear interpolation
 *              between steps; the line starts at rest). The branch current
 *              is the current from node k into the line. Lines take no
 *              events and belong to no pi-section (line = -1); a batch with
 *              lines runs forward only (EMT_EINVAL with checkpoint_every >
 *              0 or with components split over workgroups) and takes no
 *              emt_set_state.
 *              DIODE (an ideal diode, a state-dependent switch): R = its
 *              on-resistance > 0, conducting from k to m. in_service0 is
 *              its initial state; after every step a conducting diode
 *              whose current is negative blocks from the next step on and a
 *              blocking one whose voltage v_k - v_m is positive conducts
 *              from the next step on, the conductance matrix being
 *              refactorised inside the time loop (one-workgroup solvers,
 *              sweeps without a dense tail). Diodes take no events; a batch
 *              with diodes runs forward only (EMT_EINVAL with checkpoints,
 *              the dense solver or emt_steady_state). The plain trapezoidal
 *              rule rings when a diode interrupts an inductor's current, so
 *              a diode can chatter after it blocks (no damping step is
 *              added).
 *              CSWITCH (a switch driven by a control-system vertex: the
 *              control graph of Sec. III-A's basic processes reduced to one
 *              hysteresis comparator per switch): R = its on-resistance > 0;
 *              the comparator's reference r(t) = E cos(omega t + phase) + C
 *              (E, omega, phase, C finite) and half-width h = L >= 0; it
 *              measures s = v_a - v_b, the nodes a = meas[2b], b = meas[2b+1]
 *              (-1 = ground; in the switch's connected component). After
 *              step n, with e = r(n dt) - s(n): the switch conducts from
 *              step n+1 on if e > h, is open if e < -h, else keeps its state
 *              (the one-step delay breaks the algebraic loop between the
 *              controller and the network it measures); in_service0 is its
 *              state before step 1. Like diodes: refactorised inside the
 *              loop, no events, forward only, sweep solvers.
 *   E, omega, phase  source EMF E cos(omega t + phase); read for EMT_SRC only.
 *   line       pi-section line index l of the branch, or -1. Line parameters
 *              theta[3l + {0,1,2}] = (R_l, L_l, C_l) are the series R and L
 *              of each EMT_RL branch of line l and twice the capacitance of
 *              each EMT_C branch of line l (C_l / 2 at each end).
 *   n_params   3 * number of lines (0 if none).
 *   in_service0  state at t = 0 (1 = in service / switch closed); NULL means
 *              every branch in service except switches, which start open.
 *   events     at step ev_step[j] (1 <= ev_step <= n_steps; later ones are
 *              ignored) branch ev_branch[j] goes in service
 *              (ev_in_service[j] = 1) or out (0).
 *   rec_nodes  the n_rec recorded nodes (NULL = all nodes, n_rec = n_nodes).
 *   meas       [2 n_branches] the measured node pairs of CSWITCH branches
 *              (read for CSWITCH only; NULL if there is none).
 *   group, Rm, Lm, Cm  coupled three-phase groups (NULL = none; the
 *              per-component Norton equivalents of Sec. III-A's first basic
 *              process with 3 x 3 blocks): group[b] = g >= 0 puts branch b in
 *              group g, -1 in none. A group is three EMT_RL (series) or
 *              three EMT_C (shunt) branches with equal R, L, C, Rm, Lm, Cm,
 *              line = -1, no events, in service from t = 0, whose R, L or C
 *              matrix is circulant: R, L, C on the diagonal, Rm, Lm, Cm off
 *              it (positive definite: L - Lm > 0, L + 2 Lm > 0, R - Rm >= 0,
 *              R + 2 Rm >= 0; C - Cm > 0, C + 2 Cm > 0). Its trapezoidal
 *              companion is the circulant i = G u + h, h' = B i + Gamma u
 *              (RL: G = (R + 2L/dt)^-1, B = G (2L/dt - R), Gamma = G; C:
 *              G = 2C/dt, B = -I, Gamma = -G). A batch with groups runs
 *              forward only (EMT_EINVAL with checkpoint_every > 0 or with
 *              components split over workgroups); the three phases a group
 *              couples form one component.
 */
typedef struct {
  int32_t n_nodes, n_branches;
  const int32_t *k, *m, *kind;
  const double *R, *L, *C;
  const double *E, *omega, *phase;
  const int32_t *line;
  int32_t n_params;
  const uint8_t *in_service0;
  int32_t n_events;
  const int64_t *ev_step;
  const int32_t *ev_branch;
  const uint8_t *ev_in_service;
  int32_t n_rec;
  const int32_t *rec_nodes;
  const int32_t *group;
  const double *Rm, *Lm, *Cm;
  const int32_t *meas;
} emt_net;

/* Simulation settings shared by all scenarios of a context.
 *   dt > 0, n_steps >= 1 (the horizon T).
 *   checkpoint_every K: 0 = no checkpoints (emt_adjoint unavailable); else
 *     the forward run stores the branch state every K steps and the adjoint
 *     recomputes each K-step segment from its checkpoint.
 *   solver: how each connected component's G v = rhs is solved (Sec. III-A,
 *     fourth basic process). SPARSE: level-scheduled forward/backward sweeps
 *     over the LDL^T factor. DENSE: v = G^{-1} rhs with the component's whole
 *     inverse, formed by emt_factor for every topology; a component of up to
 *     128 nodes keeps it in one workgroup, a larger one (up to 2048 nodes) is
 *     split by columns over ceil(n/split_cols) workgroups that exchange
 *     partial voltages every step (all must be resident at once: EMT_EINVAL
 *     from emt_build otherwise; forward only: EMT_EINVAL with
 *     checkpoint_every > 0). AUTO: sweeps over the leading rows of the
 *     elimination order and the dense inverse of its trailing block, cut
 *     where a cost model finds fewest dependent phases.
 *     COMPENSATION (Sec. III-B's many scenarios of one network, with Sec.
 *     III-A's factorisation done once for all of them; the compensation
 *     itself is not in the paper): the first scenario's components, in
 *     their initial topology, are the base. Every scenario's component is
 *     one of them with at most 4 branches switched differently (in service
 *     or not, or present in one and not the other; branches are matched by
 *     kind, terminals, R, L, C and line). Each base's dense inverse Z =
 *     G0^-1 is formed once by emt_factor and shared: a scenario's solve in
 *     topology t is w = Z rhs followed by the Sherman-Morrison-Woodbury
 *     correction v = w - Z U K U^T w, K = (D^-1 + U^T Z U)^-1 (U: the
 *     switched branches' incidence vectors, D: their conductances, + where
 *     the scenario has the branch in service and the base not, - the
 *     reverse), and a workgroup applies Z to several scenarios' right-hand
 *     sides at once (comp_items). Components of at most 256 nodes and 2048
 *     branches; forward
 *     only (EMT_EINVAL with checkpoint_every > 0, lines, coupled groups or
 *     diodes); every scenario's pi-section parameters must equal the first
 *     scenario's where their branches are matched (emt_factor: EMT_EINVAL).
 *     The result equals the other solvers' up to rounding.
 * Launch shape (0 / -1 = chosen by the library; paper_1903_01081_amd.tune
 * times the alternatives):
 *   block_size: lanes of a one-workgroup component (64, 256 or 512);
 *     EMT_EINVAL if a component's branches or dense tail do not fit.
 *   split_cols: inverse columns per workgroup of a split component (16 or
 *     32; 0 = 32 where the lane state fits, else 16).
 *   dense_tail: AUTO solver only, the dense tail size in nodes (capped by
 *     the block size's limit); -1 = the cost model.
 *   sweep_from_global: 1 = the sweep data (factor values, row descriptors,
 *     node CSR) stay in global memory even where LDS would hold them.
 *   serial_adjoint: 1 = emt_adjoint recomputes and reverses each checkpoint
 *     segment in turn with one workgroup per item; 0 = where both fit on the
 *     device at once, a second workgroup per item recomputes segment s-1
 *     while the first reverses segment s (twice the segment buffer).
 *   split_device_scope: 1 = the workgroups of a split component always
 *     exchange their partial voltages through device-coherent memory; 0 =
 *     through the L2 of their XCD when all of them run on one XCD (the
 *     library places each component on one XCD where its workgroups fit;
 *     they check where they run at the start of every launch). Results are
 *     bitwise the same either way.
 *   pack_nodes: 0 = one work item (workgroup) per connected component; > 0 =
 *     a scenario's components are packed, largest first, into work items of
 *     at most pack_nodes nodes (a larger component stays alone), so small
 *     components share a workgroup and its lanes (their G is block-diagonal
 *     within the item). At most 128 with the dense solver.
 *   comp_items: COMPENSATION only, scenarios' components per workgroup (1 ..
 *     8; 0 = the fewest that keep the workgroups within one per compute
 *     unit); each component runs its branch phase on block_size lanes of
 *     the workgroup (COMPENSATION: 64, 128, 192 or 256; 0 = the fewest
 *     that hold its branches at up to 8 per lane), and a workgroup of
 *     block_size x comp_items lanes (at most 1024, covering the
 *     component's nodes) applies Z to all of its components at once. */
typedef struct {
  double dt;
  int64_t n_steps;
  int32_t checkpoint_every;
  int32_t solver;
  int32_t block_size;
  int32_t split_cols;
  int32_t dense_tail;
  int32_t sweep_from_global;
  int32_t serial_adjoint;
  int32_t split_device_scope;
  int32_t pack_nodes;
  int32_t comp_items;
} emt_sim;

/* Sizes of a built context (emt_info) or of a host-only analysis. */
typedef struct {
  int32_t n_scen;
  int32_t rec_stride;    /* R = max over scenarios of n_rec: rec is [S][n][R] */
  int32_t param_stride;  /* P = max over scenarios of n_params: theta/grad [S][P] */
  int32_t n_items;       /* scenario x connected-component work items */
  int32_t n_symbolic;    /* distinct symbolic factorisations (shared by isomorphic items) */
  int32_t max_item_nodes, max_item_branches;
  int64_t total_nodes, total_branches;
  int64_t nnz_L;         /* strictly-lower nonzeros of L summed over items */
  int32_t max_levels;    /* deepest forward or backward sweep, in levels */
  int32_t max_topologies;
  int64_t step;          /* steps taken so far (built contexts only) */
  int64_t device_bytes;  /* device memory owned by the context */
  int32_t dense_items;   /* items solved entirely by their dense tail inverse */
  int32_t block_size;    /* threads per work item in the step kernels */
  int32_t sweep_levels;  /* barrier-separated solve phases per step (max over items) */
  int32_t max_tail;      /* largest dense tail (nodes) */
  int32_t lds_bytes;     /* LDS per workgroup of the forward step kernel */
  int32_t lds_limit;     /* LDS per workgroup the device allows */
  int32_t lds_staged;    /* 1 if index arrays and factors are staged in LDS */
  int32_t lanes_per_block; /* branches per lane */
  int32_t split_tiles;   /* workgroups of the split dense components (0 if none) */
  int32_t split_cols;    /* inverse columns per split workgroup (16 or 32; 0 if none) */
  int32_t adjoint_pipelined; /* 1 if emt_adjoint overlaps each segment's recompute with
                                the previous segment's reversal (two workgroups per item) */
  int32_t split_local;   /* split components whose last launch exchanged through one XCD's L2
                            (0 before the first step; synchronises the device) */
  int32_t comp_families;   /* COMPENSATION: base components (dense inverses) */
  int32_t comp_max_rank;   /* COMPENSATION: most switched branches of a component and topology */
  int32_t comp_items;      /* COMPENSATION: components per workgroup (built contexts) */
  int32_t comp_blocks;     /* COMPENSATION: workgroups of the step kernel (built contexts) */
} emt_info;

/* Source: Sec. II-A and II-B (a simulation task is a model of connected
 * components plus the task's configuration, here: time step, horizon,
 * switching events, recorded outputs), Sec. III-A (the task is turned into
 * the per-step computations of the four basic processes, ordered in layers)
 * and Sec. III-B (scenarios of one topology run side by side; here also
 * networks of different sizes).
 * Validate, analyse (components, ordering, symbolic LDL^T, sweep levels) and
 * upload n_scen networks; allocates the context on the current HIP device.
 * Companion coefficients are computed from the branch values (no theta).
 * Errors: EMT_EINVAL (any invalid field), EMT_ESINGULAR (a node without a
 * conductive path to ground in some topology), EMT_ENOMEM, EMT_EDEVICE. */
emt_status emt_build(const emt_net *nets, int32_t n_scen, const emt_sim *sim, emt_ctx **out);

/* Source: Sec. III-A (the task parser and the layering of the basic
 * processes), without the upload. Host-only: the validation and analysis of
 * emt_build without any device work (same errors except
 * EMT_ENOMEM/EMT_EDEVICE); fills *info. */
emt_status emt_analyze(const emt_net *nets, int32_t n_scen, const emt_sim *sim, emt_info *info);

/* Not in the paper: sizes and launch shape of a built context (fills *info;
 * EMT_EINVAL on NULL). Synchronises the device when the context has split
 * components (to read where their last launch ran). */
emt_status emt_info_get(const emt_ctx *ctx, emt_info *info);

/* Source: Sec. III-A, first basic process (each component's Norton
 * equivalent conductance and history coefficients, from its parameters).
 * Replace the line parameters of every scenario: theta_dev is device memory
 * [S][P] (P = info.param_stride; entries past a scenario's n_params are
 * ignored). Recomputes the companion coefficients of all topologies on the
 * device, rewinds to step 0 and marks the factors stale (emt_factor next).
 * Values must be positive and finite: R_l >= 0, L_l > 0, C_l > 0 (not
 * checked on the device; a bad value shows up as EMT_ESINGULAR or NaN). */
emt_status emt_set_params(emt_ctx *ctx, const double *theta_dev, void *stream);

/* Source: Sec. III-A, third basic process (factorising the system
 * conductance matrix), done here once per topology that the switching
 * events produce, before the time loop.
 * Numerically factorise G of every topology of every scenario (LDL^T on the
 * shared symbolic pattern; with the COMPENSATION solver also each base's
 * dense inverse and every scenario's K per topology). Starts a run (clears
 * the device error flag) and synchronises `stream` to check the pivots:
 * EMT_ESINGULAR if any pivot is non-positive or not finite (or a K does not
 * exist); EMT_EINVAL if, with the COMPENSATION solver, a scenario's
 * pi-section parameters differ from the first scenario's on matched
 * branches. */
emt_status emt_factor(emt_ctx *ctx, void *stream);

/* Source: Sec. III-A, third basic process, as emt_factor: the same
 * factorisation, queued without waiting:
 * the pivot check is reported by the next emt_sync (EMT_ESINGULAR; the
 * factors are then stale again). For callers that record a whole run
 * (parameters, factorisation, forward, adjoint) into one HIP graph. */
emt_status emt_factor_async(emt_ctx *ctx, void *stream);

/* Source: Sec. III-A, the four basic processes per time step (Norton
 * equivalents, nodal injections, and the forward/back substitution through
 * the prefactored matrix), the layers run in order; Sec. III-B, all
 * scenarios at once. Advance every scenario by n steps from the current
 * step, writing the recorded node voltages to rec_dev [S][n][R] (row j =
 * step current+1+j; columns past a scenario's n_rec are left untouched;
 * rec_dev may be NULL to record nothing). Writes checkpoints when
 * checkpoint_every > 0. Queues the launches on `stream` and returns without
 * waiting for them; a split launch that gave up (EMT_EDEVICE) is reported
 * by the next synchronising call, e.g. emt_sync.
 * Errors: EMT_ESTATE before emt_factor or past n_steps; EMT_EINVAL n < 0. */
emt_status emt_step(emt_ctx *ctx, int64_t n, double *rec_dev, void *stream);

/* Not in the paper. For callers that cannot allocate device memory while
 * they step (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): emt_step with the split components' per-step
 * exchange (partial voltages, give-up flag, XCD record) in the library's
 * static exchange space, a file-scope device array of 2 MiB
 * (EMT_STATIC_SCRATCH_BYTES) that each device holds until the process ends,
 * instead of the context's own exchange buffer. Same arguments, results
 * (bitwise) and stream order as emt_step; it calls no allocating routine.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (other streams, other contexts, other threads) race and must
 * be serialised by the caller. The array keeps the last call's contents;
 * each call re-initialises what it reads (exchange tags, flag, record).
 * The array's device address is looked up once per device, at the first
 * call on that device, which must have the context's device current
 * (EMT_EDEVICE otherwise).
 * Errors: those of emt_step, and EMT_EINVAL if the context's split
 * components need more than EMT_STATIC_SCRATCH_BYTES (e.g. one 1000-node
 * component x 3 phases in 32-column tiles needs 1.5 MB; in 16-column tiles
 * 3 MB). emt_info.split_local does not report calls of this entry point. */
#define EMT_STATIC_SCRATCH_BYTES (2 * 1024 * 1024)
emt_status emt_step_noalloc(emt_ctx *ctx, int64_t n, double *rec_dev, void *stream);

/* Not in the paper: waits for the work queued on `stream` and reports
 * device-side failures of the queued work: EMT_ESINGULAR for non-positive
 * pivots of an emt_factor_async; EMT_EDEVICE if a split launch since the
 * last emt_factor / emt_reset / emt_set_params gave up waiting for its
 * workgroups (its recorded outputs are then not valid) or a pipelined
 * emt_adjoint did (its gradient is then not valid). */
emt_status emt_sync(emt_ctx *ctx, void *stream);

/* Source: Sec. IV-B and IV-C (a simulator is judged by its average time per
 * integration step). Latency floor of a step kernel, a measurement: the time
 * loop here is bound by its chain of dependent phases, not by bandwidth or
 * arithmetic. Runs n_steps steps of a kernel with the step kernel's launch
 * shape but no arithmetic and
 * returns its time per step in microseconds (HIP events on `stream`, which
 * the call synchronises):
 *   EMT_FLOOR_ONE_WORKGROUP: the one-workgroup kernel's grid, workgroup
 *     size and LDS size, each step emt_info.sweep_levels + 2 phases in which
 *     every lane reads a value another lane wrote in the previous phase,
 *     separated by LDS barriers (the gather, the solve passes and the branch
 *     update of a step).
 *   EMT_FLOOR_SPLIT: the split components' kernel with the same tiles and
 *     placement, each step storing its step-tagged partials and reading the
 *     needed nodes' partials until their tags are current, with the same
 *     barriers, but no right-hand side, partial products or branch update.
 * The simulation state and step counter are untouched; a temporary buffer is
 * allocated for the one-workgroup floor. Errors: EMT_EINVAL (no component
 * of that kind, n_steps outside 1 .. 2^30, unknown kernel), EMT_EDEVICE. */
typedef enum { EMT_FLOOR_ONE_WORKGROUP = 0, EMT_FLOOR_SPLIT = 1 } emt_floor_kernel;
emt_status emt_latency_floor(emt_ctx *ctx, int32_t kernel, int64_t n_steps, double *us_per_step, void *stream);

/* Not in the paper (its runs start from rest): return every scenario to
 * step 0 with the zero initial state; starts a run (clears the device error
 * flag, discarding a give-up not yet reported). Stream-ordered. */
emt_status emt_reset(emt_ctx *ctx, void *stream);

/* Not in the paper (its runs start from rest; the sinusoidal steady state is
 * the usual start of an EMTP-type run). Return every scenario to step 0 in
 * the periodic steady state of its initial topology (switches at their
 * initial positions, the coefficients as set by emt_build / emt_set_params)
 * under its sources, which must share one angular frequency w per scenario:
 * with z = exp(j w dt) each branch acts as the discrete admittance
 * y = (g z + gamma) / (z - beta) of its companion recursion, the node
 * phasors solve (A y A^T) V = A y E (E = E exp(j phase) on sources), and the
 * state is v = Re V, u = Re(A^T V - E), i = Re(y u). The recursion started
 * there stays on v_n = Re(V z^n) until the first event. A component without
 * sources rests at zero. One workgroup per component factorises Y on the
 * component's own symbolic pattern (complex LDL^T, allocated at the first
 * call); runs forward only afterwards (emt_adjoint needs a run from rest).
 * Synchronises. Errors: EMT_EINVAL (sources of one scenario at different
 * frequencies; distributed-parameter lines), EMT_ESINGULAR (a zero or
 * non-finite complex pivot), EMT_ENOMEM, EMT_EDEVICE. */
emt_status emt_steady_state(emt_ctx *ctx, void *stream);

/* Not in the paper, which has no gradients: an extension that
 * differentiates the paper's time loop (Sec. III-A) exactly. It is the
 * discrete adjoint of the recursion at the top of this header, with the
 * transposed solves through the factors of emt_factor.
 * Reverse-time adjoint (vector-Jacobian product) of the whole recorded
 * waveform: given dJ_drec_dev [S][T][R] returns grad_dev [S][P] = dJ/dtheta
 * (entries past a scenario's n_params are set to 0). Recomputes each
 * checkpoint segment, then runs transposed solves through the same factors
 * backwards in time; where both fit on the device at once, a second
 * workgroup per component recomputes segment s-1 while segment s is
 * reversed (emt_info.adjoint_pipelined; a give-up of those workgroups is
 * reported by emt_sync as EMT_EDEVICE; while `stream` is being captured
 * into a HIP graph the one-workgroup kernel runs instead). Stream-ordered;
 * bitwise the same gradient either way. dJ_drec_dev may be
 * NULL when no node is recorded (R = 0). Requires checkpoint_every > 0 and a
 * forward run of all n_steps since the last emt_set_params/emt_factor/
 * emt_reset (else EMT_ESTATE); EMT_EINVAL with split dense components.
 * Leaves the forward state at step n_steps. */
emt_status emt_adjoint(emt_ctx *ctx, const double *dJ_drec_dev, double *grad_dev, void *stream);

/* Not in the paper (part of the adjoint extension above): the waveform
 * mismatch of a parameter-identification run. For rec_dev and target_dev
 * [S][T][R] (device), writes dJ_drec_dev [S][T][R] = 2 (rec - target) on
 * each scenario's n_rec recorded columns (0 on the others) and loss_dev [S]
 * = sum over steps and recorded columns of (rec - target)^2, in a fixed
 * order (deterministic). Stream-ordered; rec and dJ_drec may not overlap. */
emt_status emt_mismatch(emt_ctx *ctx, const double *rec_dev, const double *target_dev, double *dJ_drec_dev,
                        double *loss_dev, void *stream);

/* Not in the paper (part of the adjoint extension above).
 * Per-branch adjoints of the companion coefficients from the last
 * emt_adjoint, in the scenario's original branch order (host arrays of
 * n_branches, any may be NULL). Synchronises the device. */
emt_status emt_branch_adjoints(emt_ctx *ctx, int32_t scen, double *gbar, double *betabar,
                               double *gammabar);

/* Source: Sec. III-A (the node voltages of the fourth basic process and the
 * branch currents of the first). Copy one scenario's current state to
 * host: v [n_nodes], i [n_branches] (original branch order; out-of-service
 * branches read 0); either may be NULL. Synchronises the device;
 * EMT_EDEVICE if a split launch of this run gave up. */
emt_status emt_get_state(emt_ctx *ctx, int32_t scen, double *v_host, double *i_host);

/* Not in the paper (its runs start from rest; used for initial states such
 * as a charged lossless L-C tank). Overwrite one scenario's state at the
 * current step from host v and i (u is recomputed as A^T v - e at the
 * current step). Synchronises. */
emt_status emt_set_state(emt_ctx *ctx, int32_t scen, const double *v_host, const double *i_host);

/* Not in the paper: free everything the context owns (NULL-safe).
 * Synchronises the device. */
void emt_destroy(emt_ctx *ctx);

/* Not in the paper: message for the last non-OK status returned on this
 * thread. */
const char *emt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EMT_H */
