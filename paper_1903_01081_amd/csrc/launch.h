// Host-callable launchers of the HIP kernels (step.hip, aux.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "comp.h"
#include "device.h"
#include "emt.h"

namespace emt {

// Sizes that decide an item's LDS footprint in the step kernels.
struct LdsShape {
  int n, d, ns, nbr, nsrc, nsv, nfdesc, nbdesc, nent, nrec;
  int nlev = 0;      // factor levels
  bool dyn = false;  // refactorised inside the loop (diodes, controlled switches)
};

// Launch shape of the step kernels, chosen once per context.
struct KernelShape {
  int bs = 256;    // threads per workgroup (64, 256 or 512)
  int bpt = 1;     // branches per lane (1, 2, 4, 6, 8, 12, 16)
  int wpt = 4;     // tail-inverse entries per lane (4, 16 or 32)
  bool sm = true;  // index arrays and factors staged in LDS
  size_t lds_fwd = 0, lds_adj = 0;
  int dmax = 0;    // largest dense tail this block size supports
  bool ext = false;  // the batch has distributed-parameter lines, coupled groups or diodes
};

struct CompanionArgs {
  const int64_t *coef_base, *br_base;
  const int32_t *nbr_of, *cnt_prefix;
  int total, n_items;
};

size_t lds_bytes(const LdsShape &s, bool sm, bool adjoint);

hipError_t launch_forward_bs64(const DevCtx &, const KernelShape &, const int32_t *, int, int64_t, int64_t,
                               double *, hipStream_t);
hipError_t launch_forward_bs256(const DevCtx &, const KernelShape &, const int32_t *, int, int64_t, int64_t,
                                double *, hipStream_t);
hipError_t launch_forward_bs512(const DevCtx &, const KernelShape &, const int32_t *, int, int64_t, int64_t,
                                double *, hipStream_t);
hipError_t launch_adjoint_bs64(const DevCtx &, const KernelShape &, const int32_t *, int, const double *,
                               hipStream_t);
hipError_t launch_adjoint_bs256(const DevCtx &, const KernelShape &, const int32_t *, int, const double *,
                                hipStream_t);
hipError_t launch_adjoint_bs512(const DevCtx &, const KernelShape &, const int32_t *, int, const double *,
                                hipStream_t);

// Pipelined adjoint (two workgroups per item, cooperative launch) and its
// resident workgroups per compute unit.
hipError_t launch_adjoint_pipe_bs64(const DevCtx &, const KernelShape &, const int32_t *, int, const double *,
                                    int32_t *, hipStream_t);
hipError_t launch_adjoint_pipe_bs256(const DevCtx &, const KernelShape &, const int32_t *, int, const double *,
                                     int32_t *, hipStream_t);
hipError_t launch_adjoint_pipe_bs512(const DevCtx &, const KernelShape &, const int32_t *, int, const double *,
                                     int32_t *, hipStream_t);
hipError_t adjoint_pipe_blocks_per_cu_bs64(const KernelShape &, int *);
hipError_t adjoint_pipe_blocks_per_cu_bs256(const KernelShape &, int *);
hipError_t adjoint_pipe_blocks_per_cu_bs512(const KernelShape &, int *);

hipError_t launch_factor(const DevCtx &c, const int32_t *pairs, int n_pairs, int max_tail, hipStream_t st);
hipError_t launch_companions(const DevCtx &c, const CompanionArgs &a, hipStream_t st);
hipError_t launch_set_params(const DevCtx &c, const double *theta, int P, const int32_t *bscen,
                             int64_t nbr_total, hipStream_t st);
hipError_t launch_reset(const DevCtx &c, const int32_t *bitem, const int32_t *blocal, int64_t nbr_total,
                        int64_t n_nodes_total, int64_t ring_doubles, hipStream_t st);
hipError_t launch_set_state(const DevCtx &c, const int32_t *bitem, const int32_t *blocal,
                            const int64_t *br_ids, int64_t b0, int64_t nb, const double *i_in, int64_t n,
                            hipStream_t st);
hipError_t launch_grad(const DevCtx &c, const int32_t *lptr, const int64_t *lent, const int32_t *line_scen,
                       const int32_t *line_id, int n_lines_total, double *grad, int P, int64_t grad_len,
                       hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);
hipError_t launch_mismatch(const double *rec, const double *target, double *dJ, double *loss, const int32_t *nrec,
                           int n_scen, int64_t T, int R, hipStream_t st);
hipError_t launch_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t st);

// Split dense components (split.hip).
size_t split_lds_bytes(int nn, int bpt, int ne, int nrec, int rt);
hipError_t launch_inverse(const DevCtx &c, const SplitCtx &s, const int32_t *jobs, int n_jobs, size_t lds,
                          hipStream_t st);
hipError_t launch_split(const DevCtx &c, const SplitCtx &s, int bpt, int rpl, int rt, int n_blocks, int64_t n0,
                        int64_t ns, double *rec, size_t lds, bool floor, hipStream_t st);
hipError_t split_blocks_per_cu(int bpt, int rpl, int rt, size_t lds, int *blocks);

// The library's static exchange space (scratch.hip, used by emt_step_noalloc):
// its size and its device address on `device`, which must be the current
// device (read once per device, then cached).
constexpr int64_t kStaticScratchBytes = EMT_STATIC_SCRATCH_BYTES;
hipError_t static_scratch_ptr(int device, void **ptr);
// dst[0] = 1 if src[0] != 0 (one lane; stream-ordered)
// Sinusoidal steady state of every item's initial topology (state at step
// 0); complex factor, pivots and solution in the scratch given, at the
// per-item offsets (in complex entries); bad counts zero pivots.
hipError_t launch_steady(const DevCtx &c, int n_items, const int64_t *off_l, const int64_t *off_n, void *Lc,
                         void *Dc, void *X, int32_t *bad, hipStream_t st);

hipError_t launch_or_flag(int32_t *dst, const int32_t *src, hipStream_t st);

// Compensation solver (comp.hip): lanes and LDS of a step workgroup of q
// items (sb lanes each for their branch phase), the (lanes per item,
// branches per lane, items) shapes that have a kernel, the step launch, and
// the factor work (bases' inverses, parameter check, K per item and topology).
int comp_lanes(int n, int q, int sb);
size_t comp_lds_bytes(int n, int nbr, int q, int ne, int nr, int ns, int sb);
bool comp_shape_exists(int sb, int bpt, int q);
hipError_t launch_comp(const DevCtx &c, const CompCtx &cc, int sb, int bpt, int q, int lanes, int n_blocks,
                       int64_t n0, int64_t ns, double *rec, size_t lds, hipStream_t st);
hipError_t launch_comp_factor(const DevCtx &c, const CompCtx &cc, hipStream_t st);

// Latency floors (floor.hip; the split floor is launch_split with floor set).
hipError_t launch_barrier_floor(int bs, int n_blocks, int phases, int64_t nsteps, size_t lds, double *out,
                                hipStream_t st);

}  // namespace emt
