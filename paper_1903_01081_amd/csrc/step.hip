// Instantiations of the step kernels for one workgroup size (EMT_BS, set by
// the build: 64, 256 or 512), so the three sizes compile in parallel.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "step.h"

#ifndef EMT_BS
#error "EMT_BS must be defined"
#endif

namespace emt {

namespace {

template <int BPT, int WPT, bool SM, bool EXT>
hipError_t fwd(const DevCtx &c, const int32_t *order, int n_items, int64_t n0, int64_t ns, double *rec,
               size_t lds, hipStream_t st) {
  auto k = step::k_forward<EMT_BS, BPT, WPT, SM, EXT>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(n_items), dim3(EMT_BS), lds, st, c, order, n0, ns, rec);
  return hipGetLastError();
}

template <int BPT, int WPT, bool SM>
hipError_t adj(const DevCtx &c, const int32_t *order, int n_items, const double *dJ, size_t lds,
               hipStream_t st) {
  auto k = step::k_adjoint<EMT_BS, BPT, WPT, SM>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(n_items), dim3(EMT_BS), lds, st, c, order, dJ);
  return hipGetLastError();
}

template <int BPT, int WPT, bool SM>
hipError_t adj_pipe(const DevCtx &c, const int32_t *order, int n_items, const double *dJ, int32_t *pipe,
                    size_t lds, hipStream_t st) {
  auto k = step::k_adjoint_pipe<EMT_BS, BPT, WPT, SM>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  DevCtx ca = c;
  const int32_t *oa = order;
  int na = n_items;
  const double *da = dJ;
  int32_t *pa = pipe;
  void *args[] = {&ca, &oa, &na, &da, &pa};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k), dim3(2 * n_items), dim3(EMT_BS), args,
                                    (unsigned)lds, st);
}

template <int BPT, int WPT, bool SM>
hipError_t adj_pipe_occupancy(size_t lds, int *blocks) {
  auto k = step::k_adjoint_pipe<EMT_BS, BPT, WPT, SM>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, reinterpret_cast<const void *>(k), EMT_BS, lds);
}

}  // namespace

#define EMT_CAT2(a, b) a##b
#define EMT_CAT(a, b) EMT_CAT2(a, b)

// Branches per lane x tail-inverse entries per lane: LDS-staged variants for
// every size, global-memory fallbacks for the larger ones.
#define EMT_SHAPES_W(X, W) \
  X(1, W, true) X(2, W, true) X(4, W, true) X(6, W, true) X(8, W, true) X(12, W, true) X(16, W, true) \
  X(4, W, false) X(8, W, false) X(16, W, false)
#if EMT_BS >= 512
#define EMT_SHAPES(X) EMT_SHAPES_W(X, 4) EMT_SHAPES_W(X, 16) EMT_SHAPES_W(X, 32)
#else
#define EMT_SHAPES(X) EMT_SHAPES_W(X, 4) EMT_SHAPES_W(X, 16)
#endif

hipError_t EMT_CAT(launch_forward_bs, EMT_BS)(const DevCtx &c, const KernelShape &ks, const int32_t *order,
                                              int n_items, int64_t n0, int64_t ns, double *rec,
                                              hipStream_t st) {
#define EMT_CASE(BPT, WPT, SM)                                                                      \
  if (ks.bpt == BPT && ks.wpt == WPT && ks.sm == SM)                                                \
    return ks.ext ? fwd<BPT, WPT, SM, true>(c, order, n_items, n0, ns, rec, ks.lds_fwd, st)          \
                  : fwd<BPT, WPT, SM, false>(c, order, n_items, n0, ns, rec, ks.lds_fwd, st);
  EMT_SHAPES(EMT_CASE)
#undef EMT_CASE
  return hipErrorInvalidValue;
}

hipError_t EMT_CAT(launch_adjoint_bs, EMT_BS)(const DevCtx &c, const KernelShape &ks, const int32_t *order,
                                              int n_items, const double *dJ, hipStream_t st) {
#define EMT_CASE(BPT, WPT, SM) \
  if (ks.bpt == BPT && ks.wpt == WPT && ks.sm == SM) return adj<BPT, WPT, SM>(c, order, n_items, dJ, ks.lds_adj, st);
  EMT_SHAPES(EMT_CASE)
#undef EMT_CASE
  return hipErrorInvalidValue;
}

hipError_t EMT_CAT(launch_adjoint_pipe_bs, EMT_BS)(const DevCtx &c, const KernelShape &ks, const int32_t *order,
                                                   int n_items, const double *dJ, int32_t *pipe, hipStream_t st) {
#define EMT_CASE(BPT, WPT, SM) \
  if (ks.bpt == BPT && ks.wpt == WPT && ks.sm == SM) return adj_pipe<BPT, WPT, SM>(c, order, n_items, dJ, pipe, ks.lds_adj, st);
  EMT_SHAPES(EMT_CASE)
#undef EMT_CASE
  return hipErrorInvalidValue;
}

hipError_t EMT_CAT(adjoint_pipe_blocks_per_cu_bs, EMT_BS)(const KernelShape &ks, int *blocks) {
#define EMT_CASE(BPT, WPT, SM) \
  if (ks.bpt == BPT && ks.wpt == WPT && ks.sm == SM) return adj_pipe_occupancy<BPT, WPT, SM>(ks.lds_adj, blocks);
  EMT_SHAPES(EMT_CASE)
#undef EMT_CASE
  return hipErrorInvalidValue;
}

}  // namespace emt
