// Latency floor of the one-workgroup step kernel (a measurement, not part of
// the time loop). The step kernel's time per step is bound by its chain of
// barrier-separated phases (gather, the sweep passes and dense tail, the
// branch update), each reading what other lanes wrote in the one before.
// k_barrier_floor runs that many such phases per step and nothing else:
// every lane reads one value another lane wrote in the previous phase,
// writes one, and the workgroup meets at an LDS barrier. Launched with the
// step kernel's grid, workgroup size and dynamic LDS size, it shares the
// compute units the same way, so its time per step is the floor the step
// kernel's phase structure sets on this device.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "step.h"

namespace emt {

namespace {

template <int BS>
__global__ __launch_bounds__(BS) void k_barrier_floor(int phases, int64_t nsteps, double *out) {
  double *a = reinterpret_cast<double *>(step::emt_lds);
  double *b = a + BS;
  const int tid = threadIdx.x;
  a[tid] = (double)tid;
  step::lds_barrier();
  double acc = 0.0;
  for (int64_t n = 0; n < nsteps; ++n) {
    for (int p = 0; p < phases; ++p) {
      // a value another lane wrote one phase ago, into the other buffer
      const double v = a[(tid + 1 + p) & (BS - 1)];
      b[tid] = v + 1.0;
      acc = acc + v;
      step::lds_barrier();
      double *t = a;
      a = b;
      b = t;
    }
  }
  out[blockIdx.x * BS + tid] = acc;  // keeps the chain live
}

template <int BS>
hipError_t floor_launch(int n_blocks, int phases, int64_t nsteps, size_t lds, double *out, hipStream_t st) {
  auto k = k_barrier_floor<BS>;
  const size_t need = 2 * BS * sizeof(double);
  if (lds < need) lds = need;
  hipError_t e =
      hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(n_blocks), dim3(BS), lds, st, phases, nsteps, out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_barrier_floor(int bs, int n_blocks, int phases, int64_t nsteps, size_t lds, double *out,
                                hipStream_t st) {
  if (n_blocks <= 0 || phases <= 0 || nsteps <= 0) return hipErrorInvalidValue;
  switch (bs) {
    case 64: return floor_launch<64>(n_blocks, phases, nsteps, lds, out, st);
    case 256: return floor_launch<256>(n_blocks, phases, nsteps, lds, out, st);
    case 512: return floor_launch<512>(n_blocks, phases, nsteps, lds, out, st);
    case 128: return floor_launch<128>(n_blocks, phases, nsteps, lds, out, st);
    case 1024: return floor_launch<1024>(n_blocks, phases, nsteps, lds, out, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace emt
