// Device code of the persistent step kernels (forward time loop and
// reverse-time adjoint), FP64, gfx950.
//
// One workgroup owns one work item (a connected component of one scenario)
// for many time steps; scenarios and components are more workgroups of the
// same launch. This is the paper's pair of parallel strategies (Sec. III-B):
// the processes of one layer run together and the layers are replayed in
// order every step; isomorphic scenarios run the same processes side by
// side. A step runs the four basic processes of an EMTP-type solver that the
// paper lists (Sec. III-A) as barrier-separated phases:
//   branch phase  (one branch per lane slot; coefficients and history in
//                 VGPRs): u = A^T v - e and i = g u + h of the previous step,
//                 the next history h = beta i + gamma u, the source EMF e and
//                 the branch injection J = g e - h into LDS;
//   gather        every node sums its incident branch ends' J in a fixed
//                 (CSR) order — a deterministic segmented sum, no atomics;
//   forward       L y = rhs over the leading part of the elimination order,
//                 one pass per level (level 0 needs none), then the dense
//                 tail's reduced right-hand side c = rhs_D - L_DS y_S;
//   tail          x_D = W c, W = (L_DD D_D L_DD^T)^{-1} held in VGPRs;
//   backward      x = D^{-1} y - L^T x, one pass per level.
// In a sweep pass each row is shared by 2^k <= 16 adjacent lanes (k per
// pass, so that a few long rows at the top of the tree use many lanes and
// many short rows one lane each); the lanes' partial sums meet in a fixed
// scan of DPP row shifts, so every run rounds identically.
// All factors of every topology are computed before the loop (k_factor,
// k_tail); a switching event swaps coefficients and factor pointers.
//
// Compiled with -ffp-contract=off so that identical formulas round
// identically in every code path (forward, checkpoint recompute, reload).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"
#include "trig.h"

namespace emt {
namespace step {

constexpr int64_t kNever = INT64_MAX;

__device__ __forceinline__ double gamma_of(uint32_t pk, double g) {
  const uint32_t c = pk >> 30;
  return c == GAMMA_PLUS_G ? g : (c == GAMMA_MINUS_G ? -g : 0.0);
}

__device__ __forceinline__ double source_emf(const DevCtx &c, int64_t gb, int64_t n) {
  const double t = (double)n * c.dt;
  return c.bE[gb] * emf_cos(c.bw[gb] * t + c.bph[gb]);
}

__device__ __forceinline__ int topo_of(const int64_t *topo, int ntopo, int64_t n) {
  int t = 0;
  while (t + 1 < ntopo && topo[t + 1] <= n) ++t;
  return t;
}

// The lane index, hidden from the optimiser at each use so that per-slot
// index and address arithmetic is recomputed inside the time loop (a few
// integer operations) instead of being hoisted out of it and held in VGPRs.
__device__ __forceinline__ int lane_id() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Workgroup barrier that orders LDS only. Lanes of a workgroup exchange
// data only through LDS here; global stores (recorded outputs, checkpoints,
// state) are read by later kernels or by the same lane, so a barrier need
// not wait for them to complete as __syncthreads() would.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Dynamic LDS of the step kernels (addressed with 32-bit offsets so that
// every access compiles to a ds_* instruction).
extern __shared__ __align__(16) char emt_lds[];

// A read-only array either in LDS (32-bit byte offset) or in global memory.
template <class T, bool SM>
struct Ref;
template <class T>
struct Ref<T, true> {
  uint32_t off;
  __device__ __forceinline__ T operator[](int i) const { return reinterpret_cast<const T *>(emt_lds + off)[i]; }
};
template <class T>
struct Ref<T, false> {
  const T *p;
  __device__ __forceinline__ T operator[](int i) const { return p[i]; }
};

// A read-write LDS array.
template <class T>
struct Lds {
  uint32_t off;
  __device__ __forceinline__ T &operator[](int i) const { return reinterpret_cast<T *>(emt_lds + off)[i]; }
};

// Per-workgroup view of an item: sizes, LDS arrays, and the sweep data in
// LDS (SM = true) or global memory.
template <bool SM>
struct View {
  int n, d, ns, nbr, nsrc, nsv, nrec, tpr, wlen;  // nbr: padded to whole lane slots
  int nfpass, nbpass;
  const int32_t *fpass, *bpass;  // (first descriptor, log2 lanes) pairs, global
  Ref<uint64_t, SM> fdesc, bdesc;
  Ref<uint16_t, SM> fcol, brow, bpos, nent, rnode, rcolumn;
  Ref<int32_t, SM> nptr, rptr;
  Lds<double> x, J, cD, dv, sv_s, dinv_s;  // x has n+1 entries, x[n] = 0
  Lds<int32_t> flag;                       // adjoint: a word for broadcasts
  Ref<double, SM> sv, dinv;
  // SM, items refactorised inside the loop: the factorisation's row
  // pointers, level pointers (rows, entries) and level rows
  Lds<int32_t> rf_rowptr, rf_flev, rf_fent_ptr;
  Lds<uint16_t> rf_rows;
};

// Tail rows are split into tpr lanes of contiguous columns: tpr = the
// largest power of two (<= 16, within one DPP row) with d * tpr <= block size.
__device__ __forceinline__ int tail_tpr(int d, int bs) {
  int t = 16;
  while (t > 1 && d * t > bs) t >>= 1;
  return t;
}

template <int BS, class T>
__device__ __forceinline__ void copy_to(uint32_t off, const T *src, int cnt) {
  T *dst = reinterpret_cast<T *>(emt_lds + off);
  for (int q = threadIdx.x; q < cnt; q += BS) dst[q] = src[q];
}

// Copy of int32 values below 65536 into uint16 LDS.
template <int BS>
__device__ __forceinline__ void copy_to_u16(uint32_t off, const int32_t *src, int cnt) {
  uint16_t *dst = reinterpret_cast<uint16_t *>(emt_lds + off);
  for (int q = threadIdx.x; q < cnt; q += BS) dst[q] = (uint16_t)src[q];
}

// LDS layout (byte offsets from emt_lds, each array 16-byte aligned):
// cD, x, J, [dv], then under SM sv, dinv, fdesc, bdesc, nptr, [rptr],
// fcol, brow, bpos, nent, rnode, rcolumn, and for an item with diodes or
// controlled switches rf_rowptr, rf_flev, rf_fent_ptr, rf_rows.
// Must match lds_bytes() on the host.
template <int BS, bool SM>
__device__ View<SM> make_view(const DevCtx &c, const ItemDesc &it, bool adjoint) {
  const SymDesc sd = c.syms[it.sym];
  View<SM> v;
  v.n = it.n;
  v.d = sd.d;
  v.ns = sd.ns;
  v.nbr = it.n_br;
  v.nsrc = it.n_src;
  v.nsv = sd.nsv;
  v.nrec = it.n_rec;
  v.tpr = tail_tpr(sd.d, BS);
  v.wlen = (sd.d + v.tpr - 1) / v.tpr;
  v.nfpass = sd.nfpass;
  v.nbpass = sd.nbpass;
  v.fpass = c.symi + sd.fpass;
  v.bpass = c.symi + sd.bpass;
  const uint64_t *g_fdesc = c.symd + sd.fdesc, *g_bdesc = c.symd + sd.bdesc;
  const uint16_t *g_fcol = c.symh + sd.fcol, *g_brow = c.symh + sd.brow, *g_bpos = c.symh + sd.bpos;
  const int32_t *g_nptr = c.nptr + it.nptr, *g_rptr = c.rptr + it.nptr;
  const uint16_t *g_nent = c.nent + it.nent, *g_rnode = c.rnode + it.rec, *g_rcolumn = c.rcolumn + it.rec;
  const int nent_cnt = g_nptr[v.n];

  uint32_t off = 0;
  auto take = [&off](int cnt, int size) {
    const uint32_t o = off;
    off += ((uint32_t)cnt * (uint32_t)size + 15u) & ~15u;
    return o;
  };
  v.cD.off = take(v.d + 1, 8);
  v.x.off = take(v.n + 1, 8);
  v.J.off = take(v.nbr, 8);
  v.dv.off = take(adjoint ? v.n : 0, 8);
  v.flag.off = take(adjoint ? 1 : 0, 4);
  if (threadIdx.x == 0) {
    v.cD[v.d] = 0.0;  // spare slot read by the last pair of the tail product
    v.x[v.n] = 0.0;   // the ground: every grounded terminal points here
  }
  if constexpr (SM) {
    v.sv_s.off = take(v.nsv, 8);
    v.dinv_s.off = take(v.ns, 8);
    v.fdesc.off = take(sd.nfdesc, 8);
    v.bdesc.off = take(sd.nbdesc, 8);
    v.nptr.off = take(v.n + 1, 4);
    v.rptr.off = take(adjoint ? v.n + 1 : 0, 4);
    v.fcol.off = take(v.nsv, 2);
    v.brow.off = take(v.nsv, 2);
    v.bpos.off = take(v.nsv, 2);
    v.nent.off = take(nent_cnt, 2);
    v.rnode.off = take(v.nrec, 2);
    v.rcolumn.off = take(v.nrec, 2);
    copy_to<BS>(v.fdesc.off, g_fdesc, sd.nfdesc);
    copy_to<BS>(v.bdesc.off, g_bdesc, sd.nbdesc);
    copy_to<BS>(v.nptr.off, g_nptr, v.n + 1);
    if (adjoint) copy_to<BS>(v.rptr.off, g_rptr, v.n + 1);
    copy_to<BS>(v.fcol.off, g_fcol, v.nsv);
    copy_to<BS>(v.brow.off, g_brow, v.nsv);
    copy_to<BS>(v.bpos.off, g_bpos, v.nsv);
    copy_to<BS>(v.nent.off, g_nent, nent_cnt);
    copy_to<BS>(v.rnode.off, g_rnode, v.nrec);
    copy_to<BS>(v.rcolumn.off, g_rcolumn, v.nrec);
    if (it.n_diodes > 0) {
      v.rf_rowptr.off = take(v.n + 1, 4);
      v.rf_flev.off = take(sd.nlev + 1, 4);
      v.rf_fent_ptr.off = take(sd.nlev + 1, 4);
      v.rf_rows.off = take(v.n, 2);
      copy_to<BS>(v.rf_rowptr.off, c.symi + sd.rowptr, v.n + 1);
      copy_to<BS>(v.rf_flev.off, c.symi + sd.flevptr, sd.nlev + 1);
      copy_to<BS>(v.rf_fent_ptr.off, c.symi + sd.fentptr, sd.nlev + 1);
      copy_to_u16<BS>(v.rf_rows.off, c.symi + sd.flevrows, v.n);
    }
    v.sv.off = v.sv_s.off;
    v.dinv.off = v.dinv_s.off;
  } else {
    v.fdesc.p = g_fdesc;
    v.bdesc.p = g_bdesc;
    v.fcol.p = g_fcol;
    v.brow.p = g_brow;
    v.bpos.p = g_bpos;
    v.nptr.p = g_nptr;
    v.rptr.p = g_rptr;
    v.nent.p = g_nent;
    v.rnode.p = g_rnode;
    v.rcolumn.p = g_rcolumn;
  }
  return v;
}

// Factor values and the tail inverse of topology t (sweep values and 1/D in
// LDS under SM; the lane's contiguous share of its tail row of W in VGPRs).
template <int BS, int WPT, bool SM>
__device__ __forceinline__ void select_factor(const DevCtx &c, const ItemDesc &it, View<SM> &v, int t,
                                              double (&w)[WPT]) {
  const double *sv = c.svals + it.sv + (int64_t)t * v.nsv;
  const double *di = c.dinv + it.dfac + (int64_t)t * v.n;
  if constexpr (SM) {
    copy_to<BS>(v.sv_s.off, sv, v.nsv);
    copy_to<BS>(v.dinv_s.off, di, v.ns);
  } else {
    v.sv.p = sv;
    v.dinv.p = di;
  }
  const double *W = c.wtail + it.w + (int64_t)t * v.d * v.d;
  const int tid = lane_id();
  const int row = tid / v.tpr, col0 = (tid % v.tpr) * v.wlen;
#pragma unroll
  for (int q = 0; q < WPT; ++q) {
    const int col = col0 + q;
    w[q] = (row < v.d && q < v.wlen && col < v.d) ? W[row * v.d + col] : 0.0;
  }
}

// Gather: x_r = sum of the signed branch injections at node r (+ dv_r in the
// adjoint), for every node; loads run four entries ahead of the in-order sum.
template <int BS, bool ADJ, bool SM>
__device__ __forceinline__ void gather_all(const View<SM> &v) {
  for (int r = lane_id(); r < v.n; r += BS) {
    double acc = 0.0;
    int e = v.nptr[r];
    const int e1 = v.nptr[r + 1];
    for (; e + 4 <= e1; e += 4) {
      const int n0 = v.nent[e], n1 = v.nent[e + 1], n2 = v.nent[e + 2], n3 = v.nent[e + 3];
      const double j0 = v.J[n0 >> 1], j1 = v.J[n1 >> 1], j2 = v.J[n2 >> 1], j3 = v.J[n3 >> 1];
      acc = (n0 & 1) ? acc - j0 : acc + j0;
      acc = (n1 & 1) ? acc - j1 : acc + j1;
      acc = (n2 & 1) ? acc - j2 : acc + j2;
      acc = (n3 & 1) ? acc - j3 : acc + j3;
    }
    for (; e < e1; ++e) {
      const int ent = v.nent[e];
      const double jv = v.J[ent >> 1];
      acc = (ent & 1) ? acc - jv : acc + jv;
    }
    if (ADJ) acc = acc + v.dv[r];
    v.x[r] = acc;
  }
  lds_barrier();
}

// DPP row_shr:K of a double: lane i receives lane i-K of its 16-lane row
// (0 where that lane is outside the row).
template <int K>
__device__ __forceinline__ double dpp_row_shr(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffu), 0x110 + K, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0x110 + K, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum over an aligned group of 2^lg <= 16 lanes (sub = lane index in the
// group) by an inclusive scan of row shifts: the group's last lane ends
// with the sum, always added in the same order.
__device__ __forceinline__ double group_sum(double s, int lg, int sub) {
  if (lg >= 1) {
    const double t = dpp_row_shr<1>(s);
    if (sub >= 1) s = s + t;
  }
  if (lg >= 2) {
    const double t = dpp_row_shr<2>(s);
    if (sub >= 2) s = s + t;
  }
  if (lg >= 3) {
    const double t = dpp_row_shr<4>(s);
    if (sub >= 4) s = s + t;
  }
  if (lg >= 4) {
    const double t = dpp_row_shr<8>(s);
    if (sub >= 8) s = s + t;
  }
  return s;
}

// One forward pass: for each row descriptor (r, q0, cnt) the row's lanes
// sum sv[q] x[fcol[q]] over their strided entries; out[r - shift] =
// x[r] - sum (out = x for the leading levels, cD with shift ns for the tail
// rows).
template <int BS, bool SM>
__device__ __forceinline__ void forward_pass(const View<SM> &v, int p0, int p1, int lg, uint32_t out_off,
                                             int shift) {
  const int tid = lane_id();
  const int G = 1 << lg, sub = tid & (G - 1);
  for (int p = p0 + (tid >> lg); p < p1; p += (BS >> lg)) {
    const uint64_t dsc = v.fdesc[p];
    const int r = (int)(dsc & 0xFFFF), q0 = (int)((dsc >> 16) & 0xFFFF), cnt = (int)(dsc >> 32);
    const double xr = v.x[r];
    double s = 0.0;
    int q = q0 + sub;
    const int q1 = q0 + cnt;
    for (; q + G < q1; q += 2 * G) {
      const int c0 = v.fcol[q], c1 = v.fcol[q + G];
      const double a0 = v.sv[q], a1 = v.sv[q + G];
      const double x0 = v.x[c0], x1 = v.x[c1];
      s = s + a0 * x0;
      s = s + a1 * x1;
    }
    if (q < q1) s = s + v.sv[q] * v.x[v.fcol[q]];
    s = group_sum(s, lg, sub);
    if (sub == G - 1) reinterpret_cast<double *>(emt_lds + out_off)[r - shift] = xr - s;
  }
  lds_barrier();
}

// One backward pass: x_r = x_r / D_r - sum over the row's column entries of
// sv[bpos[q]] x[brow[q]].
template <int BS, bool SM>
__device__ __forceinline__ void backward_pass(const View<SM> &v, int p0, int p1, int lg) {
  const int tid = lane_id();
  const int G = 1 << lg, sub = tid & (G - 1);
  for (int p = p0 + (tid >> lg); p < p1; p += (BS >> lg)) {
    const uint64_t dsc = v.bdesc[p];
    const int r = (int)(dsc & 0xFFFF), q0 = (int)((dsc >> 16) & 0xFFFF), cnt = (int)(dsc >> 32);
    const double xr = v.x[r] * v.dinv[r];
    double s = 0.0;
    int q = q0 + sub;
    const int q1 = q0 + cnt;
    for (; q + G < q1; q += 2 * G) {
      const int i0 = v.bpos[q], i1 = v.bpos[q + G];
      const int r0 = v.brow[q], r1 = v.brow[q + G];
      const double a0 = v.sv[i0], a1 = v.sv[i1];
      const double x0 = v.x[r0], x1 = v.x[r1];
      s = s + a0 * x0;
      s = s + a1 * x1;
    }
    if (q < q1) s = s + v.sv[v.bpos[q]] * v.x[v.brow[q]];
    s = group_sum(s, lg, sub);
    if (sub == G - 1) v.x[r] = xr - s;
  }
  lds_barrier();
}

// x_D = W c: each tail row is shared by tpr adjacent lanes of one wave, lane
// k owning the contiguous columns [k*wlen, (k+1)*wlen).
template <int BS, int WPT, bool SM>
__device__ __forceinline__ void tail_solve(const View<SM> &v, const double (&w)[WPT]) {
  const int tid = lane_id();
  const int row = tid / v.tpr, col0 = (tid % v.tpr) * v.wlen;
  const double *cD = reinterpret_cast<const double *>(emt_lds + v.cD.off);
  double s = 0.0;
  if (row < v.d) {
    if ((v.wlen & 1) == 0) {
      // pairs: both columns of a pair are < d or both >= d up to the spare
      // slot of cD, whose product with a zero W entry is zero
#pragma unroll
      for (int q = 0; q < WPT; q += 2) {
        if (q < v.wlen && col0 + q < v.d) {
          const double2 cc = *reinterpret_cast<const double2 *>(cD + col0 + q);
          s = s + w[q] * cc.x;
          s = s + w[q + 1] * cc.y;
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < WPT; ++q)
        if (q < v.wlen && col0 + q < v.d) s = s + w[q] * cD[col0 + q];
    }
  }
  int lg = 0;
  while ((1 << lg) < v.tpr) ++lg;
  const int sub = tid % v.tpr;
  s = group_sum(s, lg, sub);
  if (row < v.d && sub == v.tpr - 1) v.x[v.ns + row] = s;
  lds_barrier();
}

// The solve after the gather: forward passes, tail, backward passes.
template <int BS, int WPT, bool SM>
__device__ __forceinline__ void solve_after_gather(const View<SM> &v, const double (&w)[WPT]) {
  for (int k = 0; k < v.nfpass; ++k) {
    const int p0 = v.fpass[2 * k], lg = v.fpass[2 * k + 1], p1 = v.fpass[2 * k + 2];
    // the last forward pass of an item with a dense tail is the tail rows'
    const bool tail_rows = v.d > 0 && k == v.nfpass - 1;
    forward_pass<BS, SM>(v, p0, p1, lg, tail_rows ? v.cD.off : v.x.off, tail_rows ? v.ns : 0);
  }
  if (v.d > 0) tail_solve<BS, WPT, SM>(v, w);
  for (int k = 0; k < v.nbpass; ++k) {
    const int p0 = v.bpass[2 * k], lg = v.bpass[2 * k + 1], p1 = v.bpass[2 * k + 2];
    backward_pass<BS, SM>(v, p0, p1, lg);
  }
}

// Lane state of the forward loop: coefficients of the current topology for
// each slot (branches padded to whole slots with inert ones, so every slot
// is valid) and the history current of slot 0. The history of the other
// slots lives in LDS as their injection: a slot j > 0 carries no source, so
// J = -h there exactly and h = -J is read back where it is needed.
template <int BPT>
struct Lane {
  double g[BPT], be[BPT], h0;
  uint32_t pk[BPT];
  // the source of slot 0 (sources are numbered first and fit in one slot):
  // EMF parameters and the EMF of the current step
  double sE, sw, sph, e0;
};

template <int BS, int BPT>
__device__ __forceinline__ void load_lane(const DevCtx &c, const ItemDesc &it, Lane<BPT> &L) {
#pragma unroll
  for (int j = 0; j < BPT; ++j) L.pk[j] = c.bpack[it.br + threadIdx.x + j * BS];
  const int b0 = threadIdx.x;
  const bool src = b0 < it.n_src;
  L.sE = src ? c.bE[it.br + b0] : 0.0;
  L.sw = src ? c.bw[it.br + b0] : 0.0;
  L.sph = src ? c.bph[it.br + b0] : 0.0;
  L.e0 = 0.0;
}

template <int BS, int BPT>
__device__ __forceinline__ void load_coefs(const DevCtx &c, const ItemDesc &it, int t, double (&g)[BPT],
                                           double (&be)[BPT]) {
  const int64_t base = it.coef + (int64_t)t * it.n_br;
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    g[j] = c.cg[base + threadIdx.x + j * BS];
    be[j] = c.cb[base + threadIdx.x + j * BS];
  }
}

// History current h = beta*i + gamma*u from a stored state (i, u).
// History of the next step from a stored state (i, u): slot 0 into L.h0,
// the other slots straight into their injections J = -h.
template <int BS, int BPT, bool SM>
__device__ __forceinline__ void history_from_state(const double *si, const double *su, Lane<BPT> &L,
                                                   const View<SM> &v) {
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int b = threadIdx.x + j * BS;
    const double h = L.be[j] * si[b] + gamma_of(L.pk[j], L.g[j]) * su[b];
    if (j == 0)
      L.h0 = h;
    else
      v.J[b] = -h;
  }
}

// EMF of step n for the lane's slot-0 branch (0 if it is not a source).
template <int BPT>
__device__ __forceinline__ double slot0_emf(const DevCtx &c, const Lane<BPT> &L, int tid, int nsrc, int64_t n) {
  return tid < nsrc ? L.sE * emf_cos(L.sw * ((double)n * c.dt) + L.sph) : 0.0;
}

// Slot 0's injection of step n: J = g e - h (the other slots' injections
// were written with their history).
template <int BS, int BPT, bool SM>
__device__ __forceinline__ void inject(const DevCtx &c, const View<SM> &v, Lane<BPT> &L, int64_t n) {
  const int tid = lane_id();
  L.e0 = slot0_emf<BPT>(c, L, tid, v.nsrc, n);
  v.J[tid] = L.g[0] * L.e0 - L.h0;
}

// Branch phase after the solve of step n: u, i of step n with the current
// coefficients; optional stores of (i, u) to up to two places (null = none);
// if step n+1 starts a new topology its coefficients are loaded; the history
// of step n+1; and, when inj is set, the injections of step n+1.
template <int BS, int BPT, bool SM, bool PASS = false>
__device__ __forceinline__ void update_inject(const DevCtx &c, const View<SM> &v, Lane<BPT> &L, double *st_i,
                                              double *st_u, double *st2_i, double *st2_u, bool switch_next,
                                              int64_t next_coef, bool inj, int64_t n) {
  const int tid = lane_id();
  const double e_next = inj ? slot0_emf<BPT>(c, L, tid, v.nsrc, n + 1) : 0.0;
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int b = tid + j * BS;
    const uint32_t pk = L.pk[j];
    // a line end's or a coupled member's history is its injection in every
    // slot (no source there), and a pass after this update, not the update,
    // writes its next injection and its stored state (PASS: the batch has
    // such branches; the kernels of other batches carry none of this)
    const bool line = PASS && (pk >> 30) == GAMMA_PASS;
    const double vk = v.x[pk & kTermGround], vm = v.x[(pk >> 15) & kTermGround];
    const double e = j == 0 ? L.e0 : 0.0;
    const double h = (j == 0 && !line) ? L.h0 : -v.J[b];
    const double u = (L.g[j] != 0.0) ? (vk - vm) - e : 0.0;
    const double i = L.g[j] * u + h;
    if (st_i && !line) {
      st_i[b] = i;
      st_u[b] = u;
    }
    if (st2_i && !line) {
      st2_i[b] = i;
      st2_u[b] = u;
    }
    if (switch_next) {
      L.g[j] = c.cg[next_coef + b];
      L.be[j] = c.cb[next_coef + b];
    }
    const double hn = L.be[j] * i + gamma_of(pk, L.g[j]) * u;
    if (j == 0) {
      L.h0 = hn;
      if (inj && !line) v.J[b] = L.g[j] * e_next - hn;
    } else if (inj && !line) {
      v.J[b] = -hn;
    }
  }
  L.e0 = e_next;
}

// Distributed-parameter lines, one lane per line. Each end is a Norton
// equivalent to ground (1/Z) whose history current is the wave that left the
// other end tau = (D0 + f) dt earlier: h_k(n) = -[(1 - f) w_m(n - D0) +
// f w_m(n - D0 - 1)], w = g v + i, i = g v + h, w = 0 up to step 0 (the line
// starts at rest). With advance set, the waves of step n are formed from the
// solution (v.x) and the ends' injections J = -h of step n, stored, and the
// injections of step n + 1 written; otherwise only those of step n.
template <int BS, bool SM>
__device__ __forceinline__ void line_pass(const DevCtx &c, const ItemDesc &it, const View<SM> &v, int64_t n,
                                          bool advance, double *st_i, double *st_u) {
  for (int q = lane_id(); q < it.n_lines; q += BS) {
    const LineDesc ld = c.line_tab[it.lines + q];
    const double g = c.line_gf[2 * (it.lines + q)], f = c.line_gf[2 * (it.lines + q) + 1];
    double *rk = c.ring + ld.ring, *rm = rk + (ld.mask + 1);
    int64_t m = n;
    if (advance) {
      const double vk = v.x[ld.nk], vm = v.x[ld.nm];
      const double ik = g * vk - v.J[ld.bk], im = g * vm - v.J[ld.bm];
      rk[n & ld.mask] = g * vk + ik;
      rm[n & ld.mask] = g * vm + im;
      if (st_i) {  // each end's current into the line and its voltage
        st_i[ld.bk] = ik;
        st_u[ld.bk] = vk;
        st_i[ld.bm] = im;
        st_u[ld.bm] = vm;
      }
      m = n + 1;
    }
    const int64_t j0 = m - ld.d0, j1 = j0 - 1;
    const double k0 = j0 > 0 ? rk[j0 & ld.mask] : 0.0, k1 = j1 > 0 ? rk[j1 & ld.mask] : 0.0;
    const double m0 = j0 > 0 ? rm[j0 & ld.mask] : 0.0, m1 = j1 > 0 ? rm[j1 & ld.mask] : 0.0;
    v.J[ld.bk] = (1.0 - f) * m0 + f * m1;
    v.J[ld.bm] = (1.0 - f) * k0 + f * k1;
  }
}

// Coupled three-phase groups, one lane per group. A member's current and
// history involve all three members through the circulant companion: with
// the group sums S_u, S_i,
//   i_p  = g u_p + g_o (S_u - u_p) + h_p,
//   h'_p = beta i_p + sgn g u_p + beta_o (S_i - i_p) + sgn g_o (S_u - u_p),
// sgn = +1 for R-L and -1 for C groups. Members carry no source (u = v_k -
// v_m); the branch update leaves their injections and stored state to this
// pass, which reads h_p = -J and writes J = -h'_p (when inj) and the state
// (when st_i is set). With init, (i, u) are the stored state instead (the
// start of a launch) and only the injections are written. The members take
// no events, so the coefficients of topology 0 hold in every topology.
template <int BS, bool SM>
__device__ __forceinline__ void group_pass(const DevCtx &c, const ItemDesc &it, const View<SM> &v, bool init,
                                           bool inj, double *st_i, double *st_u) {
  for (int q = lane_id(); q < it.n_groups; q += BS) {
    const GroupDesc gd = c.group_tab[it.groups + q];
    const int64_t k0 = it.coef + gd.b[0];
    const double g = c.cg[k0], go = c.cgo[k0], be = c.cb[k0], bo = c.cbo[k0];
    const double sg = (double)gd.sgn;
    double u[3], i[3];
    if (init) {
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        u[p] = c.su[it.br + gd.b[p]];
        i[p] = c.si[it.br + gd.b[p]];
      }
    } else {
#pragma unroll
      for (int p = 0; p < 3; ++p) u[p] = v.x[gd.k[p]] - v.x[gd.m[p]];
      const double su = u[0] + u[1] + u[2];
#pragma unroll
      for (int p = 0; p < 3; ++p) i[p] = (g * u[p] - v.J[gd.b[p]]) + go * (su - u[p]);
      if (st_i) {
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          st_i[gd.b[p]] = i[p];
          st_u[gd.b[p]] = u[p];
        }
      }
    }
    if (init || inj) {
      const double su = u[0] + u[1] + u[2], si = i[0] + i[1] + i[2];
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        const double h = (be * i[p] + sg * g * u[p]) + (bo * (si - i[p]) + sg * go * (su - u[p]));
        v.J[gd.b[p]] = -h;
      }
    }
  }
}

// Ideal diodes (state-dependent switches). A diode is a resistive branch
// whose conductance is 1/R_on while it conducts and 0 while it blocks; its
// state lives in c.dstate and changes after a step (a conducting diode whose
// current g u went negative blocks, a blocking one whose voltage v_k - v_m
// went positive conducts), taking effect from the next step. dmask marks a
// lane's diode and controlled-switch slots, cmask the latter: a controlled
// switch's hysteresis comparator measures s = v_a - v_b of step n against
// its reference r = E cos(omega n dt + phase) + C and, with e = r - s,
// conducts from the next step if e > h, opens if e < -h, else keeps its
// state (h in the branch's L). Returns the slots that change; their new
// state is stored at once, their conductance only after the branch update
// of this step (which still uses the old one).
template <int BS, int BPT, bool SM>
__device__ __forceinline__ uint32_t diode_flips(const DevCtx &c, const ItemDesc &it, const View<SM> &v,
                                                const Lane<BPT> &L, uint32_t dmask, uint32_t cmask, int64_t n) {
  uint32_t fl = 0;
  const int tid = lane_id();
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    if (!((dmask >> j) & 1u)) continue;
    const bool on = L.g[j] != 0.0;
    bool next;
    if ((cmask >> j) & 1u) {
      const int64_t gb = it.br + tid + j * BS;
      const double s = v.x[c.bmeas[2 * gb]] - v.x[c.bmeas[2 * gb + 1]];
      const double r = c.bE[gb] * emf_cos(c.bw[gb] * ((double)n * c.dt) + c.bph[gb]) + c.bC[gb];
      const double e = r - s, h = c.bL[gb];
      next = e > h ? true : (e < -h ? false : on);
    } else {
      const uint32_t pk = L.pk[j];
      const double du = v.x[pk & kTermGround] - v.x[(pk >> 15) & kTermGround];
      next = on ? !(L.g[j] * du < 0.0) : (du > 0.0);
    }
    if (next != on) {
      fl |= 1u << j;
      c.dstate[it.br + tid + j * BS] = next ? 1 : 0;
    }
  }
  return fl;
}

// The diode slots' conductances from their stored state.
template <int BS, int BPT>
__device__ __forceinline__ void diode_conductances(const DevCtx &c, const ItemDesc &it, Lane<BPT> &L,
                                                   uint32_t dmask) {
  const int tid = lane_id();
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    if (!((dmask >> j) & 1u)) continue;
    const int64_t gb = it.br + tid + j * BS;
    L.g[j] = c.dstate[gb] ? 1.0 / c.bR[gb] : 0.0;
    L.be[j] = 0.0;
  }
}

// A workgroup barrier for data in LDS (SM) or in global memory.
template <bool SM>
__device__ __forceinline__ void wg_sync() {
  if constexpr (SM)
    lds_barrier();
  else
    __syncthreads();
}

// log2 of the lanes that share one row or entry of a factorisation level
// with cnt of them: as many as fill the workgroup, at most 16 (one DPP row).
template <int BS>
__device__ __forceinline__ int team_log2(int cnt) {
  int lg = 0;
  while (lg < 4 && (cnt << (lg + 1)) <= BS) ++lg;
  return lg;
}

// A lane's first entry of a factorisation level: its CSR position and the
// range of its share of the entry's update pairs (start already offset by
// the lane's index in its team), fetched one level ahead, and its first
// PC pairs, fetched at the start of the level, so that neither global
// load waits inside the level. Pairs are read PC at a time.
template <int PC>
struct LevelEntry {
  int p, pos, r, r1, lg;
  uint32_t pr[PC];
};

template <int BS, int PC, class LV>
__device__ __forceinline__ LevelEntry<PC> first_entry(const LV &fent_ptr, int l, const int32_t *rent) {
  const int e0 = fent_ptr[l], e1 = fent_ptr[l + 1];
  LevelEntry<PC> f;
  f.lg = team_log2<BS>(e1 - e0);
  f.p = e0 + ((int)threadIdx.x >> f.lg);
  f.pos = 0;
  f.r = f.r1 = 0;
  if (f.p < e1) {
    f.pos = rent[2 * f.p];
    f.r = rent[2 * f.p + 1] + ((int)threadIdx.x & ((1 << f.lg) - 1));
    f.r1 = rent[2 * f.p + 3];
  }
  return f;
}

template <int PC>
__device__ __forceinline__ void load_pairs(uint32_t (&pr)[PC], const uint32_t *rpair, int r, int r1, int g) {
#pragma unroll
  for (int u = 0; u < PC; ++u) pr[u] = (r + u * g < r1) ? rpair[r + u * g] : 0u;
}

// LDL^T of the assembled G (D and Lr hold its diagonal and strictly lower
// entries on entry) by the factorisation's levels; the columns of one
// elimination-tree level depend only on lower levels:
//   D_j  = G_jj - sum_{k<j} L_jk^2 D_k
//   L_ij = (G_ij - sum_{k<j} L_ik D_k L_jk) / D_j
// Each row (first phase) and each entry (second phase) of a level is shared
// by a team of 2^lg adjacent lanes, lg from the level's width: the top of
// the elimination tree is a chain of one-row levels with long rows, which
// one lane per row would walk serially. An entry's terms come from its list
// of update pairs (the CSR positions of L_ik and L_jk for every common
// column k, precomputed on the host), so no lane searches the two rows; the
// team's partial sums meet in a fixed DPP scan. The structure comes through
// accessors (LDS copies or global arrays): row pointers and columns of L by
// rows, per level its rows and the range of its entries. Non-positive
// pivots are counted in *bad.
template <int BS, bool SM, int PC, class RP, class LV, class RW, class RC>
__device__ __forceinline__ void ldl_levels(int nlev, const RP &rowptr, const LV &flev, const RW &rows,
                                           const LV &fent_ptr, const RC &rowcol, const int32_t *rent,
                                           const uint32_t *rpair, double *Lr, double *D, int32_t *bad) {
  const int tid = (int)threadIdx.x;
  LevelEntry<PC> next = first_entry<BS, PC>(fent_ptr, 0, rent);
  for (int l = 0; l < nlev; ++l) {
    LevelEntry<PC> cur = next;
    load_pairs(cur.pr, rpair, cur.r, cur.r1, 1 << cur.lg);
    if (l + 1 < nlev) next = first_entry<BS, PC>(fent_ptr, l + 1, rent);
    {
      const int p0 = flev[l], p1 = flev[l + 1];
      const int lg = team_log2<BS>(p1 - p0), g = 1 << lg, sub = tid & (g - 1);
      for (int p = p0 + (tid >> lg); p < p1; p += BS >> lg) {
        const int j = rows[p];
        const int q1 = rowptr[j + 1];
        double acc = 0.0;
        for (int q = rowptr[j] + sub; q < q1; q += g) {
          const double ljk = Lr[q];
          acc = acc + ljk * ljk * D[rowcol[q]];
        }
        acc = group_sum(acc, lg, sub);
        if (sub == g - 1) {
          const double d = D[j] - acc;
          D[j] = d;
          if (!(d > 0.0) || !isfinite(d)) atomicAdd(bad, 1);
        }
      }
    }
    wg_sync<SM>();
    {
      const int p1 = fent_ptr[l + 1];
      const int lg = team_log2<BS>(p1 - fent_ptr[l]), g = 1 << lg, sub = tid & (g - 1);
      for (int p = cur.p; p < p1; p += BS >> lg) {
        int pos = cur.pos, r = cur.r, r1 = cur.r1;
        uint32_t pr[PC];
#pragma unroll
        for (int u = 0; u < PC; ++u) pr[u] = cur.pr[u];
        if (p != cur.p) {
          pos = rent[2 * p];
          r = rent[2 * p + 1] + sub;
          r1 = rent[2 * p + 3];
          load_pairs(pr, rpair, r, r1, g);
        }
        double acc = 0.0;
        while (r < r1) {
#pragma unroll
          for (int u = 0; u < PC; ++u) {
            if (r + u * g < r1) {
              const int qi = (int)(pr[u] & 0xFFFFu), qj = (int)(pr[u] >> 16);
              acc = acc + Lr[qi] * D[rowcol[qj]] * Lr[qj];
            }
          }
          r += PC * g;
          if (r < r1) load_pairs(pr, rpair, r, r1, g);
        }
        acc = group_sum(acc, lg, sub);
        if (sub == g - 1) Lr[pos] = (Lr[pos] - acc) / D[rowcol[pos]];
      }
    }
    wg_sync<SM>();
  }
}

// The factor of an item with diodes for its current conductances (the
// lanes' L.g), computed inside the time loop into the item's dynamic slot:
// G on the item's symbolic pattern (with any coupled groups' mutual
// stamps), LDL^T by the factorisation's levels (the same arithmetic as the
// factorisation before the loop), then the sweep values and 1/D, which the
// sweeps then read (staged into LDS under SM). Such items have no dense
// tail. Non-positive pivots are counted in c.flags[4].
template <int BS, int BPT, bool SM>
__device__ void refactor_dynamic(const DevCtx &c, const ItemDesc &it, View<SM> &v, const Lane<BPT> &L) {
  const SymDesc sd = c.syms[it.sym];
  const int n = it.n;
  double *gcur = c.dyn + it.dyn;
  // Under SM the factorisation runs in LDS: without a dense tail the sweep
  // values are exactly L's nonzeros in row order (sv index = CSR position),
  // so L is built in place in the staged sweep values and D in the staged
  // 1/D, which is inverted at the end; the structure is read from LDS too
  // (the sweeps' column, row and position arrays are then L's by rows and
  // by columns). Otherwise in the dynamic slot in global memory.
  double *Lr, *D;
  if constexpr (SM) {
    Lr = reinterpret_cast<double *>(emt_lds + v.sv_s.off);
    D = reinterpret_cast<double *>(emt_lds + v.dinv_s.off);
  } else {
    Lr = gcur + it.n_br;
    D = Lr + sd.nnz;
  }
  double *sv = gcur + it.n_br + sd.nnz + n;
  double *di = sv + sd.nsv;
  const int32_t *g_rowptr = c.symi + sd.rowptr;
  const int32_t *bk = c.bk + it.br, *bm = c.bm + it.br, *gpos = c.bgpos + it.br;
  const int tid = lane_id();
#pragma unroll
  for (int j = 0; j < BPT; ++j) gcur[tid + j * BS] = L.g[j];
  __syncthreads();
  for (int r = threadIdx.x; r < n; r += BS) {
    int q0, q1;
    if constexpr (SM) {
      q0 = v.rf_rowptr[r];
      q1 = v.rf_rowptr[r + 1];
    } else {
      q0 = g_rowptr[r];
      q1 = g_rowptr[r + 1];
    }
    for (int q = q0; q < q1; ++q) Lr[q] = 0.0;
    double d = 0.0;
    const int e1 = v.nptr[r + 1];
    for (int e = v.nptr[r]; e < e1; ++e) {
      const int ent = v.nent[e];
      const int b = ent >> 1;
      const double gv = gcur[b];
      d = d + gv;
      const int other = (ent & 1) ? bk[b] : bm[b];
      if (other >= 0 && other < r) Lr[gpos[b]] = Lr[gpos[b]] - gv;
    }
    D[r] = d;
    if (it.n_groups > 0) {
      const int32_t *mp = c.mptr + it.mptr;
      const int32_t *me = c.ment + it.ment;
      const double *go = c.cgo + it.coef;
      for (int e = mp[r]; e < mp[r + 1]; ++e) {
        const int pos = me[2 * e], code = me[2 * e + 1];
        const double gv = go[code >> 1];
        Lr[pos] = (code & 1) ? Lr[pos] - gv : Lr[pos] + gv;
      }
    }
  }
  wg_sync<SM>();
  constexpr int kPC = 2;  // pairs per load round (more measured no faster)
  const int32_t *rent = c.symi + sd.rent;
  const uint32_t *rpair = reinterpret_cast<const uint32_t *>(c.symi + sd.rpair);
  if constexpr (SM) {
    ldl_levels<BS, SM, kPC>(sd.nlev, v.rf_rowptr, v.rf_flev, v.rf_rows, v.rf_fent_ptr, v.fcol, rent, rpair, Lr, D,
                       c.flags + 4);
    (void)sv;
    (void)di;
    for (int r = threadIdx.x; r < n; r += BS) D[r] = 1.0 / D[r];
    lds_barrier();
  } else {
    const int32_t *rowcol = c.symi + sd.rowcol;
    const int32_t *flevptr = c.symi + sd.flevptr, *flevrows = c.symi + sd.flevrows;
    const int32_t *fentptr = c.symi + sd.fentptr;
    const int32_t *svmap = c.symi + sd.svmap;
    ldl_levels<BS, SM, kPC>(sd.nlev, g_rowptr, flevptr, flevrows, fentptr, rowcol, rent, rpair, Lr, D, c.flags + 4);
    for (int q = threadIdx.x; q < sd.nsv; q += BS) sv[q] = Lr[svmap[q]];
    for (int r = threadIdx.x; r < n; r += BS) di[r] = 1.0 / D[r];
    __syncthreads();
    v.sv.p = sv;
    v.dinv.p = di;
  }
}

// ---------------------------------------------------------------------------
// Forward loop: steps n0+1 .. n0+nsteps for every item.
// ---------------------------------------------------------------------------
// EXT: the batch has distributed-parameter lines, coupled groups or diodes
// (the variant without them carries none of their code or registers).
template <int BS, int BPT, int WPT, bool SM, bool EXT>
__global__ __launch_bounds__(BS) void k_forward(DevCtx c, const int32_t *order, int64_t n0, int64_t nsteps,
                                                double *rec) {
  const ItemDesc it = c.items[order[blockIdx.x]];
  View<SM> v = make_view<BS, SM>(c, it, false);
  const int64_t *topo = c.topo + it.topo;
  int t = topo_of(topo, it.n_topo, n0 + 1);
  int64_t next = (t + 1 < it.n_topo) ? topo[t + 1] : kNever;
  Lane<BPT> L;
  double w[WPT];
  load_lane<BS, BPT>(c, it, L);
  load_coefs<BS, BPT>(c, it, t, L.g, L.be);
  const bool diodes = EXT && it.n_diodes > 0;  // diodes or controlled switches
  uint32_t dmask = 0, cmask = 0;
  if (diodes) {
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int kd = c.bkind[it.br + threadIdx.x + j * BS];
      if (kd == KIND_DIODE || kd == KIND_CSWITCH) dmask |= 1u << j;
      if (kd == KIND_CSWITCH) cmask |= 1u << j;
    }
    diode_conductances<BS, BPT>(c, it, L, dmask);
  }
  history_from_state<BS, BPT, SM>(c.si + it.br, c.su + it.br, L, v);
  if (diodes) {
    // no dense tail: w stays zero
#pragma unroll
    for (int q = 0; q < WPT; ++q) w[q] = 0.0;
    refactor_dynamic<BS, BPT, SM>(c, it, v, L);
  } else {
    select_factor<BS, WPT, SM>(c, it, v, t, w);
  }
  inject<BS, BPT, SM>(c, v, L, n0 + 1);
  lds_barrier();
  const bool lines = EXT && it.n_lines > 0, groups = EXT && it.n_groups > 0;
  if (lines || groups) {
    if (lines) line_pass<BS, SM>(c, it, v, n0 + 1, false, nullptr, nullptr);
    if (groups) group_pass<BS, SM>(c, it, v, true, true, nullptr, nullptr);
    lds_barrier();
  }
  const int R = c.rec_stride;
  const int64_t n_end = n0 + nsteps;
  for (int64_t n = n0 + 1; n <= n_end; ++n) {
    gather_all<BS, false, SM>(v);
    solve_after_gather<BS, WPT, SM>(v, w);
    if (rec) {
      double *row = rec + ((int64_t)it.scen * nsteps + (n - n0 - 1)) * R;
      for (int q = lane_id(); q < v.nrec; q += BS) row[v.rcolumn[q]] = v.x[v.rnode[q]];
    }
    const bool sw = (n + 1 == next);
    const uint32_t fl = diodes ? diode_flips<BS, BPT, SM>(c, it, v, L, dmask, cmask, n) : 0u;
    double *ck_i = nullptr, *ck_u = nullptr, *st_i = nullptr, *st_u = nullptr;
    if (c.K > 0 && n % c.K == 0) {
      const int64_t o = it.ck + (n / c.K) * (int64_t)v.nbr;
      ck_i = c.ck_i + o;
      ck_u = c.ck_u + o;
    }
    if (n == n_end) {
      st_i = c.si + it.br;
      st_u = c.su + it.br;
    }
    update_inject<BS, BPT, SM, EXT>(c, v, L, ck_i, ck_u, st_i, st_u, sw, it.coef + (int64_t)(t + 1) * v.nbr,
                               n < n_end, n);
    if (lines || groups) {
      lds_barrier();
      if (lines) line_pass<BS, SM>(c, it, v, n, true, st_i, st_u);
      if (groups) group_pass<BS, SM>(c, it, v, false, n < n_end, st_i, st_u);
    }
    if (diodes) {
      // a diode changed state or the topology switched: the conductances
      // of step n+1 and their factor, inside the loop
      if (__syncthreads_or(fl != 0u) || sw) {
        diode_conductances<BS, BPT>(c, it, L, dmask);
        refactor_dynamic<BS, BPT, SM>(c, it, v, L);
      }
    }
    if (sw) {
      ++t;
      next = (t + 1 < it.n_topo) ? topo[t + 1] : kNever;
      if (!diodes) select_factor<BS, WPT, SM>(c, it, v, t, w);
    }
    lds_barrier();
  }
  for (int q = threadIdx.x; q < v.n; q += BS) c.sv_state[it.node + q] = v.x[q];
}

// ---------------------------------------------------------------------------
// Reverse-time adjoint over the whole horizon, one workgroup per item. For
// each checkpoint segment (last first): recompute its forward steps from the
// checkpoint into the segment buffer, then run the discrete adjoint of the
// step backwards:
//   ibar = beta_{n+1} hbar_{n+1};  q = gamma_{n+1} hbar_{n+1} + g_n ibar
//   vbar = dJ/dv_n + A q;          w = G_n^{-T} vbar (G symmetric: same solve)
//   hbar_n = ibar - A^T w
//   gbar += hbar_n u_n, betabar += hbar_n i_{n-1}, gammabar += hbar_n u_{n-1}
// ---------------------------------------------------------------------------
// Runs f(j, g_nx, be_nx) for every slot with the coefficients of step n+1:
// those of step n (in L) unless a switching event lies between the two
// steps (t_nx != t, uniform over the workgroup), then reloaded. Two fully
// unrolled loops, so every slot index is a constant.
template <int BS, int BPT, class F>
__device__ __forceinline__ void with_next_coefs(const DevCtx &c, const ItemDesc &it, const Lane<BPT> &L, int t,
                                                int t_nx, F &&f) {
  if (t_nx == t) {
#pragma unroll
    for (int j = 0; j < BPT; ++j) f(j, L.g[j], L.be[j]);
  } else {
    const int64_t o = it.coef + (int64_t)t_nx * it.n_br + lane_id();
#pragma unroll
    for (int j = 0; j < BPT; ++j) f(j, c.cg[o + j * BS], c.cb[o + j * BS]);
  }
}

template <int BS, int BPT, bool SM>
__device__ __forceinline__ void adjoint_seed(const DevCtx &c, const ItemDesc &it, const View<SM> &v,
                                             const Lane<BPT> &L, int t, int t_nx, const double (&hb_nx)[BPT],
                                             const double *dJ, int64_t n) {
  const int tid = lane_id();
  with_next_coefs<BS, BPT>(c, it, L, t, t_nx, [&](int j, double g_nx, double be_nx) {
    const int b = tid + j * BS;
    const double ibar = be_nx * hb_nx[j];
    const double ga_nx = gamma_of(L.pk[j], g_nx);
    v.J[b] = (L.g[j] != 0.0) ? ga_nx * hb_nx[j] + L.g[j] * ibar : 0.0;
  });
  const double *drow = dJ + ((int64_t)it.scen * c.T + (n - 1)) * c.rec_stride;
  for (int r = tid; r < v.n; r += BS) {
    double acc = 0.0;
    const int e1 = v.rptr[r + 1];
    for (int e = v.rptr[r]; e < e1; ++e) acc = acc + drow[v.rcolumn[e]];
    v.dv[r] = acc;
  }
}

// Recomputes steps lo+1..hi of segment s from its checkpoint into a
// segment buffer (row 0 = the checkpoint, row n-lo = step n). Afterwards L's
// coefficients and the factors are those of step hi.
template <int BS, int BPT, int WPT, bool SM>
__device__ __forceinline__ void recompute_segment(const DevCtx &c, const ItemDesc &it, View<SM> &v,
                                                  Lane<BPT> &L, double (&w)[WPT], int64_t s, double *seg_i,
                                                  double *seg_u) {
  const int64_t *topo = c.topo + it.topo;
  const int nbr = v.nbr;
  const int64_t lo = s * c.K, hi = (lo + c.K < c.T) ? lo + c.K : c.T;
  const int64_t cko = it.ck + s * (int64_t)nbr;
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int b = threadIdx.x + j * BS;
    seg_i[b] = c.ck_i[cko + b];
    seg_u[b] = c.ck_u[cko + b];
  }
  int t = topo_of(topo, it.n_topo, lo + 1);
  int64_t next = (t + 1 < it.n_topo) ? topo[t + 1] : kNever;
  load_coefs<BS, BPT>(c, it, t, L.g, L.be);
  history_from_state<BS, BPT, SM>(c.ck_i + cko, c.ck_u + cko, L, v);
  select_factor<BS, WPT, SM>(c, it, v, t, w);
  inject<BS, BPT, SM>(c, v, L, lo + 1);
  lds_barrier();
  for (int64_t n = lo + 1; n <= hi; ++n) {
    gather_all<BS, false, SM>(v);
    solve_after_gather<BS, WPT, SM>(v, w);
    const int64_t o = (n - lo) * (int64_t)nbr;
    const bool sw = (n + 1 == next) && n < hi;
    update_inject<BS, BPT, SM>(c, v, L, seg_i + o, seg_u + o, nullptr, nullptr, sw,
                               it.coef + (int64_t)(t + 1) * nbr, n < hi, n);
    if (sw) {
      ++t;
      next = (t + 1 < it.n_topo) ? topo[t + 1] : kNever;
      select_factor<BS, WPT, SM>(c, it, v, t, w);
    }
    lds_barrier();
  }
}

// Reverses steps hi..lo+1 of segment s from its buffer. On entry L's
// coefficients and the factors are those of step hi (topology t) and hb_nx
// holds hbar of step hi+1 (0 past the horizon); on exit hb_nx holds hbar of
// step lo+1, and the gradient accumulators have taken the segment's terms.
template <int BS, int BPT, int WPT, bool SM>
__device__ __forceinline__ void reverse_segment(const DevCtx &c, const ItemDesc &it, View<SM> &v,
                                                Lane<BPT> &L, double (&w)[WPT], int64_t s, int t,
                                                const double *seg_i, const double *seg_u, double (&hb_nx)[BPT],
                                                double (&gb)[BPT], double (&bb)[BPT], double (&cb)[BPT],
                                                const double *dJ) {
  const int64_t *topo = c.topo + it.topo;
  const int nbr = v.nbr;
  const int64_t T = c.T;
  const int64_t lo = s * c.K, hi = (lo + c.K < T) ? lo + c.K : T;
  // the coefficients of step hi+1 are those of topology t_nx (unused at
  // hi = T, where hbar = 0)
  int t_nx = hi < T ? topo_of(topo, it.n_topo, hi + 1) : t;
  adjoint_seed<BS, BPT, SM>(c, it, v, L, t, t_nx, hb_nx, dJ, hi);
  lds_barrier();
  for (int64_t n = hi; n >= lo + 1; --n) {
    gather_all<BS, true, SM>(v);
    solve_after_gather<BS, WPT, SM>(v, w);
    const int64_t on = (n - lo) * (int64_t)nbr, op = (n - 1 - lo) * (int64_t)nbr;
    const int tid = lane_id();
    with_next_coefs<BS, BPT>(c, it, L, t, t_nx, [&](int j, double g_nx, double be_nx) {
      (void)g_nx;
      const int b = tid + j * BS;
      const uint32_t pk = L.pk[j];
      const double wk = v.x[pk & kTermGround], wm = v.x[(pk >> 15) & kTermGround];
      const double ibar = be_nx * hb_nx[j];
      const double hb = (L.g[j] != 0.0) ? ibar - (wk - wm) : 0.0;
      gb[j] = gb[j] + hb * seg_u[on + b];
      bb[j] = bb[j] + hb * seg_i[op + b];
      cb[j] = cb[j] + hb * seg_u[op + b];
      hb_nx[j] = hb;
    });
    // step n's coefficients become the next-step ones of step n-1
    t_nx = t;
    if (n - 1 >= lo + 1) {
      const int tp = topo_of(topo, it.n_topo, n - 1);
      if (tp != t) {
        t = tp;
        load_coefs<BS, BPT>(c, it, t, L.g, L.be);
        select_factor<BS, WPT, SM>(c, it, v, t, w);
      }
      adjoint_seed<BS, BPT, SM>(c, it, v, L, t, t_nx, hb_nx, dJ, n - 1);
    }
    lds_barrier();
  }
}

template <int BS, int BPT>
__device__ __forceinline__ void store_branch_adjoints(const DevCtx &c, const ItemDesc &it, const double (&gb)[BPT],
                                                      const double (&bb)[BPT], const double (&cb)[BPT]) {
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int b = threadIdx.x + j * BS;
    c.gbar[it.br + b] = gb[j];
    c.bbar[it.br + b] = bb[j];
    c.cbar[it.br + b] = cb[j];
  }
}

// Serial adjoint: one workgroup per item recomputes and reverses each
// segment in turn, last segment first. With 256 lanes the register budget
// is held to two waves per SIMD (two workgroups per compute unit), so a
// batch of many components runs in fewer rounds than at the one wave per
// SIMD that its largest branch-slot counts would otherwise take.
template <int BS, int BPT, int WPT, bool SM>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(BS == 256 ? 2 : 1))) void k_adjoint(
    DevCtx c, const int32_t *order, const double *dJ) {
  const ItemDesc it = c.items[order[blockIdx.x]];
  View<SM> v = make_view<BS, SM>(c, it, true);
  const int64_t nseg = (c.T + c.K - 1) / c.K;
  double *seg_i = c.seg_i + it.seg, *seg_u = c.seg_u + it.seg;
  Lane<BPT> L;
  double w[WPT];
  load_lane<BS, BPT>(c, it, L);
  // per slot: hbar of step n+1 and the three gradient accumulators
  double hb_nx[BPT], gb[BPT], bb[BPT], cb[BPT];
#pragma unroll
  for (int j = 0; j < BPT; ++j) hb_nx[j] = gb[j] = bb[j] = cb[j] = 0.0;
  for (int64_t s = nseg - 1; s >= 0; --s) {
    recompute_segment<BS, BPT, WPT, SM>(c, it, v, L, w, s, seg_i, seg_u);
    const int64_t hi = (s * c.K + c.K < c.T) ? s * c.K + c.K : c.T;
    const int t = topo_of(c.topo + it.topo, it.n_topo, hi);
    reverse_segment<BS, BPT, WPT, SM>(c, it, v, L, w, s, t, seg_i, seg_u, hb_nx, gb, bb, cb, dJ);
  }
  store_branch_adjoints<BS, BPT>(c, it, gb, bb, cb);
}

// Waits until *flag >= target: wave 0 polls (bounded), acquires at device
// scope, and the workgroup barrier releases the other waves. Returns false
// (and sets the error flag) if the wait gave up.
__device__ __forceinline__ bool wait_flag(const int32_t *flag, int32_t target, int32_t *err,
                                          Lds<int32_t> give_up) {
  if (threadIdx.x < 64) {
    int64_t spins = 0;
    bool quit = false;
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++spins > (int64_t(1) << 24) || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        quit = true;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    if (threadIdx.x == 0) {
      give_up[0] = quit ? 1 : 0;
      if (quit) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return give_up[0] == 0;
}

// Publishes *flag = value after every wave's global stores: each wave
// waits for its own stores, the workgroup barrier joins them, lane 0
// releases at device scope and stores the flag.
__device__ __forceinline__ void publish_flag(int32_t *flag, int32_t value) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(flag, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Pipelined adjoint: two workgroups per item, resident together
// (cooperative launch). Workgroup n_items + i recomputes the segments of
// item order[i], last first, into two alternating segment buffers;
// workgroup i reverses each segment as soon as it is recomputed, so the
// recompute of segment s-1 overlaps the reversal of segment s. Per item,
// pipe[2q] counts recomputed segments and pipe[2q+1] reversed ones; the
// recompute of the k-th segment waits until the (k-2)-th is reversed.
template <int BS, int BPT, int WPT, bool SM>
__global__ __launch_bounds__(BS) void k_adjoint_pipe(DevCtx c, const int32_t *order, int n_items,
                                                     const double *dJ, int32_t *pipe) {
  const bool recompute = (int)blockIdx.x >= n_items;
  const int q = order[recompute ? blockIdx.x - n_items : blockIdx.x];
  const ItemDesc it = c.items[q];
  View<SM> v = make_view<BS, SM>(c, it, true);
  const int64_t nseg = (c.T + c.K - 1) / c.K;
  const int64_t seg_len = ((c.K < c.T ? c.K : c.T) + 1) * (int64_t)v.nbr;
  int32_t *ready = pipe + 2 * q, *done = pipe + 2 * q + 1;
  Lane<BPT> L;
  double w[WPT];
  load_lane<BS, BPT>(c, it, L);
  if (recompute) {
    for (int64_t k = 0; k < nseg; ++k) {
      if (k >= 2 && !wait_flag(done, (int32_t)(k - 1), c.flags + 2, v.flag)) return;
      const int64_t o = it.seg + (k & 1) * seg_len;
      recompute_segment<BS, BPT, WPT, SM>(c, it, v, L, w, nseg - 1 - k, c.seg_i + o, c.seg_u + o);
      publish_flag(ready, (int32_t)(k + 1));
    }
    return;
  }
  double hb_nx[BPT], gb[BPT], bb[BPT], cb[BPT];
#pragma unroll
  for (int j = 0; j < BPT; ++j) hb_nx[j] = gb[j] = bb[j] = cb[j] = 0.0;
  for (int64_t k = 0; k < nseg; ++k) {
    const int64_t s = nseg - 1 - k;
    if (!wait_flag(ready, (int32_t)(k + 1), c.flags + 2, v.flag)) return;
    const int64_t hi = (s * c.K + c.K < c.T) ? s * c.K + c.K : c.T;
    const int t = topo_of(c.topo + it.topo, it.n_topo, hi);
    load_coefs<BS, BPT>(c, it, t, L.g, L.be);
    select_factor<BS, WPT, SM>(c, it, v, t, w);
    lds_barrier();
    const int64_t o = it.seg + (k & 1) * seg_len;
    reverse_segment<BS, BPT, WPT, SM>(c, it, v, L, w, s, t, c.seg_i + o, c.seg_u + o, hb_nx, gb, bb, cb, dJ);
    publish_flag(done, (int32_t)(k + 1));
  }
  store_branch_adjoints<BS, BPT>(c, it, gb, bb, cb);
}

}  // namespace step
}  // namespace emt
