// Device code of the persistent step kernels (forward time loop and
// reverse-time adjoint), FP64, gfx950.
//
// One workgroup owns one work item (a connected component of one scenario)
// for many time steps; scenarios and components are more workgroups of the
// same launch. This is the paper's pair of parallel strategies (Sec. III-B):
// the processes of one layer run together and the layers are replayed in
// order every step; isomorphic scenarios run the same processes side by side.
// Each step runs the four basic processes of an EMTP-type solver that the
// paper lists (Sec. III-A), separated by workgroup barriers:
//   1. branch phase (one branch per lane, coefficients and history in VGPRs):
//        source EMF e, branch injection J = g*e - h into LDS;
//   2. forward sweep: each row gathers its nodal injection from its incident
//        branch ends in a fixed (CSR) order — a deterministic segmented sum,
//        no atomics — and solves L y = rhs level by level over the leading
//        part of the elimination order; the dense tail rows gather
//        c = rhs_D - L_DS y_S;
//   3. tail: x_D = W c with W = (L_DD D_D L_DD^T)^{-1} held in VGPRs (a
//        dense matrix-vector product reduced across lanes with shuffles);
//      backward sweep: x = D^{-1} y - L^T x level by level;
//   4. branch phase: u = A^T v - e, i = g*u + h, next history
//        h = beta*i + gamma*u; record and checkpoint.
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

// The lane index, hidden from the optimiser once per time step so that the
// per-branch index and address arithmetic is recomputed inside the loop
// (a few integer operations) instead of being hoisted out of it and held in
// VGPRs for every branch of the lane.
__device__ __forceinline__ int lane_id() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
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

// Per-workgroup view of an item. Index arrays and factor values live in LDS
// (SM = true) or are read from global memory.
template <bool SM>
struct View {
  int n, d, ns, nbr, nsrc, nsv, nlf, nlb, nrec, tpr;
  Ref<int32_t, SM> frowptr, bptr, flevptr, blevptr, nptr, rptr;
  Ref<uint16_t, SM> fcol, brow, bpos, flevrows, blevrows, nent, rnode, rcolumn;
  Lds<double> x, J, cD, eS, dv, sv_s, dinv_s;
  Ref<double, SM> sv, dinv;
};

// Threads per tail row: the largest power of two (<= 64, one wave) with
// d * tpr <= block size.
__device__ __forceinline__ int tail_tpr(int d, int bs) {
  int t = 64;
  while (t > 1 && d * t > bs) t >>= 1;
  return t;
}

template <int BS>
__device__ __forceinline__ void copy_i32(int32_t *dst, const int32_t *src, int cnt) {
  for (int q = threadIdx.x; q < cnt; q += BS) dst[q] = src[q];
}
template <int BS>
__device__ __forceinline__ void copy_u16(uint16_t *dst, const uint16_t *src, int cnt) {
  for (int q = threadIdx.x; q < cnt; q += BS) dst[q] = src[q];
}
template <int BS>
__device__ __forceinline__ void copy_f64(double *dst, const double *src, int cnt) {
  for (int q = threadIdx.x; q < cnt; q += BS) dst[q] = src[q];
}

// LDS layout: doubles (x, J, cD, eS, [dv], [sv, dinv]), then int32, then
// uint16. Must match lds_bytes() on the host.
template <int BS>
__device__ __forceinline__ void copy_to(uint32_t off, const int32_t *src, int cnt) {
  copy_i32<BS>(reinterpret_cast<int32_t *>(emt_lds + off), src, cnt);
}
template <int BS>
__device__ __forceinline__ void copy_to(uint32_t off, const uint16_t *src, int cnt) {
  copy_u16<BS>(reinterpret_cast<uint16_t *>(emt_lds + off), src, cnt);
}

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
  v.nlf = sd.nlf;
  v.nlb = sd.nlb;
  v.nrec = it.n_rec;
  v.tpr = tail_tpr(sd.d, BS);
  const int32_t *g_frowptr = c.symi + sd.frowptr, *g_bptr = c.symi + sd.bptr;
  const int32_t *g_flevptr = c.symi + sd.sflevptr, *g_blevptr = c.symi + sd.sblevptr;
  const int32_t *g_nptr = c.nptr + it.nptr, *g_rptr = c.rptr + it.nptr;
  const uint16_t *g_fcol = c.symh + sd.fcol, *g_brow = c.symh + sd.brow, *g_bpos = c.symh + sd.bpos;
  const uint16_t *g_flevrows = c.symh + sd.sflevrows, *g_blevrows = c.symh + sd.sblevrows;
  const uint16_t *g_nent = c.nent + it.nent, *g_rnode = c.rnode + it.rec, *g_rcolumn = c.rcolumn + it.rec;
  const int nent_cnt = g_nptr[v.n];

  uint32_t off = 0;
  auto take = [&off](int cnt, int size) {
    const uint32_t o = off;
    off += (uint32_t)cnt * (uint32_t)size;
    return o;
  };
  v.x.off = take(v.n, 8);
  v.J.off = take(v.nbr, 8);
  v.cD.off = take(v.d, 8);
  v.eS.off = take(v.nsrc, 8);
  v.dv.off = take(adjoint ? v.n : 0, 8);
  if constexpr (SM) {
    v.sv_s.off = take(v.nsv, 8);
    v.dinv_s.off = take(v.ns, 8);
    v.frowptr.off = take(v.n + 1, 4);
    v.bptr.off = take(v.ns + 1, 4);
    v.flevptr.off = take(v.nlf + 1, 4);
    v.blevptr.off = take(v.nlb + 1, 4);
    v.nptr.off = take(v.n + 1, 4);
    v.rptr.off = take(adjoint ? v.n + 1 : 0, 4);
    v.fcol.off = take(v.nsv, 2);
    v.brow.off = take(v.nsv, 2);
    v.bpos.off = take(v.nsv, 2);
    v.flevrows.off = take(v.ns, 2);
    v.blevrows.off = take(v.ns, 2);
    v.nent.off = take(nent_cnt, 2);
    v.rnode.off = take(v.nrec, 2);
    v.rcolumn.off = take(v.nrec, 2);
    copy_to<BS>(v.frowptr.off, g_frowptr, v.n + 1);
    copy_to<BS>(v.bptr.off, g_bptr, v.ns + 1);
    copy_to<BS>(v.flevptr.off, g_flevptr, v.nlf + 1);
    copy_to<BS>(v.blevptr.off, g_blevptr, v.nlb + 1);
    copy_to<BS>(v.nptr.off, g_nptr, v.n + 1);
    if (adjoint) copy_to<BS>(v.rptr.off, g_rptr, v.n + 1);
    copy_to<BS>(v.fcol.off, g_fcol, v.nsv);
    copy_to<BS>(v.brow.off, g_brow, v.nsv);
    copy_to<BS>(v.bpos.off, g_bpos, v.nsv);
    copy_to<BS>(v.flevrows.off, g_flevrows, v.ns);
    copy_to<BS>(v.blevrows.off, g_blevrows, v.ns);
    copy_to<BS>(v.nent.off, g_nent, nent_cnt);
    copy_to<BS>(v.rnode.off, g_rnode, v.nrec);
    copy_to<BS>(v.rcolumn.off, g_rcolumn, v.nrec);
    v.sv.off = v.sv_s.off;
    v.dinv.off = v.dinv_s.off;
  } else {
    v.frowptr.p = g_frowptr; v.bptr.p = g_bptr; v.flevptr.p = g_flevptr; v.blevptr.p = g_blevptr;
    v.nptr.p = g_nptr; v.rptr.p = g_rptr;
    v.fcol.p = g_fcol; v.brow.p = g_brow; v.bpos.p = g_bpos; v.flevrows.p = g_flevrows;
    v.blevrows.p = g_blevrows; v.nent.p = g_nent; v.rnode.p = g_rnode; v.rcolumn.p = g_rcolumn;
  }
  return v;
}

// Factor values and the tail inverse of topology t (sweep values and 1/D in
// LDS under SM; the lane's share of W in VGPRs).
template <int BS, int WPT, bool SM>
__device__ __forceinline__ void select_factor(const DevCtx &c, const ItemDesc &it, View<SM> &v, int t,
                                              double (&w)[WPT]) {
  const double *sv = c.svals + it.sv + (int64_t)t * v.nsv;
  const double *di = c.dinv + it.dfac + (int64_t)t * v.n;
  if constexpr (SM) {
    copy_f64<BS>(reinterpret_cast<double *>(emt_lds + v.sv_s.off), sv, v.nsv);
    copy_f64<BS>(reinterpret_cast<double *>(emt_lds + v.dinv_s.off), di, v.ns);
  } else {
    v.sv.p = sv;
    v.dinv.p = di;
  }
  const double *W = c.wtail + it.w + (int64_t)t * v.d * v.d;
  const int row = threadIdx.x / v.tpr, lane = threadIdx.x % v.tpr;
#pragma unroll
  for (int q = 0; q < WPT; ++q) {
    const int col = lane + q * v.tpr;
    w[q] = (row < v.d && col < v.d) ? W[row * v.d + col] : 0.0;
  }
}

template <bool ADJ, bool SM>
__device__ __forceinline__ double gather(const View<SM> &v, int r) {
  double acc = 0.0;
  const int e1 = v.nptr[r + 1];
  for (int e = v.nptr[r]; e < e1; ++e) {
    const int ent = v.nent[e];
    const double jv = v.J[ent >> 1];
    acc = (ent & 1) ? acc - jv : acc + jv;
  }
  if (ADJ) acc = acc + v.dv[r];
  return acc;
}

// Forward sweep over the leading rows, then the tail rows' reduced
// right-hand side c = rhs_D - L_DS y_S (into cD).
template <int BS, bool ADJ, bool SM>
__device__ __forceinline__ void sweep_forward(const View<SM> &v) {
  for (int l = 0; l < v.nlf; ++l) {
    const int p1 = v.flevptr[l + 1];
    for (int p = v.flevptr[l] + (int)threadIdx.x; p < p1; p += BS) {
      const int r = v.flevrows[p];
      double acc = gather<ADJ, SM>(v, r);
      const int q1 = v.frowptr[r + 1];
      for (int q = v.frowptr[r]; q < q1; ++q) acc = acc - v.sv[q] * v.x[v.fcol[q]];
      v.x[r] = acc;
    }
    __syncthreads();
  }
  if (v.d > 0) {
    for (int a = threadIdx.x; a < v.d; a += BS) {
      const int r = v.ns + a;
      double acc = gather<ADJ, SM>(v, r);
      const int q1 = v.frowptr[r + 1];
      for (int q = v.frowptr[r]; q < q1; ++q) acc = acc - v.sv[q] * v.x[v.fcol[q]];
      v.cD[a] = acc;
    }
    __syncthreads();
  }
}

// x_D = W c: each tail row is shared by tpr adjacent lanes of one wave; the
// partial dot products are combined by a fixed butterfly of shuffles.
template <int BS, int WPT, bool SM>
__device__ __forceinline__ void tail_solve(const View<SM> &v, const double (&w)[WPT]) {
  if (v.d == 0) return;
  const int tid = lane_id();
  const int row = tid / v.tpr, lane = tid % v.tpr;
  double s = 0.0;
  if (row < v.d) {
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
      const int col = lane + q * v.tpr;
      if (col < v.d) s = s + w[q] * v.cD[col];
    }
  }
  for (int off = 1; off < v.tpr; off <<= 1) s = s + __shfl_xor(s, off);
  if (row < v.d && lane == 0) v.x[v.ns + row] = s;
  __syncthreads();
}

// Backward sweep over the leading rows: x_r = y_r / D_r - sum_c L_cr x_c.
template <int BS, bool SM>
__device__ __forceinline__ void sweep_backward(const View<SM> &v) {
  for (int l = 0; l < v.nlb; ++l) {
    const int p1 = v.blevptr[l + 1];
    for (int p = v.blevptr[l] + (int)threadIdx.x; p < p1; p += BS) {
      const int r = v.blevrows[p];
      double acc = v.x[r] * v.dinv[r];
      const int q1 = v.bptr[r + 1];
      for (int q = v.bptr[r]; q < q1; ++q) acc = acc - v.sv[v.bpos[q]] * v.x[v.brow[q]];
      v.x[r] = acc;
    }
    __syncthreads();
  }
}

template <int BS, int WPT, bool ADJ, bool SM>
__device__ __forceinline__ void solve(const View<SM> &v, const double (&w)[WPT]) {
  sweep_forward<BS, ADJ, SM>(v);
  tail_solve<BS, WPT, SM>(v, w);
  sweep_backward<BS, SM>(v);
}

// Lane state of the forward loop: coefficients of the current topology and
// the history current of the next step.
template <int BPT>
struct Lane {
  double g[BPT], be[BPT], h[BPT];
  uint32_t pk[BPT];
  // EMF parameters of the lane's first branch (sources are numbered first,
  // so only slot 0 can hold one while n_src <= block size)
  double sE, sw, sph;
};

template <int BS, int BPT>
__device__ __forceinline__ void load_lane(const DevCtx &c, const ItemDesc &it, Lane<BPT> &L) {
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int b = threadIdx.x + j * BS;
    L.pk[j] = b < it.n_br ? c.bpack[it.br + b] : (kTermGround | (kTermGround << 15));
  }
  const int b0 = threadIdx.x;
  const bool src = b0 < it.n_src;
  L.sE = src ? c.bE[it.br + b0] : 0.0;
  L.sw = src ? c.bw[it.br + b0] : 0.0;
  L.sph = src ? c.bph[it.br + b0] : 0.0;
}

template <int BS, int BPT>
__device__ __forceinline__ void load_coefs(const DevCtx &c, const ItemDesc &it, int t, double (&g)[BPT],
                                           double (&be)[BPT]) {
  const int64_t base = it.coef + (int64_t)t * it.n_br;
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int b = threadIdx.x + j * BS;
    g[j] = b < it.n_br ? c.cg[base + b] : 0.0;
    be[j] = b < it.n_br ? c.cb[base + b] : 0.0;
  }
}

// History current h = beta*i + gamma*u from a stored state (i, u).
template <int BS, int BPT>
__device__ __forceinline__ void history_from_state(const double *si, const double *su, int nbr, Lane<BPT> &L) {
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int b = threadIdx.x + j * BS;
    const double i = b < nbr ? si[b] : 0.0;
    const double u = b < nbr ? su[b] : 0.0;
    L.h[j] = L.be[j] * i + gamma_of(L.pk[j], L.g[j]) * u;
  }
}

template <int BS, int BPT, bool SM>
__device__ __forceinline__ void inject(const DevCtx &c, const ItemDesc &it, const View<SM> &v, const Lane<BPT> &L,
                                       int64_t n) {
  const double tn = (double)n * c.dt;
  const int tid = lane_id();
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int b = tid + j * BS;
    if (b < v.nbr) {
      double e = 0.0;
      if (b < v.nsrc) {
        e = (j == 0) ? L.sE * emf_cos(L.sw * tn + L.sph) : source_emf(c, it.br + b, n);
        v.eS[b] = e;
      }
      v.J[b] = L.g[j] * e - L.h[j];
    }
  }
}

// Branch update of step n with the current coefficients; optional stores of
// (i, u) to up to two places (null = none); then, if the next step starts a
// new topology, its coefficients are loaded before the next history current
// is formed.
template <int BS, int BPT, bool SM>
__device__ __forceinline__ void update(const DevCtx &c, const View<SM> &v, Lane<BPT> &L, double *st_i, double *st_u,
                                       double *st2_i, double *st2_u, bool switch_next, int64_t next_coef) {
  const int tid = lane_id();
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int b = tid + j * BS;
    if (b < v.nbr) {
      const uint32_t pk = L.pk[j];
      const uint32_t k = pk & kTermGround, m = (pk >> 15) & kTermGround;
      const double vk = k != kTermGround ? v.x[k] : 0.0;
      const double vm = m != kTermGround ? v.x[m] : 0.0;
      const double e = b < v.nsrc ? v.eS[b] : 0.0;
      const double u = (L.g[j] != 0.0) ? (vk - vm) - e : 0.0;
      const double i = L.g[j] * u + L.h[j];
      if (st_i) {
        st_i[b] = i;
        st_u[b] = u;
      }
      if (st2_i) {
        st2_i[b] = i;
        st2_u[b] = u;
      }
      if (switch_next) {
        L.g[j] = c.cg[next_coef + b];
        L.be[j] = c.cb[next_coef + b];
      }
      L.h[j] = L.be[j] * i + gamma_of(pk, L.g[j]) * u;
    }
  }
}

// ---------------------------------------------------------------------------
// Forward loop: steps n0+1 .. n0+ns for every item.
// ---------------------------------------------------------------------------
template <int BS, int BPT, int WPT, bool SM>
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
  history_from_state<BS, BPT>(c.si + it.br, c.su + it.br, v.nbr, L);
  select_factor<BS, WPT, SM>(c, it, v, t, w);
  __syncthreads();
  const int R = c.rec_stride;
  const int64_t n_end = n0 + nsteps;
  for (int64_t n = n0 + 1; n <= n_end; ++n) {
    inject<BS, BPT, SM>(c, it, v, L, n);
    __syncthreads();
    solve<BS, WPT, false, SM>(v, w);
    if (rec) {
      double *row = rec + ((int64_t)it.scen * nsteps + (n - n0 - 1)) * R;
      for (int q = threadIdx.x; q < v.nrec; q += BS) row[v.rcolumn[q]] = v.x[v.rnode[q]];
    }
    const bool sw = (n + 1 == next);
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
    update<BS, BPT, SM>(c, v, L, ck_i, ck_u, st_i, st_u, sw, it.coef + (int64_t)(t + 1) * v.nbr);
    if (sw) {
      ++t;
      next = (t + 1 < it.n_topo) ? topo[t + 1] : kNever;
      select_factor<BS, WPT, SM>(c, it, v, t, w);
    }
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
template <int BS, int BPT, int WPT, bool SM>
__global__ __launch_bounds__(BS) void k_adjoint(DevCtx c, const int32_t *order, const double *dJ) {
  const ItemDesc it = c.items[order[blockIdx.x]];
  View<SM> v = make_view<BS, SM>(c, it, true);
  const int64_t *topo = c.topo + it.topo;
  const int K = c.K;
  const int64_t T = c.T;
  const int R = c.rec_stride;
  const int64_t nseg = (T + K - 1) / K;
  double *seg_i = c.seg_i + it.seg, *seg_u = c.seg_u + it.seg;
  const int nbr = v.nbr;

  Lane<BPT> L;
  double w[WPT];
  load_lane<BS, BPT>(c, it, L);
  double g_nx[BPT], be_nx[BPT], hb_nx[BPT], ib[BPT];
  double gb[BPT], bb[BPT], cb[BPT];
#pragma unroll
  for (int j = 0; j < BPT; ++j) g_nx[j] = be_nx[j] = hb_nx[j] = gb[j] = bb[j] = cb[j] = 0.0;

  for (int64_t s = nseg - 1; s >= 0; --s) {
    const int64_t lo = s * K, hi = (lo + K < T) ? lo + K : T;
    // Recompute steps lo+1..hi from the checkpoint at lo.
    const int64_t cko = it.ck + s * (int64_t)nbr;
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int b = threadIdx.x + j * BS;
      if (b < nbr) {
        seg_i[b] = c.ck_i[cko + b];
        seg_u[b] = c.ck_u[cko + b];
      }
    }
    int t = topo_of(topo, it.n_topo, lo + 1);
    int64_t next = (t + 1 < it.n_topo) ? topo[t + 1] : kNever;
    load_coefs<BS, BPT>(c, it, t, L.g, L.be);
    history_from_state<BS, BPT>(c.ck_i + cko, c.ck_u + cko, nbr, L);
    select_factor<BS, WPT, SM>(c, it, v, t, w);
    __syncthreads();
    for (int64_t n = lo + 1; n <= hi; ++n) {
      inject<BS, BPT, SM>(c, it, v, L, n);
      __syncthreads();
      solve<BS, WPT, false, SM>(v, w);
      const int64_t o = (n - lo) * (int64_t)nbr;
      const bool sw = (n + 1 == next) && n < hi;
      update<BS, BPT, SM>(c, v, L, seg_i + o, seg_u + o, nullptr, nullptr, sw, it.coef + (int64_t)(t + 1) * nbr);
      if (sw) {
        ++t;
        next = (t + 1 < it.n_topo) ? topo[t + 1] : kNever;
        select_factor<BS, WPT, SM>(c, it, v, t, w);
      }
    }
    // L.g, L.be and the factors now belong to step hi.
    for (int64_t n = hi; n >= lo + 1; --n) {
      const int tid = lane_id();
#pragma unroll
      for (int j = 0; j < BPT; ++j) {
        const int b = tid + j * BS;
        if (b < nbr) {
          const double ibar = be_nx[j] * hb_nx[j];
          ib[j] = ibar;
          const double ga_nx = gamma_of(L.pk[j], g_nx[j]);
          v.J[b] = (L.g[j] != 0.0) ? ga_nx * hb_nx[j] + L.g[j] * ibar : 0.0;
        }
      }
      const double *drow = dJ + ((int64_t)it.scen * T + (n - 1)) * R;
      for (int r = threadIdx.x; r < v.n; r += BS) {
        double acc = 0.0;
        const int e1 = v.rptr[r + 1];
        for (int e = v.rptr[r]; e < e1; ++e) acc = acc + drow[v.rcolumn[e]];
        v.dv[r] = acc;
      }
      __syncthreads();
      solve<BS, WPT, true, SM>(v, w);
      const int64_t on = (n - lo) * (int64_t)nbr, op = (n - 1 - lo) * (int64_t)nbr;
      const int tid2 = lane_id();
#pragma unroll
      for (int j = 0; j < BPT; ++j) {
        const int b = tid2 + j * BS;
        if (b < nbr) {
          const uint32_t pk = L.pk[j];
          const uint32_t k = pk & kTermGround, m = (pk >> 15) & kTermGround;
          const double wk = k != kTermGround ? v.x[k] : 0.0;
          const double wm = m != kTermGround ? v.x[m] : 0.0;
          const double hb = (L.g[j] != 0.0) ? ib[j] - (wk - wm) : 0.0;
          gb[j] = gb[j] + hb * seg_u[on + b];
          bb[j] = bb[j] + hb * seg_i[op + b];
          cb[j] = cb[j] + hb * seg_u[op + b];
          hb_nx[j] = hb;
          g_nx[j] = L.g[j];
          be_nx[j] = L.be[j];
        }
      }
      if (n - 1 >= lo + 1) {
        const int tp = topo_of(topo, it.n_topo, n - 1);
        if (tp != t) {
          t = tp;
          load_coefs<BS, BPT>(c, it, t, L.g, L.be);
          select_factor<BS, WPT, SM>(c, it, v, t, w);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int b = threadIdx.x + j * BS;
    if (b < nbr) {
      c.gbar[it.br + b] = gb[j];
      c.bbar[it.br + b] = bb[j];
      c.cbar[it.br + b] = cb[j];
    }
  }
}

}  // namespace step
}  // namespace emt
