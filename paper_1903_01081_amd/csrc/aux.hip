// Auxiliary HIP kernels: companion coefficients, line parameters, the
// numeric factorisation (once per topology), state reset/set and the
// reduction of branch adjoints to line-parameter gradients.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"
#include "launch.h"
#include "trig.h"

namespace emt {

namespace {

__device__ __forceinline__ double emf0(const DevCtx &c, int64_t gb, int64_t n) {
  const double t = (double)n * c.dt;
  return c.bE[gb] * emf_cos(c.bw[gb] * t + c.bph[gb]);
}

__device__ __forceinline__ int topo_at(const int64_t *topo, int ntopo, int64_t n) {
  int t = 0;
  while (t + 1 < ntopo && topo[t + 1] <= n) ++t;
  return t;
}

}  // namespace

// Companion coefficients of every (item branch, topology): the trapezoidal
// Norton equivalents of the paper's first basic process (Sec. III-A):
//   R-L / source impedance: g = 1/(R + 2L/dt), beta = (2L/dt - R) g (gamma = g)
//   capacitor:              g = 2C/dt,         beta = -1            (gamma = -g)
//   resistor / switch:      g = 1/R,           beta = 0             (gamma = 0)
//   out of service:         g = beta = 0
__global__ void k_companions(DevCtx c, const int64_t *coef_base, const int64_t *br_base, const int32_t *nbr_of,
                             const int32_t *cnt_prefix, int total, int n_items) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= total) return;
  int lo = 0, hi = n_items - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (cnt_prefix[mid] <= w) lo = mid; else hi = mid - 1;
  }
  const int item = lo;
  const int local = w - cnt_prefix[item];
  const int nbr = nbr_of[item];
  const int t = local / nbr, b = local % nbr;
  const int64_t gb = br_base[item] + b;
  const int64_t ci = coef_base[item] + (int64_t)t * nbr + b;
  double g = 0.0, be = 0.0;
  if (c.bgrp && c.bgrp[gb]) {
    // member of a coupled group (always in service): the circulant
    // companion from its zero- and positive-sequence eigenvalues d + 2o and
    // d - o (a circulant's products and inverses are circulants with the
    // products and inverses of these); diagonal -> cg, cb, off-diagonal ->
    // cgo, cbo
    const double dt = c.dt;
    double go = 0.0, bo = 0.0;
    if (c.bkind[gb] == KIND_RL) {
      const double Md = c.bR[gb] + 2.0 * c.bL[gb] / dt, Mo = c.bRm[gb] + 2.0 * c.bLm[gb] / dt;
      const double Nd = 2.0 * c.bL[gb] / dt - c.bR[gb], No = 2.0 * c.bLm[gb] / dt - c.bRm[gb];
      const double l0 = Md + 2.0 * Mo, l1 = Md - Mo, m0 = Nd + 2.0 * No, m1 = Nd - No;
      const double g0 = 1.0 / l0, g1 = 1.0 / l1, b0 = m0 / l0, b1 = m1 / l1;
      g = (g0 + 2.0 * g1) / 3.0;
      go = (g0 - g1) / 3.0;
      be = (b0 + 2.0 * b1) / 3.0;
      bo = (b0 - b1) / 3.0;
    } else {
      g = 2.0 * c.bC[gb] / dt;
      go = 2.0 * c.bCm[gb] / dt;
      be = -1.0;
    }
    c.cg[ci] = g;
    c.cb[ci] = be;
    c.cgo[ci] = go;
    c.cbo[ci] = bo;
    return;
  }
  if (c.cgo) {
    c.cgo[ci] = 0.0;
    c.cbo[ci] = 0.0;
  }
  if (c.cins[ci]) {
    const double dt = c.dt;
    const int kind = c.bkind[gb];
    if (kind == KIND_RL || kind == KIND_SRC) {
      const double R = c.bR[gb], L = c.bL[gb];
      g = 1.0 / (R + 2.0 * L / dt);
      be = (2.0 * L / dt - R) * g;
    } else if (kind == KIND_C) {
      g = 2.0 * c.bC[gb] / dt;
      be = -1.0;
    } else {
      g = 1.0 / c.bR[gb];
    }
  }
  c.cg[ci] = g;
  c.cb[ci] = be;
}

// Line parameters theta [S][P] -> branch R, L, C (series: R_l, L_l; each
// shunt capacitor of the pi-section: C_l / 2).
__global__ void k_set_params(DevCtx c, const double *theta, int P, const int32_t *bscen, int64_t nbr_total) {
  const int64_t gb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gb >= nbr_total) return;
  const int l = c.bline[gb];
  if (l < 0) return;
  const double *th = theta + (int64_t)bscen[gb] * P + 3 * l;
  const int kind = c.bkind[gb];
  if (kind == KIND_RL) {
    c.bR[gb] = th[0];
    c.bL[gb] = th[1];
  } else if (kind == KIND_C) {
    c.bC[gb] = 0.5 * th[2];
  }
}

// Numeric LDL^T of the conductance matrix of every (item, topology), one
// workgroup each (the paper's third basic process, run once per topology).
// G is assembled row by row from the node CSR in a fixed order, then
// factorised level by level (the columns of one elimination-tree level only
// depend on lower levels):
//   D_j  = G_jj - sum_{k<j} L_jk^2 D_k
//   L_ij = (G_ij - sum_{k<j} L_ik D_k L_jk) / D_j
// A non-positive or non-finite pivot increments c.flags[0].
template <int BS>
__global__ __launch_bounds__(BS) void k_factor(DevCtx c, const int32_t *pairs) {
  const int item = pairs[2 * blockIdx.x], t = pairs[2 * blockIdx.x + 1];
  const ItemDesc it = c.items[item];
  const SymDesc sd = c.syms[it.sym];
  const int n = it.n;
  const int32_t *rowptr = c.symi + sd.rowptr, *rowcol = c.symi + sd.rowcol;
  const int32_t *colrow = c.symi + sd.colrow, *colpos = c.symi + sd.colpos;
  const int32_t *flevptr = c.symi + sd.flevptr, *flevrows = c.symi + sd.flevrows;
  const int32_t *fentptr = c.symi + sd.fentptr, *fent = c.symi + sd.fent;
  const int32_t *nptr = c.nptr + it.nptr;
  const uint16_t *nent = c.nent + it.nent;
  const double *g = c.cg + it.coef + (int64_t)t * it.n_br;
  const int32_t *bk = c.bk + it.br, *bm = c.bm + it.br, *gpos = c.bgpos + it.br;
  double *Lr = c.lfull + it.fac + (int64_t)t * sd.nnz;
  double *D = c.dpiv + it.dfac + (int64_t)t * n;
  for (int r = threadIdx.x; r < n; r += BS) {
    for (int q = rowptr[r]; q < rowptr[r + 1]; ++q) Lr[q] = 0.0;
    double d = 0.0;
    for (int e = nptr[r]; e < nptr[r + 1]; ++e) {
      const int ent = nent[e];
      const int b = ent >> 1;
      const double gv = g[b];
      d = d + gv;
      const int other = (ent & 1) ? bk[b] : bm[b];
      if (other >= 0 && other < r) Lr[gpos[b]] = Lr[gpos[b]] - gv;
    }
    D[r] = d;
    if (it.n_groups > 0) {
      // mutual conductances of coupled groups: +g_o between like terminals
      // of two members, -g_o between a k and an m terminal
      const int32_t *mp = c.mptr + it.mptr;
      const int32_t *me = c.ment + it.ment;
      const double *go = c.cgo + it.coef + (int64_t)t * it.n_br;
      for (int e = mp[r]; e < mp[r + 1]; ++e) {
        const int pos = me[2 * e], code = me[2 * e + 1];
        const double v = go[code >> 1];
        Lr[pos] = (code & 1) ? Lr[pos] - v : Lr[pos] + v;
      }
    }
  }
  __syncthreads();
  for (int l = 0; l < sd.nlev; ++l) {
    for (int p = flevptr[l] + threadIdx.x; p < flevptr[l + 1]; p += BS) {
      const int j = flevrows[p];
      double d = D[j];
      for (int q = rowptr[j]; q < rowptr[j + 1]; ++q) {
        const double ljk = Lr[q];
        d = d - ljk * ljk * D[rowcol[q]];
      }
      D[j] = d;
      if (!(d > 0.0) || !isfinite(d)) atomicAdd(&c.flags[0], 1);
    }
    __syncthreads();
    for (int p = fentptr[l] + threadIdx.x; p < fentptr[l + 1]; p += BS) {
      const int e = fent[p];
      const int i = colrow[e];
      const int pos = colpos[e];
      const int j = rowcol[pos];
      double s = Lr[pos];
      int qi = rowptr[i], qj = rowptr[j];
      const int qi1 = rowptr[i + 1], qj1 = rowptr[j + 1];
      while (qi < qi1 && qj < qj1) {
        const int ci = rowcol[qi], cj = rowcol[qj];
        if (ci >= j) break;
        if (ci == cj) {
          s = s - Lr[qi] * D[ci] * Lr[qj];
          ++qi;
          ++qj;
        } else if (ci < cj) {
          ++qi;
        } else {
          ++qj;
        }
      }
      Lr[pos] = s / D[j];
    }
    __syncthreads();
  }
}

// Per (item, topology): sweep values (the nonzeros of L with a column in the
// leading part), 1/D, and the inverse W of the tail's Schur complement
// S = L_DD D_D L_DD^T. L_DD (unit lower, dense) is staged in LDS; lane j
// solves S w = e_j (forward, scale, backward) into row j of W (W is
// symmetric, so rows and columns coincide).
__global__ __launch_bounds__(256) void k_tail(DevCtx c, const int32_t *pairs) {
  extern __shared__ __align__(16) char lds[];
  const int item = pairs[2 * blockIdx.x], t = pairs[2 * blockIdx.x + 1];
  const ItemDesc it = c.items[item];
  const SymDesc sd = c.syms[it.sym];
  const int n = it.n, d = sd.d, ns = sd.ns;
  const double *Lr = c.lfull + it.fac + (int64_t)t * sd.nnz;
  const double *D = c.dpiv + it.dfac + (int64_t)t * n;
  const int32_t *svmap = c.symi + sd.svmap;
  double *sv = c.svals + it.sv + (int64_t)t * sd.nsv;
  double *dinv = c.dinv + it.dfac + (int64_t)t * n;
  for (int q = threadIdx.x; q < sd.nsv; q += blockDim.x) sv[q] = Lr[svmap[q]];
  for (int r = threadIdx.x; r < n; r += blockDim.x) dinv[r] = 1.0 / D[r];
  if (d == 0) return;
  double *Ld = reinterpret_cast<double *>(lds);  // d x d, row-major, strictly lower
  const int32_t *rowptr = c.symi + sd.rowptr, *rowcol = c.symi + sd.rowcol;
  for (int q = threadIdx.x; q < d * d; q += blockDim.x) Ld[q] = 0.0;
  __syncthreads();
  for (int a = threadIdx.x; a < d; a += blockDim.x) {
    const int r = ns + a;
    for (int q = rowptr[r]; q < rowptr[r + 1]; ++q) {
      const int col = rowcol[q];
      if (col >= ns) Ld[a * d + (col - ns)] = Lr[q];
    }
  }
  __syncthreads();
  double *W = c.wtail + it.w + (int64_t)t * d * d;
  for (int j = threadIdx.x; j < d; j += blockDim.x) {
    double *z = W + (int64_t)j * d;
    for (int a = 0; a < j; ++a) z[a] = 0.0;
    for (int a = j; a < d; ++a) {
      double s = (a == j) ? 1.0 : 0.0;
      for (int b = j; b < a; ++b) s = s - Ld[a * d + b] * z[b];
      z[a] = s;
    }
    for (int a = 0; a < d; ++a) z[a] = z[a] / D[ns + a];
    for (int a = d - 1; a >= 0; --a) {
      double s = z[a];
      for (int b = a + 1; b < d; ++b) s = s - Ld[b * d + a] * z[b];
      z[a] = s;
    }
  }
}

// State at step 0: v = 0, i = 0, u = -e(0) on in-service branches; writes
// checkpoint 0 when checkpoints are on.
__global__ void k_reset(DevCtx c, const int32_t *bitem, const int32_t *blocal, int64_t nbr_total) {
  const int64_t gb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gb >= nbr_total) return;
  const ItemDesc it = c.items[bitem[gb]];
  const int b = blocal[gb];
  const bool on = c.cins[it.coef + b] != 0;
  const double e = (b < it.n_src) ? emf0(c, gb, 0) : 0.0;
  const double u = on ? (0.0 - 0.0) - e : 0.0;
  c.si[gb] = 0.0;
  c.su[gb] = u;
  if (c.K > 0) {
    c.ck_i[it.ck + b] = 0.0;
    c.ck_u[it.ck + b] = u;
  }
  // a diode or a controlled switch starts in its initial state
  if (c.dstate && (c.bkind[gb] == KIND_DIODE || c.bkind[gb] == KIND_CSWITCH)) c.dstate[gb] = on ? 1 : 0;
}

__global__ void k_fill_f64(double *p, int64_t n, double v) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) p[q] = v;
}

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) p[q] = v;
}

// Waveform mismatch of scenario blockIdx.x over its recorded columns:
// dJ = 2 (rec - target) and loss = sum (rec - target)^2, summed by each
// lane over a fixed stride and then by a fixed tree, so every run rounds
// identically. Columns past the scenario's n_rec get dJ = 0.
__global__ __launch_bounds__(256) void k_mismatch(const double *rec, const double *target, double *dJ, double *loss,
                                                  const int32_t *nrec, int64_t T, int R) {
  __shared__ double part[256];
  const int s = blockIdx.x, nr = nrec[s];
  const int64_t base = (int64_t)s * T * R, cnt = T * R;
  double acc = 0.0;
  for (int64_t q = threadIdx.x; q < cnt; q += 256) {
    const int col = (int)(q % R);
    const double d = col < nr ? rec[base + q] - target[base + q] : 0.0;
    dJ[base + q] = 2.0 * d;
    acc = acc + d * d;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] = part[threadIdx.x] + part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[s] = part[0];
}

__global__ void k_or_flag(int32_t *dst, const int32_t *src) {
  if (threadIdx.x == 0 && src[0] != 0) dst[0] = 1;
}

// State at step n from node voltages (already in c.sv_state) and branch
// currents: u = A^T v - e(n) and i on in-service branches, 0 elsewhere.
__global__ void k_set_state(DevCtx c, const int32_t *bitem, const int32_t *blocal, const int64_t *br_ids,
                            int64_t b0, int64_t nb, const double *i_in, int64_t n) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nb) return;
  const int64_t gb = br_ids[b0 + q];
  const ItemDesc it = c.items[bitem[gb]];
  const int b = blocal[gb];
  const int t = topo_at(c.topo + it.topo, it.n_topo, n);
  const bool on = c.cins[it.coef + (int64_t)t * it.n_br + b] != 0;
  const double *x = c.sv_state + it.node;
  const int k = c.bk[gb], m = c.bm[gb];
  const double vk = k >= 0 ? x[k] : 0.0, vm = m >= 0 ? x[m] : 0.0;
  const double e = (b < it.n_src) ? emf0(c, gb, n) : 0.0;
  c.su[gb] = on ? (vk - vm) - e : 0.0;
  c.si[gb] = on ? i_in[q] : 0.0;
}

// dJ/dtheta per (scenario, line) from the branch adjoints, in a fixed order:
//   series R-L:  dJ/dR += (gbar + gammabar)(-g^2) + betabar(-(4L/dt) g^2)
//                dJ/dL += (gbar + gammabar)(-(2/dt) g^2) + betabar((4R/dt) g^2)
//   shunt C/2:   dJ/dC += (gbar - gammabar) / dt
__global__ void k_grad(DevCtx c, const int32_t *lptr, const int64_t *lent, const int32_t *line_scen,
                       const int32_t *line_id, int n_lines_total, double *grad, int P) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_lines_total) return;
  const double dt = c.dt;
  double dR = 0.0, dL = 0.0, dC = 0.0;
  for (int e = lptr[q]; e < lptr[q + 1]; ++e) {
    const int64_t gb = lent[e];
    const int kind = c.bkind[gb];
    if (kind == KIND_RL) {
      const double R = c.bR[gb], L = c.bL[gb];
      const double g0 = 1.0 / (R + 2.0 * L / dt);
      const double g2 = g0 * g0;
      const double s = c.gbar[gb] + c.cbar[gb];
      dR = dR + s * (-g2) + c.bbar[gb] * (-(4.0 * L / dt) * g2);
      dL = dL + s * (-(2.0 / dt) * g2) + c.bbar[gb] * ((4.0 * R / dt) * g2);
    } else if (kind == KIND_C) {
      dC = dC + (c.gbar[gb] - c.cbar[gb]) / dt;
    }
  }
  double *gr = grad + (int64_t)line_scen[q] * P + 3 * line_id[q];
  gr[0] = dR;
  gr[1] = dL;
  gr[2] = dC;
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------

size_t lds_bytes(const LdsShape &s, bool sm, bool adjoint) {
  auto arr = [](size_t cnt, size_t size) { return (cnt * size + 15) & ~(size_t)15; };
  size_t b = arr(s.d + 1, 8) + arr(s.n + 1, 8) + arr(s.nbr, 8) + arr(adjoint ? s.n : 0, 8) + arr(adjoint ? 1 : 0, 4);
  if (sm) {
    b += arr(s.nsv, 8) + arr(s.ns, 8) + arr(s.nfdesc, 8) + arr(s.nbdesc, 8) + arr(s.n + 1, 4) +
         arr(adjoint ? s.n + 1 : 0, 4) + 3 * arr(s.nsv, 2) + arr(s.nent, 2) + 2 * arr(s.nrec, 2);
    // the factorisation's own structure for the refactorisations inside the
    // loop: row pointers, level pointers (rows, entries) and level rows
    if (s.dyn) b += arr(s.n + 1, 4) + 2 * arr(s.nlev + 1, 4) + arr(s.n, 2);
  }
  return b;
}

static unsigned blocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_factor(const DevCtx &c, const int32_t *pairs, int n_pairs, int max_tail, hipStream_t st) {
  if (n_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_factor<256>, dim3(n_pairs), dim3(256), 0, st, c, pairs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)max_tail * max_tail * sizeof(double) + 16;
  e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_tail), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tail, dim3(n_pairs), dim3(256), lds, st, c, pairs);
  return hipGetLastError();
}

hipError_t launch_companions(const DevCtx &c, const CompanionArgs &a, hipStream_t st) {
  if (a.total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_companions, dim3(blocks(a.total, 256)), dim3(256), 0, st, c, a.coef_base, a.br_base,
                     a.nbr_of, a.cnt_prefix, a.total, a.n_items);
  return hipGetLastError();
}

hipError_t launch_set_params(const DevCtx &c, const double *theta, int P, const int32_t *bscen,
                             int64_t nbr_total, hipStream_t st) {
  hipLaunchKernelGGL(k_set_params, dim3(blocks(nbr_total, 256)), dim3(256), 0, st, c, theta, P, bscen, nbr_total);
  return hipGetLastError();
}

hipError_t launch_reset(const DevCtx &c, const int32_t *bitem, const int32_t *blocal, int64_t nbr_total,
                        int64_t n_nodes_total, int64_t ring_doubles, hipStream_t st) {
  hipLaunchKernelGGL(k_reset, dim3(blocks(nbr_total, 256)), dim3(256), 0, st, c, bitem, blocal, nbr_total);
  hipLaunchKernelGGL(k_fill_f64, dim3(blocks(n_nodes_total, 256)), dim3(256), 0, st, c.sv_state, n_nodes_total,
                     0.0);
  // travelling-wave histories: every line starts at rest
  if (ring_doubles > 0)
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks(ring_doubles, 256)), dim3(256), 0, st, c.ring, ring_doubles, 0.0);
  return hipGetLastError();
}

hipError_t launch_set_state(const DevCtx &c, const int32_t *bitem, const int32_t *blocal, const int64_t *br_ids,
                            int64_t b0, int64_t nb, const double *i_in, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_set_state, dim3(blocks(nb, 256)), dim3(256), 0, st, c, bitem, blocal, br_ids, b0, nb, i_in,
                     n);
  return hipGetLastError();
}

hipError_t launch_grad(const DevCtx &c, const int32_t *lptr, const int64_t *lent, const int32_t *line_scen,
                       const int32_t *line_id, int n_lines_total, double *grad, int P, int64_t grad_len,
                       hipStream_t st) {
  if (grad_len > 0)
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks(grad_len, 256)), dim3(256), 0, st, grad, grad_len, 0.0);
  if (n_lines_total > 0)
    hipLaunchKernelGGL(k_grad, dim3(blocks(n_lines_total, 256)), dim3(256), 0, st, c, lptr, lent, line_scen,
                       line_id, n_lines_total, grad, P);
  return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i64, dim3(blocks(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_mismatch(const double *rec, const double *target, double *dJ, double *loss, const int32_t *nrec,
                           int n_scen, int64_t T, int R, hipStream_t st) {
  if (n_scen == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mismatch, dim3(n_scen), dim3(256), 0, st, rec, target, dJ, loss, nrec, T, R);
  return hipGetLastError();
}

hipError_t launch_or_flag(int32_t *dst, const int32_t *src, hipStream_t st) {
  hipLaunchKernelGGL(k_or_flag, dim3(1), dim3(64), 0, st, dst, src);
  return hipGetLastError();
}

}  // namespace emt
