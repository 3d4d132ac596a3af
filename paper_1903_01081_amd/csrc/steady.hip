// Sinusoidal steady state of every item's initial topology, the usual start
// of an EMTP-type run (not one of the paper's basic processes). With all
// sources of a scenario at one angular frequency w, the companion recursion
// i_n = g u_n + h_n, h_{n+1} = beta i_n + gamma u_n has the periodic solution
// x_n = Re(X z^n), z = exp(j w dt), in which each branch acts as the discrete
// admittance y = (g z + gamma) / (z - beta). One workgroup per item solves
// (A y A^T) V = A y E on the item's own symbolic LDL^T pattern (complex
// symmetric, no pivoting: the real part of Y is positive definite when every
// node reaches ground through resistance, and a zero or non-finite pivot is
// counted and reported), then writes the state at step 0: v = Re V,
// u = Re(A^T V - E), i = Re(y u) on in-service branches.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"
#include "launch.h"

namespace emt {

namespace {

struct cplx {
  double re, im;
};

__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// Scalar discrete admittance (g z + gamma) / (z - beta).
__device__ __forceinline__ cplx scalar_admittance(double g, double gam, double be, cplx z) {
  const cplx num = {g * z.re + gam, g * z.im};
  const cplx den = {z.re - be, z.im};
  return (g == 0.0 && gam == 0.0) ? cplx{0.0, 0.0} : cdiv(num, den);
}

// Discrete admittance of local branch b of an item in topology 0; for a
// member of a coupled group (class "pass": lines are refused before this
// kernel runs) the diagonal of its circulant admittance, with the
// off-diagonal in *mutual: per sequence (zero: d + 2o, positive: d - o) the
// scalar admittance, then back to the circulant.
__device__ __forceinline__ cplx admittance(const DevCtx &c, const ItemDesc &it, int b, cplx z,
                                           cplx *mutual = nullptr) {
  const double g = c.cg[it.coef + b], be = c.cb[it.coef + b];
  const uint32_t cls = c.bpack[it.br + b] >> 30;
  if (cls == GAMMA_PASS) {
    const double go = c.cgo[it.coef + b], bo = c.cbo[it.coef + b];
    const double sg = c.bkind[it.br + b] == KIND_C ? -1.0 : 1.0;
    const cplx y0 = scalar_admittance(g + 2.0 * go, sg * (g + 2.0 * go), be + 2.0 * bo, z);
    const cplx y1 = scalar_admittance(g - go, sg * (g - go), be - bo, z);
    if (mutual) *mutual = {(y0.re - y1.re) / 3.0, (y0.im - y1.im) / 3.0};
    return {(y0.re + 2.0 * y1.re) / 3.0, (y0.im + 2.0 * y1.im) / 3.0};
  }
  if (mutual) *mutual = {0.0, 0.0};
  const double gam = cls == GAMMA_PLUS_G ? g : (cls == GAMMA_MINUS_G ? -g : 0.0);
  return scalar_admittance(g, gam, be, z);
}

// Source phasor E exp(j phase) of local branch b (0 for other branches).
__device__ __forceinline__ cplx source_phasor(const DevCtx &c, const ItemDesc &it, int b) {
  if (b >= it.n_src) return {0.0, 0.0};
  const int64_t gb = it.br + b;
  double s, co;
  sincos(c.bph[gb], &s, &co);
  return {c.bE[gb] * co, c.bE[gb] * s};
}

template <int BS>
__global__ __launch_bounds__(BS) void k_steady(DevCtx c, const int64_t *off_l, const int64_t *off_n, cplx *Lc,
                                               cplx *Dc, cplx *X, int32_t *bad) {
  const ItemDesc it = c.items[blockIdx.x];
  const SymDesc sd = c.syms[it.sym];
  const int n = it.n;
  const int32_t *rowptr = c.symi + sd.rowptr, *rowcol = c.symi + sd.rowcol;
  const int32_t *colptr = c.symi + sd.colptr, *colrow = c.symi + sd.colrow, *colpos = c.symi + sd.colpos;
  const int32_t *flevptr = c.symi + sd.flevptr, *flevrows = c.symi + sd.flevrows;
  const int32_t *fentptr = c.symi + sd.fentptr, *fent = c.symi + sd.fent;
  const int32_t *blevptr = c.symi + sd.blevptr, *blevrows = c.symi + sd.blevrows;
  const int32_t *nptr = c.nptr + it.nptr;
  const uint16_t *nent = c.nent + it.nent;
  const int32_t *bk = c.bk + it.br, *bm = c.bm + it.br, *gpos = c.bgpos + it.br;
  cplx *L = Lc + off_l[blockIdx.x];
  cplx *D = Dc + off_n[blockIdx.x];
  cplx *x = X + off_n[blockIdx.x];
  // the scenario's frequency, from the item's first source (sources are
  // numbered first); an item without sources rests at zero
  cplx z = {1.0, 0.0};
  const bool driven = it.n_src > 0;
  if (driven) sincos(c.bw[it.br] * c.dt, &z.im, &z.re);

  if (driven) {
    // Y on the pattern of L (strictly lower part) and its diagonal; the
    // right-hand side A y E from the sources
    for (int r = threadIdx.x; r < n; r += BS) {
      for (int q = rowptr[r]; q < rowptr[r + 1]; ++q) L[q] = {0.0, 0.0};
      cplx d = {0.0, 0.0}, rhs = {0.0, 0.0};
      for (int e = nptr[r]; e < nptr[r + 1]; ++e) {
        const int ent = nent[e];
        const int b = ent >> 1;
        const cplx y = admittance(c, it, b, z);
        d = cadd(d, y);
        const cplx yE = cmul(y, source_phasor(c, it, b));
        rhs = (ent & 1) ? csub(rhs, yE) : cadd(rhs, yE);
        const int other = (ent & 1) ? bk[b] : bm[b];
        if (other >= 0 && other < r) L[gpos[b]] = csub(L[gpos[b]], y);
      }
      D[r] = d;
      x[r] = rhs;
      if (it.n_groups > 0) {
        // mutual admittances of coupled groups (+y_o between like terminals
        // of two members, -y_o between a k and an m terminal)
        const int32_t *mp = c.mptr + it.mptr;
        const int32_t *me = c.ment + it.ment;
        for (int e = mp[r]; e < mp[r + 1]; ++e) {
          const int pos = me[2 * e], code = me[2 * e + 1];
          cplx yo;
          admittance(c, it, code >> 1, z, &yo);
          L[pos] = (code & 1) ? csub(L[pos], yo) : cadd(L[pos], yo);
        }
      }
    }
    __syncthreads();
    // LDL^T by the factorisation's levels: pivots of a level's rows, then the
    // entries of their columns
    for (int l = 0; l < sd.nlev; ++l) {
      for (int p = flevptr[l] + threadIdx.x; p < flevptr[l + 1]; p += BS) {
        const int j = flevrows[p];
        cplx d = D[j];
        for (int q = rowptr[j]; q < rowptr[j + 1]; ++q) d = csub(d, cmul(cmul(L[q], L[q]), D[rowcol[q]]));
        D[j] = d;
        const double m2 = d.re * d.re + d.im * d.im;
        if (!(m2 > 0.0) || !isfinite(m2)) atomicAdd(bad, 1);
      }
      __syncthreads();
      for (int p = fentptr[l] + threadIdx.x; p < fentptr[l + 1]; p += BS) {
        const int e = fent[p];
        const int i = colrow[e];
        const int pos = colpos[e];
        const int j = rowcol[pos];
        cplx s = L[pos];
        int qi = rowptr[i], qj = rowptr[j];
        const int qi1 = rowptr[i + 1], qj1 = rowptr[j + 1];
        while (qi < qi1 && qj < qj1) {
          const int ci = rowcol[qi], cj = rowcol[qj];
          if (ci >= j) break;
          if (ci == cj) {
            s = csub(s, cmul(cmul(L[qi], D[ci]), L[qj]));
            ++qi;
            ++qj;
          } else if (ci < cj) {
            ++qi;
          } else {
            ++qj;
          }
        }
        L[pos] = cdiv(s, D[j]);
      }
      __syncthreads();
    }
    // L w = rhs by forward levels, w / D, L^T x = w by backward levels
    for (int l = 0; l < sd.nlev; ++l) {
      for (int p = flevptr[l] + threadIdx.x; p < flevptr[l + 1]; p += BS) {
        const int j = flevrows[p];
        cplx s = x[j];
        for (int q = rowptr[j]; q < rowptr[j + 1]; ++q) s = csub(s, cmul(L[q], x[rowcol[q]]));
        x[j] = s;
      }
      __syncthreads();
    }
    for (int r = threadIdx.x; r < n; r += BS) x[r] = cdiv(x[r], D[r]);
    __syncthreads();
    for (int l = 0; l < sd.nlevb; ++l) {
      for (int p = blevptr[l] + threadIdx.x; p < blevptr[l + 1]; p += BS) {
        const int j = blevrows[p];
        cplx s = x[j];
        for (int e = colptr[j]; e < colptr[j + 1]; ++e) s = csub(s, cmul(L[colpos[e]], x[colrow[e]]));
        x[j] = s;
      }
      __syncthreads();
    }
  } else {
    for (int r = threadIdx.x; r < n; r += BS) x[r] = {0.0, 0.0};
    __syncthreads();
  }
  // the state at step 0
  for (int r = threadIdx.x; r < n; r += BS) c.sv_state[it.node + r] = x[r].re;
  for (int b = threadIdx.x; b < it.n_br; b += BS) {
    const int64_t gb = it.br + b;
    const bool on = c.cins[it.coef + b] != 0;
    double iv = 0.0, uv = 0.0;
    if (on && driven) {
      const cplx vk = bk[b] >= 0 ? x[bk[b]] : cplx{0.0, 0.0};
      const cplx vm = bm[b] >= 0 ? x[bm[b]] : cplx{0.0, 0.0};
      const cplx u = csub(csub(vk, vm), source_phasor(c, it, b));
      iv = cmul(admittance(c, it, b, z), u).re;
      uv = u.re;
    } else if (on) {
      // no source in the item: at rest, u = -e(0) = 0
      uv = 0.0;
    }
    // a coupled member's current needs the other members' voltages: the
    // group loop below writes it
    if (!(driven && (c.bpack[gb] >> 30) == GAMMA_PASS)) c.si[gb] = iv;
    c.su[gb] = uv;
    if (c.K > 0) {
      c.ck_i[it.ck + b] = iv;
      c.ck_u[it.ck + b] = uv;
    }
  }
  if (it.n_groups > 0 && driven) {
    // members of coupled groups: i_p = y_d u_p + y_o (S_u - u_p) (members
    // carry no source; coupled groups take no checkpoints)
    for (int q = threadIdx.x; q < it.n_groups; q += BS) {
      const GroupDesc gd = c.group_tab[it.groups + q];
      cplx u[3], su = {0.0, 0.0};
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        const cplx vk = gd.k[p] < n ? x[gd.k[p]] : cplx{0.0, 0.0};
        const cplx vm = gd.m[p] < n ? x[gd.m[p]] : cplx{0.0, 0.0};
        u[p] = csub(vk, vm);
        su = cadd(su, u[p]);
      }
      cplx yo;
      const cplx yd = admittance(c, it, gd.b[0], z, &yo);
#pragma unroll
      for (int p = 0; p < 3; ++p) c.si[it.br + gd.b[p]] = cadd(cmul(yd, u[p]), cmul(yo, csub(su, u[p]))).re;
    }
  }
}

}  // namespace

hipError_t launch_steady(const DevCtx &c, int n_items, const int64_t *off_l, const int64_t *off_n, void *Lc,
                         void *Dc, void *X, int32_t *bad, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_steady<256>, dim3(n_items), dim3(256), 0, st, c, off_l, off_n, static_cast<cplx *>(Lc),
                     static_cast<cplx *>(Dc), static_cast<cplx *>(X), bad);
  return hipGetLastError();
}

}  // namespace emt
