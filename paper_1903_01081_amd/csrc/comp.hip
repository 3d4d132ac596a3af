// Compensation solver kernels (the method is described in comp.h), FP64,
// gfx950.
//
// emt_factor: per family the base matrix G0 is assembled densely from the
// base item's conductances and inverted in place (Gauss-Jordan: G0 is
// symmetric positive definite, so no pivoting), the pi-section branches that
// items share with their base are checked for equal parameters, and per item
// and topology the r x r matrix K = (D^-1 + U^T Z U)^-1 is formed.
//
// k_comp, the time loop: one workgroup holds nq <= Q items of one family,
// each with its branch state in VGPRs (the same branch phase as k_forward)
// and its injections, right-hand side and voltages in LDS. Per step:
//   gather      rhs of every item in the base's node order;
//   product     w = Z rhs for all items at once, one row of Z per lane, Z
//               read from L2 once per workgroup and step and applied to
//               every item's right-hand side;
//   correction  v = w - (Z U) K (U^T w) for the items whose topology
//               differs from the base (U^T w reads two entries of w per
//               switched branch, Z U two rows of Z);
//   branch      record, u = A^T v - e, i = g u + h, next history and
//               injections.
// FP64 matrix cores would not help the product: the MI355X runs FP64 MFMA at
// the FP64 vector rate, and a workgroup holds only a few right-hand sides.
#include <hip/hip_runtime.h>

#include "comp.h"
#include "launch.h"
#include "step.h"

namespace emt {

namespace {

using step::emt_lds;
using step::lds_barrier;

__global__ __launch_bounds__(kCompBS) void k_comp_assemble(DevCtx c, CompCtx cc) {
  const CompFamily F = cc.fam[blockIdx.x];
  const ItemDesc it = c.items[F.base];
  double *Z = cc.z + F.z;
  const int n = F.n;
  const int32_t *nptr = c.nptr + it.nptr;
  const uint16_t *nent = c.nent + it.nent;
  for (int r = threadIdx.x; r < n; r += kCompBS) {
    double *row = Z + (int64_t)r * n;
    for (int j = 0; j < n; ++j) row[j] = 0.0;
    double diag = 0.0;
    for (int e = nptr[r]; e < nptr[r + 1]; ++e) {
      const int ent = nent[e];
      const int j = ent >> 1;
      const double g = c.cg[it.coef + j];  // topology 0
      const int other = (ent & 1) ? c.bk[it.br + j] : c.bm[it.br + j];
      diag += g;
      if (other >= 0) row[other] -= g;
    }
    row[r] += diag;
  }
}

// In-place Gauss-Jordan inversion of one family's G0 (symmetric positive
// definite): after pivot p, a_pp <- 1/a_pp, row p scaled by it, column p
// scaled by -1/a_pp, the rest updated a_ij -= a_ip a_pj / a_pp; then
// symmetrised (the two triangles round differently). A non-positive or
// non-finite pivot is counted in flags[0].
constexpr int kInvBS = 512;
__global__ __launch_bounds__(kInvBS) void k_comp_invert(CompCtx cc, int32_t *flags) {
  const CompFamily F = cc.fam[blockIdx.x];
  double *A = cc.z + F.z;
  const int n = F.n;
  __shared__ double rowp[kCompMaxNodes], colp[kCompMaxNodes];
  const int nn = n * n;
  for (int p = 0; p < n; ++p) {
    for (int j = threadIdx.x; j < n; j += kInvBS) {
      rowp[j] = A[(int64_t)p * n + j];
      colp[j] = A[(int64_t)j * n + p];
    }
    __syncthreads();
    const double piv = rowp[p];
    const bool ok = piv > 0.0 && piv < INFINITY;
    if (!ok && threadIdx.x == 0) atomicAdd(flags, 1);
    const double d = ok ? 1.0 / piv : 0.0;
    for (int e = threadIdx.x; e < nn; e += kInvBS) {
      const int i = e / n, j = e - i * n;
      double a;
      if (i == p)
        a = (j == p) ? d : rowp[j] * d;
      else if (j == p)
        a = -(colp[i] * d);
      else
        a = A[e] - colp[i] * (rowp[j] * d);
      A[e] = a;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nn; e += kInvBS) {
    const int i = e / n, j = e - i * n;
    if (i < j) {
      const double s = 0.5 * (A[e] + A[(int64_t)j * n + i]);
      A[e] = s;
      A[(int64_t)j * n + i] = s;
    }
  }
}

// Pi-section branches matched to their base take R, L, C from their own
// scenario's theta: they must equal the base's (counted in flags[5]).
__global__ void k_comp_check(DevCtx c, CompCtx cc) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= cc.n_pairs) return;
  const int64_t a = cc.pairs[2 * q], b = cc.pairs[2 * q + 1];
  if (c.bR[a] != c.bR[b] || c.bL[a] != c.bL[b] || c.bC[a] != c.bC[b]) atomicAdd(c.flags + 5, 1);
}

// K = (D^-1 + U^T Z U)^-1 of every (item, topology), r x r, by Gauss-Jordan
// with partial pivoting; a zero or non-finite pivot is counted in flags[6].
__global__ void k_comp_k(DevCtx c, CompCtx cc) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= cc.n_mods) return;
  const CompMod md = cc.mods[q];
  double *Kq = cc.K + (int64_t)q * 16;
  for (int e = 0; e < 16; ++e) Kq[e] = 0.0;
  const int r = md.r;
  if (r == 0) return;
  const CompFamily F = cc.fam[md.fam];
  const double *Z = cc.z + F.z;
  const int n = F.n;
  auto z = [&](int i, int j) { return (i < 0 || j < 0) ? 0.0 : Z[(int64_t)i * n + j]; };
  double M[kCompMaxRank][2 * kCompMaxRank];
  for (int a = 0; a < r; ++a) {
    for (int b = 0; b < r; ++b) {
      const double v = z(md.k[a], md.k[b]) - z(md.k[a], md.m[b]) - z(md.m[a], md.k[b]) + z(md.m[a], md.m[b]);
      M[a][b] = v;
      M[a][r + b] = (a == b) ? 1.0 : 0.0;
    }
    const double g = c.cg[md.g[a]];
    M[a][a] += 1.0 / ((double)md.sgn[a] * g);
  }
  bool ok = true;
  for (int p = 0; p < r; ++p) {
    int best = p;
    for (int i = p + 1; i < r; ++i)
      if (fabs(M[i][p]) > fabs(M[best][p])) best = i;
    if (best != p)
      for (int j = 0; j < 2 * r; ++j) {
        const double t = M[p][j];
        M[p][j] = M[best][j];
        M[best][j] = t;
      }
    const double piv = M[p][p];
    if (!(fabs(piv) > 0.0) || !(fabs(piv) < INFINITY)) {
      ok = false;
      break;
    }
    const double d = 1.0 / piv;
    for (int j = 0; j < 2 * r; ++j) M[p][j] *= d;
    for (int i = 0; i < r; ++i) {
      if (i == p) continue;
      const double f = M[i][p];
      for (int j = 0; j < 2 * r; ++j) M[i][j] -= f * M[p][j];
    }
  }
  if (!ok) {
    atomicAdd(c.flags + 6, 1);
    return;
  }
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < r; ++b) Kq[a * 4 + b] = M[a][r + b];
}

// Layout of a k_comp workgroup. Item q of the workgroup is run by lanes
// q*SB .. q*SB+SB-1 (its "sub-group": branch phase, gather and correction);
// the product uses every lane. Per item slot (byte offsets, 16-byte
// aligned parts):
//   meta   int32 [16]: scen, n_src, n_rec, n_topo, mod0, r, k[4], m[4];
//          int64 [8] from byte 64: br, coef, node, topo
//   K      [16]  the current topology's K (leading dimension 4)
//   x      [n+1] voltages in the item's node order (x[n] = 0: the ground);
//                between the gather and the correction the same array
//                holds the right-hand side in the base's node order
//   J      [nbr] branch injections
//   zu     [4n]  Z u_a of the current topology's switched branches
//   perm   [2n]  uint16: item -> base node map, base -> item
//   nptr   [n+1] int32, nent [ne] uint16: the item's node CSR
//   rnode, rcol [nr] uint16: recorded nodes and their columns
//   src    [ns][3] the sources' E, omega, phase (slot 0 of the first ns lanes)
// After the Q slots: the product's partial sums P [KS][Q][n].
struct CompSlot {
  uint32_t meta, K, x, J, zu, perm, nptr, nent, rnode, rcol, src, bytes;
};
__host__ __device__ inline uint32_t align16(uint32_t b) { return (b + 15u) & ~15u; }
__host__ __device__ inline CompSlot comp_slot(int n, int nbr, int ne, int nr, int ns) {
  CompSlot s;
  uint32_t o = 0;
  auto take = [&o](uint32_t b) {
    const uint32_t r = o;
    o += align16(b);
    return r;
  };
  s.meta = take(128);
  s.K = take(16 * 8);
  s.x = take((uint32_t)(n + 1) * 8u);
  s.J = take((uint32_t)nbr * 8u);
  s.zu = take((uint32_t)kCompMaxRank * n * 8u);
  s.perm = take((uint32_t)(2 * n) * 2u);
  s.nptr = take((uint32_t)(n + 1) * 4u);
  s.nent = take((uint32_t)ne * 2u);
  s.rnode = take((uint32_t)nr * 2u);
  s.rcol = take((uint32_t)nr * 2u);
  s.src = take(3u * 8u * (uint32_t)ns);
  s.bytes = o;
  return s;
}
// k-splits of the product: lanes are (split, row) pairs over rows rounded
// up to whole waves, at most 4 splits.
__host__ __device__ inline int comp_ksplits(int n, int bs) {
  const int rw = (n + 63) / 64 * 64;
  const int ks = bs / rw;
  return ks < 1 ? 1 : (ks > 4 ? 4 : ks);
}
__host__ __device__ inline uint32_t comp_lds(int n, int nbr, int ne, int nr, int ns, int q, int bs) {
  return (uint32_t)q * comp_slot(n, nbr, ne, nr, ns).bytes + align16((uint32_t)(comp_ksplits(n, bs) * q * n) * 8u);
}

// A value hidden from the optimiser at each use, so that per-slot index and
// address arithmetic inside the time loop is recomputed there (a few
// integer operations) instead of being hoisted out of it into VGPRs.
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Values that are the same in every lane of a wave (a sub-group is whole
// waves), moved to scalar registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

enum { M_SCEN = 0, M_NSRC, M_NREC, M_NTOPO, M_MOD0, M_R, M_K, M_M = M_K + 4 };
enum { M64_BR = 8, M64_COEF, M64_NODE, M64_TOPO };

constexpr int kChunk = 8;        // k ranges of the product splits are multiples of this
constexpr int kCompQMax = kCompMaxItems;  // accumulators per lane of the product

// SB lanes per item, BPT branch slots per lane; Q = blockDim.x / SB items.
template <int SB, int BPT>
__global__ __launch_bounds__(1024) void k_comp(DevCtx c, CompCtx cc, int Q, int64_t n0, int64_t nsteps, double *rec) {
  const CompBlock blk = cc.blocks[blockIdx.x];
  const int nq = blk.nq;
  const int BS = blockDim.x;  // at least SB * Q; the lanes past them join the gather, product and correction
  const CompFamily F = cc.fam[blk.family];
  const int n = F.n;
  const double *Z = cc.z + F.z;
  const int tid = threadIdx.x;
  const int sq = uni(tid / SB);   // this lane's item slot (whole waves)
  const int jl = tid - sq * SB;   // lane within the sub-group
  const bool mine = sq < nq;      // the slot holds an item
  const int nbr = SB * BPT;
  const CompSlot S = comp_slot(n, nbr, cc.ne_max, cc.nr_max, cc.ns_max);
  char *slot = emt_lds + sq * S.bytes;
  int32_t *m32 = reinterpret_cast<int32_t *>(slot + S.meta);
  int64_t *m64 = reinterpret_cast<int64_t *>(slot + S.meta);
  double *Kq = reinterpret_cast<double *>(slot + S.K);
  double *x = reinterpret_cast<double *>(slot + S.x);
  double *J = reinterpret_cast<double *>(slot + S.J);
  double *zu = reinterpret_cast<double *>(slot + S.zu);
  uint16_t *perm = reinterpret_cast<uint16_t *>(slot + S.perm);
  int32_t *nptr = reinterpret_cast<int32_t *>(slot + S.nptr);
  uint16_t *nent = reinterpret_cast<uint16_t *>(slot + S.nent);
  uint16_t *rnode = reinterpret_cast<uint16_t *>(slot + S.rnode);
  uint16_t *rcol = reinterpret_cast<uint16_t *>(slot + S.rcol);
  double *src = reinterpret_cast<double *>(slot + S.src);
  const int KS = comp_ksplits(n, BS);
  double *P = reinterpret_cast<double *>(emt_lds + Q * S.bytes);  // [KS][Q][n]

  // the correction data of topology t: r, terminals, K and the vectors
  // Z u_a (rows k_a and m_a of Z, Z being symmetric), by the sub-group
  auto load_corr = [&](int mod0, int t) {
    const int mi = mod0 + t;
    const CompMod *md = cc.mods + mi;
    const int r = md->r;
    if (jl == 0) {
      m32[M_R] = r;
      for (int a = 0; a < kCompMaxRank; ++a) {
        m32[M_K + a] = md->k[a];
        m32[M_M + a] = md->m[a];
      }
    }
    if (jl < 16) Kq[jl] = cc.K[(int64_t)mi * 16 + jl];
    for (int a = 0; a < r; ++a) {
      const int ka = md->k[a], ma = md->m[a];
      for (int i = jl; i < n; i += SB) {
        const double zk = ka >= 0 ? Z[(int64_t)ka * n + i] : 0.0;
        const double zm = ma >= 0 ? Z[(int64_t)ma * n + i] : 0.0;
        zu[a * n + i] = zk - zm;
      }
    }
  };

  // Branch state of this lane's slots (the same recursion as k_forward's
  // branch phase): packed terminals, coefficients, the source of slot 0.
  uint32_t pk[BPT];
  double g[BPT], be[BPT];
  double h0 = 0.0, e0 = 0.0;
  int t = 0;
  int64_t next = step::kNever;
  int nsrc = 0;
  int64_t br = 0, coef = 0;
  if (mine) {
    const int item = uni(cc.list[blk.q0 + sq]);
    const ItemDesc it = c.items[item];
    const int64_t *topo = c.topo + it.topo;
    t = uni(step::topo_of(topo, it.n_topo, n0 + 1));
    next = uni64((t + 1 < it.n_topo) ? topo[t + 1] : step::kNever);
    nsrc = uni(it.n_src);
    br = uni64(it.br);
    coef = uni64(it.coef);
    if (jl == 0) {
      m32[M_SCEN] = it.scen;
      m32[M_NSRC] = it.n_src;
      m32[M_NREC] = it.n_rec;
      m32[M_NTOPO] = it.n_topo;
      m32[M_MOD0] = cc.mod0[item];
      m64[M64_BR] = it.br;
      m64[M64_COEF] = it.coef;
      m64[M64_NODE] = it.node;
      m64[M64_TOPO] = it.topo;
      x[n] = 0.0;
    }
    const uint16_t *g_perm = cc.perm + cc.poff[item];
    for (int i = jl; i < 2 * n; i += SB) perm[i] = g_perm[i];
    const int32_t *g_nptr = c.nptr + it.nptr;
    const uint16_t *g_nent = c.nent + it.nent;
    for (int r = jl; r <= n; r += SB) nptr[r] = g_nptr[r];
    const int ne = g_nptr[n];
    for (int e = jl; e < ne; e += SB) nent[e] = g_nent[e];
    for (int e = jl; e < it.n_rec; e += SB) {
      rnode[e] = c.rnode[it.rec + e];
      rcol[e] = c.rcolumn[it.rec + e];
    }
    load_corr(cc.mod0[item], t);
    const int64_t cb0 = coef + (int64_t)t * nbr;
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int b = jl + j * SB;
      pk[j] = c.bpack[br + b];
      g[j] = c.cg[cb0 + b];
      be[j] = c.cb[cb0 + b];
      const double h = be[j] * c.si[br + b] + step::gamma_of(pk[j], g[j]) * c.su[br + b];
      if (j == 0)
        h0 = h;
      else
        J[b] = -h;
    }
    if (jl < nsrc) {
      const double sE = c.bE[br + jl], sw = c.bw[br + jl], sph = c.bph[br + jl];
      src[3 * jl] = sE;
      src[3 * jl + 1] = sw;
      src[3 * jl + 2] = sph;
      e0 = sE * emf_cos(sw * ((double)(n0 + 1) * c.dt) + sph);
    }
    J[jl] = g[0] * e0 - h0;
  } else {
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      pk[j] = 0;
      g[j] = 0.0;
      be[j] = 0.0;
    }
  }
  step::lds_barrier();

  const int R = c.rec_stride;
  const int64_t n_end = n0 + nsteps;
  // product lanes: (split g, row pr); k range of split g
  const int rw = (n + 63) / 64 * 64;
  const int pg = uni(tid / rw), pr = tid - pg * rw;
  const int kc = ((n + KS - 1) / KS + kChunk - 1) / kChunk * kChunk;
  const int KSe = (n + kc - 1) / kc;  // splits with a non-empty k range (<= KS)
  const int k0 = pg * kc, k1 = (pg + 1) * kc < n ? (pg + 1) * kc : n;
  const bool prod = pg < KSe && pr < n;
  for (int64_t s = n0 + 1; s <= n_end; ++s) {
    // gather: every (item, node) pair of the workgroup, the right-hand
    // side into the item's x in the base's node order
    for (int p = tid; p < nq * n; p += BS) {
      const int q = p / n, r = p - q * n;
      char *sl = emt_lds + q * S.bytes;
      const int32_t *np = reinterpret_cast<const int32_t *>(sl + S.nptr);
      const uint16_t *ne = reinterpret_cast<const uint16_t *>(sl + S.nent);
      const double *Jq = reinterpret_cast<const double *>(sl + S.J);
      double acc = 0.0;
      int e = np[r];
      const int e1 = np[r + 1];
      for (; e + 4 <= e1; e += 4) {
        const int a0 = ne[e], a1 = ne[e + 1], a2 = ne[e + 2], a3 = ne[e + 3];
        const double j0 = Jq[a0 >> 1], j1 = Jq[a1 >> 1], j2 = Jq[a2 >> 1], j3 = Jq[a3 >> 1];
        acc = (a0 & 1) ? acc - j0 : acc + j0;
        acc = (a1 & 1) ? acc - j1 : acc + j1;
        acc = (a2 & 1) ? acc - j2 : acc + j2;
        acc = (a3 & 1) ? acc - j3 : acc + j3;
      }
      for (; e < e1; ++e) {
        const int a0 = ne[e];
        const double j0 = Jq[a0 >> 1];
        acc = (a0 & 1) ? acc - j0 : acc + j0;
      }
      const uint16_t *pm = reinterpret_cast<const uint16_t *>(sl + S.perm);
      reinterpret_cast<double *>(sl + S.x)[pm[r]] = acc;
    }
    step::lds_barrier();
    // product: partial sums of w = Z rhs over this lane's k range for every
    // item of the workgroup (row pr of Z is its column pr). Z comes from L2
    // in chunks of kChunk rows, the next chunk in flight while the current
    // one is multiplied.
    if (prod) {
      double w[kCompQMax];
#pragma unroll
      for (int q = 0; q < kCompQMax; ++q) w[q] = 0.0;
      const double *zc = Z + opaque(pr);
      constexpr int CH = 8;
      const int nch = (k1 - k0) / CH, kf = k0 + nch * CH;
      // the workgroups of a family walk their chunks from different starts,
      // so that they do not all ask the same L2 channels for the same rows
      // at once
      const int c0 = nch > 0 ? (int)(blockIdx.x % (unsigned)nch) : 0;
      double zb[CH];
      if (nch > 0) {
        const int ks = k0 + c0 * CH;
#pragma unroll
        for (int u = 0; u < CH; ++u) zb[u] = zc[(int64_t)(ks + u) * n];
      }
      for (int ci = 0; ci < nch; ++ci) {
        int cc0 = c0 + ci;
        if (cc0 >= nch) cc0 -= nch;
        const int k = k0 + cc0 * CH;
        int cn = cc0 + 1;
        if (cn >= nch) cn -= nch;
        const int kn = k0 + cn * CH;
        double zn[CH];
        const bool more = ci + 1 < nch;
        if (more) {
#pragma unroll
          for (int u = 0; u < CH; ++u) zn[u] = zc[(int64_t)(kn + u) * n];
        }
#pragma unroll
        for (int q = 0; q < kCompQMax; ++q) {
          if (q >= nq) break;
          const double2 *xb = reinterpret_cast<const double2 *>(
              reinterpret_cast<const double *>(emt_lds + q * S.bytes + S.x) + k);
#pragma unroll
          for (int u = 0; u < CH / 2; ++u) {
            const double2 a = xb[u];
            w[q] = __builtin_fma(zb[2 * u], a.x, w[q]);
            w[q] = __builtin_fma(zb[2 * u + 1], a.y, w[q]);
          }
        }
        if (more) {
#pragma unroll
          for (int u = 0; u < CH; ++u) zb[u] = zn[u];
        }
      }
      if (kf < k1) {
        double zt[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) zt[u] = (kf + u < k1) ? zc[(int64_t)(kf + u) * n] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (kf + u >= k1) break;
#pragma unroll
          for (int q = 0; q < kCompQMax; ++q) {
            if (q >= nq) break;
            const double *xb = reinterpret_cast<const double *>(emt_lds + q * S.bytes + S.x);
            w[q] = __builtin_fma(zt[u], xb[kf + u], w[q]);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < kCompQMax; ++q) {
        if (q >= nq) break;
        P[(pg * Q + q) * n + pr] = w[q];
      }
    }
    step::lds_barrier();
    // correction: w = sum of the partials; v = w - sum_a (K y)_a Z u_a with
    // y_a = u_a^T w; the voltages into x in the item's node order; every
    // (item, node) pair of the workgroup
    for (int p = tid; p < nq * n; p += BS) {
      const int q = p / n, i = p - q * n;
      char *sl = emt_lds + q * S.bytes;
      const int32_t *mq = reinterpret_cast<const int32_t *>(sl + S.meta);
      const int r = mq[M_R];
      double v = 0.0;
      for (int gg = 0; gg < KSe; ++gg) v = v + P[(gg * Q + q) * n + i];
      if (r > 0) {
        const double *Kr = reinterpret_cast<const double *>(sl + S.K);
        const double *zq = reinterpret_cast<const double *>(sl + S.zu);
        double y[kCompMaxRank];
#pragma unroll
        for (int a = 0; a < kCompMaxRank; ++a) {
          y[a] = 0.0;
          if (a < r) {
            const int ka = mq[M_K + a], ma = mq[M_M + a];
            for (int gg = 0; gg < KSe; ++gg) {
              const double *pw = P + (gg * Q + q) * n;
              const double wk = ka >= 0 ? pw[ka] : 0.0, wm = ma >= 0 ? pw[ma] : 0.0;
              y[a] = y[a] + (wk - wm);
            }
          }
        }
#pragma unroll
        for (int a = 0; a < kCompMaxRank; ++a) {
          if (a >= r) continue;
          double za = 0.0;
#pragma unroll
          for (int b = 0; b < kCompMaxRank; ++b)
            if (b < r) za = za + Kr[a * 4 + b] * y[b];
          v = v - za * zq[a * n + i];
        }
      }
      const uint16_t *pm = reinterpret_cast<const uint16_t *>(sl + S.perm);
      reinterpret_cast<double *>(sl + S.x)[pm[n + i]] = v;
    }
    step::lds_barrier();
    // record, branch update, next injections
    if (mine) {
      if (rec) {
        double *row = rec + ((int64_t)uni(m32[M_SCEN]) * nsteps + (s - n0 - 1)) * R;
        const int nrec = uni(m32[M_NREC]);
        for (int e = jl; e < nrec; e += SB) row[rcol[e]] = x[rnode[e]];
      }
      const bool swn = (s + 1 == next);
      const bool inj = s < n_end;
      const int64_t ncoef = coef + (int64_t)(t + 1) * nbr;
      double e_next = 0.0;
      if (inj && jl < nsrc) e_next = src[3 * jl] * emf_cos(src[3 * jl + 1] * ((double)(s + 1) * c.dt) + src[3 * jl + 2]);
      const int jo = opaque(jl);
#pragma unroll
      for (int j = 0; j < BPT; ++j) {
        const int b = jo + j * SB;
        const double vk = x[pk[j] & kTermGround], vm = x[(pk[j] >> 15) & kTermGround];
        const double e = j == 0 ? e0 : 0.0;
        const double h = j == 0 ? h0 : -J[b];
        const double u = (g[j] != 0.0) ? (vk - vm) - e : 0.0;
        const double i = g[j] * u + h;
        if (s == n_end) {
          c.si[br + b] = i;
          c.su[br + b] = u;
        }
        if (swn) {
          g[j] = c.cg[ncoef + b];
          be[j] = c.cb[ncoef + b];
        }
        const double hn = be[j] * i + step::gamma_of(pk[j], g[j]) * u;
        if (j == 0) {
          h0 = hn;
          if (inj) J[b] = g[j] * e_next - hn;
        } else if (inj) {
          J[b] = -hn;
        }
      }
      e0 = e_next;
      if (swn) {
        ++t;
        const int64_t *topo = c.topo + uni64(m64[M64_TOPO]);
        next = uni64((t + 1 < uni(m32[M_NTOPO])) ? topo[t + 1] : step::kNever);
        load_corr(uni(m32[M_MOD0]), t);
      }
    }
    step::lds_barrier();
  }
  if (mine) {
    const int64_t node = uni64(m64[M64_NODE]);
    for (int r = jl; r < n; r += SB) c.sv_state[node + r] = x[r];
  }
}

template <int SB, int BPT>
hipError_t comp_launch(const DevCtx &c, const CompCtx &cc, int q, int lanes, int n_blocks, int64_t n0, int64_t ns,
                       double *rec, size_t lds, hipStream_t st) {
  auto k = k_comp<SB, BPT>;
  hipError_t e =
      hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(n_blocks), dim3(lanes), lds, st, c, cc, q, n0, ns, rec);
  return hipGetLastError();
}

int blocks_of(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

}  // namespace

int comp_lanes(int n, int q, int sb) {
  const int pairs = (n * q + 63) / 64 * 64;  // (item, node) pairs in whole waves
  const int l = sb * q > pairs ? sb * q : pairs;
  return l > 1024 ? 1024 : l;
}

size_t comp_lds_bytes(int n, int nbr, int q, int ne, int nr, int ns, int sb) {
  return comp_lds(n, nbr, ne, nr, ns, q, comp_lanes(n, q, sb));
}

// (lanes per item, branch slots per lane) pairs with an instantiated kernel
#define EMT_COMP_SB(X, SB) X(SB, 1) X(SB, 2) X(SB, 3) X(SB, 4) X(SB, 5) X(SB, 6) X(SB, 7) X(SB, 8)
#define EMT_COMP_SHAPES(X) EMT_COMP_SB(X, 64) EMT_COMP_SB(X, 128) EMT_COMP_SB(X, 192) EMT_COMP_SB(X, 256)

bool comp_shape_exists(int sb, int bpt, int q) {
  if (q < 1 || q > kCompQMax || sb * q > 1024) return false;
#define EMT_CASE(SB, B) \
  if (sb == SB && bpt == B) return true;
  EMT_COMP_SHAPES(EMT_CASE)
#undef EMT_CASE
  return false;
}

hipError_t launch_comp(const DevCtx &c, const CompCtx &cc, int sb, int bpt, int q, int lanes, int n_blocks,
                       int64_t n0, int64_t ns, double *rec, size_t lds, hipStream_t st) {
  if (!comp_shape_exists(sb, bpt, q) || lanes < sb * q || lanes > 1024 || lanes % 64) return hipErrorInvalidValue;
#define EMT_CASE(SB, B) \
  if (sb == SB && bpt == B) return comp_launch<SB, B>(c, cc, q, lanes, n_blocks, n0, ns, rec, lds, st);
  EMT_COMP_SHAPES(EMT_CASE)
#undef EMT_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_comp_factor(const DevCtx &c, const CompCtx &cc, hipStream_t st) {
  if (cc.n_fam <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_comp_assemble, dim3(cc.n_fam), dim3(kCompBS), 0, st, c, cc);
  hipLaunchKernelGGL(k_comp_invert, dim3(cc.n_fam), dim3(kInvBS), 0, st, cc, c.flags);
  if (cc.n_pairs > 0)
    hipLaunchKernelGGL(k_comp_check, dim3(blocks_of(cc.n_pairs, 256)), dim3(256), 0, st, c, cc);
  if (cc.n_mods > 0) hipLaunchKernelGGL(k_comp_k, dim3(blocks_of(cc.n_mods, 64)), dim3(64), 0, st, c, cc);
  return hipGetLastError();
}

}  // namespace emt
