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
using step::Lane;
using step::View;

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

// LDS of k_comp per item slot: x [n+1] (item order, x[n] = 0 is the
// ground), J [nbr], xb [n] (right-hand side, base order), wb [n+1] (w, base
// order, wb[n] = 0).
__host__ __device__ inline uint32_t align16(uint32_t b) { return (b + 15u) & ~15u; }
__host__ __device__ inline uint32_t comp_slot_bytes(int n, int nbr) {
  return align16((uint32_t)(n + 1) * 8u) + align16((uint32_t)nbr * 8u) + align16((uint32_t)n * 8u) +
         align16((uint32_t)(n + 1) * 8u);
}

constexpr int kChunk = 8;  // rows of Z in flight per lane

template <int BPT, int Q>
__global__ __launch_bounds__(kCompBS) void k_comp(DevCtx c, CompCtx cc, int64_t n0, int64_t nsteps, double *rec) {
  constexpr int BS = kCompBS;
  const CompBlock blk = cc.blocks[blockIdx.x];
  const int nq = blk.nq;
  const CompFamily F = cc.fam[blk.family];
  const int n = F.n;
  const double *Z = cc.z + F.z;
  const int tid = threadIdx.x;
  const int nbr = BS * BPT;
  const uint32_t slot = comp_slot_bytes(n, nbr);
  const uint32_t o_x = 0, o_j = align16((uint32_t)(n + 1) * 8u), o_xb = o_j + align16((uint32_t)nbr * 8u),
                 o_wb = o_xb + align16((uint32_t)n * 8u);
  auto X = [&](int q) { return reinterpret_cast<double *>(emt_lds + q * slot + o_x); };
  auto XB = [&](int q) { return reinterpret_cast<double *>(emt_lds + q * slot + o_xb); };
  auto WB = [&](int q) { return reinterpret_cast<double *>(emt_lds + q * slot + o_wb); };
  auto view = [&](int q, int nsrc) {
    View<false> v{};
    v.n = n;
    v.nbr = nbr;
    v.nsrc = nsrc;
    v.x.off = q * slot + o_x;
    v.J.off = q * slot + o_j;
    return v;
  };

  Lane<BPT> L[Q];
  int t[Q], pf[Q], pi[Q];
  int64_t next[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    t[q] = 0;
    next[q] = step::kNever;
    pf[q] = 0;
    pi[q] = 0;
    if (q < nq) {
      const ItemDesc it = c.items[cc.list[blk.q0 + q]];
      const int64_t *topo = c.topo + it.topo;
      t[q] = step::topo_of(topo, it.n_topo, n0 + 1);
      next[q] = (t[q] + 1 < it.n_topo) ? topo[t[q] + 1] : step::kNever;
      const uint16_t *perm = cc.perm + cc.poff[cc.list[blk.q0 + q]];
      if (tid < n) {
        pf[q] = perm[tid];
        pi[q] = perm[n + tid];
      }
      step::load_lane<BS, BPT>(c, it, L[q]);
      step::load_coefs<BS, BPT>(c, it, t[q], L[q].g, L[q].be);
      View<false> v = view(q, it.n_src);
      step::history_from_state<BS, BPT, false>(c.si + it.br, c.su + it.br, L[q], v);
      step::inject<BS, BPT, false>(c, v, L[q], n0 + 1);
      if (tid == 0) {
        X(q)[n] = 0.0;
        WB(q)[n] = 0.0;
      }
    } else {
      // an empty slot: its right-hand side stays zero
      for (int r = tid; r < n; r += BS) XB(q)[r] = 0.0;
    }
  }
  lds_barrier();

  const int R = c.rec_stride;
  const int64_t n_end = n0 + nsteps;
  for (int64_t s = n0 + 1; s <= n_end; ++s) {
    // gather: rhs in the base's node order
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (q >= nq) continue;
      const ItemDesc *ip = c.items + cc.list[blk.q0 + q];
      const int32_t *nptr = c.nptr + ip->nptr;
      const uint16_t *nent = c.nent + ip->nent;
      const double *J = reinterpret_cast<const double *>(emt_lds + q * slot + o_j);
      if (tid < n) {
        double acc = 0.0;
        const int e1 = nptr[tid + 1];
        for (int e = nptr[tid]; e < e1; ++e) {
          const int ent = nent[e];
          const double jv = J[ent >> 1];
          acc = (ent & 1) ? acc - jv : acc + jv;
        }
        XB(q)[pf[q]] = acc;
      }
    }
    lds_barrier();
    // product: w = Z rhs for every item (row tid of Z is column tid). Z is
    // read from L2 in chunks of kChunk rows, the next chunk's loads in
    // flight while the current one is multiplied; fused multiply-adds.
    double w[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) w[q] = 0.0;
    if (tid < n) {
      const double *zc = Z + tid;
      const int nfull = n / kChunk * kChunk;
      double zb[kChunk];
      if (nfull > 0) {
#pragma unroll
        for (int u = 0; u < kChunk; ++u) zb[u] = zc[(int64_t)u * n];
      }
      for (int k = 0; k < nfull; k += kChunk) {
        double zn[kChunk];
        const bool more = k + kChunk < nfull;
        if (more) {
#pragma unroll
          for (int u = 0; u < kChunk; ++u) zn[u] = zc[(int64_t)(k + kChunk + u) * n];
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const double2 *xb = reinterpret_cast<const double2 *>(XB(q) + k);
#pragma unroll
          for (int u = 0; u < kChunk / 2; ++u) {
            const double2 a = xb[u];
            w[q] = __builtin_fma(zb[2 * u], a.x, w[q]);
            w[q] = __builtin_fma(zb[2 * u + 1], a.y, w[q]);
          }
        }
        if (more) {
#pragma unroll
          for (int u = 0; u < kChunk; ++u) zb[u] = zn[u];
        }
      }
      for (int k = nfull; k < n; ++k) {
        const double zk = zc[(int64_t)k * n];
#pragma unroll
        for (int q = 0; q < Q; ++q) w[q] = __builtin_fma(zk, XB(q)[k], w[q]);
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) WB(q)[tid] = w[q];
    }
    lds_barrier();
    // correction, then the voltages in each item's own node order
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (q >= nq) continue;
      const int item = cc.list[blk.q0 + q];
      const int mi = cc.mod0[item] + t[q];
      const CompMod *md = cc.mods + mi;
      const int r = md->r;
      double v = w[q];
      if (r > 0) {
        const double *Kq = cc.K + (int64_t)mi * 16;
        const double *wb = WB(q);
        double y[kCompMaxRank];
#pragma unroll
        for (int a = 0; a < kCompMaxRank; ++a) {
          y[a] = 0.0;
          if (a < r) {
            const int ka = md->k[a], ma = md->m[a];
            y[a] = wb[ka < 0 ? n : ka] - wb[ma < 0 ? n : ma];
          }
        }
#pragma unroll
        for (int a = 0; a < kCompMaxRank; ++a) {
          if (a >= r) continue;
          double za = 0.0;
#pragma unroll
          for (int b = 0; b < kCompMaxRank; ++b)
            if (b < r) za = za + Kq[a * 4 + b] * y[b];
          if (tid < n) {
            const int ka = md->k[a], ma = md->m[a];
            const double zk = ka >= 0 ? Z[(int64_t)ka * n + tid] : 0.0;
            const double zm = ma >= 0 ? Z[(int64_t)ma * n + tid] : 0.0;
            v = v - za * (zk - zm);
          }
        }
      }
      if (tid < n) X(q)[pi[q]] = v;
    }
    lds_barrier();
    // record, branch update, next injections
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (q >= nq) continue;
      const ItemDesc *ip = c.items + cc.list[blk.q0 + q];
      const double *x = X(q);
      if (rec) {
        double *row = rec + ((int64_t)ip->scen * nsteps + (s - n0 - 1)) * R;
        const uint16_t *rnode = c.rnode + ip->rec, *rcol = c.rcolumn + ip->rec;
        for (int e = tid; e < ip->n_rec; e += BS) row[rcol[e]] = x[rnode[e]];
      }
      const bool sw = (s + 1 == next[q]);
      double *st_i = nullptr, *st_u = nullptr;
      if (s == n_end) {
        st_i = c.si + ip->br;
        st_u = c.su + ip->br;
      }
      const View<false> v = view(q, ip->n_src);
      step::update_inject<BS, BPT, false, false>(c, v, L[q], nullptr, nullptr, st_i, st_u, sw,
                                                 ip->coef + (int64_t)(t[q] + 1) * nbr, s < n_end, s);
      if (sw) {
        ++t[q];
        const int64_t *topo = c.topo + ip->topo;
        next[q] = (t[q] + 1 < ip->n_topo) ? topo[t[q] + 1] : step::kNever;
      }
    }
    lds_barrier();
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (q >= nq) continue;
    const ItemDesc *ip = c.items + cc.list[blk.q0 + q];
    for (int r = tid; r < n; r += BS) c.sv_state[ip->node + r] = X(q)[r];
  }
}

template <int BPT, int Q>
hipError_t comp_launch(const DevCtx &c, const CompCtx &cc, int n_blocks, int64_t n0, int64_t ns, double *rec,
                       size_t lds, hipStream_t st) {
  auto k = k_comp<BPT, Q>;
  hipError_t e =
      hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(n_blocks), dim3(kCompBS), lds, st, c, cc, n0, ns, rec);
  return hipGetLastError();
}

int blocks_of(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

}  // namespace

size_t comp_lds_bytes(int n, int nbr, int q) { return (size_t)q * comp_slot_bytes(n, nbr); }

// (branches per lane, items per workgroup) pairs with an instantiated kernel
#define EMT_COMP_SHAPES(X)                                          \
  X(1, 1) X(1, 2) X(1, 3) X(1, 4) X(1, 5) X(1, 6)                   \
  X(2, 1) X(2, 2) X(2, 3) X(2, 4) X(2, 5) X(2, 6)                   \
  X(4, 1) X(4, 2) X(4, 3) X(4, 4) X(4, 5) X(4, 6)                   \
  X(6, 1) X(6, 2) X(6, 3) X(6, 4) X(6, 5) X(6, 6)                   \
  X(8, 1) X(8, 2) X(8, 3) X(8, 4) X(12, 1) X(12, 2) X(12, 3)        \
  X(16, 1) X(16, 2)

bool comp_shape_exists(int bpt, int q) {
#define EMT_CASE(B, Q) \
  if (bpt == B && q == Q) return true;
  EMT_COMP_SHAPES(EMT_CASE)
#undef EMT_CASE
  return false;
}

hipError_t launch_comp(const DevCtx &c, const CompCtx &cc, int bpt, int q, int n_blocks, int64_t n0, int64_t ns,
                       double *rec, size_t lds, hipStream_t st) {
#define EMT_CASE(B, Q) \
  if (bpt == B && q == Q) return comp_launch<B, Q>(c, cc, n_blocks, n0, ns, rec, lds, st);
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
