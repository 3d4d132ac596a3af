// Dense-inverse solve of components too large for one workgroup (Sec.
// III-A's fourth process done as v = G^{-1} rhs, with G^{-1} formed once per
// topology; Sec. III-B's single-task strategy spread over many compute
// units). A component's inverse is split by columns over P workgroups
// ("tiles"); tile p owns rt nodes (a block of a breadth-first order,
// so a tile's branches touch few other nodes) and every branch incident to
// them. Per step, a tile:
//   1. sums the injections of its own nodes (fixed CSR order, DPP scan);
//   2. multiplies them into its columns of G^{-1}: a partial voltage for
//      every node, written to the component's exchange buffer (four
//      consecutive nodes' partials of one tile side by side);
//   3. reads the P partials of each node its branches touch, polling until
//      each carries the step's tag, and sums them in tile order, so every
//      tile obtains bitwise the same voltages;
//   4. updates its branches (u, i, history, next injection) as the one-
//      workgroup kernel does.
// The exchange needs no flags or fences: every partial is one 8-byte
// store whose two lowest mantissa bits hold (step / 2) mod 4 (a change of
// at most 3 ulp, the same in every tile), and readers use 8-byte loads, so
// a value read is either the old one or the new one and the tag tells
// which. The buffer is double-buffered by step parity: a tile writes the
// buffer of step n+2 only after reading step n+1's partials from every
// tile, each of which wrote them only after reading step n's; steps n and
// n-2 share a buffer and differ in tag. The host fills both buffers with
// non-matching tags before each launch.
// The host places each component's tiles on one XCD where they fit (one
// L2 per XCD); the tiles confirm it at the start of the launch and then
// exchange through that L2, else through device-coherent memory.
// All tiles of a launch must be resident together: the launch is
// cooperative, and a poll that outlasts kSpinLimit rounds sets an error
// flag and ends every tile's loop instead of hanging.
#include <hip/hip_runtime.h>

#include "device.h"
#include "launch.h"
#include "step.h"

namespace emt {

namespace {

using step::gamma_of;
using step::group_sum;
using step::kNever;
using step::lds_barrier;
using step::topo_of;

constexpr int64_t kSpinLimit = int64_t(1) << 22;
// rows whose partials each tile stores last (components here have more nodes)
constexpr int kHintRows = 8;

__device__ __forceinline__ int tid_() { return step::lane_id(); }

// Position of node r's first partial in an exchange buffer (its partials
// follow at a stride of kSplitRowBlock).
__device__ __forceinline__ int64_t node_base(int r, int Pp) {
  static_assert(kSplitRowBlock == 4, "shifts below");
  const unsigned u = (unsigned)r;  // node ids are >= 0
  return (int64_t)(((u >> 2) * (unsigned)Pp) << 2) + (u & 3u);
}

// Accesses to an exchange buffer. Device-wide (the component's tiles span
// XCDs): 8-byte relaxed atomics at agent scope, served by device-coherent
// memory. XCD-local (all its tiles on one XCD): stores at workgroup scope,
// which go through the CU's write-through L1 into the XCD's L2, and raw
// buffer loads with the workgroup-scope and non-temporal bits (sc0 nt),
// which are not served from the L1 (a line there could be stale: other CUs'
// stores do not update it) but from that L2. A workgroup-scope load without
// the non-temporal bit may hit such a stale L1 line and never see the new
// value. Either way a value read is one aligned 8-byte access, old or new,
// and the step tag tells which; poll loops hold a compiler barrier so every
// round issues its loads again.
__device__ __forceinline__ void xput(bool local, uint64_t *p, uint64_t v) {
  if (local)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  else
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// raw buffer load, sc0 nt, at a byte offset (offsets past the resource's
// size read 0)
__device__ __forceinline__ uint64_t l2_load_off(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 3));
}

// Loads a lane's share of one node's P partials (q = sub + k * 2^lg): all of
// them, or (stale_only) those whose tag is not `tag`. Slots past P read as
// current.
template <int K>
__device__ __forceinline__ void load_partials(bool local, __amdgpu_buffer_rsrc_t rs, const uint64_t *base,
                                              uint64_t (&pv)[K], const uint64_t *row, int sub, int lg, int P,
                                              uint64_t tag, bool stale_only) {
  uint64_t *r = const_cast<uint64_t *>(row);
  if (!local) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int q = sub + (k << lg);
      if (stale_only && (pv[k] & 3) == tag) continue;
      pv[k] = q < P ? __hip_atomic_load(r + q * kSplitRowBlock, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : tag;
    }
    return;
  }
  const int off0 = (int)((row - base) * 8);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int q = sub + (k << lg);
    if (stale_only && (pv[k] & 3) == tag) continue;
    pv[k] = q < P ? l2_load_off(rs, off0 + q * (8 * kSplitRowBlock)) : tag;
  }
}

}  // namespace

// Columns of G^{-1} = (L D L^T)^{-1} for one (split item, topology, block of
// cb columns): forward substitution L y = e_j level by level, then
// x = D^{-1} y - L^T x level by level (backward levels over all rows), with
// the block's columns side by side in LDS ([row][cb]). Column j is written
// to its tile's slot in gt.
__global__ __launch_bounds__(256) void k_inverse(DevCtx c, SplitCtx s, const int32_t *jobs) {
  double *Y = reinterpret_cast<double *>(step::emt_lds);
  const int si = jobs[3 * blockIdx.x], t = jobs[3 * blockIdx.x + 1], j0 = jobs[3 * blockIdx.x + 2];
  const SplitItem sp = s.items[si];
  const ItemDesc it = c.items[sp.item];
  const SymDesc sd = c.syms[it.sym];
  const int n = it.n, cb = sp.cb;
  const int nc = min(cb, n - j0);
  const double *Lr = c.lfull + it.fac + (int64_t)t * sd.nnz;
  const double *D = c.dpiv + it.dfac + (int64_t)t * n;
  const int32_t *rowptr = c.symi + sd.rowptr, *rowcol = c.symi + sd.rowcol;
  const int32_t *colptr = c.symi + sd.colptr, *colrow = c.symi + sd.colrow, *colpos = c.symi + sd.colpos;
  const int32_t *flevptr = c.symi + sd.flevptr, *flevrows = c.symi + sd.flevrows;
  const int32_t *blevptr = c.symi + sd.blevptr, *blevrows = c.symi + sd.blevrows;
  for (int l = 0; l < sd.nlev; ++l) {
    const int p0 = flevptr[l], cnt = (flevptr[l + 1] - p0) * cb;
    for (int idx = threadIdx.x; idx < cnt; idx += blockDim.x) {
      const int i = flevrows[p0 + idx / cb], cc = idx % cb;
      double acc = (i == j0 + cc) ? 1.0 : 0.0;
      for (int q = rowptr[i]; q < rowptr[i + 1]; ++q) acc = acc - Lr[q] * Y[rowcol[q] * cb + cc];
      Y[i * cb + cc] = acc;
    }
    __syncthreads();
  }
  for (int l = 0; l < sd.nlevb; ++l) {
    const int p0 = blevptr[l], cnt = (blevptr[l + 1] - p0) * cb;
    for (int idx = threadIdx.x; idx < cnt; idx += blockDim.x) {
      const int i = blevrows[p0 + idx / cb], cc = idx % cb;
      double acc = Y[i * cb + cc] / D[i];
      for (int e = colptr[i]; e < colptr[i + 1]; ++e) acc = acc - Lr[colpos[e]] * Y[colrow[e] * cb + cc];
      Y[i * cb + cc] = acc;
    }
    __syncthreads();
  }
  const int32_t *pos = s.i32 + sp.pos;
  for (int cc = 0; cc < nc; ++cc) {
    const int tp = pos[j0 + cc];
    double *dst = s.gt + sp.gt + ((int64_t)t * sp.P * sp.rt + tp) * n;
    for (int r = threadIdx.x; r < n; r += blockDim.x) dst[r] = Y[r * cb + cc];
  }
}

// Forward time loop of the split components: one workgroup per tile, all
// steps n0+1 .. n0+nsteps. FLOOR (a measurement) keeps the placement check,
// the tagged exchange and the barriers of every step but drops the
// arithmetic (right-hand side, partial products, branch update) and writes
// no state or output: its time per step is the floor the exchange sets.
template <int BPT, int RPL, int RT, bool FLOOR>
__global__ __launch_bounds__(kSplitBS) void k_split(DevCtx c, SplitCtx s, int64_t n0, int64_t nsteps,
                                                   double *rec) {
  constexpr int BS = kSplitBS;
  static_assert(RT * 16 <= BS, "16 lanes per owned node");
  constexpr int kPPL = split_max_partials(RT);  // partials summed per lane
  const int tix = s.blk[blockIdx.x];
  if (tix < 0) return;  // a block on an XCD left without tiles
  const SplitTile tl = s.tiles[tix];
  const SplitItem sp = s.items[tl.sitem];
  const ItemDesc it = c.items[sp.item];
  const int n = it.n, nn = tl.nn, P = sp.P, Pp = (P + 7) & ~7, n4 = split_rows_padded(n);
  // lanes that sum one node's partials, chosen per component so that one
  // round covers every tile's nodes
  const int lq_lg = sp.lq_lg;
  const int slot0 = (int)threadIdx.x >> lq_lg;
  const int64_t row0 = slot0 < nn ? node_base(s.i32[tl.need + slot0], Pp) : 0;
  // readiness hint: the partials of one of the component's last kHintRows
  // nodes (each tile stores those last), spread over the reading tiles so
  // that no one row draws every tile's polls
  const int64_t row0_hint = node_base(n - 1 - tl.p % kHintRows, Pp);

  // LDS: x[nn + 1] (x[nn] = 0 for grounded terminals), J[BS * BPT],
  // rhs[RT], need[nn], nptr[RT + 1], nent[ne], rec[nrec], abort flag and
  // exchange scope.
  auto take = [](uint32_t &off, size_t bytes) {
    const uint32_t o = off;
    off += (uint32_t)((bytes + 15) & ~(size_t)15);
    return o;
  };
  uint32_t off = 0;
  const uint32_t ox = take(off, (size_t)(nn + 1) * 8), oJ = take(off, (size_t)BS * BPT * 8),
                 orhs = take(off, RT * 8), oneed = take(off, (size_t)nn * 4), onp = take(off, (RT + 1) * 4),
                 one = take(off, (size_t)tl.ne * 2), orec = take(off, (size_t)tl.nrec * 4),
                 oab = take(off, 8);
  step::Lds<double> x{ox}, J{oJ}, rhs{orhs};
  step::Lds<int32_t> need{oneed}, nptr{onp}, abort_flag{oab};  // [0] abort, [1] XCD-local exchange
  step::Lds<uint16_t> nent{one};
  step::Lds<uint32_t> recl{orec};
  for (int q = threadIdx.x; q < nn; q += BS) need[q] = s.i32[tl.need + q];
  for (int q = threadIdx.x; q <= RT; q += BS) nptr[q] = q <= tl.cnt ? s.i32[tl.nptr + q] : s.i32[tl.nptr + tl.cnt];
  for (int q = threadIdx.x; q < tl.ne; q += BS) nent[q] = s.u16[tl.nent + q];
  for (int q = threadIdx.x; q < tl.nrec; q += BS) recl[q] = s.u32[tl.rec + q];
  for (int q = threadIdx.x; q < RT; q += BS) rhs[q] = 0.0;
  if (threadIdx.x == 0) {
    x[nn] = 0.0;
    abort_flag[0] = 0;
  }

  const int64_t *topo = c.topo + it.topo;
  int t = topo_of(topo, it.n_topo, n0 + 1);
  int64_t next = (t + 1 < it.n_topo) ? topo[t + 1] : kNever;

  // Branch slots of this lane: item-local branch (or -1), owner bit, packed
  // terminals, coefficients and history.
  int bid[BPT];
  bool own[BPT];
  uint32_t pk[BPT];
  double g[BPT], be[BPT], h[BPT];
  const int tid0 = threadIdx.x;
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int v = s.i32[tl.br + tid0 + j * BS];
    bid[j] = v < 0 ? -1 : (v & 0x3FFFFFFF);
    own[j] = v >= 0 && ((v >> 30) & 1);
    pk[j] = s.u32[tl.bpack + tid0 + j * BS];
    const int64_t cbase = it.coef + (int64_t)t * it.n_br;
    g[j] = bid[j] >= 0 ? c.cg[cbase + bid[j]] : 0.0;
    be[j] = bid[j] >= 0 ? c.cb[cbase + bid[j]] : 0.0;
    h[j] = bid[j] >= 0 ? be[j] * c.si[it.br + bid[j]] + gamma_of(pk[j], g[j]) * c.su[it.br + bid[j]] : 0.0;
  }
  const bool src = tid0 < tl.nsrc;
  const double sE = src ? c.bE[it.br + bid[0]] : 0.0, sw = src ? c.bw[it.br + bid[0]] : 0.0,
               sph = src ? c.bph[it.br + bid[0]] : 0.0;
  auto emf = [&](int64_t m) { return src ? sE * emf_cos(sw * ((double)m * c.dt) + sph) : 0.0; };

  // This tile's columns of G^{-1} for the rows r = lane + rr * BS.
  double w[RPL * RT];
  auto load_inverse = [&](int tt) {
    const double *gsrc = s.gt + sp.gt + ((int64_t)tt * P + tl.p) * RT * (int64_t)n;
#pragma unroll
    for (int rr = 0; rr < RPL; ++rr) {
      const int r = tid0 + rr * BS;
#pragma unroll
      for (int k = 0; k < RT; ++k) w[rr * RT + k] = r < n ? gsrc[(int64_t)k * n + r] : 0.0;
    }
  };
  load_inverse(t);

  double e0 = emf(n0 + 1);
#pragma unroll
  for (int j = 0; j < BPT; ++j) J[tid0 + j * BS] = g[j] * (j == 0 ? e0 : 0.0) - h[j];

  // Exchange scope. Every tile publishes the XCD it runs on (the XCC_ID
  // hardware register, id in bits 3:0) and reads its component's: when all
  // tiles share one XCD, partials travel through that XCD's L2 (xput and
  // load_partials above), else through device-coherent memory. The tiles
  // read the same P entries, so they all choose alike. Either way the step
  // tags decide which values are current; the scope only sets the latency.
  if (tid0 < 64) {
    int xcc;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
    xcc &= 0xF;
    if (tid0 == 0) __hip_atomic_store(s.xcc + tix, xcc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool same = true, quit = false;
    for (int64_t spins = 0;;) {
      bool ok = true;
      same = true;
      for (int q = tid0; q < P; q += 64) {
        const int v = __hip_atomic_load(s.xcc + sp.t0 + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = ok && v >= 0;
        same = same && v == xcc;
      }
      if (__all(ok)) break;
      if ((++spins & 255) == 0 &&
          (spins > kSpinLimit || __hip_atomic_load(s.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
        quit = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    same = __all(same);
    if (tid0 == 0) {
      abort_flag[1] = (same && s.allow_local) ? 1 : 0;
      if (quit) {
        __hip_atomic_store(s.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        abort_flag[0] = 1;
      }
    }
  }
  __syncthreads();
  if (abort_flag[0]) return;
  const bool xcd_local = abort_flag[1] != 0;

  double *xb = s.xbuf + sp.xbuf;
  // the component's two exchange buffers as one raw buffer resource (no
  // stride, size in bytes, 32-bit data format) for the XCD-local loads
  const uint64_t *xbase = reinterpret_cast<const uint64_t *>(xb);
  const __amdgpu_buffer_rsrc_t xrs = __builtin_amdgcn_make_buffer_rsrc(xb, 0, 2 * n4 * Pp * 8, 0x00020000);
  const int R = c.rec_stride;
  const int64_t n_end = n0 + nsteps;
  for (int64_t m = n0 + 1; m <= n_end; ++m) {
    const int tid = tid_();
    // 1. injections of the owned nodes, 16 lanes per node
    if constexpr (!FLOOR) {
      const int node = tid >> 4, sub = tid & 15;
      double acc = 0.0;
      if (node < tl.cnt) {
        for (int e = nptr[node] + sub; e < nptr[node + 1]; e += 16) {
          const int ent = nent[e];
          const double jv = J[ent >> 1];
          acc = (ent & 1) ? acc - jv : acc + jv;
        }
      }
      acc = group_sum(acc, 4, sub);
      if (node < tl.cnt && sub == 15) rhs[node] = acc;
    }
    lds_barrier();
    // 2. partial voltages of every node from this tile's columns
    double rv[RT];
#pragma unroll
    for (int k = 0; k < RT; ++k) rv[k] = rhs[k];
    double *xw = xb + (int64_t)(m & 1) * n4 * Pp;
    const uint64_t tag = (uint64_t)((m >> 1) & 3);
    uint64_t hint_bits = 0;
    int hint_r = -1;
#pragma unroll
    for (int rr = 0; rr < RPL; ++rr) {
      const int r = tid + rr * BS;
      // four independent fused multiply-add chains (columns k mod 4), then
      // a fixed pairing: every tile rounds its partials the same way
      double a[4] = {0.0, 0.0, 0.0, 0.0};
      if constexpr (!FLOOR) {
#pragma unroll
        for (int k = 0; k < RT; ++k) a[k & 3] = __builtin_fma(w[rr * RT + k], rv[k], a[k & 3]);
      }
      const double acc = (a[0] + a[1]) + (a[2] + a[3]);
      // tagged, device-coherent 8-byte store: the two lowest mantissa bits
      // carry the step's tag, so readers recognise this step's value. The
      // last kHintRows nodes' partials are stored after the others (below,
      // at most one per lane): readers poll them as the sign that the
      // tile's partials have landed.
      const uint64_t bits = (__builtin_bit_cast(uint64_t, acc) & ~uint64_t(3)) | tag;
      if (r >= n - kHintRows && r < n) {
        hint_bits = bits;
        hint_r = r;
      } else if (r < n) {
        xput(xcd_local, reinterpret_cast<uint64_t *>(xw) + node_base(r, Pp) + tl.p * kSplitRowBlock, bits);
      }
    }
    lds_barrier();
    if (hint_r >= 0)
      xput(xcd_local, reinterpret_cast<uint64_t *>(xw) + node_base(hint_r, Pp) + tl.p * kSplitRowBlock,
           hint_bits);
    // the next step's source EMF does not depend on this step's voltages:
    // computed here, it overlaps the reads below
    const bool last = (m == n_end);
    double e_next = last ? 0.0 : emf(m + 1);
    asm volatile("" : "+v"(e_next));  // keep it here, ahead of the reads
    // 3. voltages of the needed nodes: each lane loads its share of a node's
    // P partials and reloads any whose tag is not this step's until all are
    // (8-byte atomic accesses: a value is either the old or the new one),
    // then the partials are summed in tile order (the same lanes-per-node
    // split in every tile of the component, so all tiles round alike). The
    // first round's node offsets sit in a register.
    {
      const uint64_t *xr = reinterpret_cast<const uint64_t *>(xb) + (int64_t)(m & 1) * n4 * Pp;
      bool quit = false;
      // readiness hint (device-wide exchange only): wave 0 polls the P
      // partials of its hint row, among each tile's final stores (P loads a
      // round, as cheap as arrival flags), before everyone reads, which
      // spares device memory the polls of every lane; the tags decide
      // correctness. Through one XCD's L2 polling is cheap and every lane
      // polls its own partials at once.
      if (tid < 64 && !xcd_local) {
        uint64_t *hint = const_cast<uint64_t *>(xr) + row0_hint;
        for (int64_t spins = 0;;) {
          bool ok = true;
          asm volatile("" ::: "memory");  // reload every round
          for (int q = tid; q < P; q += 64)
            ok = ok && (__hip_atomic_load(hint + q * kSplitRowBlock, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 3) ==
                           tag;
          if (__all(ok)) break;
          if ((++spins & 255) == 0 &&
              (spins > kSpinLimit || __hip_atomic_load(s.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
            quit = true;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      lds_barrier();
      const int sub = tid & ((1 << lq_lg) - 1);
      int round = 0;
      for (int slot = tid >> lq_lg; slot < nn; slot += BS >> lq_lg, ++round) {
        uint64_t *row = const_cast<uint64_t *>(xr) + (round == 0 ? row0 : node_base(need[slot], Pp));
        uint64_t pv[kPPL];
        load_partials(xcd_local, xrs, xbase, pv, row, sub, lq_lg, P, tag, false);
        for (int64_t spins = 0;;) {
          bool ok = true;
#pragma unroll
          for (int k = 0; k < kPPL; ++k) ok = ok && (pv[k] & 3) == tag;
          if (ok) break;
          if ((++spins & 255) == 0 &&
              (spins > kSpinLimit || __hip_atomic_load(s.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
            quit = true;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          asm volatile("" ::: "memory");  // reload every round
          load_partials(xcd_local, xrs, xbase, pv, row, sub, lq_lg, P, tag, true);
        }
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < kPPL; ++k) {
          const int q = sub + (k << lq_lg);
          acc = acc + (q < P ? __builtin_bit_cast(double, pv[k]) : 0.0);
        }
        acc = group_sum(acc, lq_lg, sub);
        if (sub == (1 << lq_lg) - 1) x[slot] = acc;
      }
      if (quit) {
        __hip_atomic_store(s.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        abort_flag[0] = 1;
      }
    }
    lds_barrier();
    if (abort_flag[0]) break;
    if constexpr (FLOOR) {
      e0 = e_next;
      lds_barrier();
      continue;
    }
    // 4. record, branch update, next injection
    if (rec) {
      double *row = rec + ((int64_t)it.scen * nsteps + (m - n0 - 1)) * R;
      for (int q = tid; q < tl.nrec; q += BS) {
        const uint32_t pr = recl[q];
        row[pr >> 16] = x[(int)(pr & 0xFFFF)];
      }
    }
    const bool swn = (m + 1 == next);
    const int64_t ncoef = it.coef + (int64_t)(t + 1) * it.n_br;
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const double vk = x[(int)(pk[j] & kTermGround)], vm = x[(int)((pk[j] >> 15) & kTermGround)];
      const double e = j == 0 ? e0 : 0.0;
      const double u = (g[j] != 0.0) ? (vk - vm) - e : 0.0;
      const double i = g[j] * u + h[j];
      if (last && own[j]) {
        c.si[it.br + bid[j]] = i;
        c.su[it.br + bid[j]] = u;
      }
      if (swn) {
        g[j] = bid[j] >= 0 ? c.cg[ncoef + bid[j]] : 0.0;
        be[j] = bid[j] >= 0 ? c.cb[ncoef + bid[j]] : 0.0;
      }
      h[j] = be[j] * i + gamma_of(pk[j], g[j]) * u;
      if (!last) J[tid + j * BS] = g[j] * (j == 0 ? e_next : 0.0) - h[j];
    }
    e0 = e_next;
    if (swn) {
      ++t;
      next = (t + 1 < it.n_topo) ? topo[t + 1] : kNever;
      load_inverse(t);
    }
    if (last)
      for (int q = tid; q < tl.cnt; q += BS) c.sv_state[it.node + need[q]] = x[q];
    lds_barrier();
  }
}

size_t split_lds_bytes(int nn, int bpt, int ne, int nrec, int rt) {
  auto arr = [](size_t bytes) { return (bytes + 15) & ~(size_t)15; };
  return arr((size_t)(nn + 1) * 8) + arr((size_t)kSplitBS * bpt * 8) + arr((size_t)rt * 8) + arr((size_t)nn * 4) +
         arr((size_t)(rt + 1) * 4) + arr((size_t)ne * 2) + arr((size_t)nrec * 4) + arr(8);
}

hipError_t launch_inverse(const DevCtx &c, const SplitCtx &s, const int32_t *jobs, int n_jobs, size_t lds,
                          hipStream_t st) {
  if (n_jobs == 0) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_inverse),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_inverse, dim3(n_jobs), dim3(256), lds, st, c, s, jobs);
  return hipGetLastError();
}

namespace {

template <int BPT, int RPL, int RT, bool FLOOR>
hipError_t split_launch(const DevCtx &c, const SplitCtx &s, int n_blocks, int64_t n0, int64_t ns, double *rec,
                        size_t lds, hipStream_t st) {
  auto k = k_split<BPT, RPL, RT, FLOOR>;
  hipError_t e =
      hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  DevCtx ca = c;
  SplitCtx sa = s;
  void *args[] = {&ca, &sa, &n0, &ns, &rec};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k), dim3(n_blocks), dim3(kSplitBS), args,
                                    (unsigned)lds, st);
}

template <int BPT, int RPL, int RT>
hipError_t split_occupancy(int *blocks_per_cu, size_t lds) {
  auto k = k_split<BPT, RPL, RT, false>;
  hipError_t e =
      hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, reinterpret_cast<const void *>(k), kSplitBS,
                                                      lds);
}

}  // namespace

// (branch slots per lane, inverse rows per lane, columns per tile); 32
// columns only where the lane state fits the VGPRs without spilling
#define EMT_SPLIT_SHAPES(X)                                                                          \
  X(1, 1, 16) X(1, 2, 16) X(1, 4, 16) X(2, 1, 16) X(2, 2, 16) X(2, 4, 16) X(4, 1, 16) X(4, 2, 16) \
  X(4, 4, 16) X(1, 1, 32) X(1, 2, 32) X(2, 1, 32) X(2, 2, 32) X(4, 1, 32)

hipError_t launch_split(const DevCtx &c, const SplitCtx &s, int bpt, int rpl, int rt, int n_blocks, int64_t n0,
                        int64_t ns, double *rec, size_t lds, bool floor, hipStream_t st) {
#define EMT_CASE(B, R, W)                                                                               \
  if (bpt == B && rpl == R && rt == W)                                                                  \
    return floor ? split_launch<B, R, W, true>(c, s, n_blocks, n0, ns, nullptr, lds, st)               \
                 : split_launch<B, R, W, false>(c, s, n_blocks, n0, ns, rec, lds, st);
  EMT_SPLIT_SHAPES(EMT_CASE)
#undef EMT_CASE
  return hipErrorInvalidValue;
}

hipError_t split_blocks_per_cu(int bpt, int rpl, int rt, size_t lds, int *blocks) {
#define EMT_CASE(B, R, W) \
  if (bpt == B && rpl == R && rt == W) return split_occupancy<B, R, W>(blocks, lds);
  EMT_SPLIT_SHAPES(EMT_CASE)
#undef EMT_CASE
  return hipErrorInvalidValue;
}

}  // namespace emt
