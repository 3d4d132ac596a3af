// Device-side data layout shared by the kernels and the host code that
// uploads it. Everything is flattened into a few big arrays addressed by
// per-item offsets (structure of arrays; one work item = one connected
// component of one scenario).
#pragma once

#include <cstdint>

namespace emt {

enum : int {
  KIND_RL = 0, KIND_C = 1, KIND_R = 2, KIND_SWITCH = 3, KIND_SRC = 4, KIND_LINE = 5, KIND_DIODE = 6, KIND_CSWITCH = 7
};

// Packed branch descriptor for the step kernels: local terminals in 15 bits
// each (a grounded terminal holds the node count n: the step kernels keep a
// zero at x[n]) and the history-coefficient class in 2 bits: gamma = g (R-L
// and sources), -g (capacitors) or 0 (resistors, switches), or a branch
// whose history a pass after the branch update writes into its injection
// (a line end: the other end's travelling wave; a member of a coupled
// group: its circulant companion with the other members' currents and
// voltages).
constexpr uint32_t kTermGround = 0x7FFF;  // mask of one packed terminal
constexpr int kMaxItemNodes = 0x7FFF;
enum : uint32_t { GAMMA_PLUS_G = 0, GAMMA_MINUS_G = 1, GAMMA_ZERO = 2, GAMMA_PASS = 3 };

// Symbolic factor and sweep plan (shared by isomorphic items). Offsets index
// DevCtx::symi (int32) or DevCtx::symh (uint16).
struct SymDesc {
  int32_t n, d, ns, nnz;        // nodes, dense-tail size, leading size, nonzeros of L
  int32_t nsv, nfpass, nbpass, nlev;  // sweep entries, sweep passes, factor levels
  int32_t nfdesc, nbdesc, nlevb, pad1;  // row descriptors of the passes; backward levels
  // int32 (symi): full factor structure for the numeric factorisation
  int64_t rowptr, rowcol, colptr, colrow, colpos, flevptr, flevrows, fentptr, fent;
  // int32 (symi): backward levels over all n rows (explicit inverse)
  int64_t blevptr, blevrows;
  // int32 (symi): sweep plan: sv entry -> L entry; per pass (first row
  // descriptor, log2 lanes per row) pairs, nfpass+1 / nbpass+1 of them
  int64_t svmap, fpass, bpass;
  // uint16 (symh): sweep plan
  int64_t fcol, brow, bpos;
  // uint64 (symd): row descriptors (row | first << 16 | count << 32)
  int64_t fdesc, bdesc;
  // int32 (symi), symbolics refactorised inside the time loop (else -1):
  // per level entry (in fent order) its CSR position and the start of its
  // update pairs, nnz+1 of them; the pairs (qi | qj << 16), the CSR
  // positions of L_ik and L_jk for every column k < j common to rows i and j
  int64_t rent, rpair;
};

struct ItemDesc {
  int32_t scen, sym, n, n_br, n_src, n_topo, n_rec, n_lines;
  int64_t br;    // per-branch arrays
  int64_t coef;  // coefficient arrays [n_topo][n_br] (g, beta, in-service)
  int64_t nptr;  // node CSR pointers [n+1] (int32); also recorded-node pointers rptr
  int64_t nent;  // node CSR entries (uint16: local branch << 1 | end-is-m)
  int64_t node;  // per-node state [n]
  int64_t fac;   // full L values [n_topo][nnz] (factorisation work)
  int64_t dfac;  // pivots D and 1/D [n_topo][n]
  int64_t sv;    // sweep values [n_topo][nsv]
  int64_t w;     // tail inverse [n_topo][d*d]
  int64_t rec;   // recorded pairs (uint16 local node, uint16 column) [n_rec]
  int64_t topo;  // scenario topology start steps [n_topo]
  int64_t ck;    // checkpoints (i, u) [n_ck][n_br]
  int64_t seg;   // adjoint segment buffer (i, u) [K+1][n_br]
  int64_t lines; // distributed-parameter lines: first entry of line_tab / line_gf
  int32_t n_groups, pad2;  // coupled three-phase groups
  int64_t groups;  // first entry of group_tab
  int64_t mptr;    // mutual stamps by row of L [n+1] (int32), into ment
  int64_t ment;    // mutual stamps: (L position, local branch << 1 | negative) pairs (int32)
  int32_t n_diodes, pad3;  // ideal diodes (state-dependent switches)
  int64_t dyn;     // items with diodes: the factor refreshed inside the time loop, in DevCtx::dyn:
                   // current conductances [n_br], L [nnz], D [n], sweep values [nsv], 1/D [n]
};

// One coupled three-phase group: its members' local branches and terminals
// (a grounded terminal is the item's zero node slot n) and the sign of its
// Gamma (+1: R-L, Gamma = G; -1: C, Gamma = -G).
struct GroupDesc {
  int32_t b[3], k[3], m[3], sgn;
};

// One distributed-parameter line: its two local branches (k end, m end),
// their local nodes, the integer part D0 of tau / dt and the offset of its
// two wave rings (k end, then m end) in DevCtx::ring. Each ring holds
// mask + 1 doubles, a power of two >= D0 + 2; step n's wave sits at n & mask.
struct LineDesc {
  int32_t bk, bm, nk, nm, d0, mask;
  int64_t ring;
};

// Components too large for one workgroup's dense tail, solved with their
// whole inverse G^{-1} split by columns over P workgroups ("tiles"), each
// tile holding rt (16 or 32) columns in VGPRs. Per step a tile forms the
// right-hand side of its own nodes, multiplies it into a partial voltage
// vector for every node, writes that with a step tag, and sums the P
// partials of the nodes its branches touch once their tags are current.
constexpr int kSplitColsMax = 32;
constexpr int kSplitBS = 512;
// Most partials one lane sums for a node: a component has at most
// 2048 / rt tiles, and the lanes per node are raised until each lane's share
// fits (smaller for 32-column tiles, whose weight cache fills the registers).
constexpr int split_max_partials(int rt) { return rt >= 32 ? 8 : 16; }
// Exchange buffer layout: the partials of kSplitRowBlock consecutive nodes
// are interleaved per tile ([node / 4][tile][node % 4]), so one wave's
// stores of consecutive nodes land in 32-byte runs (a quarter of the
// memory transactions of one node per row) while a node's P partials still
// span few cache lines. Rows are padded to a multiple of kSplitRowBlock.
constexpr int kSplitRowBlock = 4;
constexpr int split_rows_padded(int n) { return (n + kSplitRowBlock - 1) / kSplitRowBlock * kSplitRowBlock; }

struct SplitItem {
  int32_t item, P, cb, rt;   // item, tiles, inverse columns per workgroup of k_inverse, columns per tile
  int32_t lq_lg;             // log2 of the lanes that sum one node's partials (same in every tile)
  int32_t t0;                // index of its first tile (its tiles are t0 .. t0 + P - 1)
  int64_t pos;               // SplitCtx::i32: [n] tile position of each column (tile * rt + k)
  int64_t gt;                // SplitCtx::gt: [n_topo][P][rt][n] inverse columns
  int64_t xbuf;              // SplitCtx::xbuf: [2][n4 / 4][Pp][4] tagged partial voltages (Pp = P rounded up
                             // to 8, n4 = n rounded up to 4)
};

struct SplitTile {
  int32_t sitem, p, cnt, nn;  // split item, tile index, owned columns, needed nodes (owned first)
  int32_t nsrc, nrec, ne, pad;  // sources (first tile slots), owned recorded nodes, owned-node CSR entries
  int64_t need;   // i32: [nn] item-local node of each slot
  int64_t br;     // i32: [kSplitBS * bpt] item-local branch | writer << 30 (-1 = padding)
  int64_t bpack;  // u32: [kSplitBS * bpt] slot terminals (ground = nn) | gamma class << 30
  int64_t nptr;   // i32: [cnt + 1] owned-node CSR of branch ends
  int64_t nent;   // u16: (tile slot << 1 | end is m)
  int64_t rec;    // u32: slot | output column << 16
};

struct SplitCtx {
  const SplitItem *items;
  const SplitTile *tiles;
  const int32_t *blk;  // [grid] tile of each workgroup, -1 = none (workgroup b runs on XCD b mod n_xcc)
  const int32_t *i32;
  const uint32_t *u32;
  const uint16_t *u16;
  double *gt, *xbuf;
  int32_t *err;  // set when a tile gives up waiting (the launch then ends early)
  int32_t *xcc;  // [n_tiles] XCD each tile ran on in the last launch (-1 before it starts)
  int32_t allow_local;  // 0: always exchange through device-coherent memory
};

// Everything a kernel needs, passed by value.
struct DevCtx {
  const ItemDesc *items;
  const SymDesc *syms;
  const int32_t *symi;
  const uint16_t *symh;
  const uint64_t *symd;
  // per item-branch arrays (ItemDesc::br + local branch)
  const uint32_t *bpack;
  const int32_t *bk, *bm, *bkind, *bline, *bgpos;
  const double *bE, *bw, *bph;
  double *bR, *bL, *bC;
  double *si, *su;             // branch state i, u
  double *gbar, *bbar, *cbar;  // adjoint accumulators
  // coefficients (ItemDesc::coef + t * n_br + b)
  double *cg, *cb;
  const uint8_t *cins;
  // node data
  const int32_t *nptr, *rptr;  // node CSR and recorded-column pointers (ItemDesc::nptr)
  const uint16_t *nent;        // (ItemDesc::nent)
  const uint16_t *rnode, *rcolumn;  // (ItemDesc::rec)
  double *sv_state;            // node voltages (ItemDesc::node)
  // numeric factors
  double *lfull, *dpiv, *dinv, *svals, *wtail;
  const int64_t *topo;
  double *ck_i, *ck_u, *seg_i, *seg_u;
  int32_t *flags;  // [0] = bad pivots
  double dt;
  int64_t T;
  int32_t K;
  int32_t rec_stride;
  // distributed-parameter lines (ItemDesc::lines + q): descriptor, (1/Z,
  // fractional delay f) pairs, and the wave rings
  const LineDesc *line_tab;
  const double *line_gf;
  double *ring;
  // coupled groups: descriptors, mutual stamps, per-branch mutual values and
  // member flags, and the mutual companion coefficients g_o, beta_o per
  // (topology, branch) beside cg, cb
  const GroupDesc *group_tab;
  const int32_t *mptr, *ment;
  const double *bRm, *bLm, *bCm;
  const int32_t *bgrp;
  double *cgo, *cbo;
  // ideal diodes and controlled switches: the dynamic factor slots and the
  // conducting state per branch (meaningful for those branches)
  double *dyn;
  int32_t *dstate;
  // controlled switches: per item-branch the measured node pair, item-local
  // (the ground is the item's zero node slot n); null when there is none
  const int32_t *bmeas;
};

}  // namespace emt
