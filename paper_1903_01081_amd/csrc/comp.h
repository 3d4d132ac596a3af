// Compensation solver: the descriptors that the host builds and the
// compensation kernels (comp.hip) read.
//
// Scenarios that share one base network and differ from it by a few
// switched branches (the N-1 contingencies of Sec. III-B's multi-scenario
// strategy: every scenario is the same grid with one branch out and one
// fault in) share one dense base inverse Z = G0^-1 per connected component
// ("family"). A work item's conductance matrix in topology t is
// G = G0 + U D U^T, U holding the incidence vectors of the r <= 4 branches
// whose state differs from the base and D their signed conductances, and
//   G^-1 rhs = w - (Z U) K (U^T w),  w = Z rhs,  K = (D^-1 + U^T Z U)^-1
// (Sherman-Morrison-Woodbury). Every item of a family applies the same Z,
// so a workgroup holds several items of one family and streams Z once per
// step for all of them.
#pragma once

#include <cstdint>

namespace emt {

constexpr int kCompBS = 256;        // lanes of a workgroup of the factor kernels
constexpr int kCompMaxNodes = 256;  // nodes of a family (a connected component)
constexpr int kCompMaxRank = 4;     // switched branches per item and topology
constexpr int kCompMaxItems = 6;    // items per workgroup of the step kernel

// One family: its nodes, its base item (the first scenario's component, in
// its initial topology) and the offset of its Z in CompCtx::z (n x n,
// row-major, symmetric; local node ids are the base item's).
struct CompFamily {
  int32_t n, base;
  int64_t z;
};

// Modifications of one item in one topology: r branches, each with its
// base-local terminals (-1 = ground), the index of its conductance in
// DevCtx::cg and its sign (+1: in service here but not in the base, -1: in
// service in the base but not here); fam is the item's family.
struct CompMod {
  int32_t r, fam;
  int32_t k[kCompMaxRank], m[kCompMaxRank], sgn[kCompMaxRank];
  int64_t g[kCompMaxRank];
};

// One workgroup of the step kernel: nq items of one family, list[q0 ..].
struct CompBlock {
  int32_t family, q0, nq, pad;
};

struct CompCtx {
  const CompFamily *fam;
  const CompBlock *blocks;
  const int32_t *list;     // items of the blocks, in block order
  const int32_t *mod0;     // per item: index of its topology-0 CompMod (topology t: mod0 + t)
  const int64_t *poff;     // per item: offset of its node maps in perm
  const uint16_t *perm;    // per item: [n] item-local -> base-local, then [n] base-local -> item-local
  const CompMod *mods;
  double *K;               // [n_mods][16]: K of each CompMod (r x r, row-major, leading dimension 4)
  double *z;               // the families' Z
  const int64_t *pairs;    // (item branch, base branch) pairs of pi-section branches, global branch ids
  int64_t n_pairs;
  int32_t n_fam, n_mods;
  int32_t ne_max, nr_max, ns_max;  // most node-CSR entries, recorded nodes and sources of an item
};

}  // namespace emt
