// Host-side plan of the compensation solver: families of work items that
// share a base conductance matrix, the node maps between each item and its
// family's base, and per item and topology the switched branches that make
// its matrix differ from the base. No device code and no HIP calls.
#pragma once

#include <cstdint>
#include <vector>

#include "analysis.h"
#include "comp.h"

namespace emt {

// Where a modification's conductance lives before the device layout is
// known: item, topology and local branch of the coefficient arrays.
struct CompRef {
  int item = -1, topo = 0, local = 0;
};

struct CompPlan {
  std::vector<CompFamily> fams;   // z offsets in doubles, summed over the families
  std::vector<int> item_family;   // per item
  std::vector<int32_t> mod0;      // per item: its topology-0 entry of mods
  std::vector<CompMod> mods;      // g[] unresolved (see gref)
  std::vector<CompRef> gref;      // [mods.size() * kCompMaxRank]
  std::vector<int64_t> poff;      // per item: offset in perm
  std::vector<uint16_t> perm;     // per item: item -> base node map, then base -> item
  std::vector<int32_t> pairs;     // (item, local branch, base item, base local branch) of
                                  // matched pi-section branches
  int max_rank = 0;
  int64_t z_doubles = 0;
};

// Validates that the batch suits the compensation solver and builds its
// plan; throws Error (EMT_EINVAL) when it does not: a component of a
// scenario that is not a component of the first scenario, more than
// kCompMaxRank switched branches in a component and topology, a component
// above kCompMaxNodes nodes, checkpoints, lines, coupled groups or diodes.
CompPlan plan_compensation(const Analysis &A, const emt_net *nets, const emt_sim &sim);

}  // namespace emt
