// Host-side plan of the compensation solver (see comp.h for the method).
//
// Families: the first scenario's work items, each in its initial topology,
// are the bases; an item of another scenario belongs to the family whose
// base holds exactly its nodes. Branches are matched to the base's by what
// fixes their conductance (kind, terminals, R, L, C, pi-section line), as a
// multiset; a matched pair in service on both sides contributes the same
// g a a^T to both matrices, so only the branches whose state differs (and
// unmatched branches in service) enter U and D. Matched pi-section branches
// take their R, L, C from each scenario's theta: the factorisation checks on
// the device that the two sides' values agree.
#include "comp_plan.h"

#include <algorithm>
#include <map>
#include <string>
#include <tuple>

namespace emt {
namespace {

[[noreturn]] void fail(std::string msg) { throw Error{EMT_EINVAL, "compensation solver: " + std::move(msg)}; }

// What fixes a branch's contribution to G, with base-local terminals in
// ascending order (the sign of a a^T does not depend on the orientation).
using Key = std::tuple<int, int, int, double, double, double, int>;

Key key_of(const emt_net &net, int b, int a, int c) {
  if (a > c) std::swap(a, c);
  const int kd = net.kind[b];
  const double R = (kd == EMT_C) ? 0.0 : net.R[b];
  const double L = (kd == EMT_RL || kd == EMT_SRC) ? net.L[b] : 0.0;
  const double C = (kd == EMT_C) ? net.C[b] : 0.0;
  return Key{kd == EMT_SRC ? EMT_RL : kd, a, c, R, L, C, net.line ? net.line[b] : -1};
}

}  // namespace

CompPlan plan_compensation(const Analysis &A, const emt_net *nets, const emt_sim &sim) {
  if (sim.checkpoint_every > 0) fail("runs forward only (checkpoint_every must be 0)");
  for (size_t s = 0; s < A.scens.size(); ++s) {
    const emt_net &net = nets[s];
    for (int b = 0; b < net.n_branches; ++b) {
      if (net.kind[b] == EMT_LINE) fail("distributed-parameter lines are not supported");
      if (net.kind[b] == EMT_DIODE || net.kind[b] == EMT_CSWITCH)
        fail("diodes and controlled switches are not supported (they refactorise inside the loop)");
      if (net.group && net.group[b] >= 0) fail("coupled three-phase groups are not supported");
    }
  }
  const Scenario &s0 = A.scens[0];
  const int NI = (int)A.items.size();
  CompPlan P;
  P.item_family.assign(NI, -1);
  std::vector<int> fam_of_base(NI, -1);
  for (int q = 0; q < NI; ++q) {
    const Item &it = A.items[q];
    if (it.scen != 0) continue;
    if (it.n > kCompMaxNodes)
      fail("a connected component has " + std::to_string(it.n) + " nodes; at most " +
           std::to_string(kCompMaxNodes));
    CompFamily f{};
    f.n = it.n;
    f.base = q;
    f.z = P.z_doubles;
    P.z_doubles += (int64_t)it.n * it.n;
    fam_of_base[q] = (int)P.fams.size();
    P.fams.push_back(f);
  }

  // Node maps.
  P.poff.assign(NI, 0);
  for (int q = 0; q < NI; ++q) {
    const Item &it = A.items[q];
    const int s = it.scen;
    const int g0 = it.gnode[0];
    if (g0 >= s0.n_nodes)
      fail("scenario " + std::to_string(s) + " has a node that the first scenario does not have");
    const int base = s0.node_item[g0];
    if (A.items[base].n != it.n)
      fail("scenario " + std::to_string(s) + "'s component of node " + std::to_string(g0) +
           " is not a component of the first scenario");
    std::vector<uint16_t> fwd(it.n), inv(it.n, 0xFFFF);
    for (int i = 0; i < it.n; ++i) {
      const int g = it.gnode[i];
      if (g >= s0.n_nodes || s0.node_item[g] != base)
        fail("scenario " + std::to_string(s) + "'s component of node " + std::to_string(g0) +
             " is not a component of the first scenario");
      const int l = s0.node_local[g];
      fwd[i] = (uint16_t)l;
      inv[l] = (uint16_t)i;
    }
    P.item_family[q] = fam_of_base[base];
    P.poff[q] = (int64_t)P.perm.size();
    P.perm.insert(P.perm.end(), fwd.begin(), fwd.end());
    P.perm.insert(P.perm.end(), inv.begin(), inv.end());
  }

  // Base branches by key, per family.
  std::vector<std::map<Key, std::vector<int>>> base_keys(P.fams.size());
  for (size_t f = 0; f < P.fams.size(); ++f) {
    const Item &bi = A.items[P.fams[f].base];
    for (int j = 0; j < (int)bi.br.size(); ++j) {
      const int b = bi.br[j];
      if (b < 0) continue;
      base_keys[f][key_of(nets[0], b, bi.bk[j], bi.bm[j])].push_back(j);
    }
  }

  P.mod0.assign(NI, 0);
  for (int q = 0; q < NI; ++q) {
    const Item &it = A.items[q];
    const int s = it.scen;
    const Scenario &sc = A.scens[s];
    const int f = P.item_family[q];
    const int qb = P.fams[f].base;
    const Item &bi = A.items[qb];
    const uint16_t *fwd = P.perm.data() + P.poff[q];
    auto base_local = [&](int t) { return t < 0 ? -1 : (int)fwd[t]; };
    // multiset matching of the item's branches to the base's
    std::map<Key, size_t> taken;
    std::vector<int> match(it.br.size(), -1);
    std::vector<char> base_used(bi.br.size(), 0);
    for (int j = 0; j < (int)it.br.size(); ++j) {
      const int b = it.br[j];
      if (b < 0) continue;
      const Key k = key_of(nets[s], b, base_local(it.bk[j]), base_local(it.bm[j]));
      auto e = base_keys[f].find(k);
      if (e == base_keys[f].end()) continue;
      size_t &used = taken[k];
      if (used >= e->second.size()) continue;
      match[j] = e->second[used++];
      base_used[match[j]] = 1;
      if (std::get<6>(k) >= 0) {
        P.pairs.push_back(q);
        P.pairs.push_back(j);
        P.pairs.push_back(qb);
        P.pairs.push_back(match[j]);
      }
    }
    P.mod0[q] = (int32_t)P.mods.size();
    for (int t = 0; t < sc.n_topo; ++t) {
      CompMod md{};
      md.fam = f;
      std::vector<CompRef> refs;
      auto add = [&](int sgn, int k, int m, CompRef ref) {
        if (md.r == kCompMaxRank)
          fail("scenario " + std::to_string(s) + " differs from the first scenario's initial topology in more than " +
               std::to_string(kCompMaxRank) + " branches of a component (from step " +
               std::to_string(sc.topo_step[t]) + ")");
        md.k[md.r] = k;
        md.m[md.r] = m;
        md.sgn[md.r] = sgn;
        md.r++;
        refs.push_back(ref);
      };
      for (int j = 0; j < (int)it.br.size(); ++j) {
        const int b = it.br[j];
        if (b < 0) continue;
        const bool on = sc.ins[t][b] != 0;
        const int j0 = match[j];
        const bool on0 = j0 >= 0 && s0.ins[0][bi.br[j0]] != 0;
        if (on && !on0) add(+1, base_local(it.bk[j]), base_local(it.bm[j]), CompRef{q, t, j});
        if (!on && on0) add(-1, bi.bk[j0], bi.bm[j0], CompRef{qb, 0, j0});
      }
      for (int j0 = 0; j0 < (int)bi.br.size(); ++j0) {
        const int b0 = bi.br[j0];
        if (b0 < 0 || base_used[j0] || !s0.ins[0][b0]) continue;
        add(-1, bi.bk[j0], bi.bm[j0], CompRef{qb, 0, j0});
      }
      P.max_rank = std::max(P.max_rank, md.r);
      refs.resize(kCompMaxRank);
      P.gref.insert(P.gref.end(), refs.begin(), refs.end());
      P.mods.push_back(md);
    }
  }
  return P;
}

}  // namespace emt
