// Host-side analysis: validation, topology schedule, connected components,
// minimum-degree ordering, symbolic LDL^T and sweep level sets.
//
// The conductance matrix G = A diag(g) A^T of every topology shares one
// nonzero pattern per connected component: the union of all branches that
// are ever in service (a removed branch only zeroes entries, a switch to
// ground only changes a diagonal). So one symbolic factorisation serves every
// topology, and every scenario whose component graph is the same (the
// isomorphic scenarios of the paper's multi-scenario strategy, Sec. III-B).
#include "analysis.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <set>
#include <utility>

namespace emt {
namespace {

[[noreturn]] void fail(emt_status st, std::string msg) { throw Error{st, std::move(msg)}; }

std::string where(int s, const char *what, long idx = -1) {
  std::string r = "scenario " + std::to_string(s) + ": " + what;
  if (idx >= 0) r += " (index " + std::to_string(idx) + ")";
  return r;
}

bool finite(double x) { return std::isfinite(x); }

void validate(const emt_net &n, int s, const emt_sim &sim) {
  if (n.n_nodes < 1) fail(EMT_EINVAL, where(s, "n_nodes must be >= 1"));
  if (n.n_branches < 1) fail(EMT_EINVAL, where(s, "n_branches must be >= 1"));
  if (!n.k || !n.m || !n.kind || !n.R || !n.L || !n.C)
    fail(EMT_EINVAL, where(s, "k, m, kind, R, L, C are required"));
  if (n.n_params < 0 || n.n_params % 3) fail(EMT_EINVAL, where(s, "n_params must be 3 * lines"));
  const int n_lines = n.n_params / 3;
  for (int b = 0; b < n.n_branches; ++b) {
    const int k = n.k[b], m = n.m[b], kd = n.kind[b];
    if (k < -1 || k >= n.n_nodes || m < -1 || m >= n.n_nodes)
      fail(EMT_EINVAL, where(s, "branch terminal out of range", b));
    if (k == m) fail(EMT_EINVAL, where(s, "branch with both terminals equal (or both ground)", b));
    if (kd < EMT_RL || kd > EMT_CSWITCH) fail(EMT_EINVAL, where(s, "unknown branch kind", b));
    const double R = n.R[b], L = n.L[b], C = n.C[b];
    switch (kd) {
      case EMT_RL:
      case EMT_SRC:
        if (!finite(R) || R < 0 || !finite(L) || !(L > 0))
          fail(EMT_EINVAL, where(s, "R-L branch needs R >= 0 and L > 0", b));
        if (kd == EMT_SRC) {
          if (!n.E || !n.omega || !n.phase) fail(EMT_EINVAL, where(s, "source needs E, omega, phase"));
          if (!finite(n.E[b]) || !finite(n.omega[b]) || !finite(n.phase[b]))
            fail(EMT_EINVAL, where(s, "source EMF parameters must be finite", b));
        }
        break;
      case EMT_C:
        if (!finite(C) || !(C > 0)) fail(EMT_EINVAL, where(s, "capacitor needs C > 0", b));
        break;
      case EMT_DIODE:
        if (!finite(R) || !(R > 0)) fail(EMT_EINVAL, where(s, "a diode needs its on-resistance R > 0", b));
        if (sim.checkpoint_every > 0)
          fail(EMT_EINVAL, where(s, "diodes run forward only (no checkpoints)", b));
        if (sim.solver == EMT_SOLVER_DENSE)
          fail(EMT_EINVAL, where(s, "diodes need the sweep solvers (auto or sparse), refactorised in the loop", b));
        if (n.group && n.group[b] >= 0) fail(EMT_EINVAL, where(s, "a diode cannot belong to a coupled group", b));
        break;
      case EMT_CSWITCH: {
        if (!finite(R) || !(R > 0))
          fail(EMT_EINVAL, where(s, "a controlled switch needs its on-resistance R > 0", b));
        if (!finite(L) || !(L >= 0))
          fail(EMT_EINVAL, where(s, "a controlled switch needs its hysteresis half-width L >= 0", b));
        if (!finite(C)) fail(EMT_EINVAL, where(s, "a controlled switch's reference offset C must be finite", b));
        if (!n.E || !n.omega || !n.phase || !finite(n.E[b]) || !finite(n.omega[b]) || !finite(n.phase[b]))
          fail(EMT_EINVAL, where(s, "a controlled switch's reference E, omega, phase must be finite", b));
        if (!n.meas) fail(EMT_EINVAL, where(s, "controlled switches need meas (their measured nodes)", b));
        for (int e2 = 0; e2 < 2; ++e2)
          if (n.meas[2 * b + e2] < -1 || n.meas[2 * b + e2] >= n.n_nodes)
            fail(EMT_EINVAL, where(s, "a controlled switch's measured node is out of range", b));
        if (sim.checkpoint_every > 0)
          fail(EMT_EINVAL, where(s, "controlled switches run forward only (no checkpoints)", b));
        if (sim.solver == EMT_SOLVER_DENSE)
          fail(EMT_EINVAL, where(s, "controlled switches need the sweep solvers, refactorised in the loop", b));
        if (n.group && n.group[b] >= 0)
          fail(EMT_EINVAL, where(s, "a controlled switch cannot belong to a coupled group", b));
        break;
      }
      case EMT_LINE:
        if (k < 0 || m < 0) fail(EMT_EINVAL, where(s, "a line joins two nodes (neither end at ground)", b));
        if (!finite(R) || !(R > 0)) fail(EMT_EINVAL, where(s, "a line needs its surge impedance R > 0", b));
        if (!finite(L) || !(L >= sim.dt))
          fail(EMT_EINVAL, where(s, "a line needs its travel time L >= dt", b));
        if (C != 0.0) fail(EMT_EINVAL, where(s, "a line's C must be 0 (lossless)", b));
        break;
      default:
        if (!finite(R) || !(R > 0)) fail(EMT_EINVAL, where(s, "resistor/switch needs R > 0", b));
    }
    const int l = n.line ? n.line[b] : -1;
    if (l < -1 || l >= n_lines) fail(EMT_EINVAL, where(s, "line index out of range", b));
    if (l >= 0 && kd == EMT_SRC) fail(EMT_EINVAL, where(s, "a source cannot belong to a line", b));
    if (l >= 0 && kd != EMT_RL && kd != EMT_C)
      fail(EMT_EINVAL, where(s, "only R-L and C branches can belong to a line", b));
    if (kd == EMT_LINE && sim.checkpoint_every > 0)
      fail(EMT_EINVAL, where(s, "distributed-parameter lines run forward only (no checkpoints)", b));
  }
  if (n.n_events < 0) fail(EMT_EINVAL, where(s, "n_events < 0"));
  if (n.n_events > 0 && (!n.ev_step || !n.ev_branch || !n.ev_in_service))
    fail(EMT_EINVAL, where(s, "event arrays are required"));
  for (int j = 0; j < n.n_events; ++j) {
    if (n.ev_step[j] < 1) fail(EMT_EINVAL, where(s, "event step must be >= 1", j));
    if (n.ev_branch[j] < 0 || n.ev_branch[j] >= n.n_branches)
      fail(EMT_EINVAL, where(s, "event branch out of range", j));
    if (n.ev_in_service[j] > 1) fail(EMT_EINVAL, where(s, "ev_in_service must be 0 or 1", j));
    if (n.kind[n.ev_branch[j]] == EMT_LINE)
      fail(EMT_EINVAL, where(s, "distributed-parameter lines take no switching events", j));
    if (n.kind[n.ev_branch[j]] == EMT_DIODE)
      fail(EMT_EINVAL, where(s, "diodes switch by their own state, not by events", j));
    if (n.kind[n.ev_branch[j]] == EMT_CSWITCH)
      fail(EMT_EINVAL, where(s, "controlled switches switch by their controller, not by events", j));
  }
  if (n.group) {
    if (!n.Rm || !n.Lm || !n.Cm) fail(EMT_EINVAL, where(s, "coupled groups need Rm, Lm and Cm"));
    std::map<int, std::vector<int>> members;
    for (int b = 0; b < n.n_branches; ++b) {
      if (n.group[b] < -1) fail(EMT_EINVAL, where(s, "group index must be >= -1", b));
      if (n.group[b] >= 0) members[n.group[b]].push_back(b);
    }
    if (!members.empty() && sim.checkpoint_every > 0)
      fail(EMT_EINVAL, where(s, "coupled three-phase groups run forward only (no checkpoints)"));
    for (auto &kv : members) {
      const std::vector<int> &mem = kv.second;
      if (mem.size() != 3) fail(EMT_EINVAL, where(s, "a coupled group has exactly three branches", mem[0]));
      const int b0 = mem[0];
      for (int b : mem) {
        const int kd = n.kind[b];
        if (kd != n.kind[b0] || (kd != EMT_RL && kd != EMT_C))
          fail(EMT_EINVAL, where(s, "a coupled group is three R-L or three C branches", b));
        if ((n.line && n.line[b] >= 0))
          fail(EMT_EINVAL, where(s, "a coupled group's branches belong to no pi-section line", b));
        if (n.R[b] != n.R[b0] || n.L[b] != n.L[b0] || n.C[b] != n.C[b0] || n.Rm[b] != n.Rm[b0] ||
            n.Lm[b] != n.Lm[b0] || n.Cm[b] != n.Cm[b0])
          fail(EMT_EINVAL, where(s, "a coupled group's branches have equal R, L, C, Rm, Lm, Cm", b));
        if (n.in_service0 && !n.in_service0[b])
          fail(EMT_EINVAL, where(s, "a coupled group is in service from t = 0", b));
      }
      const double R = n.R[b0], L = n.L[b0], C = n.C[b0], Rm = n.Rm[b0], Lm = n.Lm[b0], Cm = n.Cm[b0];
      const bool ok = n.kind[b0] == EMT_RL
                          ? (finite(Rm) && finite(Lm) && L - Lm > 0 && L + 2 * Lm > 0 && R - Rm >= 0 && R + 2 * Rm >= 0)
                          : (finite(Cm) && C - Cm > 0 && C + 2 * Cm > 0);
      if (!ok) fail(EMT_EINVAL, where(s, "a coupled group's circulant matrix is not positive definite", b0));
    }
    for (int j = 0; j < n.n_events; ++j)
      if (n.group[n.ev_branch[j]] >= 0)
        fail(EMT_EINVAL, where(s, "coupled groups take no switching events", j));
  }
  if (n.rec_nodes) {
    if (n.n_rec < 0) fail(EMT_EINVAL, where(s, "n_rec < 0"));
    for (int r = 0; r < n.n_rec; ++r)
      if (n.rec_nodes[r] < 0 || n.rec_nodes[r] >= n.n_nodes)
        fail(EMT_EINVAL, where(s, "recorded node out of range", r));
  } else if (n.n_rec != 0 && n.n_rec != n.n_nodes) {
    fail(EMT_EINVAL, where(s, "rec_nodes == NULL requires n_rec == n_nodes (or 0)"));
  }
}

struct DSU {
  std::vector<int> p;
  explicit DSU(int n) : p(n) { std::iota(p.begin(), p.end(), 0); }
  int find(int x) {
    while (p[x] != x) x = p[x] = p[p[x]];
    return x;
  }
  void join(int a, int b) {
    a = find(a);
    b = find(b);
    if (a != b) p[std::max(a, b)] = std::min(a, b);
  }
};

// Minimum-degree elimination on an explicit elimination graph (ties broken
// by the smaller node id, so the result is deterministic). Returns the order
// (position -> node) and, per eliminated node, its neighbours at elimination
// time: exactly the row indices of its column of L.
void min_degree(int n, std::vector<std::vector<int>> adj, std::vector<int> &order,
                std::vector<std::vector<int>> &reach) {
  std::set<std::pair<int, int>> pq;
  for (int v = 0; v < n; ++v) pq.insert({(int)adj[v].size(), v});
  std::vector<uint8_t> gone(n, 0);
  order.clear();
  reach.assign(n, {});
  std::vector<int> tmp;
  while (!pq.empty()) {
    const int p = pq.begin()->second;
    pq.erase(pq.begin());
    gone[p] = 1;
    order.push_back(p);
    const std::vector<int> nb = adj[p];
    reach[p] = nb;
    for (int q : nb) {
      pq.erase({(int)adj[q].size(), q});
      tmp.clear();
      std::set_union(adj[q].begin(), adj[q].end(), nb.begin(), nb.end(), std::back_inserter(tmp));
      adj[q].clear();
      for (int x : tmp)
        if (x != q && x != p && !gone[x]) adj[q].push_back(x);
      pq.insert({(int)adj[q].size(), q});
    }
    adj[p].clear();
  }
}

// Builds the symbolic factor of a component given in canonical labels
// (0..n-1) with sorted adjacency lists. perm[canonical] = local id.
void symbolic(int n, const std::vector<std::vector<int>> &adj, Symbolic &S, std::vector<int> &perm) {
  std::vector<int> order;
  std::vector<std::vector<int>> reach;
  min_degree(n, adj, order, reach);
  perm.assign(n, 0);
  for (int i = 0; i < n; ++i) perm[order[i]] = i;
  S.n = n;
  // Column pattern of L: column j = perm[p] has rows perm[q] for q in reach[p].
  std::vector<std::vector<int>> cols(n);
  for (int j = 0; j < n; ++j) {
    for (int q : reach[order[j]]) cols[j].push_back(perm[q]);
    std::sort(cols[j].begin(), cols[j].end());
  }
  S.lcol_ptr.assign(n + 1, 0);
  for (int j = 0; j < n; ++j) S.lcol_ptr[j + 1] = S.lcol_ptr[j] + (int)cols[j].size();
  S.lcol_row.clear();
  for (int j = 0; j < n; ++j) S.lcol_row.insert(S.lcol_row.end(), cols[j].begin(), cols[j].end());
  const int nnz = S.lcol_ptr[n];
  // Rows: transpose (columns ascending within a row because j increases).
  std::vector<int> cnt(n + 1, 0);
  for (int e = 0; e < nnz; ++e) cnt[S.lcol_row[e] + 1]++;
  for (int i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  S.lrow_ptr = cnt;
  S.lrow_col.assign(nnz, 0);
  S.lcol_pos.assign(nnz, 0);
  std::vector<int> fillp(S.lrow_ptr.begin(), S.lrow_ptr.end() - 1);
  for (int j = 0; j < n; ++j)
    for (int e = S.lcol_ptr[j]; e < S.lcol_ptr[j + 1]; ++e) {
      const int i = S.lcol_row[e];
      const int pos = fillp[i]++;
      S.lrow_col[pos] = j;
      S.lcol_pos[e] = pos;
    }
  // Forward sweep levels: row i waits for the rows of its nonzero columns.
  std::vector<int> lev(n, 0);
  int nlev = 0;
  for (int i = 0; i < n; ++i) {
    int l = 0;
    for (int e = S.lrow_ptr[i]; e < S.lrow_ptr[i + 1]; ++e) l = std::max(l, lev[S.lrow_col[e]] + 1);
    lev[i] = l;
    nlev = std::max(nlev, l + 1);
  }
  auto group = [n](const std::vector<int> &lv, int nl, std::vector<int> &ptr, std::vector<int> &rows) {
    ptr.assign(nl + 1, 0);
    for (int i = 0; i < n; ++i) ptr[lv[i] + 1]++;
    for (int l = 0; l < nl; ++l) ptr[l + 1] += ptr[l];
    rows.assign(n, 0);
    std::vector<int> f(ptr.begin(), ptr.end() - 1);
    for (int i = 0; i < n; ++i) rows[f[lv[i]]++] = i;
  };
  group(lev, nlev, S.flev_ptr, S.flev_rows);
  // Backward sweep levels: row i of L^T waits for the rows below it in its column.
  std::vector<int> blev(n, 0);
  int nb = 0;
  for (int i = n - 1; i >= 0; --i) {
    int l = 0;
    for (int e = S.lcol_ptr[i]; e < S.lcol_ptr[i + 1]; ++e) l = std::max(l, blev[S.lcol_row[e]] + 1);
    blev[i] = l;
    nb = std::max(nb, l + 1);
  }
  group(blev, nb, S.blev_ptr, S.blev_rows);
  // Numeric factorisation schedule: the columns of one forward level only
  // depend on columns of lower levels, so their entries are computed together.
  S.fent_ptr.assign(nlev + 1, 0);
  S.fent.clear();
  for (int l = 0; l < nlev; ++l) {
    for (int p = S.flev_ptr[l]; p < S.flev_ptr[l + 1]; ++p) {
      const int j = S.flev_rows[p];
      for (int e = S.lcol_ptr[j]; e < S.lcol_ptr[j + 1]; ++e) S.fent.push_back(e);
    }
    S.fent_ptr[l + 1] = (int)S.fent.size();
  }
}

}  // namespace

SweepPlan plan_sweeps(const Symbolic &S, int d) {
  const int n = S.n;
  SweepPlan P;
  P.d = d;
  P.ns = n - d;
  const int ns = P.ns;
  std::vector<int> sv_of(S.nnz(), -1);  // full CSR position -> sv index
  P.frow_ptr.assign(n + 1, 0);
  for (int r = 0; r < n; ++r) {
    for (int q = S.lrow_ptr[r]; q < S.lrow_ptr[r + 1]; ++q) {
      const int c = S.lrow_col[q];
      if (c >= ns) continue;
      sv_of[q] = (int)P.fcol.size();
      P.fcol.push_back(c);
      P.svmap.push_back(q);
    }
    P.frow_ptr[r + 1] = (int)P.fcol.size();
  }
  // Backward: column r of L (rows c > r), for r < ns.
  P.bptr.assign(ns + 1, 0);
  for (int r = 0; r < ns; ++r) {
    for (int e = S.lcol_ptr[r]; e < S.lcol_ptr[r + 1]; ++e) {
      P.brow.push_back(S.lcol_row[e]);
      P.bpos.push_back(sv_of[S.lcol_pos[e]]);
    }
    P.bptr[r + 1] = (int)P.brow.size();
  }
  // Forward levels of the leading rows (unchanged by the tail).
  std::vector<int> lev(ns, 0);
  int nlf = 0;
  for (int i = 0; i < ns; ++i) {
    int l = 0;
    for (int q = S.lrow_ptr[i]; q < S.lrow_ptr[i + 1]; ++q) l = std::max(l, lev[S.lrow_col[q]] + 1);
    lev[i] = l;
    nlf = std::max(nlf, l + 1);
  }
  // Backward levels: tail nodes are final before the backward sweep starts.
  std::vector<int> blev(ns, 0);
  int nlb = 0;
  for (int i = ns - 1; i >= 0; --i) {
    int l = 0;
    for (int e = S.lcol_ptr[i]; e < S.lcol_ptr[i + 1]; ++e) {
      const int c = S.lcol_row[e];
      if (c < ns) l = std::max(l, blev[c] + 1);
    }
    blev[i] = l;
    nlb = std::max(nlb, l + 1);
  }
  auto group = [ns](const std::vector<int> &lv, int nl, std::vector<int> &ptr, std::vector<int> &rows) {
    ptr.assign(nl + 1, 0);
    for (int i = 0; i < ns; ++i) ptr[lv[i] + 1]++;
    for (int l = 0; l < nl; ++l) ptr[l + 1] += ptr[l];
    rows.assign(ns, 0);
    std::vector<int> f(ptr.begin(), ptr.end() - 1);
    for (int i = 0; i < ns; ++i) rows[f[lv[i]]++] = i;
  };
  group(lev, nlf, P.flev_ptr, P.flev_rows);
  group(blev, nlb, P.blev_ptr, P.blev_rows);
  auto desc = [](int row, int q0, int cnt) {
    return (uint64_t)(uint32_t)row | ((uint64_t)(uint32_t)q0 << 16) | ((uint64_t)(uint32_t)cnt << 32);
  };
  P.fpass_ptr.assign(1, 0);
  for (int l = 1; l < nlf; ++l) {
    int mx = 0;
    for (int p = P.flev_ptr[l]; p < P.flev_ptr[l + 1]; ++p) {
      const int r = P.flev_rows[p];
      const int cnt = P.frow_ptr[r + 1] - P.frow_ptr[r];
      P.fdesc.push_back(desc(r, P.frow_ptr[r], cnt));
      mx = std::max(mx, cnt);
    }
    P.fpass_ptr.push_back((int)P.fdesc.size());
    P.fpass_maxcnt.push_back(mx);
  }
  if (d > 0) {
    int mx = 0;
    for (int r = ns; r < n; ++r) {
      const int cnt = P.frow_ptr[r + 1] - P.frow_ptr[r];
      P.fdesc.push_back(desc(r, P.frow_ptr[r], cnt));
      mx = std::max(mx, cnt);
    }
    P.fpass_ptr.push_back((int)P.fdesc.size());
    P.fpass_maxcnt.push_back(mx);
  }
  P.bpass_ptr.assign(1, 0);
  for (int l = 0; l < nlb; ++l) {
    int mx = 0;
    for (int p = P.blev_ptr[l]; p < P.blev_ptr[l + 1]; ++p) {
      const int r = P.blev_rows[p];
      const int cnt = P.bptr[r + 1] - P.bptr[r];
      P.bdesc.push_back(desc(r, P.bptr[r], cnt));
      mx = std::max(mx, cnt);
    }
    P.bpass_ptr.push_back((int)P.bdesc.size());
    P.bpass_maxcnt.push_back(mx);
  }
  return P;
}

int choose_tail(const Symbolic &S, int dmax) {
  const int n = S.n;
  dmax = std::min(dmax, n);
  // forward level of every row (full factor); the leading part's levels are
  // a prefix maximum of it
  std::vector<int> flev(n, 0);
  for (int i = 0; i < n; ++i)
    for (int q = S.lrow_ptr[i]; q < S.lrow_ptr[i + 1]; ++q) flev[i] = std::max(flev[i], flev[S.lrow_col[q]] + 1);
  std::vector<int> pre(n + 1, 0);  // pre[ns] = levels of rows < ns
  for (int i = 0; i < n; ++i) pre[i + 1] = std::max(pre[i], flev[i] + 1);
  double best = 1e300;
  int best_d = 0;
  std::vector<int> blev(n);
  for (int d = 0; d <= dmax; ++d) {
    const int ns = n - d;
    int nlb = 0;
    for (int i = ns - 1; i >= 0; --i) {
      int l = 0;
      for (int e = S.lcol_ptr[i]; e < S.lcol_ptr[i + 1]; ++e) {
        const int c = S.lcol_row[e];
        if (c < ns) l = std::max(l, blev[c] + 1);
      }
      blev[i] = l;
      nlb = std::max(nlb, l + 1);
    }
    const double cost = pre[ns] + nlb + (d > 0 ? 2 : 0) + d / 64.0;
    if (cost < best - 1e-9) {
      best = cost;
      best_d = d;
    }
  }
  return best_d;
}

Analysis analyze(const emt_net *nets, int n_scen, const emt_sim &sim) {
  if (!nets || n_scen < 1) fail(EMT_EINVAL, "need at least one network");
  if (!(sim.dt > 0) || !std::isfinite(sim.dt)) fail(EMT_EINVAL, "dt must be positive and finite");
  if (sim.n_steps < 1) fail(EMT_EINVAL, "n_steps must be >= 1");
  if (sim.checkpoint_every < 0) fail(EMT_EINVAL, "checkpoint_every must be >= 0");
  if (sim.solver < EMT_SOLVER_AUTO || sim.solver > EMT_SOLVER_COMPENSATION)
    fail(EMT_EINVAL, "unknown solver");
  if (sim.comp_items < 0 || sim.comp_items > 6) fail(EMT_EINVAL, "comp_items must be 0..6");
  if (sim.solver == EMT_SOLVER_COMPENSATION) {
    if (sim.block_size != 0 && sim.block_size != 64 && sim.block_size != 128 && sim.block_size != 192 &&
        sim.block_size != 256)
      fail(EMT_EINVAL, "compensation solver: block_size (lanes per component) must be 0, 64, 128, 192 or 256");
  } else if (sim.block_size != 0 && sim.block_size != 64 && sim.block_size != 256 && sim.block_size != 512) {
    fail(EMT_EINVAL, "block_size must be 0, 64, 256 or 512");
  }
  if (sim.split_cols != 0 && sim.split_cols != 16 && sim.split_cols != 32)
    fail(EMT_EINVAL, "split_cols must be 0, 16 or 32");
  if (sim.dense_tail < -1) fail(EMT_EINVAL, "dense_tail must be >= -1");
  if (sim.sweep_from_global != 0 && sim.sweep_from_global != 1) fail(EMT_EINVAL, "sweep_from_global must be 0 or 1");
  if (sim.serial_adjoint != 0 && sim.serial_adjoint != 1) fail(EMT_EINVAL, "serial_adjoint must be 0 or 1");
  if (sim.split_device_scope != 0 && sim.split_device_scope != 1)
    fail(EMT_EINVAL, "split_device_scope must be 0 or 1");
  if (sim.pack_nodes < 0 || sim.pack_nodes > 32766) fail(EMT_EINVAL, "pack_nodes must be 0..32766");
  if (sim.pack_nodes > 128 && sim.solver == EMT_SOLVER_DENSE)
    fail(EMT_EINVAL, "the dense solver packs components into work items of at most 128 nodes");

  Analysis A;
  std::map<std::vector<int64_t>, std::pair<int, std::vector<int>>> sym_cache;  // key -> (sym, perm)

  for (int s = 0; s < n_scen; ++s) {
    const emt_net &net = nets[s];
    validate(net, s, sim);
    Scenario sc;
    sc.n_nodes = net.n_nodes;
    sc.n_branches = net.n_branches;
    sc.n_rec = net.rec_nodes ? net.n_rec : net.n_nodes;
    sc.n_params = net.n_params;
    const int N = net.n_nodes, B = net.n_branches;

    // Topology schedule: one topology per distinct event step within the horizon.
    std::vector<uint8_t> ins(B);
    for (int b = 0; b < B; ++b)
      ins[b] = net.in_service0 ? (net.in_service0[b] ? 1 : 0) : (net.kind[b] == EMT_SWITCH ? 0 : 1);
    std::vector<int> ev;
    for (int j = 0; j < net.n_events; ++j)
      if (net.ev_step[j] <= sim.n_steps) ev.push_back(j);
    std::stable_sort(ev.begin(), ev.end(), [&](int a, int b) { return net.ev_step[a] < net.ev_step[b]; });
    sc.ins.push_back(ins);
    sc.topo_step.push_back(0);
    for (size_t q = 0; q < ev.size();) {
      const int64_t st = net.ev_step[ev[q]];
      while (q < ev.size() && net.ev_step[ev[q]] == st) {
        ins[net.ev_branch[ev[q]]] = net.ev_in_service[ev[q]];
        ++q;
      }
      sc.ins.push_back(ins);
      sc.topo_step.push_back(st);
    }
    sc.n_topo = (int)sc.ins.size();
    A.max_topo = std::max(A.max_topo, sc.n_topo);

    // Every topology: each island of in-service branches must reach ground.
    for (int t = 0; t < sc.n_topo; ++t) {
      DSU d(N + 1);  // node N = ground
      for (int b = 0; b < B; ++b) {
        if (!sc.ins[t][b]) continue;
        const int k = net.k[b] < 0 ? N : net.k[b], m = net.m[b] < 0 ? N : net.m[b];
        if (net.kind[b] == EMT_LINE) {  // each end a Norton equivalent to ground
          d.join(k, N);
          d.join(m, N);
          continue;
        }
        d.join(k, m);
      }
      for (int v = 0; v < N; ++v)
        if (d.find(v) != d.find(N))
          fail(EMT_ESINGULAR, where(s, "node has no conductive path to ground in topology", v) +
                                  " topology " + std::to_string(t));
    }

    // Union graph over all topologies -> connected components (items).
    std::vector<uint8_t> ever(B, 0);
    for (int t = 0; t < sc.n_topo; ++t)
      for (int b = 0; b < B; ++b) ever[b] |= sc.ins[t][b];
    // a diode may conduct at any step, whatever its initial state
    for (int b = 0; b < B; ++b)
      if (net.kind[b] == EMT_DIODE || net.kind[b] == EMT_CSWITCH) ever[b] = 1;
    DSU d(N);
    for (int b = 0; b < B; ++b)
      if (ever[b] && net.k[b] >= 0 && net.m[b] >= 0) d.join(net.k[b], net.m[b]);
    // coupled groups couple the terminals of their members
    std::map<int, std::vector<int>> groups;  // group -> its branches
    if (net.group)
      for (int b = 0; b < B; ++b)
        if (net.group[b] >= 0) groups[net.group[b]].push_back(b);
    for (auto &kv : groups) {
      int first = -1;
      for (int b : kv.second)
        for (int t : {net.k[b], net.m[b]}) {
          if (t < 0) continue;
          if (first < 0) first = t;
          else d.join(first, t);
        }
    }
    // Work items: one per component, or with packing, components packed
    // first-fit by decreasing size into items of at most pack_nodes nodes
    // (a larger component stays alone). An item's G is then block-diagonal.
    std::map<int, int> comp_size;
    for (int v = 0; v < N; ++v) comp_size[d.find(v)]++;
    std::map<int, int> bundle;  // component root -> item key (the root of its first component)
    if (sim.pack_nodes > 0) {
      std::vector<std::pair<int, int>> by_size;  // (-size, root): largest first, ties by root
      for (auto &kv : comp_size) by_size.push_back({-kv.second, kv.first});
      std::sort(by_size.begin(), by_size.end());
      std::vector<std::pair<int, int>> bins;  // (key, nodes)
      for (auto &e : by_size) {
        const int sz = -e.first;
        size_t q = 0;
        while (q < bins.size() && bins[q].second + sz > sim.pack_nodes) ++q;
        if (q == bins.size()) bins.push_back({e.second, 0});
        bins[q].second += sz;
        bundle[e.second] = bins[q].first;
      }
    } else {
      for (auto &kv : comp_size) bundle[kv.first] = kv.first;
    }
    std::vector<int> key_of(N);
    for (int v = 0; v < N; ++v) key_of[v] = bundle[d.find(v)];
    auto item_key = [&](int node) { return key_of[node]; };
    std::map<int, std::vector<int>> comps;  // item key -> sorted nodes
    for (int v = 0; v < N; ++v) comps[item_key(v)].push_back(v);

    sc.node_item.assign(N, -1);
    sc.node_local.assign(N, -1);
    sc.br_item.assign(B, -1);
    sc.br_local.assign(B, -1);

    for (auto &kv : comps) {
      const std::vector<int> &nodes = kv.second;
      const int n = (int)nodes.size();
      std::map<int, int> canon;
      for (int i = 0; i < n; ++i) canon[nodes[i]] = i;
      std::vector<std::vector<int>> adj(n);
      std::vector<int64_t> key;
      key.push_back(n);
      for (int v : nodes) key.push_back(v);
      std::vector<std::pair<int, int>> edges;
      for (int b = 0; b < B; ++b) {
        if (!ever[b] || net.k[b] < 0 || net.m[b] < 0 || net.kind[b] == EMT_LINE) continue;
        if (item_key(net.k[b]) != kv.first) continue;
        int a = canon[net.k[b]], c = canon[net.m[b]];
        if (a > c) std::swap(a, c);
        edges.push_back({a, c});
      }
      // mutual couplings of the groups in this item: every pair of terminals
      // of two different members
      for (auto &g : groups) {
        const std::vector<int> &mem = g.second;
        if (item_key(net.k[mem[0]] >= 0 ? net.k[mem[0]] : net.m[mem[0]]) != kv.first) continue;
        for (size_t p = 0; p < mem.size(); ++p)
          for (size_t q = p + 1; q < mem.size(); ++q)
            for (int ta : {net.k[mem[p]], net.m[mem[p]]})
              for (int te : {net.k[mem[q]], net.m[mem[q]]}) {
                if (ta < 0 || te < 0 || ta == te) continue;
                int a = canon[ta], c = canon[te];
                if (a > c) std::swap(a, c);
                edges.push_back({a, c});
              }
      }
      std::sort(edges.begin(), edges.end());
      edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
      for (auto &e : edges) {
        adj[e.first].push_back(e.second);
        adj[e.second].push_back(e.first);
        key.push_back(((int64_t)e.first << 32) | e.second);
      }
      for (auto &a : adj) std::sort(a.begin(), a.end());

      int sym_id;
      std::vector<int> perm;
      auto it = sym_cache.find(key);
      if (it != sym_cache.end()) {
        sym_id = it->second.first;
        perm = it->second.second;
      } else {
        Symbolic S;
        symbolic(n, adj, S, perm);
        sym_id = (int)A.syms.size();
        A.syms.push_back(std::move(S));
        sym_cache.emplace(std::move(key), std::make_pair(sym_id, perm));
      }
      const Symbolic &S = A.syms[sym_id];

      Item it_;
      it_.scen = s;
      it_.sym = sym_id;
      it_.n = n;
      it_.gnode.assign(n, 0);
      const int item_id = (int)A.items.size();
      for (int i = 0; i < n; ++i) {
        it_.gnode[perm[i]] = nodes[i];
        sc.node_item[nodes[i]] = item_id;
        sc.node_local[nodes[i]] = perm[i];
      }
      // Branches of this component that are ever in service; sources first.
      std::vector<int> srcs, rest;
      for (int b = 0; b < B; ++b) {
        if (!ever[b]) continue;
        const int term = net.k[b] >= 0 ? net.k[b] : net.m[b];
        if (item_key(term) != kv.first) continue;
        (net.kind[b] == EMT_SRC ? srcs : rest).push_back(b);
      }
      it_.n_src = (int)srcs.size();
      it_.br = srcs;
      // a line is two local branches: its k end, then its m end
      std::vector<int> line_end;  // per local branch: 0, 1 = k end, 2 = m end
      line_end.assign(srcs.size(), 0);
      for (int b : rest) {
        it_.br.push_back(b);
        line_end.push_back(net.kind[b] == EMT_LINE ? 1 : 0);
        if (net.kind[b] == EMT_LINE) {
          it_.br.push_back(b);
          line_end.push_back(2);
        }
      }
      it_.n_br = (int)it_.br.size();
      it_.n_br_real = it_.n_br;
      it_.bk.resize(it_.n_br);
      it_.bm.resize(it_.n_br);
      it_.gpos.assign(it_.n_br, -1);
      for (int j = 0; j < it_.n_br; ++j) {
        const int b = it_.br[j];
        if (line_end[j]) {
          const int node = line_end[j] == 1 ? net.k[b] : net.m[b];
          it_.bk[j] = sc.node_local[node];
          it_.bm[j] = -1;
          if (line_end[j] == 1) {
            sc.br_item[b] = item_id;
            sc.br_local[b] = j;
            const double D = net.L[b] / sim.dt;
            const int D0 = (int)std::floor(D);
            it_.line_bk.push_back(j);
            it_.line_bm.push_back(j + 1);
            it_.line_nk.push_back(sc.node_local[net.k[b]]);
            it_.line_nm.push_back(sc.node_local[net.m[b]]);
            it_.line_d0.push_back(D0);
            it_.line_f.push_back(D - (double)D0);
          }
          continue;
        }
        it_.bk[j] = net.k[b] >= 0 ? sc.node_local[net.k[b]] : -1;
        it_.bm[j] = net.m[b] >= 0 ? sc.node_local[net.m[b]] : -1;
        sc.br_item[b] = item_id;
        sc.br_local[b] = j;
        if (it_.bk[j] >= 0 && it_.bm[j] >= 0) {
          const int r = std::max(it_.bk[j], it_.bm[j]), c = std::min(it_.bk[j], it_.bm[j]);
          const int *lo = &S.lrow_col[S.lrow_ptr[r]], *hi = &S.lrow_col[S.lrow_ptr[r + 1]];
          const int *f = std::lower_bound(lo, hi, c);
          if (f == hi || *f != c) fail(EMT_EDEVICE, "internal: branch missing from the L pattern");
          it_.gpos[j] = S.lrow_ptr[r] + (int)(f - lo);
        }
      }
      // Coupled groups: members' local branches and the mutual stamps.
      if (!groups.empty()) {
        std::map<int, std::vector<int>> gl;  // group -> local branches of its members
        for (int j = 0; j < it_.n_br; ++j) {
          const int b = it_.br[j];
          if (b >= 0 && !line_end[j] && net.group[b] >= 0) gl[net.group[b]].push_back(j);
        }
        std::vector<std::vector<std::pair<int, int>>> rows(n);
        for (auto &g : gl) {
          const std::vector<int> &mem = g.second;
          for (int j : mem) it_.grp_b.push_back(j);
          for (size_t p = 0; p < mem.size(); ++p)
            for (size_t q = p + 1; q < mem.size(); ++q) {
              const int jp = mem[p], jq = mem[q];
              const int tp[2] = {it_.bk[jp], it_.bm[jp]}, tq[2] = {it_.bk[jq], it_.bm[jq]};
              for (int ea = 0; ea < 2; ++ea)
                for (int ee = 0; ee < 2; ++ee) {
                  if (tp[ea] < 0 || tq[ee] < 0) continue;
                  const int r = std::max(tp[ea], tq[ee]), cc = std::min(tp[ea], tq[ee]);
                  const int *lo = &S.lrow_col[S.lrow_ptr[r]], *hi = &S.lrow_col[S.lrow_ptr[r + 1]];
                  const int *f = std::lower_bound(lo, hi, cc);
                  if (f == hi || *f != cc) fail(EMT_EDEVICE, "internal: mutual coupling missing from the L pattern");
                  rows[r].push_back({S.lrow_ptr[r] + (int)(f - lo), (jp << 1) | (ea != ee ? 1 : 0)});
                }
            }
        }
        it_.mptr.assign(n + 1, 0);
        for (int r = 0; r < n; ++r) {
          it_.mptr[r + 1] = it_.mptr[r] + (int)rows[r].size();
          for (auto &e : rows[r]) {
            it_.mpos.push_back(e.first);
            it_.mcode.push_back(e.second);
          }
        }
      }
      // Node CSR of incident branch ends, in increasing local branch order.
      it_.nptr.assign(n + 1, 0);
      for (int j = 0; j < it_.n_br; ++j) {
        if (it_.bk[j] >= 0) it_.nptr[it_.bk[j] + 1]++;
        if (it_.bm[j] >= 0) it_.nptr[it_.bm[j] + 1]++;
      }
      for (int i = 0; i < n; ++i) it_.nptr[i + 1] += it_.nptr[i];
      it_.nent.assign(it_.nptr[n], 0);
      std::vector<int> f(it_.nptr.begin(), it_.nptr.end() - 1);
      for (int j = 0; j < it_.n_br; ++j) {
        if (it_.bk[j] >= 0) it_.nent[f[it_.bk[j]]++] = (j << 1);
        if (it_.bm[j] >= 0) it_.nent[f[it_.bm[j]]++] = (j << 1) | 1;
      }
      sc.items.push_back(item_id);
      A.items.push_back(std::move(it_));
    }
    // A controlled switch's controller reads nodes of its own component
    // (the workgroup that steps it holds their voltages).
    for (int b = 0; b < B; ++b) {
      if (net.kind[b] != EMT_CSWITCH) continue;
      for (int e2 = 0; e2 < 2; ++e2) {
        const int a = net.meas[2 * b + e2];
        if (a >= 0 && sc.node_item[a] != sc.br_item[b])
          fail(EMT_EINVAL, where(s, "a controlled switch measures a node outside its connected component", b));
      }
    }
    // Recorded nodes -> (item, local node, column).
    for (int r = 0; r < sc.n_rec; ++r) {
      const int g = net.rec_nodes ? net.rec_nodes[r] : r;
      Item &it_ = A.items[sc.node_item[g]];
      it_.rec_node.push_back(sc.node_local[g]);
      it_.rec_col.push_back(r);
    }
    A.rec_stride = std::max(A.rec_stride, sc.n_rec);
    A.param_stride = std::max(A.param_stride, sc.n_params);
    A.scens.push_back(std::move(sc));
  }
  return A;
}

void fill_info(const Analysis &a, emt_info *info) {
  emt_info z{};
  z.n_scen = (int32_t)a.scens.size();
  z.rec_stride = a.rec_stride;
  z.param_stride = a.param_stride;
  z.n_items = (int32_t)a.items.size();
  z.n_symbolic = (int32_t)a.syms.size();
  z.max_topologies = a.max_topo;
  for (const auto &it : a.items) {
    z.max_item_nodes = std::max(z.max_item_nodes, it.n);
    z.max_item_branches = std::max(z.max_item_branches, it.n_br_real);
    z.total_nodes += it.n;
    z.total_branches += it.n_br_real;
    const Symbolic &S = a.syms[it.sym];
    z.nnz_L += S.nnz();
    z.max_levels = std::max(z.max_levels, std::max(S.levels_f(), S.levels_b()));
  }
  *info = z;
}

}  // namespace emt
