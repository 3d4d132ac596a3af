// C ABI of the EMT library (include/emt.h): context management, device
// layout, and the calls that queue the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "analysis.h"
#include "comp.h"
#include "comp_plan.h"
#include "device.h"
#include "emt.h"
#include "launch.h"

namespace {

thread_local std::string g_last_error;

emt_status set_error(emt_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

void hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return;
  const emt_status st = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? EMT_ENOMEM : EMT_EDEVICE;
  throw emt::Error{st, std::string(what) + ": " + hipGetErrorString(e)};
}

template <class F>
emt_status guarded(F &&f) {
  try {
    return f();
  } catch (const emt::Error &e) {
    return set_error(e.status, e.msg);
  } catch (const std::bad_alloc &) {
    return set_error(EMT_ENOMEM, "host allocation failed");
  } catch (...) {
    return set_error(EMT_EDEVICE, "unexpected internal error");
  }
}

}  // namespace

struct emt_ctx {
  emt::Analysis A;
  emt_sim sim{};
  int device = 0;
  emt::KernelShape ks;
  std::vector<void *> allocs;
  int64_t device_bytes = 0;
  emt::DevCtx dc{};
  int n_items = 0;
  int32_t *d_order = nullptr;
  int32_t *d_pairs = nullptr;
  int n_pairs = 0;
  emt::CompanionArgs ca{};
  int32_t *d_bscen = nullptr, *d_bitem = nullptr, *d_blocal = nullptr;
  int64_t nbr_total = 0, nodes_total = 0;
  int64_t *d_br_ids = nullptr;
  std::vector<int64_t> scen_br_off;  // into d_br_ids
  int32_t *d_lptr = nullptr, *d_line_scen = nullptr, *d_line_id = nullptr;
  int32_t *d_nrec = nullptr;  // recorded nodes per scenario
  int64_t *d_lent = nullptr;
  int n_lines_total = 0;
  double *d_stage = nullptr;  // staging for set_state currents
  std::vector<emt::ItemDesc> items;
  bool sm_fwd = true, sm_adj = true, ks_adj_ok = true;
  // pipelined adjoint: two workgroups per item resident together, two
  // segment buffers per item, per-item progress counters
  bool adj_pipe = false;
  int32_t *d_pipe = nullptr;
  int bpt_global = 0;
  int max_tail = 0, dense_items = 0, sweep_levels = 0, lds_limit = 0;
  // items solved in one workgroup (k_forward launches the first n_fwd of
  // d_order) and split dense components (k_split, one workgroup per tile)
  int n_fwd = 0;
  std::vector<char> is_split;
  emt::SplitCtx sc{};
  int n_tiles = 0, split_bpt = 1, split_rpl = 1, split_rt = 16;
  int split_grid = 0;                            // workgroups of a split launch (idle ones included)
  std::vector<std::pair<int, int>> split_range;  // (first tile, tiles) per split item
  size_t split_lds = 0, inverse_lds = 0;
  int32_t *d_inv_jobs = nullptr;
  int n_inv_jobs = 0;
  std::vector<std::pair<int64_t, int64_t>> split_xbuf;  // (offset, doubles per step parity) per split item
  int64_t xbuf_doubles = 0;                             // both parities of every split item
  // device-side status words of queued work, read by the synchronising
  // calls after their wait: the split give-up flag (sc.err, sticky for the
  // run), the pivot count of an emt_factor_async (dc.flags[0]) and the
  // pipelined adjoint's give-up flag (dc.flags[2])
  bool pivots_pending = false, adjoint_pending = false;
  int64_t ring_doubles = 0;  // wave rings of the distributed-parameter lines
  // steady-state solve: scenarios whose sources run at different
  // frequencies, and (allocated at the first emt_steady_state) per-item
  // offsets of the complex factor, pivots and solution
  std::vector<char> scen_mixed_freq;
  int64_t *d_ss_offl = nullptr, *d_ss_offn = nullptr;
  double *ss_L = nullptr, *ss_D = nullptr, *ss_X = nullptr;
  // compensation solver: device tables, items per workgroup, workgroups
  bool comp = false;
  emt::CompCtx cc{};
  int comp_q = 0, comp_blocks = 0, comp_max_rank = 0, comp_lanes = 0;
  size_t comp_lds = 0;
  int64_t step = 0;
  bool factored = false;
  bool clean = true;  // state evolved from the zero state with no set_state since

  template <class T>
  T *alloc(size_t count) {
    if (count == 0) count = 1;
    void *p = nullptr;
    hip_check(hipMalloc(&p, count * sizeof(T)), "hipMalloc");
    allocs.push_back(p);
    device_bytes += (int64_t)(count * sizeof(T));
    return static_cast<T *>(p);
  }
  template <class T>
  T *upload(const std::vector<T> &v) {
    T *p = alloc<T>(v.size());
    if (!v.empty()) hip_check(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "upload");
    return p;
  }
  ~emt_ctx() {
    for (void *p : allocs) (void)hipFree(p);
  }
};

namespace {

// Largest dense tail whose inverse fits the lanes of one workgroup: 16
// entries per lane up to 256 lanes (d <= 4 sqrt(lanes)), 32 with 512 lanes.
int tail_max(int bs) { return bs >= 512 ? 128 : (bs >= 256 ? 64 : 32); }

int tpr_of(int d, int bs) {
  int t = 16;
  while (t > 1 && d * t > bs) t >>= 1;
  return t;
}

}  // namespace

// Fills the per-branch arrays that need the original networks.
static void fill_branch_params(emt_ctx &c, const emt_net *nets, std::vector<int32_t> &bkind,
                               std::vector<int32_t> &bline, std::vector<double> &bE, std::vector<double> &bw,
                               std::vector<double> &bph, std::vector<double> &bR, std::vector<double> &bL,
                               std::vector<double> &bC, std::vector<uint32_t> &bpack, std::vector<uint8_t> &cins,
                               std::vector<int64_t> &br_ids) {
  const emt::Analysis &A = c.A;
  for (size_t q = 0; q < A.items.size(); ++q) {
    const emt::Item &it = A.items[q];
    const emt_net &net = nets[it.scen];
    for (int j = 0; j < it.n_br; ++j) {
      const int b = it.br[j];
      if (b < 0) {
        // padding: a resistor between the always-zero node slot and itself,
        // never in service
        bkind.push_back(EMT_R);
        bline.push_back(-1);
        bE.push_back(0.0);
        bw.push_back(0.0);
        bph.push_back(0.0);
        bR.push_back(1.0);
        bL.push_back(0.0);
        bC.push_back(0.0);
        bpack.push_back((uint32_t)it.n | ((uint32_t)it.n << 15) | ((uint32_t)emt::GAMMA_ZERO << 30));
        continue;
      }
      const int kind = net.kind[b];
      bkind.push_back(kind);
      bline.push_back(net.line ? net.line[b] : -1);
      // a source's EMF, or a controlled switch's comparator reference
      const bool src = kind == EMT_SRC || kind == EMT_CSWITCH;
      bE.push_back(src ? net.E[b] : 0.0);
      bw.push_back(src ? net.omega[b] : 0.0);
      bph.push_back(src ? net.phase[b] : 0.0);
      bR.push_back(net.R[b]);
      bL.push_back(net.L[b]);
      bC.push_back(net.C[b]);
      // ground terminals point at the node slot n, which holds 0
      const uint32_t k = it.bk[j] >= 0 ? (uint32_t)it.bk[j] : (uint32_t)it.n;
      const uint32_t m = it.bm[j] >= 0 ? (uint32_t)it.bm[j] : (uint32_t)it.n;
      const bool pass = kind == EMT_LINE || (net.group && net.group[b] >= 0);
      const uint32_t cls = pass ? emt::GAMMA_PASS
                                : ((kind == EMT_RL || kind == EMT_SRC)
                                       ? emt::GAMMA_PLUS_G
                                       : (kind == EMT_C ? emt::GAMMA_MINUS_G : emt::GAMMA_ZERO));
      bpack.push_back(k | (m << 15) | (cls << 30));
    }
  }
  for (size_t q = 0; q < A.items.size(); ++q) {
    const emt::Item &it = A.items[q];
    const emt::Scenario &sc = A.scens[it.scen];
    for (int t = 0; t < sc.n_topo; ++t)
      for (int j = 0; j < it.n_br; ++j) cins.push_back(it.br[j] < 0 ? 0 : sc.ins[t][it.br[j]]);
  }
  c.scen_br_off.clear();
  for (size_t s = 0; s < A.scens.size(); ++s) {
    c.scen_br_off.push_back((int64_t)br_ids.size());
    const emt::Scenario &sc = A.scens[s];
    for (int b = 0; b < sc.n_branches; ++b) {
      if (sc.br_item[b] < 0) continue;
      br_ids.push_back(c.items[sc.br_item[b]].br + sc.br_local[b]);
    }
  }
  c.scen_br_off.push_back((int64_t)br_ids.size());
}

static emt::LdsShape shape_of(const emt::Item &it, const emt::Symbolic &S, const emt::SweepPlan &P, bool dyn) {
  return emt::LdsShape{it.n, P.d, P.ns, it.n_br, it.n_src, P.nsv(), (int)P.fdesc.size(), (int)P.bdesc.size(),
                       it.nptr[it.n], (int)it.rec_node.size(), S.levels_f(), dyn};
}

// log2 of the lanes that share one row in a sweep pass: enough lanes that
// the pass's rows fill the workgroup, but no more than its longest row needs
// and at most 16 (one DPP row).
static int pass_lanes_log2(int rows, int maxcnt, int bs) {
  int lg = 0;
  while (lg < 4 && (rows << (lg + 1)) <= bs && (1 << lg) < maxcnt) ++lg;
  return lg;
}

// Tiles of the split dense components: a breadth-first order of each
// component's nodes cut into blocks of rt columns; a tile takes every
// branch incident to its block (a branch between two blocks belongs to both,
// and the block of its k terminal writes its state), the nodes those
// branches touch, the CSR of its own nodes' branch ends and its recorded
// nodes. Then the device arrays, the inverse jobs and the launch shape.
static bool split_shape_exists(int bpt, int rpl, int rt) { return rt == 16 || (rpl <= 2 && bpt * rpl <= 4); }

static bool build_split_with(emt_ctx &c, const std::vector<uint32_t> &bpack, int rt);

static void build_split(emt_ctx &c, const std::vector<uint32_t> &bpack) {
  // columns per tile: 32 halves the tiles and the partials each node sums;
  // 16 where the lane state of 32 would not fit the VGPRs
  const int want = c.sim.split_cols == 16 ? 16 : 32;
  if (!build_split_with(c, bpack, want)) {
    if (c.sim.split_cols == 32)
      throw emt::Error{EMT_EINVAL, "split_cols = 32 does not fit these components' lane state; use 16 or 0"};
    (void)build_split_with(c, bpack, 16);
  }
}

static bool build_split_with(emt_ctx &c, const std::vector<uint32_t> &bpack, int rt) {
  using namespace emt;
  const Analysis &A = c.A;
  const int NI = (int)A.items.size();
  int max_split_n = 0;
  for (int q = 0; q < NI; ++q)
    if (c.is_split[q]) max_split_n = std::max(max_split_n, A.items[q].n);
  if (max_split_n == 0) return true;
  const int rpl = (max_split_n + kSplitBS - 1) / kSplitBS;
  if (rpl > 4) throw Error{EMT_EINVAL, "the dense solver splits components of at most " +
                                           std::to_string(4 * kSplitBS) + " nodes"};
  c.split_rpl = rpl <= 1 ? 1 : (rpl <= 2 ? 2 : 4);
  if (!split_shape_exists(1, c.split_rpl, rt)) return false;
  c.split_rt = rt;
  c.split_xbuf.clear();
  const int RT = rt;
  std::vector<SplitItem> sitems;
  std::vector<SplitTile> tiles;
  std::vector<int32_t> i32;
  std::vector<uint32_t> u32;
  std::vector<uint16_t> u16;
  std::vector<int32_t> jobs;
  int64_t gt_off = 0, xb_off = 0;
  int max_slots = 0;
  size_t inv_lds = 0;
  struct TileLists {
    std::vector<int> br, need, nptr, nent;
    std::vector<uint32_t> pack, rec;
    int cnt = 0, nsrc = 0;
  };
  std::vector<std::vector<TileLists>> all;
  for (int q = 0; q < NI; ++q) {
    if (!c.is_split[q]) continue;
    const Item &it = A.items[q];
    const Scenario &sc = A.scens[it.scen];
    const int n = it.n;
    // adjacency over real branches, breadth-first order from node 0
    std::vector<std::vector<int>> adj(n);
    for (int b = 0; b < it.n_br; ++b) {
      if (it.br[b] < 0 || it.bk[b] < 0 || it.bm[b] < 0) continue;
      adj[it.bk[b]].push_back(it.bm[b]);
      adj[it.bm[b]].push_back(it.bk[b]);
    }
    std::vector<int> bfs, pos(n, -1);
    for (int root = 0; root < n; ++root) {
      if (pos[root] >= 0) continue;
      pos[root] = (int)bfs.size();
      bfs.push_back(root);
      for (size_t h = bfs.size() - 1; h < bfs.size(); ++h) {
        std::vector<int> nb = adj[bfs[h]];
        std::sort(nb.begin(), nb.end());
        for (int v : nb)
          if (pos[v] < 0) {
            pos[v] = (int)bfs.size();
            bfs.push_back(v);
          }
      }
    }
    const int P = (n + RT - 1) / RT;
    SplitItem si{};
    si.item = q;
    si.P = P;
    si.rt = RT;
    si.cb = std::max(1, std::min(16, 20000 / n));
    si.pos = (int64_t)i32.size();
    i32.insert(i32.end(), pos.begin(), pos.end());
    si.gt = gt_off;
    si.xbuf = xb_off;
    gt_off += (int64_t)sc.n_topo * P * RT * n;
    c.split_xbuf.emplace_back(xb_off, (int64_t)split_rows_padded(n) * ((P + 7) & ~7));
    xb_off += 2 * (int64_t)split_rows_padded(n) * ((P + 7) & ~7);
    inv_lds = std::max(inv_lds, (size_t)si.cb * n * sizeof(double));
    for (int t = 0; t < sc.n_topo; ++t)
      for (int j0 = 0; j0 < n; j0 += si.cb) {
        jobs.push_back((int32_t)sitems.size());
        jobs.push_back(t);
        jobs.push_back(j0);
      }
    std::vector<TileLists> tl(P);
    auto tile_of = [&](int node) { return pos[node] / RT; };
    for (int p = 0; p < P; ++p) {
      TileLists &T = tl[p];
      const int a0 = p * RT, a1 = std::min(n, a0 + RT);
      T.cnt = a1 - a0;
      std::vector<int> slot(n, -1);
      for (int a = a0; a < a1; ++a) {
        slot[bfs[a]] = (int)T.need.size();
        T.need.push_back(bfs[a]);
      }
      auto in_tile = [&](int node) { return node >= 0 && tile_of(node) == p; };
      std::vector<int> srcs, rest;
      for (int b = 0; b < it.n_br; ++b) {
        if (it.br[b] < 0) continue;
        if (!in_tile(it.bk[b]) && !in_tile(it.bm[b])) continue;
        (b < it.n_src ? srcs : rest).push_back(b);
      }
      T.nsrc = (int)srcs.size();
      std::vector<int> brs = srcs;
      brs.insert(brs.end(), rest.begin(), rest.end());
      std::vector<int> halo;
      for (int b : brs)
        for (int v : {it.bk[b], it.bm[b]})
          if (v >= 0 && slot[v] < 0) {
            slot[v] = -2;
            halo.push_back(v);
          }
      std::sort(halo.begin(), halo.end());
      for (int v : halo) {
        slot[v] = (int)T.need.size();
        T.need.push_back(v);
      }
      const uint32_t gnd = (uint32_t)T.need.size();
      for (int b : brs) {
        const int writer = it.bk[b] >= 0 ? tile_of(it.bk[b]) : tile_of(it.bm[b]);
        T.br.push_back(b | ((writer == p ? 1 : 0) << 30));
        const uint32_t k = it.bk[b] >= 0 ? (uint32_t)slot[it.bk[b]] : gnd;
        const uint32_t m = it.bm[b] >= 0 ? (uint32_t)slot[it.bm[b]] : gnd;
        T.pack.push_back(k | (m << 15) | (bpack[c.items[q].br + b] & 0xC0000000u));
      }
      T.nptr.push_back(0);
      for (int a = 0; a < T.cnt; ++a) {
        const int node = T.need[a];
        for (int j = 0; j < (int)brs.size(); ++j) {
          if (it.bk[brs[j]] == node) T.nent.push_back(j << 1);
          if (it.bm[brs[j]] == node) T.nent.push_back((j << 1) | 1);
        }
        T.nptr.push_back((int)T.nent.size());
      }
      for (size_t r = 0; r < it.rec_node.size(); ++r)
        if (in_tile(it.rec_node[r]))
          T.rec.push_back((uint32_t)slot[it.rec_node[r]] | ((uint32_t)it.rec_col[r] << 16));
      if ((int)T.need.size() > kMaxItemNodes - 1 || T.nent.size() > 65535)
        throw Error{EMT_EINVAL, "a split tile touches too many nodes"};
      if (2 * (int)brs.size() > 65535) throw Error{EMT_EINVAL, "a split tile has too many branches"};
      max_slots = std::max(max_slots, (int)brs.size());
    }
    sitems.push_back(si);
    all.push_back(std::move(tl));
  }
  if (sitems.empty()) return true;
  int bpt = 0;
  for (int cand : {1, 2, 4})
    if (cand * kSplitBS >= max_slots) {
      bpt = cand;
      break;
    }
  if (bpt == 0) throw Error{EMT_EINVAL, "a split tile has more than " + std::to_string(4 * kSplitBS) + " branches"};
  if (!split_shape_exists(bpt, c.split_rpl, rt)) return false;
  c.split_bpt = bpt;
  const int slots = bpt * kSplitBS;
  size_t lds = 0;
  for (size_t k = 0; k < sitems.size(); ++k) {
    sitems[k].t0 = (int32_t)tiles.size();
    for (int p = 0; p < sitems[k].P; ++p) {
      TileLists &T = all[k][p];
      SplitTile d{};
      d.sitem = (int32_t)k;
      d.p = p;
      d.cnt = T.cnt;
      d.nn = (int32_t)T.need.size();
      d.nsrc = T.nsrc;
      d.nrec = (int32_t)T.rec.size();
      d.ne = (int32_t)T.nent.size();
      d.need = (int64_t)i32.size();
      i32.insert(i32.end(), T.need.begin(), T.need.end());
      d.br = (int64_t)i32.size();
      for (int j = 0; j < slots; ++j) i32.push_back(j < (int)T.br.size() ? T.br[j] : -1);
      d.bpack = (int64_t)u32.size();
      for (int j = 0; j < slots; ++j)
        u32.push_back(j < (int)T.pack.size() ? T.pack[j]
                                             : ((uint32_t)d.nn | ((uint32_t)d.nn << 15) | (GAMMA_ZERO << 30)));
      d.nptr = (int64_t)i32.size();
      i32.insert(i32.end(), T.nptr.begin(), T.nptr.end());
      d.nent = (int64_t)u16.size();
      for (int e : T.nent) u16.push_back((uint16_t)e);
      d.rec = (int64_t)u32.size();
      u32.insert(u32.end(), T.rec.begin(), T.rec.end());
      lds = std::max(lds, split_lds_bytes(d.nn, bpt, d.ne, d.nrec, RT));
      tiles.push_back(d);
    }
  }
  // Lanes per node for the partial sums, per component: the most lanes
  // (fewest loads each, at most split_max_partials) with which one round of
  // the 512 lanes covers the largest tile's nodes.
  for (size_t k = 0; k < sitems.size(); ++k) {
    int max_nn = 0;
    for (int p = 0; p < sitems[k].P; ++p) max_nn = std::max(max_nn, (int)all[k][p].need.size());
    int lg = 3;
    while (lg > 0 && (kSplitBS >> lg) < max_nn) --lg;
    while ((sitems[k].P + (1 << lg) - 1) >> lg > split_max_partials(RT)) ++lg;
    sitems[k].lq_lg = lg;
  }
  if (lds > (size_t)c.lds_limit) throw Error{EMT_EINVAL, "a split tile needs more LDS than a workgroup has"};
  c.n_tiles = (int)tiles.size();
  c.split_lds = lds;
  c.inverse_lds = inv_lds;
  int per_cu = 0, n_cu = 0;
  hip_check(split_blocks_per_cu(c.split_bpt, c.split_rpl, c.split_rt, lds, &per_cu), "split occupancy");
  hip_check(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c.device), "CU count");
  if ((int64_t)per_cu * n_cu < c.n_tiles)
    throw Error{EMT_EINVAL, "the split components need " + std::to_string(c.n_tiles) +
                                " workgroups resident at once; the device holds " + std::to_string(per_cu * n_cu)};
  // Placement over the XCDs, each with its own L2. Workgroups are handed
  // to the XCDs in turn (workgroup b on XCD b mod n_xcc), so the block
  // order decides where a tile runs. Components are taken largest first; a
  // component whose tiles fit the room left on one XCD goes to the XCD with
  // the most room (its tiles can then exchange through that XCD's L2), the
  // others are spread over what remains. Unused workgroup slots stay idle.
  int n_xcc = 1;
  if (hipDeviceGetAttribute(&n_xcc, hipDeviceAttributeNumberOfXccs, c.device) != hipSuccess || n_xcc < 1 ||
      n_cu % n_xcc != 0)
    n_xcc = 1;
  const int room = per_cu * (n_cu / n_xcc);
  std::vector<std::vector<int32_t>> on_xcd(n_xcc);
  auto roomiest = [&]() {
    int best = 0;
    for (int x = 1; x < n_xcc; ++x)
      if (on_xcd[x].size() < on_xcd[best].size()) best = x;
    return best;
  };
  std::vector<int> by_size(sitems.size());
  for (size_t k = 0; k < sitems.size(); ++k) by_size[k] = (int)k;
  std::stable_sort(by_size.begin(), by_size.end(), [&](int a, int b) { return sitems[a].P > sitems[b].P; });
  std::vector<int> spread;
  for (int k : by_size) {
    const int x = roomiest();
    if (room - (int)on_xcd[x].size() >= sitems[k].P) {
      for (int p = 0; p < sitems[k].P; ++p) on_xcd[x].push_back(sitems[k].t0 + p);
    } else {
      spread.push_back(k);
    }
  }
  for (int k : spread)
    for (int p = 0; p < sitems[k].P; ++p) on_xcd[roomiest()].push_back(sitems[k].t0 + p);
  size_t rows = 0;
  for (const auto &v : on_xcd) rows = std::max(rows, v.size());
  std::vector<int32_t> blk((size_t)n_xcc * rows, -1);
  for (int x = 0; x < n_xcc; ++x)
    for (size_t j = 0; j < on_xcd[x].size(); ++j) blk[x + (size_t)n_xcc * j] = on_xcd[x][j];
  c.split_grid = (int)blk.size();
  c.split_range.clear();
  for (const SplitItem &si : sitems) c.split_range.emplace_back(si.t0, si.P);
  c.sc.blk = c.upload(blk);
  c.sc.xcc = c.alloc<int32_t>(tiles.size());
  hip_check(hipMemset(c.sc.xcc, 0xFF, tiles.size() * sizeof(int32_t)), "split placement record");  // all -1
  c.sc.allow_local = c.sim.split_device_scope ? 0 : 1;
  c.sc.items = c.upload(sitems);
  c.sc.tiles = c.upload(tiles);
  c.sc.i32 = c.upload(i32);
  c.sc.u32 = c.upload(u32);
  c.sc.u16 = c.upload(u16);
  c.sc.gt = c.alloc<double>(gt_off);
  hip_check(hipMemset(c.sc.gt, 0, (size_t)gt_off * sizeof(double)), "clear inverse");
  c.sc.xbuf = c.alloc<double>(xb_off);
  c.xbuf_doubles = xb_off;
  c.sc.err = c.dc.flags + 1;
  c.d_inv_jobs = c.upload(jobs);
  c.n_inv_jobs = (int)jobs.size() / 3;
  return true;
}

// Compensation solver tables: the plan's modifications with their
// conductances' device indices, matched pi-section branches as global branch
// ids, and the workgroups (items of one family, comp_items per workgroup).
static void build_comp(emt_ctx &c, const emt_net *nets) {
  using namespace emt;
  const CompPlan P = plan_compensation(c.A, nets, c.sim);
  const int NI = (int)c.A.items.size();
  const int nbr = c.ks.bs * c.ks.bpt;
  int max_n = 0;
  for (const CompFamily &f : P.fams) max_n = std::max(max_n, f.n);
  std::vector<CompMod> mods = P.mods;
  for (size_t m = 0; m < mods.size(); ++m) {
    CompMod &md = mods[m];
    const int n = P.fams[md.fam].n;
    for (int a = 0; a < md.r; ++a) {
      const CompRef &ref = P.gref[m * kCompMaxRank + a];
      const ItemDesc &d = c.items[ref.item];
      md.g[a] = d.coef + (int64_t)ref.topo * d.n_br + ref.local;
      if (md.k[a] < -1 || md.k[a] >= n || md.m[a] < -1 || md.m[a] >= n || (md.k[a] < 0 && md.m[a] < 0) ||
          (md.sgn[a] != 1 && md.sgn[a] != -1) || ref.local < 0 || ref.local >= d.n_br || ref.topo >= d.n_topo)
        throw Error{EMT_EDEVICE, "internal: a compensation entry is out of range"};
    }
  }
  for (int q = 0; q < NI; ++q) {
    const int n = P.fams[P.item_family[q]].n;
    if (c.items[q].n != n || c.items[q].n_br != nbr || P.poff[q] + 2 * n > (int64_t)P.perm.size())
      throw Error{EMT_EDEVICE, "internal: a compensation item does not match its family"};
    for (int i = 0; i < 2 * n; ++i)
      if (P.perm[P.poff[q] + i] >= n) throw Error{EMT_EDEVICE, "internal: a compensation node map is out of range"};
  }
  std::vector<int64_t> pairs;
  for (size_t e = 0; e + 3 < P.pairs.size(); e += 4) {
    pairs.push_back(c.items[P.pairs[e]].br + P.pairs[e + 1]);
    pairs.push_back(c.items[P.pairs[e + 2]].br + P.pairs[e + 3]);
  }
  // items per workgroup: the fewest that keep the workgroups within one per
  // compute unit, among the shapes whose kernel exists and whose LDS fits
  std::vector<int> per_fam(P.fams.size(), 0);
  for (int q = 0; q < NI; ++q) per_fam[P.item_family[q]]++;
  auto n_blocks = [&](int Q) {
    int64_t b = 0;
    for (int k : per_fam) b += (k + Q - 1) / Q;
    return b;
  };
  int ne_max = 0, nr_max = 0, ns_max = 0;
  for (const Item &it : c.A.items) {
    ne_max = std::max(ne_max, (int)it.nent.size());
    nr_max = std::max(nr_max, (int)it.rec_node.size());
    ns_max = std::max(ns_max, it.n_src);
  }
  if (ns_max > c.ks.bs)
    throw Error{EMT_EINVAL, "compensation solver: a component has more sources than lanes"};
  auto fits = [&](int Q) {
    return comp_shape_exists(c.ks.bs, c.ks.bpt, Q) &&
           comp_lds_bytes(max_n, nbr, Q, ne_max, nr_max, ns_max, c.ks.bs) <= (size_t)c.lds_limit;
  };
  int n_cu = 0;
  hip_check(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c.device), "CU count");
  int Q = c.sim.comp_items;
  if (Q > 0) {
    if (!fits(Q))
      throw Error{EMT_EINVAL, "compensation solver: comp_items = " + std::to_string(Q) + " does not fit a " +
                                  "workgroup (" + std::to_string(c.ks.bs) + " lanes per component, " +
                                  std::to_string(max_n) + " nodes, LDS)"};
  } else {
    // the fewest items per workgroup that keep the workgroups within one
    // per compute unit, else the most that fit
    for (int cand = 1; cand <= kCompMaxItems; ++cand) {
      if (!fits(cand)) continue;
      Q = cand;
      if (n_blocks(cand) <= n_cu) break;
    }
    if (Q == 0)
      throw Error{EMT_EINVAL, "compensation solver: a component (" + std::to_string(max_n) + " nodes, " +
                                  std::to_string(nbr) + " branch slots) does not fit the compensation kernel"};
  }
  std::vector<int32_t> list;
  std::vector<CompBlock> blocks;
  for (size_t f = 0; f < P.fams.size(); ++f) {
    std::vector<int32_t> mine;
    for (int q = 0; q < NI; ++q)
      if (P.item_family[q] == (int)f) mine.push_back(q);
    for (size_t i = 0; i < mine.size(); i += Q) {
      CompBlock b{};
      b.family = (int32_t)f;
      b.q0 = (int32_t)list.size();
      b.nq = (int32_t)std::min<size_t>(Q, mine.size() - i);
      for (int k = 0; k < b.nq; ++k) list.push_back(mine[i + k]);
      blocks.push_back(b);
    }
  }
  CompCtx &cc = c.cc;
  cc.fam = c.upload(P.fams);
  cc.blocks = c.upload(blocks);
  cc.list = c.upload(list);
  cc.mod0 = c.upload(P.mod0);
  cc.poff = c.upload(P.poff);
  cc.perm = c.upload(P.perm);
  cc.mods = c.upload(mods);
  cc.K = c.alloc<double>(16 * std::max<size_t>(mods.size(), 1));
  cc.z = c.alloc<double>((size_t)P.z_doubles);
  cc.pairs = pairs.empty() ? nullptr : c.upload(pairs);
  cc.n_pairs = (int64_t)pairs.size() / 2;
  cc.n_fam = (int32_t)P.fams.size();
  cc.n_mods = (int32_t)mods.size();
  cc.ne_max = ne_max;
  cc.nr_max = nr_max;
  cc.ns_max = ns_max;
  c.comp = true;
  c.comp_q = Q;
  c.comp_blocks = (int)blocks.size();
  c.comp_lds = comp_lds_bytes(max_n, nbr, Q, ne_max, nr_max, ns_max, c.ks.bs);
  c.comp_lanes = comp_lanes(max_n, Q, c.ks.bs);
  c.comp_max_rank = P.max_rank;
}

static void upload_all(emt_ctx &c, const emt_net *nets) {
  using namespace emt;
  Analysis &A = c.A;
  const emt_sim &sim = c.sim;
  const int K = sim.checkpoint_every;
  const int64_t T = sim.n_steps;
  const int64_t n_ck = K > 0 ? T / K + 1 : 0;
  const int64_t seg_rows = K > 0 ? std::min<int64_t>(K, T) + 1 : 0;
  const int NI = (int)A.items.size();

  // Limits of the packed (15/16-bit) index formats.
  if (A.rec_stride > 65535) throw Error{EMT_EINVAL, "at most 65535 recorded nodes per scenario"};
  // The dense solver splits components larger than the biggest one-
  // workgroup dense tail over several workgroups.
  c.is_split.assign(NI, 0);
  int max_nbr = 0, max_n = 0;
  for (int q = 0; q < NI; ++q) {
    const Item &it = A.items[q];
    if (it.n > kMaxItemNodes - 1)
      throw Error{EMT_EINVAL, "a connected component has more than 32766 nodes"};
    if (it.n_br > 32767) throw Error{EMT_EINVAL, "a connected component has more than 32767 branches"};
    if (sim.solver == EMT_SOLVER_DENSE && it.n > tail_max(512)) {
      if (!it.line_bk.empty())
        throw Error{EMT_EINVAL, "components with distributed-parameter lines run in one workgroup; the dense "
                                "solver would split one of " + std::to_string(it.n) + " nodes"};
      if (!it.grp_b.empty())
        throw Error{EMT_EINVAL, "components with coupled three-phase groups run in one workgroup; the dense "
                                "solver would split one of " + std::to_string(it.n) + " nodes"};
      c.is_split[q] = 1;
      continue;
    }
    max_n = std::max(max_n, it.n);
    max_nbr = std::max(max_nbr, it.n_br);
  }
  if (K > 0 && std::count(c.is_split.begin(), c.is_split.end(), 1) > 0)
    throw Error{EMT_EINVAL, "checkpoints (the adjoint) need every component in one workgroup; the dense solver "
                            "splits components above " + std::to_string(tail_max(512)) + " nodes and runs forward only"};

  // Workgroup size and branches per lane.
  int max_lds = 65536;
  (void)hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c.device);
  c.lds_limit = max_lds;
  // The smallest workgroup that holds the largest component's branches with
  // at most 8 per lane (12 with 512 lanes); 512 lanes run 2 waves per SIMD,
  // which leaves 256 VGPRs per lane for the branch state and tail inverse.
  int bs = sim.block_size;
  if (sim.solver == EMT_SOLVER_COMPENSATION) {
    // lanes per scenario component: the fewest that hold its branches at
    // up to 8 per lane
    if (bs == 0) {
      for (int cand : {64, 128, 192, 256})
        if ((max_nbr + cand - 1) / cand <= 8) {
          bs = cand;
          break;
        }
      if (bs == 0)
        throw Error{EMT_EINVAL, "compensation solver: a component has " + std::to_string(max_nbr) +
                                    " branches; at most 2048"};
    }
    if ((max_nbr + bs - 1) / bs > 8)
      throw Error{EMT_EINVAL, "compensation solver: a component has " + std::to_string(max_nbr) +
                                  " branches, more than 8 per lane at " + std::to_string(bs) + " lanes"};
  }
  if (bs == 0) {
    bs = 512;
    for (int cand : {64, 256})
      if ((max_nbr + cand - 1) / cand <= 8 && (c.sim.solver != EMT_SOLVER_DENSE || tail_max(cand) >= max_n)) {
        bs = cand;
        break;
      }
  }
  int bpt = 0;
  const bool comp = sim.solver == EMT_SOLVER_COMPENSATION;
  // the compensation kernel exists for every count up to 8 (it is the only
  // step kernel a compensation context launches)
  const std::vector<int> bpts = comp ? std::vector<int>{1, 2, 3, 4, 5, 6, 7, 8}
                                     : std::vector<int>{1, 2, 4, 6, 8, 12, 16};
  for (int cand : bpts)
    if (cand * bs >= std::max(max_nbr, 1)) {
      bpt = cand;
      break;
    }
  if (bpt == 0)
    throw Error{EMT_EINVAL, "a connected component has " + std::to_string(max_nbr) +
                                " branches; the step kernel holds at most " + std::to_string(16 * bs)};
  c.ks.bs = bs;
  c.ks.bpt = bpt;
  c.ks.ext = false;
  for (const Item &it : A.items) {
    if (!it.line_bk.empty() || !it.grp_b.empty()) c.ks.ext = true;
    for (int b : it.br)
      if (b >= 0 && (nets[it.scen].kind[b] == EMT_DIODE || nets[it.scen].kind[b] == EMT_CSWITCH)) c.ks.ext = true;
  }
  c.ks.dmax = tail_max(bs);
  // Pad every item's branch list to whole lane slots with inert branches, so
  // the step kernels need no per-slot bounds (each runs exactly bs * bpt
  // slots); sources must fit slot 0.
  auto pad_items = [&]() {
    for (Item &it : A.items) {
      if (c.is_split[&it - &A.items[0]]) continue;
      if (it.n_src > bs)
        throw Error{EMT_EINVAL, "a connected component has more sources (" + std::to_string(it.n_src) +
                                    ") than lanes (" + std::to_string(bs) + ")"};
      const int pad = bs * bpt;
      it.br.resize(pad, -1);
      it.bk.resize(pad, -1);
      it.bm.resize(pad, -1);
      it.gpos.resize(pad, -1);
      it.n_br = pad;
    }
  };
  pad_items();

  // Sweep plans. SPARSE: level-scheduled sweeps only; DENSE: the whole
  // component is the dense tail (it must fit one workgroup's tail); AUTO:
  // dense tail chosen by cost and grown where the LDS would overflow.
  std::vector<SweepPlan> plans(A.syms.size());
  const int forced_tail = sim.dense_tail;
  const int solver = c.sim.solver;
  std::vector<char> sym_split(A.syms.size(), 0);
  for (int q = 0; q < NI; ++q)
    if (c.is_split[q]) sym_split[A.items[q].sym] = 1;
  // items with diodes refactorise inside the time loop: sweeps only (the
  // dense tail's inverse would have to be recomputed there too)
  std::vector<char> sym_diode(A.syms.size(), 0), item_diode(NI, 0);
  for (int q = 0; q < NI; ++q) {
    const Item &it = A.items[q];
    for (int b : it.br)
      if (b >= 0 && (nets[it.scen].kind[b] == EMT_DIODE || nets[it.scen].kind[b] == EMT_CSWITCH))
        sym_diode[it.sym] = item_diode[q] = 1;
  }
  for (size_t q = 0; q < A.syms.size(); ++q) {
    const int n = A.syms[q].n;
    int d;
    if (sym_split[q] || sym_diode[q]) {
      d = 0;  // factor values only; the split kernels use the explicit inverse
    } else if (solver == EMT_SOLVER_SPARSE || solver == EMT_SOLVER_COMPENSATION) {
      d = 0;  // compensation: the factors only check the pivots of every topology
    } else if (solver == EMT_SOLVER_DENSE) {
      if (n > c.ks.dmax)
        throw Error{EMT_EINVAL, "the dense solver holds components of at most " + std::to_string(c.ks.dmax) +
                                    " nodes at this block size; a component has " + std::to_string(n)};
      d = n;
    } else {
      d = forced_tail >= 0 ? std::min({forced_tail, n, c.ks.dmax}) : choose_tail(A.syms[q], c.ks.dmax);
    }
    plans[q] = plan_sweeps(A.syms[q], d);
  }
  auto item_lds = [&](const Item &it, bool adj) {
    return lds_bytes(shape_of(it, A.syms[it.sym], plans[it.sym], item_diode[&it - &A.items[0]]), true, adj);
  };
  if (solver == EMT_SOLVER_AUTO) {
    for (const Item &it : A.items) {
      if (c.is_split[&it - &A.items[0]]) continue;
      SweepPlan &P = plans[it.sym];
      if (!sym_diode[it.sym] && item_lds(it, false) > (size_t)max_lds && P.d < std::min(c.ks.dmax, it.n))
        P = plan_sweeps(A.syms[it.sym], std::min(c.ks.dmax, it.n));
    }
  }
  size_t f_sm = 0, a_sm = 0, f_gl = 0, a_gl = 0;
  int wpt = 1;
  auto lds_figures = [&]() {
    f_sm = a_sm = f_gl = a_gl = 0;
    wpt = 1;
    for (const Item &it : A.items) {
      if (c.is_split[&it - &A.items[0]]) continue;
      const LdsShape sh = shape_of(it, A.syms[it.sym], plans[it.sym], item_diode[&it - &A.items[0]]);
      f_sm = std::max(f_sm, lds_bytes(sh, true, false));
      a_sm = std::max(a_sm, lds_bytes(sh, true, true));
      f_gl = std::max(f_gl, lds_bytes(sh, false, false));
      a_gl = std::max(a_gl, lds_bytes(sh, false, true));
      const int d = plans[it.sym].d;
      if (d > 0) wpt = std::max(wpt, (d + tpr_of(d, bs) - 1) / tpr_of(d, bs));
      if (plans[it.sym].nsv() > 65535) throw Error{EMT_EINVAL, "a connected component's factor is too large"};
    }
    c.sm_fwd = f_sm <= (size_t)max_lds && !sim.sweep_from_global;
    c.sm_adj = a_sm <= (size_t)max_lds && !sim.sweep_from_global;
  };
  lds_figures();
  if (!comp && (!c.sm_fwd || !c.sm_adj)) {
    // The global-memory variants exist for 4, 8 and 16 branches per lane and
    // run every one of those slots: items padded for fewer (1, 2, 6, 12)
    // are padded again to the global variant's count, which every kernel
    // (LDS-staged ones too) then uses, and the LDS figures are retaken.
    const int bg = bpt <= 4 ? 4 : (bpt <= 8 ? 8 : 16);
    if (bg != bpt) {
      bpt = bg;
      c.ks.bpt = bpt;
      pad_items();
      lds_figures();
    }
    c.bpt_global = bpt;
  }
  // every step kernel runs exactly bs * ks.bpt branch slots per item
  for (const Item &it : A.items)
    if (!c.is_split[&it - &A.items[0]] && it.n_br != bs * c.ks.bpt)
      throw Error{EMT_EDEVICE, "internal: an item's branch padding differs from the step kernels' slots"};
  c.ks.wpt = wpt <= 4 ? 4 : (wpt <= 16 ? 16 : 32);
  if (wpt > 32 || (wpt > 16 && bs < 512)) throw Error{EMT_EINVAL, "internal: dense tail too large for the block size"};
  c.ks.lds_fwd = c.sm_fwd ? f_sm : f_gl;
  c.ks.lds_adj = c.sm_adj ? a_sm : a_gl;
  if (f_gl > (size_t)max_lds) throw Error{EMT_EINVAL, "a connected component needs more LDS than a workgroup has"};
  c.ks_adj_ok = a_gl <= (size_t)max_lds;
  // Pipelined adjoint where both workgroups of every item fit on the device
  // at once (cooperative launch) and it was not turned off.
  c.adj_pipe = false;
  if (K > 0 && c.ks_adj_ok && !sim.serial_adjoint) {
    KernelShape ks = c.ks;
    ks.sm = c.sm_adj;
    if (!ks.sm) ks.bpt = c.bpt_global;
    int per_cu = 0, n_cu = 0, n_fwd = 0;
    for (int q = 0; q < NI; ++q) n_fwd += c.is_split[q] ? 0 : 1;
    hipError_t e = bs == 64 ? adjoint_pipe_blocks_per_cu_bs64(ks, &per_cu)
                            : (bs == 256 ? adjoint_pipe_blocks_per_cu_bs256(ks, &per_cu)
                                         : adjoint_pipe_blocks_per_cu_bs512(ks, &per_cu));
    hip_check(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c.device), "CU count");
    c.adj_pipe = e == hipSuccess && (int64_t)per_cu * n_cu >= 2 * (int64_t)n_fwd;
  }

  // Symbolic arrays.
  std::vector<int32_t> symi;
  std::vector<uint16_t> symh;
  std::vector<uint64_t> symd;
  std::vector<SymDesc> sdesc;
  auto put = [&symi](const std::vector<int> &v) {
    const int64_t off = (int64_t)symi.size();
    symi.insert(symi.end(), v.begin(), v.end());
    return off;
  };
  auto puth = [&symh](const std::vector<int> &v) {
    const int64_t off = (int64_t)symh.size();
    for (int x : v) symh.push_back((uint16_t)x);
    return off;
  };
  int max_tail = 0;
  auto passes = [&](const std::vector<int> &ptr, const std::vector<int> &maxcnt) {
    std::vector<int> v;
    for (size_t k = 0; k + 1 < ptr.size(); ++k) {
      v.push_back(ptr[k]);
      v.push_back(pass_lanes_log2(ptr[k + 1] - ptr[k], maxcnt[k], bs));
    }
    v.push_back(ptr.back());
    v.push_back(0);
    return v;
  };
  for (size_t q = 0; q < A.syms.size(); ++q) {
    const Symbolic &S = A.syms[q];
    const SweepPlan &P = plans[q];
    SymDesc d{};
    d.n = S.n;
    d.d = P.d;
    d.ns = P.ns;
    d.nnz = (int32_t)S.nnz();
    d.nsv = P.nsv();
    d.nfpass = P.nfpass();
    d.nbpass = P.nbpass();
    d.nlev = S.levels_f();
    d.nfdesc = (int32_t)P.fdesc.size();
    d.nbdesc = (int32_t)P.bdesc.size();
    d.rowptr = put(S.lrow_ptr);
    d.rowcol = put(S.lrow_col);
    d.colptr = put(S.lcol_ptr);
    d.colrow = put(S.lcol_row);
    d.colpos = put(S.lcol_pos);
    d.flevptr = put(S.flev_ptr);
    d.flevrows = put(S.flev_rows);
    d.fentptr = put(S.fent_ptr);
    d.fent = put(S.fent);
    d.nlevb = S.levels_b();
    d.blevptr = put(S.blev_ptr);
    d.blevrows = put(S.blev_rows);
    d.svmap = put(P.svmap);
    d.fpass = put(passes(P.fpass_ptr, P.fpass_maxcnt));
    d.bpass = put(passes(P.bpass_ptr, P.bpass_maxcnt));
    d.fcol = puth(P.fcol);
    d.brow = puth(P.brow);
    d.bpos = puth(P.bpos);
    d.rent = d.rpair = -1;
    if (sym_diode[q]) {
      // update pairs of the factorisation inside the loop, level entry by
      // level entry, columns ascending (the order of a merge of the rows)
      std::vector<int> rent, rpair;
      for (size_t p = 0; p < S.fent.size(); ++p) {
        const int e = S.fent[p], i = S.lcol_row[e], pos = S.lcol_pos[e], j = S.lrow_col[pos];
        rent.push_back(pos);
        rent.push_back((int)rpair.size());
        int qi = S.lrow_ptr[i], qj = S.lrow_ptr[j];
        while (qi < S.lrow_ptr[i + 1] && qj < S.lrow_ptr[j + 1]) {
          const int ci = S.lrow_col[qi], cj = S.lrow_col[qj];
          if (ci >= j) break;
          if (ci == cj) {
            rpair.push_back((int)((uint32_t)qi | ((uint32_t)qj << 16)));
            ++qi;
            ++qj;
          } else if (ci < cj) {
            ++qi;
          } else {
            ++qj;
          }
        }
      }
      rent.push_back(0);
      rent.push_back((int)rpair.size());
      d.rent = put(rent);
      d.rpair = put(rpair);
    }
    d.fdesc = (int64_t)symd.size();
    symd.insert(symd.end(), P.fdesc.begin(), P.fdesc.end());
    d.bdesc = (int64_t)symd.size();
    symd.insert(symd.end(), P.bdesc.begin(), P.bdesc.end());
    sdesc.push_back(d);
    max_tail = std::max(max_tail, P.d);
  }
  c.max_tail = max_tail;
  std::vector<int64_t> topo, scen_topo_off;
  for (const Scenario &sc : A.scens) {
    scen_topo_off.push_back((int64_t)topo.size());
    topo.insert(topo.end(), sc.topo_step.begin(), sc.topo_step.end());
  }

  c.items.assign(NI, ItemDesc{});
  std::vector<int32_t> bk, bm, bgpos, bscen, bitem, blocal, nptr, rptr;
  std::vector<uint16_t> nent, rnode, rcolumn;
  int64_t coef_off = 0, fac_off = 0, dfac_off = 0, sv_off = 0, w_off = 0, ck_off = 0, seg_off = 0, node_off = 0;
  int64_t dyn_off = 0;
  std::vector<GroupDesc> group_tab;
  std::vector<int32_t> mptr_all, ment_all;
  std::vector<LineDesc> line_tab;
  std::vector<double> line_gf;
  int64_t ring_off = 0;
  std::vector<int64_t> ca_coef, ca_br;
  std::vector<int32_t> ca_nbr, ca_prefix;
  int64_t work = 0;
  std::vector<int32_t> pairs;
  c.dense_items = 0;
  for (int q = 0; q < NI; ++q) {
    const Item &it = A.items[q];
    const Scenario &sc = A.scens[it.scen];
    const Symbolic &S = A.syms[it.sym];
    const SweepPlan &P = plans[it.sym];
    if (P.d == it.n || c.is_split[q]) c.dense_items++;
    ItemDesc d{};
    d.scen = it.scen;
    d.sym = it.sym;
    d.n = it.n;
    d.n_br = it.n_br;
    d.n_src = it.n_src;
    d.n_topo = sc.n_topo;
    d.n_rec = (int32_t)it.rec_node.size();
    d.br = (int64_t)bk.size();
    d.coef = coef_off;
    d.nptr = (int64_t)nptr.size();
    d.nent = (int64_t)nent.size();
    d.node = node_off;
    d.fac = fac_off;
    d.dfac = dfac_off;
    d.sv = sv_off;
    d.w = w_off;
    d.rec = (int64_t)rnode.size();
    d.topo = scen_topo_off[it.scen];
    d.ck = ck_off;
    d.seg = seg_off;
    d.n_diodes = 0;
    for (int b : it.br)
      if (b >= 0 && (nets[it.scen].kind[b] == EMT_DIODE || nets[it.scen].kind[b] == EMT_CSWITCH)) d.n_diodes++;
    d.dyn = dyn_off;
    if (d.n_diodes > 0) dyn_off += (int64_t)it.n_br + S.nnz() + 2 * (int64_t)it.n + plans[it.sym].nsv();
    d.n_groups = (int32_t)(it.grp_b.size() / 3);
    d.groups = (int64_t)group_tab.size();
    for (size_t g = 0; g + 2 < it.grp_b.size(); g += 3) {
      GroupDesc gd{};
      for (int p = 0; p < 3; ++p) {
        const int j = it.grp_b[g + p];
        gd.b[p] = j;
        gd.k[p] = it.bk[j] >= 0 ? it.bk[j] : it.n;
        gd.m[p] = it.bm[j] >= 0 ? it.bm[j] : it.n;
      }
      gd.sgn = nets[it.scen].kind[it.br[it.grp_b[g]]] == EMT_C ? -1 : 1;
      group_tab.push_back(gd);
    }
    d.mptr = (int64_t)mptr_all.size();
    d.ment = (int64_t)ment_all.size();
    if (!it.grp_b.empty()) {
      for (int r = 0; r <= it.n; ++r) mptr_all.push_back(it.mptr[r]);
      for (size_t e = 0; e < it.mpos.size(); ++e) {
        ment_all.push_back(it.mpos[e]);
        ment_all.push_back(it.mcode[e]);
      }
    }
    d.n_lines = (int32_t)it.line_bk.size();
    d.lines = (int64_t)line_tab.size();
    for (size_t l = 0; l < it.line_bk.size(); ++l) {
      const int b = it.br[it.line_bk[l]];
      LineDesc ld{};
      ld.bk = it.line_bk[l];
      ld.bm = it.line_bm[l];
      ld.nk = it.line_nk[l];
      ld.nm = it.line_nm[l];
      ld.d0 = it.line_d0[l];
      int32_t len = 1;  // ring length: a power of two holding steps n - D0 - 1 .. n
      while (len < ld.d0 + 2) len *= 2;
      ld.mask = len - 1;
      ld.ring = ring_off;
      ring_off += 2 * (int64_t)len;
      line_tab.push_back(ld);
      line_gf.push_back(1.0 / nets[it.scen].R[b]);
      line_gf.push_back(it.line_f[l]);
    }
    c.items[q] = d;
    coef_off += (int64_t)sc.n_topo * it.n_br;
    fac_off += (int64_t)sc.n_topo * S.nnz();
    dfac_off += (int64_t)sc.n_topo * it.n;
    sv_off += (int64_t)sc.n_topo * P.nsv();
    w_off += (int64_t)sc.n_topo * P.d * P.d;
    ck_off += n_ck * it.n_br;
    seg_off += (c.adj_pipe ? 2 : 1) * seg_rows * it.n_br;
    node_off += it.n;
    for (int t = 0; t < sc.n_topo; ++t) {
      pairs.push_back(q);
      pairs.push_back(t);
    }
    ca_coef.push_back(d.coef);
    ca_br.push_back(d.br);
    ca_nbr.push_back(it.n_br);
    ca_prefix.push_back((int32_t)work);
    work += (int64_t)it.n_br * sc.n_topo;
    for (int j = 0; j < it.n_br; ++j) {
      bk.push_back(it.bk[j]);
      bm.push_back(it.bm[j]);
      bgpos.push_back(it.gpos[j]);
      bscen.push_back(it.scen);
      bitem.push_back(q);
      blocal.push_back(j);
    }
    nptr.insert(nptr.end(), it.nptr.begin(), it.nptr.end());
    for (int e : it.nent) nent.push_back((uint16_t)e);
    std::vector<int> idx(it.rec_node.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return it.rec_node[a] < it.rec_node[b]; });
    std::vector<int32_t> rp(it.n + 1, 0);
    for (int e : idx) {
      rnode.push_back((uint16_t)it.rec_node[e]);
      rcolumn.push_back((uint16_t)it.rec_col[e]);
      rp[it.rec_node[e] + 1]++;
    }
    for (int r = 0; r < it.n; ++r) rp[r + 1] += rp[r];
    rptr.insert(rptr.end(), rp.begin(), rp.end());
  }
  if (work > INT32_MAX) throw Error{EMT_EINVAL, "too many branch-topology pairs"};
  c.n_items = NI;
  c.n_pairs = (int)pairs.size() / 2;
  c.nbr_total = (int64_t)bk.size();
  c.nodes_total = node_off;

  std::vector<int32_t> bkind, bline;
  std::vector<double> bE, bw, bph, bR, bL, bC;
  std::vector<uint32_t> bpack;
  std::vector<uint8_t> cins;
  std::vector<int64_t> br_ids;
  fill_branch_params(c, nets, bkind, bline, bE, bw, bph, bR, bL, bC, bpack, cins, br_ids);
  c.scen_mixed_freq.assign(A.scens.size(), 0);
  for (size_t q = 0; q < A.scens.size(); ++q) {
    const emt_net &net = nets[q];
    bool any = false;
    double w = 0.0;
    for (int b = 0; b < net.n_branches; ++b) {
      if (net.kind[b] != EMT_SRC) continue;
      if (any && net.omega[b] != w) c.scen_mixed_freq[q] = 1;
      w = net.omega[b];
      any = true;
    }
  }

  // Line -> branches (global item-branch index), per scenario, fixed order.
  std::vector<int32_t> lptr{0}, line_scen, line_id;
  std::vector<int64_t> lent;
  for (size_t s = 0; s < A.scens.size(); ++s) {
    const Scenario &sc = A.scens[s];
    const int nl = sc.n_params / 3;
    std::vector<std::vector<int64_t>> per(nl);
    for (int b = 0; b < sc.n_branches; ++b) {
      const int l = nets[s].line ? nets[s].line[b] : -1;
      if (l < 0 || sc.br_item[b] < 0) continue;
      per[l].push_back(c.items[sc.br_item[b]].br + sc.br_local[b]);
    }
    for (int l = 0; l < nl; ++l) {
      lent.insert(lent.end(), per[l].begin(), per[l].end());
      lptr.push_back((int32_t)lent.size());
      line_scen.push_back((int32_t)s);
      line_id.push_back(l);
    }
  }
  c.n_lines_total = (int)line_id.size();

  // One-workgroup items, largest first so their workgroups start first.
  std::vector<int32_t> order;
  for (int q = 0; q < NI; ++q)
    if (!c.is_split[q]) order.push_back(q);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (int64_t)A.items[a].n + A.items[a].n_br_real > (int64_t)A.items[b].n + A.items[b].n_br_real;
  });
  c.n_fwd = (int)order.size();
  if (order.empty()) order.push_back(0);

  DevCtx &dc = c.dc;
  dc.items = c.upload(c.items);
  dc.syms = c.upload(sdesc);
  dc.symi = c.upload(symi);
  dc.symh = c.upload(symh);
  dc.symd = c.upload(symd);
  dc.bpack = c.upload(bpack);
  dc.bk = c.upload(bk);
  dc.bm = c.upload(bm);
  dc.bkind = c.upload(bkind);
  dc.bline = c.upload(bline);
  dc.bgpos = c.upload(bgpos);
  dc.bE = c.upload(bE);
  dc.bw = c.upload(bw);
  dc.bph = c.upload(bph);
  dc.bR = c.upload(bR);
  dc.bL = c.upload(bL);
  dc.bC = c.upload(bC);
  dc.si = c.alloc<double>(c.nbr_total);
  dc.su = c.alloc<double>(c.nbr_total);
  dc.gbar = c.alloc<double>(c.nbr_total);
  dc.bbar = c.alloc<double>(c.nbr_total);
  dc.cbar = c.alloc<double>(c.nbr_total);
  dc.cg = c.alloc<double>(coef_off);
  dc.cb = c.alloc<double>(coef_off);
  dc.cins = c.upload(cins);
  dc.nptr = c.upload(nptr);
  dc.rptr = c.upload(rptr);
  dc.nent = c.upload(nent);
  dc.rnode = c.upload(rnode);
  dc.rcolumn = c.upload(rcolumn);
  dc.sv_state = c.alloc<double>(node_off);
  dc.lfull = c.alloc<double>(fac_off);
  dc.dpiv = c.alloc<double>(dfac_off);
  dc.dinv = c.alloc<double>(dfac_off);
  dc.svals = c.alloc<double>(sv_off);
  dc.wtail = c.alloc<double>(w_off);
  dc.topo = c.upload(topo);
  dc.ck_i = K > 0 ? c.alloc<double>(ck_off) : nullptr;
  dc.ck_u = K > 0 ? c.alloc<double>(ck_off) : nullptr;
  dc.seg_i = K > 0 ? c.alloc<double>(seg_off) : nullptr;
  dc.seg_u = K > 0 ? c.alloc<double>(seg_off) : nullptr;
  if (c.adj_pipe) c.d_pipe = c.alloc<int32_t>(2 * (size_t)NI);
  dc.line_tab = line_tab.empty() ? nullptr : c.upload(line_tab);
  dc.line_gf = line_gf.empty() ? nullptr : c.upload(line_gf);
  dc.ring = ring_off > 0 ? c.alloc<double>(ring_off) : nullptr;
  c.ring_doubles = ring_off;
  if (dyn_off > 0) {
    dc.dyn = c.alloc<double>(dyn_off);
    dc.dstate = c.alloc<int32_t>(c.nbr_total);
    // controlled switches' measured node pairs, item-local (ground: n)
    bool any_cs = false;
    std::vector<int32_t> bmeas(2 * (size_t)c.nbr_total, 0);
    for (int q = 0; q < NI; ++q) {
      const Item &it = A.items[q];
      const Scenario &sc = A.scens[it.scen];
      const emt_net &net = nets[it.scen];
      for (int j = 0; j < it.n_br; ++j) {
        const int b = it.br[j];
        const int64_t gb = c.items[q].br + j;
        bmeas[2 * gb] = bmeas[2 * gb + 1] = it.n;
        if (b < 0 || net.kind[b] != EMT_CSWITCH) continue;
        any_cs = true;
        for (int e2 = 0; e2 < 2; ++e2) {
          const int a = net.meas[2 * b + e2];
          if (a >= 0 && sc.node_item[a] != q)
            throw Error{EMT_EDEVICE, "internal: a controlled switch measures a node of another work item"};
          bmeas[2 * gb + e2] = a >= 0 ? sc.node_local[a] : it.n;
        }
      }
    }
    if (any_cs) dc.bmeas = c.upload(bmeas);
  }
  if (!group_tab.empty()) {
    // per-branch mutual values and member flags, in the branch arrays' order
    std::vector<double> bRm, bLm, bCm;
    std::vector<int32_t> bgrp;
    for (const Item &it : A.items) {
      const emt_net &net = nets[it.scen];
      for (int j = 0; j < it.n_br; ++j) {
        const int b = it.br[j];
        const bool g = b >= 0 && net.group && net.group[b] >= 0 && net.kind[b] != EMT_LINE;
        bgrp.push_back(g ? 1 : 0);
        bRm.push_back(g ? net.Rm[b] : 0.0);
        bLm.push_back(g ? net.Lm[b] : 0.0);
        bCm.push_back(g ? net.Cm[b] : 0.0);
      }
    }
    dc.group_tab = c.upload(group_tab);
    dc.mptr = c.upload(mptr_all);
    dc.ment = ment_all.empty() ? nullptr : c.upload(ment_all);
    dc.bRm = c.upload(bRm);
    dc.bLm = c.upload(bLm);
    dc.bCm = c.upload(bCm);
    dc.bgrp = c.upload(bgrp);
    dc.cgo = c.alloc<double>(coef_off);
    dc.cbo = c.alloc<double>(coef_off);
  }
  dc.flags = c.alloc<int32_t>(8);
  hip_check(launch_fill_i32(dc.flags, 8, 0, nullptr), "clear flags");
  dc.dt = sim.dt;
  dc.T = T;
  dc.K = K;
  dc.rec_stride = A.rec_stride;
  c.d_order = c.upload(order);
  c.d_pairs = c.upload(pairs);
  c.ca.coef_base = c.upload(ca_coef);
  c.ca.br_base = c.upload(ca_br);
  c.ca.nbr_of = c.upload(ca_nbr);
  c.ca.cnt_prefix = c.upload(ca_prefix);
  c.ca.total = (int)work;
  c.ca.n_items = NI;
  c.d_bscen = c.upload(bscen);
  c.d_bitem = c.upload(bitem);
  c.d_blocal = c.upload(blocal);
  c.d_br_ids = c.upload(br_ids);
  c.d_lptr = c.upload(lptr);
  c.d_lent = c.upload(lent);
  c.d_line_scen = c.upload(line_scen);
  c.d_line_id = c.upload(line_id);
  {
    std::vector<int32_t> nrec(A.scens.size());
    for (size_t q = 0; q < A.scens.size(); ++q) nrec[q] = A.scens[q].n_rec;
    c.d_nrec = c.upload(nrec);
  }
  int64_t max_scen_br = 0;
  for (size_t s = 0; s + 1 < c.scen_br_off.size(); ++s)
    max_scen_br = std::max(max_scen_br, c.scen_br_off[s + 1] - c.scen_br_off[s]);
  c.d_stage = c.alloc<double>(max_scen_br);
  build_split(c, bpack);
  if (sim.solver == EMT_SOLVER_COMPENSATION) build_comp(c, nets);
  // statistics
  c.sweep_levels = 0;
  for (const Item &it : A.items)
    c.sweep_levels = std::max(c.sweep_levels, plans[it.sym].nfpass() + plans[it.sym].nbpass() + (plans[it.sym].d > 0 ? 1 : 0));
}

static hipError_t launch_comp_step(emt_ctx &c, int64_t n0, int64_t ns, double *rec, hipStream_t st) {
  return emt::launch_comp(c.dc, c.cc, c.ks.bs, c.ks.bpt, c.comp_q, c.comp_lanes, c.comp_blocks, n0, ns, rec,
                          c.comp_lds, st);
}

// The compensation solver's factor work after the LDL^T factors: the bases'
// inverses, the parameter check of matched pi-section branches (flags[5])
// and every K (flags[6]).
static void launch_comp_factor(emt_ctx &c, hipStream_t st) {
  if (!c.comp) return;
  hip_check(emt::launch_fill_i32(c.dc.flags + 5, 2, 0, st), "clear flags");
  hip_check(emt::launch_comp_factor(c.dc, c.cc, st), "compensation factor");
}

// Status words of a factorisation (after its work has finished).
static void check_factor_flags(emt_ctx &c) {
  int32_t f[8] = {0};
  hip_check(hipMemcpy(f, c.dc.flags, sizeof(f), hipMemcpyDeviceToHost), "status flags");
  if (f[0] != 0) {
    c.factored = false;
    throw emt::Error{EMT_ESINGULAR, std::to_string(f[0]) + " non-positive or non-finite pivots"};
  }
  if (c.comp && f[5] != 0) {
    c.factored = false;
    throw emt::Error{EMT_EINVAL, "compensation solver: " + std::to_string(f[5]) +
                                     " pi-section branches have parameters that differ from the first scenario's"};
  }
  if (c.comp && f[6] != 0) {
    c.factored = false;
    throw emt::Error{EMT_ESINGULAR, "compensation solver: " + std::to_string(f[6]) +
                                        " switched topologies have no Sherman-Morrison-Woodbury correction"};
  }
}

static hipError_t launch_forward(emt_ctx &c, int64_t n0, int64_t ns, double *rec, hipStream_t st) {
  emt::KernelShape ks = c.ks;
  ks.sm = c.sm_fwd;
  if (!ks.sm) ks.bpt = c.bpt_global;
  switch (ks.bs) {
    case 64: return emt::launch_forward_bs64(c.dc, ks, c.d_order, c.n_fwd, n0, ns, rec, st);
    case 256: return emt::launch_forward_bs256(c.dc, ks, c.d_order, c.n_fwd, n0, ns, rec, st);
    default: return emt::launch_forward_bs512(c.dc, ks, c.d_order, c.n_fwd, n0, ns, rec, st);
  }
}

// The split components' launch: both exchange buffers hold values whose
// tag matches neither of the first two steps ((step / 2) mod 4 in the two
// lowest bits, step parity choosing the buffer) and the tiles' XCD record is
// empty. The give-up flag is not cleared here: it stays set from the launch
// that gave up until the next run starts (arm_split_flag) and is read by the
// synchronising calls.
static void launch_split_with(emt_ctx &c, const emt::SplitCtx &sc, int64_t n0, int64_t ns, double *rec,
                              hipStream_t st, bool floor) {
  for (const auto &f : c.split_xbuf)
    for (int64_t m = n0 + 1; m <= n0 + 2; ++m) {
      const int64_t stale = (((m >> 1) & 3) + 2) & 3;
      int64_t *buf = reinterpret_cast<int64_t *>(sc.xbuf + f.first + (m & 1) * f.second);
      hip_check(emt::launch_fill_i64(buf, f.second, stale, st), "split exchange buffer");
    }
  hip_check(emt::launch_fill_i32(sc.xcc, c.n_tiles, -1, st), "split placement record");
  hip_check(emt::launch_split(c.dc, sc, c.split_bpt, c.split_rpl, c.split_rt, c.split_grid, n0, ns, rec,
                              c.split_lds, floor, st),
            floor ? "split latency floor" : "split forward");
}

static void launch_split_step(emt_ctx &c, int64_t n0, int64_t ns, double *rec, hipStream_t st,
                              bool floor = false) {
  launch_split_with(c, c.sc, n0, ns, rec, st, floor);
}

// Layout of the static exchange space for this context's split components:
// partials at offset 0, then the give-up flag, then the XCD record (256-byte
// aligned parts). Returns the bytes needed.
static int64_t static_layout(const emt_ctx &c, int64_t *err_off, int64_t *xcc_off) {
  auto up = [](int64_t b) { return (b + 255) & ~int64_t(255); };
  *err_off = up(c.xbuf_doubles * 8);
  *xcc_off = *err_off + 256;
  return *xcc_off + up((int64_t)c.n_tiles * 4);
}

// Clears the split give-up flag at the start of a run (factor, reset,
// set_params), in stream order.
static void arm_split_flag(emt_ctx &c, hipStream_t st) {
  if (c.n_tiles == 0) return;
  hip_check(emt::launch_fill_i32(c.sc.err, 1, 0, st), "split error flag");
}

static int32_t read_flag(const int32_t *dev) {
  int32_t v = 0;
  hip_check(hipMemcpy(&v, dev, sizeof(int32_t), hipMemcpyDeviceToHost), "status flag");
  return v;
}

// After the work of this run has finished: a split launch gave up waiting
// for its workgroups (its outputs are not valid).
static void report_split(const emt_ctx &c) {
  if (c.n_tiles > 0 && read_flag(c.sc.err) != 0)
    throw emt::Error{EMT_EDEVICE, "a split-component launch gave up waiting for its workgroups"};
}

// After the queued work has finished: every status word it may have set
// (split give-up, pivots of an asynchronous factorisation, pipelined
// adjoint give-up).
static void report_all(emt_ctx &c) {
  report_split(c);
  if (c.pivots_pending) {
    c.pivots_pending = false;
    check_factor_flags(c);
  }
  if (c.adjoint_pending) {
    c.adjoint_pending = false;
    if (read_flag(c.dc.flags + 2) != 0)
      throw emt::Error{EMT_EDEVICE, "the pipelined adjoint gave up waiting for its recompute workgroups"};
  }
  if (c.dc.dyn) {
    // pivots of the factorisations inside the time loop (diode changes)
    const int32_t bad = read_flag(c.dc.flags + 4);
    if (bad != 0) {
      hip_check(emt::launch_fill_i32(c.dc.flags + 4, 1, 0, nullptr), "clear flag");
      throw emt::Error{EMT_ESINGULAR, std::to_string(bad) + " non-positive or non-finite pivots in the loop"};
    }
  }
}

static hipError_t launch_adjoint(emt_ctx &c, const double *dJ, hipStream_t st) {
  emt::KernelShape ks = c.ks;
  ks.sm = c.sm_adj;
  if (!ks.sm) ks.bpt = c.bpt_global;
  switch (ks.bs) {
    case 64: return emt::launch_adjoint_bs64(c.dc, ks, c.d_order, c.n_fwd, dJ, st);
    case 256: return emt::launch_adjoint_bs256(c.dc, ks, c.d_order, c.n_fwd, dJ, st);
    default: return emt::launch_adjoint_bs512(c.dc, ks, c.d_order, c.n_fwd, dJ, st);
  }
}

extern "C" {

const char *emt_last_error(void) { return g_last_error.c_str(); }

emt_status emt_analyze(const emt_net *nets, int32_t n_scen, const emt_sim *sim, emt_info *info) {
  return guarded([&]() -> emt_status {
    if (!sim || !info) return set_error(EMT_EINVAL, "sim and info are required");
    emt::Analysis A = emt::analyze(nets, n_scen, *sim);
    emt::fill_info(A, info);
    if (sim->solver == EMT_SOLVER_COMPENSATION) {
      const emt::CompPlan P = emt::plan_compensation(A, nets, *sim);
      info->comp_families = (int32_t)P.fams.size();
      info->comp_max_rank = P.max_rank;
    }
    return EMT_OK;
  });
}

emt_status emt_build(const emt_net *nets, int32_t n_scen, const emt_sim *sim, emt_ctx **out) {
  return guarded([&]() -> emt_status {
    if (!out || !sim) return set_error(EMT_EINVAL, "sim and out are required");
    *out = nullptr;
    emt::Analysis A = emt::analyze(nets, n_scen, *sim);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return set_error(EMT_EDEVICE, "no HIP device");
    std::unique_ptr<emt_ctx> c(new emt_ctx);
    c->A = std::move(A);
    c->sim = *sim;
    hip_check(hipGetDevice(&c->device), "hipGetDevice");
    upload_all(*c, nets);
    hip_check(emt::launch_companions(c->dc, c->ca, nullptr), "companions");
    hip_check(emt::launch_reset(c->dc, c->d_bitem, c->d_blocal, c->nbr_total, c->nodes_total, c->ring_doubles, nullptr), "reset");
    hip_check(hipDeviceSynchronize(), "build");
    *out = c.release();
    return EMT_OK;
  });
}

emt_status emt_info_get(const emt_ctx *ctx, emt_info *info) {
  return guarded([&]() -> emt_status {
    if (!ctx || !info) return set_error(EMT_EINVAL, "ctx and info are required");
    emt::fill_info(ctx->A, info);
    info->step = ctx->step;
    info->device_bytes = ctx->device_bytes;
    info->block_size = ctx->ks.bs;
    info->dense_items = ctx->dense_items;
    info->sweep_levels = ctx->sweep_levels;
    info->max_tail = ctx->max_tail;
    info->lds_bytes = (int32_t)ctx->ks.lds_fwd;
    info->lds_limit = ctx->lds_limit;
    info->lds_staged = ctx->sm_fwd ? 1 : 0;
    info->lanes_per_block = ctx->ks.bpt;
    info->split_tiles = ctx->n_tiles;
    info->adjoint_pipelined = ctx->adj_pipe ? 1 : 0;
    info->split_cols = ctx->n_tiles > 0 ? ctx->split_rt : 0;
    info->comp_families = ctx->cc.n_fam;
    info->comp_max_rank = ctx->comp_max_rank;
    info->comp_items = ctx->comp_q;
    info->comp_blocks = ctx->comp_blocks;
    if (ctx->comp) info->lds_bytes = (int32_t)ctx->comp_lds;
    info->split_local = 0;
    if (ctx->n_tiles > 0 && ctx->sc.allow_local) {
      // the XCD record of the last launch (all -1 before the first one)
      std::vector<int32_t> xcc(ctx->n_tiles);
      hip_check(hipDeviceSynchronize(), "sync");
      hip_check(hipMemcpy(xcc.data(), ctx->sc.xcc, xcc.size() * sizeof(int32_t), hipMemcpyDeviceToHost),
                "split placement record");
      for (const auto &r : ctx->split_range) {
        bool same = xcc[r.first] >= 0;
        for (int p = 1; p < r.second; ++p) same = same && xcc[r.first + p] == xcc[r.first];
        info->split_local += same ? 1 : 0;
      }
    }
    return EMT_OK;
  });
}

emt_status emt_set_params(emt_ctx *ctx, const double *theta_dev, void *stream) {
  return guarded([&]() -> emt_status {
    if (!ctx || !theta_dev) return set_error(EMT_EINVAL, "ctx and theta are required");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hip_check(emt::launch_set_params(ctx->dc, theta_dev, ctx->A.param_stride, ctx->d_bscen, ctx->nbr_total, st),
              "set_params");
    hip_check(emt::launch_companions(ctx->dc, ctx->ca, st), "companions");
    hip_check(emt::launch_reset(ctx->dc, ctx->d_bitem, ctx->d_blocal, ctx->nbr_total, ctx->nodes_total, ctx->ring_doubles, st),
              "reset");
    arm_split_flag(*ctx, st);
    ctx->step = 0;
    ctx->factored = false;
    ctx->clean = true;
    return EMT_OK;
  });
}

emt_status emt_factor(emt_ctx *ctx, void *stream) {
  return guarded([&]() -> emt_status {
    if (!ctx) return set_error(EMT_EINVAL, "ctx is required");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hip_check(emt::launch_fill_i32(ctx->dc.flags, 1, 0, st), "clear flags");
    arm_split_flag(*ctx, st);
    hip_check(emt::launch_factor(ctx->dc, ctx->d_pairs, ctx->n_pairs, ctx->max_tail, st), "factor");
    if (ctx->n_tiles > 0)
      hip_check(emt::launch_inverse(ctx->dc, ctx->sc, ctx->d_inv_jobs, ctx->n_inv_jobs, ctx->inverse_lds, st),
                "inverse");
    launch_comp_factor(*ctx, st);
    hip_check(hipStreamSynchronize(st), "factor sync");
    ctx->pivots_pending = false;
    check_factor_flags(*ctx);
    ctx->factored = true;
    return EMT_OK;
  });
}

emt_status emt_factor_async(emt_ctx *ctx, void *stream) {
  return guarded([&]() -> emt_status {
    if (!ctx) return set_error(EMT_EINVAL, "ctx is required");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hip_check(emt::launch_fill_i32(ctx->dc.flags, 1, 0, st), "clear flags");
    arm_split_flag(*ctx, st);
    hip_check(emt::launch_factor(ctx->dc, ctx->d_pairs, ctx->n_pairs, ctx->max_tail, st), "factor");
    if (ctx->n_tiles > 0)
      hip_check(emt::launch_inverse(ctx->dc, ctx->sc, ctx->d_inv_jobs, ctx->n_inv_jobs, ctx->inverse_lds, st),
                "inverse");
    launch_comp_factor(*ctx, st);
    ctx->factored = true;
    ctx->pivots_pending = true;
    return EMT_OK;
  });
}

emt_status emt_step(emt_ctx *ctx, int64_t n, double *rec_dev, void *stream) {
  return guarded([&]() -> emt_status {
    if (!ctx) return set_error(EMT_EINVAL, "ctx is required");
    if (n < 0) return set_error(EMT_EINVAL, "n must be >= 0");
    if (!ctx->factored) return set_error(EMT_ESTATE, "emt_factor has not succeeded since the last change");
    if (ctx->step + n > ctx->sim.n_steps) return set_error(EMT_ESTATE, "stepping past n_steps");
    if (n == 0) return EMT_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (ctx->comp)
      hip_check(launch_comp_step(*ctx, ctx->step, n, rec_dev, st), "compensation forward");
    else if (ctx->n_fwd > 0)
      hip_check(launch_forward(*ctx, ctx->step, n, rec_dev, st), "forward");
    if (ctx->n_tiles > 0) launch_split_step(*ctx, ctx->step, n, rec_dev, st);
    ctx->step += n;
    return EMT_OK;
  });
}

emt_status emt_step_noalloc(emt_ctx *ctx, int64_t n, double *rec_dev, void *stream) {
  return guarded([&]() -> emt_status {
    if (!ctx) return set_error(EMT_EINVAL, "ctx is required");
    if (n < 0) return set_error(EMT_EINVAL, "n must be >= 0");
    if (!ctx->factored) return set_error(EMT_ESTATE, "emt_factor has not succeeded since the last change");
    if (ctx->step + n > ctx->sim.n_steps) return set_error(EMT_ESTATE, "stepping past n_steps");
    int64_t err_off = 0, xcc_off = 0;
    const int64_t need = ctx->n_tiles > 0 ? static_layout(*ctx, &err_off, &xcc_off) : 0;
    if (need > emt::kStaticScratchBytes)
      return set_error(EMT_EINVAL, "the split components' exchange needs " + std::to_string(need) +
                                       " bytes; the static exchange space holds " +
                                       std::to_string(emt::kStaticScratchBytes));
    if (n == 0) return EMT_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (ctx->comp)
      hip_check(launch_comp_step(*ctx, ctx->step, n, rec_dev, st), "compensation forward");
    else if (ctx->n_fwd > 0)
      hip_check(launch_forward(*ctx, ctx->step, n, rec_dev, st), "forward");
    if (ctx->n_tiles > 0) {
      void *base = nullptr;
      hip_check(emt::static_scratch_ptr(ctx->device, &base), "static scratch address");
      char *b = static_cast<char *>(base);
      emt::SplitCtx sc = ctx->sc;
      sc.xbuf = reinterpret_cast<double *>(b);
      sc.err = reinterpret_cast<int32_t *>(b + err_off);
      sc.xcc = reinterpret_cast<int32_t *>(b + xcc_off);
      hip_check(emt::launch_fill_i32(sc.err, 1, 0, st), "split error flag");
      launch_split_with(*ctx, sc, ctx->step, n, rec_dev, st, false);
      // a give-up joins the run's sticky flag
      hip_check(emt::launch_or_flag(ctx->sc.err, sc.err, st), "split error flag");
    }
    ctx->step += n;
    return EMT_OK;
  });
}

emt_status emt_mismatch(emt_ctx *ctx, const double *rec_dev, const double *target_dev, double *dJ_drec_dev,
                        double *loss_dev, void *stream) {
  return guarded([&]() -> emt_status {
    if (!ctx || !rec_dev || !target_dev || !dJ_drec_dev || !loss_dev)
      return set_error(EMT_EINVAL, "ctx, rec, target, dJ_drec and loss are required");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hip_check(emt::launch_mismatch(rec_dev, target_dev, dJ_drec_dev, loss_dev, ctx->d_nrec, (int)ctx->A.scens.size(),
                                   ctx->sim.n_steps, ctx->A.rec_stride, st),
              "mismatch");
    return EMT_OK;
  });
}

emt_status emt_sync(emt_ctx *ctx, void *stream) {
  return guarded([&]() -> emt_status {
    if (!ctx) return set_error(EMT_EINVAL, "ctx is required");
    hip_check(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "sync");
    report_all(*ctx);
    return EMT_OK;
  });
}

emt_status emt_latency_floor(emt_ctx *ctx, int32_t kernel, int64_t n_steps, double *us_per_step, void *stream) {
  // events and the scratch output are released on every path
  struct Scratch {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double *out = nullptr;
    ~Scratch() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      if (out) (void)hipFree(out);
    }
  };
  return guarded([&]() -> emt_status {
    if (!ctx || !us_per_step) return set_error(EMT_EINVAL, "ctx and us_per_step are required");
    if (n_steps <= 0 || n_steps > (int64_t(1) << 30)) return set_error(EMT_EINVAL, "n_steps must be in 1 .. 2^30");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scratch sc;
    hip_check(hipEventCreate(&sc.e0), "event");
    hip_check(hipEventCreate(&sc.e1), "event");
    if (kernel == EMT_FLOOR_ONE_WORKGROUP && ctx->comp) {
      // the compensation kernel's four phases per step (gather, product,
      // correction, branch update) in its grid, workgroup and LDS size
      int fb = 64;  // the floor kernel's lanes: a power of two, at least the workgroup's
      while (fb < ctx->comp_lanes) fb *= 2;
      hip_check(hipMalloc(reinterpret_cast<void **>(&sc.out), (size_t)ctx->comp_blocks * fb * sizeof(double)),
                "hipMalloc");
      hip_check(hipEventRecord(sc.e0, st), "event");
      hip_check(emt::launch_barrier_floor(fb, ctx->comp_blocks, 4, n_steps, ctx->comp_lds, sc.out, st),
                "barrier floor");
      hip_check(hipEventRecord(sc.e1, st), "event");
    } else if (kernel == EMT_FLOOR_ONE_WORKGROUP) {
      if (ctx->n_fwd == 0) return set_error(EMT_EINVAL, "no component of this batch runs in one workgroup");
      hip_check(hipMalloc(reinterpret_cast<void **>(&sc.out), (size_t)ctx->n_fwd * ctx->ks.bs * sizeof(double)),
                "hipMalloc");
      hip_check(hipEventRecord(sc.e0, st), "event");
      hip_check(emt::launch_barrier_floor(ctx->ks.bs, ctx->n_fwd, ctx->sweep_levels + 2, n_steps, ctx->ks.lds_fwd,
                                          sc.out, st),
                "barrier floor");
      hip_check(hipEventRecord(sc.e1, st), "event");
    } else if (kernel == EMT_FLOOR_SPLIT) {
      if (ctx->n_tiles == 0) return set_error(EMT_EINVAL, "no split component in this batch");
      hip_check(hipStreamSynchronize(st), "sync");
      report_split(*ctx);
      arm_split_flag(*ctx, st);
      hip_check(hipEventRecord(sc.e0, st), "event");
      launch_split_step(*ctx, 0, n_steps, nullptr, st, true);
      hip_check(hipEventRecord(sc.e1, st), "event");
    } else {
      return set_error(EMT_EINVAL, "kernel must be EMT_FLOOR_ONE_WORKGROUP or EMT_FLOOR_SPLIT");
    }
    hip_check(hipEventSynchronize(sc.e1), "sync");
    float ms = 0.0f;
    hip_check(hipEventElapsedTime(&ms, sc.e0, sc.e1), "event time");
    if (kernel == EMT_FLOOR_SPLIT) report_split(*ctx);
    *us_per_step = (double)ms * 1e3 / (double)n_steps;
    return EMT_OK;
  });
}

emt_status emt_steady_state(emt_ctx *ctx, void *stream) {
  return guarded([&]() -> emt_status {
    if (!ctx) return set_error(EMT_EINVAL, "ctx is required");
    for (const emt::Item &it : ctx->A.items)
      if (!it.line_bk.empty())
        return set_error(EMT_EINVAL, "distributed-parameter lines start from rest (no steady state)");
    if (ctx->dc.dyn)
      return set_error(EMT_EINVAL, "diodes and controlled switches switch by their own state (no steady state)");
    for (size_t q = 0; q < ctx->scen_mixed_freq.size(); ++q)
      if (ctx->scen_mixed_freq[q])
        return set_error(EMT_EINVAL, "scenario " + std::to_string(q) +
                                         ": sources at different frequencies have no single steady state");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int NI = (int)ctx->A.items.size();
    if (!ctx->ss_L) {
      std::vector<int64_t> offl(NI), offn(NI);
      int64_t nl = 0, nn = 0;
      for (int q = 0; q < NI; ++q) {
        offl[q] = nl;
        offn[q] = nn;
        nl += ctx->A.syms[ctx->A.items[q].sym].nnz();
        nn += ctx->A.items[q].n;
      }
      ctx->d_ss_offl = ctx->upload(offl);
      ctx->d_ss_offn = ctx->upload(offn);
      ctx->ss_L = ctx->alloc<double>(2 * (size_t)std::max<int64_t>(nl, 1));
      ctx->ss_D = ctx->alloc<double>(2 * (size_t)std::max<int64_t>(nn, 1));
      ctx->ss_X = ctx->alloc<double>(2 * (size_t)std::max<int64_t>(nn, 1));
    }
    hip_check(emt::launch_fill_i32(ctx->dc.flags + 3, 1, 0, st), "clear flag");
    arm_split_flag(*ctx, st);
    hip_check(emt::launch_steady(ctx->dc, NI, ctx->d_ss_offl, ctx->d_ss_offn, ctx->ss_L, ctx->ss_D, ctx->ss_X,
                                 ctx->dc.flags + 3, st),
              "steady state");
    int32_t bad = 0;
    hip_check(hipMemcpyAsync(&bad, ctx->dc.flags + 3, sizeof(int32_t), hipMemcpyDeviceToHost, st), "flag");
    hip_check(hipStreamSynchronize(st), "steady-state sync");
    ctx->step = 0;
    ctx->clean = false;
    if (bad) return set_error(EMT_ESINGULAR, std::to_string(bad) + " zero or non-finite complex pivots");
    return EMT_OK;
  });
}

emt_status emt_reset(emt_ctx *ctx, void *stream) {
  return guarded([&]() -> emt_status {
    if (!ctx) return set_error(EMT_EINVAL, "ctx is required");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hip_check(emt::launch_reset(ctx->dc, ctx->d_bitem, ctx->d_blocal, ctx->nbr_total, ctx->nodes_total, ctx->ring_doubles, st),
              "reset");
    arm_split_flag(*ctx, st);
    ctx->step = 0;
    ctx->clean = true;
    return EMT_OK;
  });
}

emt_status emt_adjoint(emt_ctx *ctx, const double *dJ_drec_dev, double *grad_dev, void *stream) {
  return guarded([&]() -> emt_status {
    if (!ctx || !grad_dev) return set_error(EMT_EINVAL, "ctx and grad are required");
    if (!dJ_drec_dev && ctx->A.rec_stride > 0) return set_error(EMT_EINVAL, "dJ_drec is required");
    if (ctx->sim.checkpoint_every <= 0) return set_error(EMT_ESTATE, "built without checkpoints");
    if (!ctx->factored || !ctx->clean || ctx->step != ctx->sim.n_steps)
      return set_error(EMT_ESTATE, "needs a complete forward run from step 0 since the last change");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!ctx->ks_adj_ok) return set_error(EMT_EINVAL, "a connected component is too large for the adjoint kernel");
    if (ctx->n_tiles > 0) return set_error(EMT_EINVAL, "the split dense solver runs forward only");
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hip_check(hipStreamIsCapturing(st, &cap), "capture status");
    // the pipelined kernel is a cooperative launch: not recorded into graphs
    if (ctx->adj_pipe && cap == hipStreamCaptureStatusNone) {
      emt::KernelShape ks = ctx->ks;
      ks.sm = ctx->sm_adj;
      if (!ks.sm) ks.bpt = ctx->bpt_global;
      hip_check(emt::launch_fill_i32(ctx->d_pipe, 2 * (int64_t)ctx->A.items.size(), 0, st), "pipe counters");
      hip_check(emt::launch_fill_i32(ctx->dc.flags + 2, 1, 0, st), "pipe error flag");
      const int n = ctx->n_fwd;
      hip_check(ks.bs == 64 ? emt::launch_adjoint_pipe_bs64(ctx->dc, ks, ctx->d_order, n, dJ_drec_dev, ctx->d_pipe, st)
                : ks.bs == 256
                    ? emt::launch_adjoint_pipe_bs256(ctx->dc, ks, ctx->d_order, n, dJ_drec_dev, ctx->d_pipe, st)
                    : emt::launch_adjoint_pipe_bs512(ctx->dc, ks, ctx->d_order, n, dJ_drec_dev, ctx->d_pipe, st),
                "adjoint");
      ctx->adjoint_pending = true;
    } else {
      hip_check(launch_adjoint(*ctx, dJ_drec_dev, st), "adjoint");
    }
    const int P = ctx->A.param_stride;
    hip_check(emt::launch_grad(ctx->dc, ctx->d_lptr, ctx->d_lent, ctx->d_line_scen, ctx->d_line_id,
                               ctx->n_lines_total, grad_dev, P, (int64_t)ctx->A.scens.size() * P, st),
              "grad");
    return EMT_OK;
  });
}

emt_status emt_branch_adjoints(emt_ctx *ctx, int32_t scen, double *gbar, double *betabar, double *gammabar) {
  return guarded([&]() -> emt_status {
    if (!ctx || scen < 0 || scen >= (int)ctx->A.scens.size()) return set_error(EMT_EINVAL, "bad scenario");
    hip_check(hipDeviceSynchronize(), "sync");
    const emt::Scenario &sc = ctx->A.scens[scen];
    double *outs[3] = {gbar, betabar, gammabar};
    double *srcs[3] = {ctx->dc.gbar, ctx->dc.bbar, ctx->dc.cbar};
    std::vector<double> buf(ctx->nbr_total);
    for (int w = 0; w < 3; ++w) {
      if (!outs[w]) continue;
      hip_check(hipMemcpy(buf.data(), srcs[w], buf.size() * sizeof(double), hipMemcpyDeviceToHost), "copy");
      for (int b = 0; b < sc.n_branches; ++b)
        outs[w][b] = sc.br_item[b] < 0 ? 0.0 : buf[ctx->items[sc.br_item[b]].br + sc.br_local[b]];
    }
    return EMT_OK;
  });
}

emt_status emt_get_state(emt_ctx *ctx, int32_t scen, double *v_host, double *i_host) {
  return guarded([&]() -> emt_status {
    if (!ctx || scen < 0 || scen >= (int)ctx->A.scens.size()) return set_error(EMT_EINVAL, "bad scenario");
    hip_check(hipDeviceSynchronize(), "sync");
    report_split(*ctx);
    const emt::Scenario &sc = ctx->A.scens[scen];
    if (v_host) {
      std::vector<double> sv(ctx->nodes_total);
      hip_check(hipMemcpy(sv.data(), ctx->dc.sv_state, sv.size() * sizeof(double), hipMemcpyDeviceToHost), "copy v");
      for (int a = 0; a < sc.n_nodes; ++a)
        v_host[a] = sv[ctx->items[sc.node_item[a]].node + sc.node_local[a]];
    }
    if (i_host) {
      std::vector<double> si(ctx->nbr_total);
      hip_check(hipMemcpy(si.data(), ctx->dc.si, si.size() * sizeof(double), hipMemcpyDeviceToHost), "copy i");
      for (int b = 0; b < sc.n_branches; ++b)
        i_host[b] = sc.br_item[b] < 0 ? 0.0 : si[ctx->items[sc.br_item[b]].br + sc.br_local[b]];
    }
    return EMT_OK;
  });
}

emt_status emt_set_state(emt_ctx *ctx, int32_t scen, const double *v_host, const double *i_host) {
  return guarded([&]() -> emt_status {
    if (!ctx || scen < 0 || scen >= (int)ctx->A.scens.size() || !v_host || !i_host)
      return set_error(EMT_EINVAL, "bad arguments");
    const emt::Scenario &sc = ctx->A.scens[scen];
    for (int q : sc.items)
      if (!ctx->A.items[q].line_bk.empty())
        return set_error(EMT_EINVAL, "a scenario with distributed-parameter lines starts from rest (no set_state)");
    for (int a = 0; a < sc.n_nodes; ++a)
      if (!std::isfinite(v_host[a])) return set_error(EMT_EINVAL, "non-finite voltage");
    for (int b = 0; b < sc.n_branches; ++b)
      if (!std::isfinite(i_host[b])) return set_error(EMT_EINVAL, "non-finite current");
    hip_check(hipDeviceSynchronize(), "sync");
    for (int q : sc.items) {
      const emt::Item &it = ctx->A.items[q];
      std::vector<double> v(it.n);
      for (int a = 0; a < it.n; ++a) v[a] = v_host[it.gnode[a]];
      hip_check(hipMemcpy(ctx->dc.sv_state + ctx->items[q].node, v.data(), v.size() * sizeof(double),
                          hipMemcpyHostToDevice),
                "copy v");
    }
    std::vector<double> iv;
    for (int b = 0; b < sc.n_branches; ++b)
      if (sc.br_item[b] >= 0) iv.push_back(i_host[b]);
    const int64_t b0 = ctx->scen_br_off[scen], nb = ctx->scen_br_off[scen + 1] - b0;
    if (nb > 0) {
      hip_check(hipMemcpy(ctx->d_stage, iv.data(), nb * sizeof(double), hipMemcpyHostToDevice), "copy i");
      hip_check(emt::launch_set_state(ctx->dc, ctx->d_bitem, ctx->d_blocal, ctx->d_br_ids, b0, nb, ctx->d_stage,
                                      ctx->step, nullptr),
                "set_state");
    }
    hip_check(hipDeviceSynchronize(), "sync");
    ctx->clean = false;
    return EMT_OK;
  });
}

void emt_destroy(emt_ctx *ctx) {
  if (!ctx) return;
  (void)hipDeviceSynchronize();
  delete ctx;
}

}  // extern "C"
