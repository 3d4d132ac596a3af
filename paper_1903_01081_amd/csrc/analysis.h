// Host-side analysis of a batch of networks: validation, topologies,
// connected components, fill-reducing ordering, symbolic LDL^T and the level
// schedules of the two triangular sweeps. No device code and no HIP calls.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "emt.h"

namespace emt {

// Thrown inside the library only; converted to a status at the C boundary.
struct Error {
  emt_status status;
  std::string msg;
};

// Symbolic LDL^T of one connected component. Local node ids are positions in
// the elimination order, so L is strictly lower triangular in them.
struct Symbolic {
  int n = 0;
  std::vector<int> lrow_ptr, lrow_col;  // L by rows (columns ascending)
  std::vector<int> lcol_ptr, lcol_row;  // L by columns (rows ascending)
  std::vector<int> lcol_pos;            // CSC entry -> CSR entry of the same nonzero
  std::vector<int> flev_ptr, flev_rows; // forward sweep: rows grouped by level
  std::vector<int> blev_ptr, blev_rows; // backward sweep: rows grouped by level
  std::vector<int> fent_ptr, fent;      // per forward level: CSC entries of its columns
  int64_t nnz() const { return (int64_t)lrow_col.size(); }
  int levels_f() const { return (int)flev_ptr.size() - 1; }
  int levels_b() const { return (int)blev_ptr.size() - 1; }
};

// Sweep plan of a symbolic factor with a dense tail of d nodes. The last d
// nodes of the elimination order (the top of the elimination tree, where the
// factor is dense and the level schedule degenerates into a chain) are solved
// in one step with the precomputed inverse of their Schur complement; the
// leading ns = n - d nodes keep level-scheduled sparse sweeps. Sweep entries
// ("sv") are the nonzeros L_rc with c < ns, stored once in row order.
struct SweepPlan {
  int d = 0, ns = 0;
  std::vector<int> frow_ptr;             // [n+1] row r's sv entries
  std::vector<int> fcol;                 // [nsv] column of each sv entry
  std::vector<int> svmap;                // [nsv] CSR position of the entry in the full L
  std::vector<int> bptr;                 // [ns+1] column r's sv entries (backward sweep)
  std::vector<int> brow, bpos;           // [nsv] row and sv index of each
  std::vector<int> flev_ptr, flev_rows;  // forward levels over rows < ns
  std::vector<int> blev_ptr, blev_rows;  // backward levels over rows < ns
  // Row descriptors for the device sweeps: row | first entry << 16 | count
  // << 32. Forward passes: levels 1.. of the leading rows (level 0 rows have
  // no entries), then one pass over the tail rows; backward passes: the
  // backward levels. Per pass: start, row count, largest count.
  std::vector<uint64_t> fdesc, bdesc;
  std::vector<int> fpass_ptr, fpass_maxcnt, bpass_ptr, bpass_maxcnt;
  int nsv() const { return (int)fcol.size(); }
  int nfpass() const { return (int)fpass_ptr.size() - 1; }
  int nbpass() const { return (int)bpass_ptr.size() - 1; }
  int nlf() const { return (int)flev_ptr.size() - 1; }
  int nlb() const { return (int)blev_ptr.size() - 1; }
};

SweepPlan plan_sweeps(const Symbolic &S, int d);

// Dense-tail size minimising the barrier-separated phases of one solve
// (forward levels + backward levels + 2 for the tail), with a small penalty
// per tail node, over d <= dmax.
int choose_tail(const Symbolic &S, int dmax);

// One work item: one connected component of one scenario.
struct Item {
  int scen = 0, sym = 0, n = 0, n_br = 0, n_src = 0;
  int n_br_real = 0;        // branches before padding to whole lane slots
  std::vector<int> gnode;   // local node -> scenario node id
  std::vector<int> br;      // local branch -> scenario branch id (sources first; -1 = padding)
  std::vector<int> bk, bm;  // local terminals (-1 = ground)
  std::vector<int> nptr, nent;  // node CSR of incident branch ends: (local branch << 1) | (end is m)
  std::vector<int> gpos;    // per local branch: CSR entry of L for its off-diagonal, -1 if none
  std::vector<int> rec_node, rec_col;  // recorded local node and its output column
  // distributed-parameter lines: each is two local branches (its k end and
  // its m end, Norton equivalents to ground) whose histories come from each
  // other's travelling waves; per line its two local branches and nodes and
  // its delay tau / dt = D0 + f
  std::vector<int> line_bk, line_bm, line_nk, line_nm, line_d0;
  std::vector<double> line_f;
  // coupled three-phase groups: the local branches of each group's three
  // members, and the groups' mutual conductance stamps by row of L (CSR:
  // entry = L position, and local branch << 1 | 1 if the stamp is -g_o)
  std::vector<int> grp_b;
  std::vector<int> mptr, mpos, mcode;
};

struct Scenario {
  int n_nodes = 0, n_branches = 0, n_rec = 0, n_params = 0, n_topo = 1;
  std::vector<int64_t> topo_step;           // topo_step[t] = first step of topology t (t >= 1)
  std::vector<std::vector<uint8_t>> ins;    // [topology][branch] in service
  std::vector<int> node_item, node_local;   // scenario node -> (item, local id)
  std::vector<int> br_item, br_local;       // scenario branch -> (item, local id) or -1
  std::vector<int> items;
};

struct Analysis {
  std::vector<Symbolic> syms;
  std::vector<Item> items;
  std::vector<Scenario> scens;
  int rec_stride = 0, param_stride = 0, max_topo = 1;
};

// Validates and analyses; throws Error on invalid input or singular topology.
Analysis analyze(const emt_net *nets, int n_scen, const emt_sim &sim);

void fill_info(const Analysis &a, emt_info *info);

}  // namespace emt
