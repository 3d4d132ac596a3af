// Host-side analysis under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Reads networks written by test_host_sanitizers.py (one batch per file:
// int32 count, then per network its counts and arrays in the order of
// emt_net), analyses the batch with every solver and launch-shape setting
// the ABI accepts, and some invalid inputs, and prints one line per
// analysis. Built with g++ -fsanitize=address,undefined and
// -fno-sanitize-recover, so any memory or UB error ends the run non-zero.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "analysis.h"
#include "comp_plan.h"

namespace {

struct Net {
  int32_t n_nodes = 0, n_branches = 0, n_params = 0, n_events = 0, n_rec = 0;
  std::vector<int32_t> k, m, kind, line, ev_branch, rec_nodes;
  std::vector<double> R, L, C, E, omega, phase;
  std::vector<uint8_t> in_service0, ev_in_service;
  std::vector<int64_t> ev_step;
  bool has_ins = false, has_rec = false;
};

template <class T>
bool rd(FILE *f, T *p, size_t n) {
  return n == 0 || std::fread(p, sizeof(T), n, f) == n;
}

template <class T>
bool rdv(FILE *f, std::vector<T> &v, size_t n) {
  v.resize(n);
  return rd(f, v.data(), n);
}

bool read_net(FILE *f, Net &n) {
  int32_t h[7];
  if (!rd(f, h, 7)) return false;
  n.n_nodes = h[0];
  n.n_branches = h[1];
  n.n_params = h[2];
  n.n_events = h[3];
  n.n_rec = h[4];
  n.has_ins = h[5] != 0;
  n.has_rec = h[6] != 0;
  const size_t B = (size_t)n.n_branches, V = (size_t)n.n_events;
  return rdv(f, n.k, B) && rdv(f, n.m, B) && rdv(f, n.kind, B) && rdv(f, n.R, B) && rdv(f, n.L, B) &&
         rdv(f, n.C, B) && rdv(f, n.E, B) && rdv(f, n.omega, B) && rdv(f, n.phase, B) && rdv(f, n.line, B) &&
         rdv(f, n.in_service0, n.has_ins ? B : 0) && rdv(f, n.ev_step, V) && rdv(f, n.ev_branch, V) &&
         rdv(f, n.ev_in_service, V) && rdv(f, n.rec_nodes, n.has_rec ? (size_t)n.n_rec : 0);
}

emt_net view(const Net &n) {
  emt_net e{};
  e.n_nodes = n.n_nodes;
  e.n_branches = n.n_branches;
  e.k = n.k.data();
  e.m = n.m.data();
  e.kind = n.kind.data();
  e.R = n.R.data();
  e.L = n.L.data();
  e.C = n.C.data();
  e.E = n.E.data();
  e.omega = n.omega.data();
  e.phase = n.phase.data();
  e.line = n.line.data();
  e.n_params = n.n_params;
  e.in_service0 = n.has_ins ? n.in_service0.data() : nullptr;
  e.n_events = n.n_events;
  e.ev_step = n.ev_step.data();
  e.ev_branch = n.ev_branch.data();
  e.ev_in_service = n.ev_in_service.data();
  e.n_rec = n.n_rec;
  e.rec_nodes = n.has_rec ? n.rec_nodes.data() : nullptr;
  return e;
}

// One analysis: prints the status and, on success, the sizes that must not
// depend on the launch shape (items, symbolic patterns, nonzeros of L).
int run(const char *label, const std::vector<emt_net> &nets, const emt_sim &sim) {
  emt_info info{};
  try {
    emt::Analysis a = emt::analyze(nets.data(), (int)nets.size(), sim);
    emt::fill_info(a, &info);
    std::printf("%s ok items %d symbolic %d nnz_L %lld levels %d\n", label, info.n_items, info.n_symbolic,
                (long long)info.nnz_L, info.max_levels);
    return 0;
  } catch (const emt::Error &e) {
    std::printf("%s error %d\n", label, (int)e.status);
    return (int)e.status;
  }
}

// The compensation solver's plan on top of the analysis (families, node
// maps, branch matching, switched branches).
int run_comp(const char *label, const std::vector<emt_net> &nets, const emt_sim &sim) {
  try {
    emt::Analysis a = emt::analyze(nets.data(), (int)nets.size(), sim);
    emt::CompPlan p = emt::plan_compensation(a, nets.data(), sim);
    std::printf("%s comp families %d rank %d mods %d\n", label, (int)p.fams.size(), p.max_rank, (int)p.mods.size());
    return 0;
  } catch (const emt::Error &e) {
    std::printf("%s error %d\n", label, (int)e.status);
    return (int)e.status;
  }
}

}  // namespace

int main(int argc, char **argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: %s batch.bin\n", argv[0]);
    return 2;
  }
  FILE *f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t count = 0;
  if (!rd(f, &count, 1) || count < 1) return 2;
  std::vector<Net> nets((size_t)count);
  for (Net &n : nets)
    if (!read_net(f, n)) return 2;
  std::fclose(f);
  std::vector<emt_net> views;
  for (const Net &n : nets) views.push_back(view(n));

  emt_sim base{};
  base.dt = 20e-6;
  base.n_steps = 400;
  base.dense_tail = -1;
  int bad = 0;
  // every solver and launch-shape setting the ABI accepts
  for (int solver : {0, 1, 2})
    for (int bs : {0, 64, 256, 512})
      for (int K : {0, 50}) {
        emt_sim s = base;
        s.solver = solver;
        s.block_size = bs;
        s.checkpoint_every = K;
        char label[96];
        std::snprintf(label, sizeof label, "solver %d block %d K %d", solver, bs, K);
        const int st = run(label, views, s);
        if (st != 0 && st != EMT_EINVAL) bad = 1;
      }
  for (int K : {0, 50}) {
    emt_sim s = base;
    s.solver = EMT_SOLVER_COMPENSATION;
    s.checkpoint_every = K;
    char label[64];
    std::snprintf(label, sizeof label, "compensation K %d", K);
    const int st = run_comp(label, views, s);
    if (st != 0 && st != EMT_EINVAL) bad = 1;
  }
  for (int d : {0, 16, 48, 128}) {
    emt_sim s = base;
    s.dense_tail = d;
    char label[64];
    std::snprintf(label, sizeof label, "dense_tail %d", d);
    if (run(label, views, s) != 0) bad = 1;
  }
  for (int p : {64, 256, 30000}) {
    emt_sim s = base;
    s.pack_nodes = p;
    char label[64];
    std::snprintf(label, sizeof label, "pack_nodes %d", p);
    const int st = run(label, views, s);
    if (st != 0 && st != EMT_EINVAL) bad = 1;
  }
  // invalid inputs are reported, not crashed on
  {
    std::vector<Net> broken = nets;
    broken[0].k[0] = broken[0].n_nodes + 7;  // terminal out of range
    std::vector<emt_net> v;
    for (const Net &n : broken) v.push_back(view(n));
    if (run("terminal out of range", v, base) != EMT_EINVAL) bad = 1;
  }
  {
    std::vector<Net> broken = nets;
    if (broken[0].n_events > 0) broken[0].ev_step[0] = -3;  // event before the horizon
    else broken[0].kind[0] = 99;
    std::vector<emt_net> v;
    for (const Net &n : broken) v.push_back(view(n));
    if (run("bad event or kind", v, base) != EMT_EINVAL) bad = 1;
  }
  {
    emt_sim s = base;
    s.dt = -1.0;
    if (run("negative dt", views, s) != EMT_EINVAL) bad = 1;
  }
  return bad;
}
