// CPU oracle for the EMT nodal-analysis time loop — TEST INFRASTRUCTURE ONLY.
//
// Only the test suite, the smoke check and the benchmark's CPU-baseline leg
// may load this library. It shares no code with the GPU library: it reads the
// same network description (branch list, parameters, events) and nothing else.
//
// What it computes (the paper, Sec. III-A, lists the four basic processes of
// an EMTP-type solver: update each component's Norton equivalent (history
// current and conductance), assemble nodal injected currents, factorise the
// nodal conductance matrix, forward/back substitute for node voltages; the
// formulas are the textbook trapezoidal companion models of the EMTP method
// the paper cites as its reference [2]):
//
//   companion (per in-service branch b, time step dt):
//     series R-L (and source impedance):  g = 1/(R + 2L/dt),
//                                         beta = (2L/dt - R) g, gamma = g
//     capacitor:                          g = 2C/dt, beta = -1, gamma = -g
//     resistor / closed switch:           g = 1/R,   beta = gamma = 0
//     out-of-service branch:              g = beta = gamma = 0, u = i = 0
//   state at step 0: v_0 = 0, i_0 = 0, u_0 = A^T v_0 - e_0 (zero state,
//     sources active from t = 0), unless an initial state is supplied.
//   for n = 1..T (t_n = n dt):
//     apply the events of step n (switches change, G is re-assembled and
//       re-factorised: the new topology produces v_n);
//     h_n   = beta * i_{n-1} + gamma * u_{n-1}              (history current)
//     e_n   = E cos(omega t_n + phase)       (source branches; 0 elsewhere)
//     rhs_n = A (g * e_n - h_n)                          (nodal injections)
//     v_n   = G^{-1} rhs_n,  G = A diag(g) A^T    (dense LU, partial pivot)
//     u_n   = A^T v_n - e_n,  i_n = g * u_n + h_n         (branch update)
//   A is the node-by-branch incidence matrix (+1 at k_b, -1 at m_b, ground
//   rows dropped), u_b is the voltage across the branch's passive part and
//   i_b flows from k_b to m_b.
//
// Discrete adjoint of that recursion (reverse time, hbar_{T+1} = 0):
//     ibar_n = beta_{n+1} hbar_{n+1}
//     q_n    = gamma_{n+1} hbar_{n+1} + g_n ibar_n            (= ubar_n)
//     vbar_n = dJ/dv_n + A q_n,   w_n = G_n^{-T} vbar_n
//     hbar_n = ibar_n - A^T w_n
//     gbar += hbar_n u_n, betabar += hbar_n i_{n-1}, gammabar += hbar_n u_{n-1}
//   then the chain rule to the per-line parameters (R_l, L_l, C_l).
//
// Distributed-parameter (travelling-wave, Bergeron) lines, kind 5, between
// nodes k and m with surge impedance Z (field R) and travel time tau (field
// L, tau >= dt): the lossless line of the EMTP method (the paper's reference
// [2]). Each end is a Norton equivalent to ground, g = 1/Z, whose history
// current is the wave that left the other end tau earlier:
//     i_k(n) = g v_k(n) + h_k(n),   h_k(n) = -w_m(t_n - tau),
//     w_m(n) = g v_m(n) + i_m(n)    (and the same with k and m swapped),
// i_k the current from node k into the line. t_n - tau falls between steps:
// with tau / dt = D0 + f (0 <= f < 1), w(t_n - tau) = (1 - f) w(n - D0) +
// f w(n - D0 - 1), and w = 0 before step 1 (the line starts at rest). The
// branch current i of a line is i_k; its u is v_k. Lines run forward only
// (the adjoint rejects them), take no events and no initial state.
//
// Everything is plain loops over dense arrays in the scalar type T (double,
// or std::complex<double> for complex-step differentiation; pivots are chosen
// by |Re| so that the complex run stays analytic).

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

enum { K_RL = 0, K_C = 1, K_R = 2, K_SWITCH = 3, K_SRC = 4, K_LINE = 5, K_DIODE = 6, K_CSWITCH = 7 };

}  // namespace

extern "C" {

// Network description as plain arrays (layout mirrors the generator's
// Network object; the GPU library has its own declaration of this shape).
struct OracleNet {
  int32_t n_nodes, n_branches;
  const int32_t *k, *m, *kind;
  const double *R, *L, *C, *E, *omega, *phase;
  const int32_t *line;
  int32_t n_params;
  const uint8_t *in_service0;  // may be null: all in service, switches open
  int32_t n_events;
  const int64_t *ev_step;
  const int32_t *ev_branch;
  const uint8_t *ev_in_service;
  int32_t n_rec;
  const int32_t *rec_nodes;  // may be null: every node
  // coupled three-phase groups (may be null): group id per branch or -1, and
  // the mutual entries of each group's circulant R, L or C matrix
  const int32_t *group;
  const double *Rm, *Lm, *Cm;
  // controlled switches (may be null if there is none): the measured node
  // pair of each branch, [2 n_branches]
  const int32_t *meas;
};

}  // extern "C"

namespace {

using cplx = std::complex<double>;

inline double re(double x) { return x; }
inline double re(const cplx &x) { return x.real(); }

template <class T>
struct Companions {
  std::vector<T> g, beta, gamma;
  // mutual coefficients of coupled groups (0 elsewhere): the off-diagonal
  // entries of the group's circulant G, B and Gamma
  std::vector<T> go, bo, co;
};

// Members of each coupled group (three branches), in branch order.
std::vector<std::vector<int>> group_members(const OracleNet &net) {
  std::vector<std::vector<int>> gm;
  if (!net.group) return gm;
  for (int b = 0; b < net.n_branches; ++b) {
    const int g = net.group[b];
    if (g < 0) continue;
    if ((int)gm.size() <= g) gm.resize(g + 1);
    gm[g].push_back(b);
  }
  return gm;
}

// Per-branch R, L, C with the line parameters theta applied (series branch:
// R_l, L_l; each shunt capacitor of a pi-section: C_l / 2).
template <class T>
void branch_values(const OracleNet &net, const T *theta, int b, T &R, T &L, T &C) {
  R = T(net.R[b]);
  L = T(net.L[b]);
  C = T(net.C[b]);
  const int l = net.line[b];
  if (theta && l >= 0) {
    if (net.kind[b] == K_RL) {
      R = theta[3 * l + 0];
      L = theta[3 * l + 1];
    } else if (net.kind[b] == K_C) {
      C = theta[3 * l + 2] / 2.0;
    }
  }
}

template <class T>
void companions(const OracleNet &net, const T *theta, double dt,
                const std::vector<uint8_t> &ins, Companions<T> &c) {
  const int B = net.n_branches;
  c.g.assign(B, T(0));
  c.beta.assign(B, T(0));
  c.gamma.assign(B, T(0));
  for (int b = 0; b < B; ++b) {
    if (!ins[b]) continue;
    T R, L, C;
    branch_values(net, theta, b, R, L, C);
    switch (net.kind[b]) {
      case K_RL:
      case K_SRC: {
        T g = T(1) / (R + T(2) * L / dt);
        c.g[b] = g;
        c.beta[b] = (T(2) * L / dt - R) * g;
        c.gamma[b] = g;
        break;
      }
      case K_C: {
        T g = T(2) * C / dt;
        c.g[b] = g;
        c.beta[b] = T(-1);
        c.gamma[b] = -g;
        break;
      }
      default: {  // resistor, closed switch, or a line end's 1/Z
        c.g[b] = T(1) / R;
        break;
      }
    }
  }
  // Coupled groups: 3 x 3 circulant companions, i = G u + h and
  // h' = B i + Gamma u per group (RL: G = (R + 2L/dt)^{-1}, B = G (2L/dt -
  // R), Gamma = G; C: G = 2C/dt, B = -I, Gamma = -G). A 3 x 3 circulant with diagonal d and off-diagonal o has eigenvalues
  // d + 2o (zero sequence) and d - o (positive and negative sequence), and
  // products and inverses of circulants are circulants with the products
  // and inverses of these eigenvalues.
  c.go.assign(B, T(0));
  c.bo.assign(B, T(0));
  c.co.assign(B, T(0));
  if (!net.group) return;
  auto diag_off = [](T e0, T e1, T &d, T &o) {  // circulant from its two eigenvalues
    d = (e0 + T(2) * e1) / T(3);
    o = (e0 - e1) / T(3);
  };
  for (int b = 0; b < B; ++b) {
    if (net.group[b] < 0 || !ins[b]) continue;
    if (net.kind[b] == K_RL) {
      const T Md = T(net.R[b]) + T(2) * T(net.L[b]) / dt, Mo = T(net.Rm[b]) + T(2) * T(net.Lm[b]) / dt;
      const T Nd = T(2) * T(net.L[b]) / dt - T(net.R[b]), No = T(2) * T(net.Lm[b]) / dt - T(net.Rm[b]);
      const T l0 = Md + T(2) * Mo, l1 = Md - Mo, m0 = Nd + T(2) * No, m1 = Nd - No;
      diag_off(T(1) / l0, T(1) / l1, c.g[b], c.go[b]);        // G = M^{-1}
      diag_off(m0 / l0, m1 / l1, c.beta[b], c.bo[b]);         // B = G N
      c.gamma[b] = c.g[b];                                    // Gamma = G
      c.co[b] = c.go[b];
    } else {  // capacitor group: G = 2 C / dt, B = -I, Gamma = -G
      c.g[b] = T(2) * T(net.C[b]) / dt;
      c.go[b] = T(2) * T(net.Cm[b]) / dt;
      c.beta[b] = T(-1);
      c.bo[b] = T(0);
      c.gamma[b] = -c.g[b];
      c.co[b] = -c.go[b];
    }
  }
}

// Dense LU with partial pivoting (row swaps), in place, row-major n x n.
template <class T>
struct DenseLU {
  int n = 0;
  std::vector<T> a;
  std::vector<int> piv;
  // pivot on |Re| (complex step: the imaginary parts are perturbations) or,
  // for genuinely complex systems, on the modulus
  bool by_modulus = false;
  double mag(const T &x) const { return by_modulus ? std::abs(x) : std::fabs(re(x)); }

  bool factor(const std::vector<T> &G, int n_) {
    n = n_;
    a = G;
    piv.resize(n);
    for (int j = 0; j < n; ++j) {
      int p = j;
      double best = mag(a[(size_t)j * n + j]);
      for (int i = j + 1; i < n; ++i) {
        double v = mag(a[(size_t)i * n + j]);
        if (v > best) {
          best = v;
          p = i;
        }
      }
      piv[j] = p;
      if (best == 0.0) return false;
      if (p != j)
        for (int c = 0; c < n; ++c) std::swap(a[(size_t)j * n + c], a[(size_t)p * n + c]);
      const T d = a[(size_t)j * n + j];
      for (int i = j + 1; i < n; ++i) {
        T f = a[(size_t)i * n + j] / d;
        a[(size_t)i * n + j] = f;
        if (f == T(0)) continue;
        T *ri = &a[(size_t)i * n];
        const T *rj = &a[(size_t)j * n];
        for (int c = j + 1; c < n; ++c) ri[c] -= f * rj[c];
      }
    }
    return true;
  }

  // Solve G x = b: P G = L U.
  void solve(std::vector<T> &x) const {
    for (int j = 0; j < n; ++j)
      if (piv[j] != j) std::swap(x[j], x[piv[j]]);
    for (int i = 0; i < n; ++i) {
      T s = x[i];
      const T *ri = &a[(size_t)i * n];
      for (int c = 0; c < i; ++c) s -= ri[c] * x[c];
      x[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
      T s = x[i];
      const T *ri = &a[(size_t)i * n];
      for (int c = i + 1; c < n; ++c) s -= ri[c] * x[c];
      x[i] = s / ri[i];
    }
  }

  // Solve G^T x = b: G^T = U^T L^T P, so U^T y = b, L^T z = y, x = P^T z.
  void solve_transposed(std::vector<T> &x) const {
    for (int i = 0; i < n; ++i) {
      T s = x[i];
      for (int c = 0; c < i; ++c) s -= a[(size_t)c * n + i] * x[c];
      x[i] = s / a[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      T s = x[i];
      for (int c = i + 1; c < n; ++c) s -= a[(size_t)c * n + i] * x[c];
      x[i] = s;
    }
    for (int j = n - 1; j >= 0; --j)
      if (piv[j] != j) std::swap(x[j], x[piv[j]]);
  }
};

template <class T>
void assemble(const OracleNet &net, const Companions<T> &c, std::vector<T> &G) {
  const int N = net.n_nodes;
  G.assign((size_t)N * N, T(0));
  for (int b = 0; b < net.n_branches; ++b) {
    const int k = net.k[b], m = net.m[b];
    const T g = c.g[b];
    if (k >= 0) G[(size_t)k * N + k] += g;
    if (m >= 0) G[(size_t)m * N + m] += g;
    if (net.kind[b] == K_LINE) continue;  // two Norton equivalents to ground
    if (k >= 0 && m >= 0) {
      G[(size_t)k * N + m] -= g;
      G[(size_t)m * N + k] -= g;
    }
  }
  // coupled groups: A Gm A^T with Gm's off-diagonal go between members
  for (const auto &mem : group_members(net))
    for (int p : mem)
      for (int q : mem) {
        if (p == q) continue;
        const int tp[2] = {net.k[p], net.m[p]}, tq[2] = {net.k[q], net.m[q]};
        for (int a = 0; a < 2; ++a)
          for (int e = 0; e < 2; ++e) {
            if (tp[a] < 0 || tq[e] < 0) continue;
            const T v = (a == e) ? c.go[p] : -c.go[p];
            G[(size_t)tp[a] * N + tq[e]] += v;
          }
      }
}

inline double emf(const OracleNet &net, int b, int64_t n, double dt) {
  if (net.kind[b] != K_SRC) return 0.0;
  const double t = (double)n * dt;
  return net.E[b] * std::cos(net.omega[b] * t + net.phase[b]);
}

bool valid(const OracleNet &net, double dt, int64_t T) {
  if (!(dt > 0) || T < 0 || net.n_nodes <= 0 || net.n_branches < 0) return false;
  for (int b = 0; b < net.n_branches; ++b) {
    const int k = net.k[b], m = net.m[b];
    if (k < -1 || k >= net.n_nodes || m < -1 || m >= net.n_nodes) return false;
    if (k < 0 && m < 0) return false;
    if (net.kind[b] < 0 || net.kind[b] > 7) return false;
    if (net.kind[b] == K_CSWITCH) {
      if (!(net.R[b] > 0) || !(net.L[b] >= 0) || !std::isfinite(net.L[b]) || !std::isfinite(net.C[b]) ||
          !std::isfinite(net.E[b]) || !std::isfinite(net.omega[b]) || !std::isfinite(net.phase[b]) || !net.meas ||
          net.line[b] >= 0 || (net.group && net.group[b] >= 0))
        return false;
      for (int e2 = 0; e2 < 2; ++e2)
        if (net.meas[2 * b + e2] < -1 || net.meas[2 * b + e2] >= net.n_nodes) return false;
    }
    if (net.kind[b] == K_DIODE && (!(net.R[b] > 0) || net.line[b] >= 0 || (net.group && net.group[b] >= 0)))
      return false;
    if (net.kind[b] == K_LINE &&
        (k < 0 || m < 0 || k == m || !(net.R[b] > 0) || !(net.L[b] >= dt) || net.C[b] != 0.0 || net.line[b] >= 0))
      return false;
  }
  for (int j = 0; j < net.n_events; ++j) {
    if (net.ev_step[j] < 1) return false;
    if (net.ev_branch[j] < 0 || net.ev_branch[j] >= net.n_branches) return false;
    if (net.kind[net.ev_branch[j]] == K_LINE || net.kind[net.ev_branch[j]] == K_DIODE ||
        net.kind[net.ev_branch[j]] == K_CSWITCH)
      return false;
  }
  for (int r = 0; r < net.n_rec; ++r)
    if (net.rec_nodes && (net.rec_nodes[r] < 0 || net.rec_nodes[r] >= net.n_nodes)) return false;
  if (net.group) {
    if (!net.Rm || !net.Lm || !net.Cm) return false;
    for (int b = 0; b < net.n_branches; ++b)
      if (net.group[b] < -1) return false;
    for (const auto &mem : group_members(net)) {
      if (mem.size() != 3) return false;
      const int b0 = mem[0];
      for (int b : mem) {
        if (net.kind[b] != net.kind[b0] || (net.kind[b] != K_RL && net.kind[b] != K_C) || net.line[b] >= 0)
          return false;
        if (net.R[b] != net.R[b0] || net.L[b] != net.L[b0] || net.C[b] != net.C[b0] || net.Rm[b] != net.Rm[b0] ||
            net.Lm[b] != net.Lm[b0] || net.Cm[b] != net.Cm[b0])
          return false;
        if (net.in_service0 && !net.in_service0[b]) return false;
        for (int j = 0; j < net.n_events; ++j)
          if (net.ev_branch[j] == b) return false;
      }
      if (net.kind[b0] == K_RL) {
        if (!(net.L[b0] - net.Lm[b0] > 0) || !(net.L[b0] + 2 * net.Lm[b0] > 0) ||
            !(net.R[b0] - net.Rm[b0] >= 0) || !(net.R[b0] + 2 * net.Rm[b0] >= 0))
          return false;
      } else if (!(net.C[b0] - net.Cm[b0] > 0) || !(net.C[b0] + 2 * net.Cm[b0] > 0)) {
        return false;
      }
    }
  }
  return true;
}

bool has_groups(const OracleNet &net) { return !group_members(net).empty(); }

// Diodes and controlled switches: branches whose state the run itself sets.
bool has_diodes(const OracleNet &net) {
  for (int b = 0; b < net.n_branches; ++b)
    if (net.kind[b] == K_DIODE || net.kind[b] == K_CSWITCH) return true;
  return false;
}

inline int rec_node(const OracleNet &net, int r) { return net.rec_nodes ? net.rec_nodes[r] : r; }

bool has_lines(const OracleNet &net) {
  for (int b = 0; b < net.n_branches; ++b)
    if (net.kind[b] == K_LINE) return true;
  return false;
}

// The travelling waves of the lines: w[end][step] for every line, end 0 = k,
// end 1 = m; step 0 and earlier read 0 (the line at rest).
template <class T>
struct Waves {
  std::vector<int> lines;                 // branch ids of the lines
  std::vector<std::vector<T>> w[2];       // [end][line][step]
  double dt = 0;
  void init(const OracleNet &net, double dt_, int64_t Tn) {
    dt = dt_;
    for (int b = 0; b < net.n_branches; ++b)
      if (net.kind[b] == K_LINE) lines.push_back(b);
    for (int e = 0; e < 2; ++e) w[e].assign(lines.size(), std::vector<T>(Tn + 1, T(0)));
  }
  T at(int e, size_t q, int64_t j) const { return j <= 0 ? T(0) : w[e][q][j]; }
  // w of end e of line q at t_n - tau (linear interpolation between steps)
  T delayed(const OracleNet &net, int e, size_t q, int64_t n) const {
    const double D = net.L[lines[q]] / dt;
    const int64_t D0 = (int64_t)std::floor(D);
    const double f = D - (double)D0;
    return (1.0 - f) * at(e, q, n - D0) + f * at(e, q, n - D0 - 1);
  }
};

// One forward run. Optional outputs may be null. Trajectories have T+1 rows
// (row 0 = initial state). Returns 0 on success, 1 on bad input, 2 on a
// singular conductance matrix.
template <class T>
int forward(const OracleNet &net, const T *theta, double dt, int64_t Tn,
            const double *v0, const double *i0, T *rec, T *v_traj, T *i_traj, T *u_traj,
            std::vector<int> *topo_of_step, std::vector<Companions<T>> *topos,
            std::vector<DenseLU<T>> *lus) {
  if (!valid(net, dt, Tn)) return 1;
  if (has_lines(net) && (v0 || i0)) return 1;
  const int N = net.n_nodes, B = net.n_branches;
  std::vector<uint8_t> ins(B);
  for (int b = 0; b < B; ++b)
    ins[b] = net.in_service0 ? net.in_service0[b] : (net.kind[b] == K_SWITCH ? 0 : 1);

  Companions<T> c;
  companions(net, theta, dt, ins, c);
  std::vector<T> G;
  assemble(net, c, G);
  DenseLU<T> lu;
  if (!lu.factor(G, N)) return 2;
  if (topos) {
    topos->clear();
    topos->push_back(c);
  }
  if (lus) {
    lus->clear();
    lus->push_back(lu);
  }
  if (topo_of_step) topo_of_step->assign(Tn + 1, 0);

  std::vector<T> v(N, T(0)), i(B, T(0)), u(B, T(0)), h(B), e(B), x(N);
  if (v0)
    for (int a = 0; a < N; ++a) v[a] = T(v0[a]);
  if (i0)
    for (int b = 0; b < B; ++b) i[b] = ins[b] ? T(i0[b]) : T(0);
  for (int b = 0; b < B; ++b) {
    if (!ins[b]) continue;
    T vk = net.k[b] >= 0 ? v[net.k[b]] : T(0);
    T vm = net.m[b] >= 0 ? v[net.m[b]] : T(0);
    u[b] = vk - vm - emf(net, b, 0, dt);
  }
  if (v_traj) std::copy(v.begin(), v.end(), v_traj);
  if (i_traj) std::copy(i.begin(), i.end(), i_traj);
  if (u_traj) std::copy(u.begin(), u.end(), u_traj);

  Waves<T> waves;
  waves.init(net, dt, Tn);
  const std::vector<std::vector<int>> groups = group_members(net);

  // Events sorted by step (stable order within a step).
  std::vector<int> ev(net.n_events);
  for (int j = 0; j < net.n_events; ++j) ev[j] = j;
  std::stable_sort(ev.begin(), ev.end(),
                   [&](int a, int b) { return net.ev_step[a] < net.ev_step[b]; });
  size_t next_ev = 0;
  int topo = 0;
  // ideal diodes (state-dependent switches): a conducting diode (1/R_on)
  // whose current is negative after a step blocks from the next step on; a
  // blocking one whose voltage v_k - v_m is positive conducts from the next
  // step on
  bool flipped = false;

  for (int64_t n = 1; n <= Tn; ++n) {
    bool changed = flipped;
    flipped = false;
    while (next_ev < ev.size() && net.ev_step[ev[next_ev]] == n) {
      const int j = ev[next_ev++];
      ins[net.ev_branch[j]] = net.ev_in_service[j] ? 1 : 0;
      changed = true;
    }
    while (next_ev < ev.size() && net.ev_step[ev[next_ev]] < n) ++next_ev;
    if (changed) {
      companions(net, theta, dt, ins, c);
      assemble(net, c, G);
      if (!lu.factor(G, N)) return 2;
      ++topo;
      if (topos) topos->push_back(c);
      if (lus) lus->push_back(lu);
    }
    if (topo_of_step) (*topo_of_step)[n] = topo;

    for (int b = 0; b < B; ++b) {
      h[b] = c.beta[b] * i[b] + c.gamma[b] * u[b];
      e[b] = T(emf(net, b, n, dt));
    }
    for (const auto &mem : groups) {  // mutual terms: the other members' i, u
      T si = T(0), su = T(0);
      for (int q : mem) {
        si += i[q];
        su += u[q];
      }
      for (int p : mem) h[p] += c.bo[p] * (si - i[p]) + c.co[p] * (su - u[p]);
    }
    std::fill(x.begin(), x.end(), T(0));
    for (int b = 0; b < B; ++b) {
      if (net.kind[b] == K_LINE) continue;
      const T j = c.g[b] * e[b] - h[b];
      if (net.k[b] >= 0) x[net.k[b]] += j;
      if (net.m[b] >= 0) x[net.m[b]] -= j;
    }
    // lines: each end injects minus its history current (the wave that left
    // the other end tau earlier)
    std::vector<T> hk(waves.lines.size()), hm(waves.lines.size());
    for (size_t q = 0; q < waves.lines.size(); ++q) {
      const int b = waves.lines[q];
      hk[q] = -waves.delayed(net, 1, q, n);
      hm[q] = -waves.delayed(net, 0, q, n);
      x[net.k[b]] -= hk[q];
      x[net.m[b]] -= hm[q];
    }
    lu.solve(x);
    v = x;
    for (int b = 0; b < B; ++b) {
      if (!ins[b]) {
        u[b] = T(0);
        i[b] = T(0);
        continue;
      }
      if (net.kind[b] == K_LINE) continue;
      T vk = net.k[b] >= 0 ? v[net.k[b]] : T(0);
      T vm = net.m[b] >= 0 ? v[net.m[b]] : T(0);
      u[b] = vk - vm - e[b];
      i[b] = c.g[b] * u[b] + h[b];
    }
    for (const auto &mem : groups) {
      T su = T(0);
      for (int q : mem) su += u[q];
      for (int p : mem) i[p] += c.go[p] * (su - u[p]);
    }
    for (int b = 0; b < B; ++b) {
      if (net.kind[b] != K_DIODE) continue;
      const T vk = net.k[b] >= 0 ? v[net.k[b]] : T(0);
      const T vm = net.m[b] >= 0 ? v[net.m[b]] : T(0);
      if (ins[b] && re(i[b]) < 0.0) {
        ins[b] = 0;
        flipped = true;
      } else if (!ins[b] && re(vk - vm) > 0.0) {
        ins[b] = 1;
        flipped = true;
      }
    }
    // controlled switches: a hysteresis comparator on the measured voltage
    // s = v_a - v_b of this step against the reference r = E cos(w t + phi)
    // + C at this step's time sets the switch for the next step: on above
    // the band (e = r - s > h), off below it (e < -h), unchanged inside
    for (int b = 0; b < B; ++b) {
      if (net.kind[b] != K_CSWITCH) continue;
      const int a0 = net.meas[2 * b], a1 = net.meas[2 * b + 1];
      const double sv = re(a0 >= 0 ? v[a0] : T(0)) - re(a1 >= 0 ? v[a1] : T(0));
      const double r = net.E[b] * std::cos(net.omega[b] * ((double)n * dt) + net.phase[b]) + net.C[b];
      const double err = r - sv, hw = net.L[b];
      const uint8_t want = err > hw ? 1 : (err < -hw ? 0 : ins[b]);
      if (want != ins[b]) {
        ins[b] = want;
        flipped = true;
      }
    }
    for (size_t q = 0; q < waves.lines.size(); ++q) {
      const int b = waves.lines[q];
      const T g = c.g[b], vk = v[net.k[b]], vm = v[net.m[b]];
      const T ik = g * vk + hk[q], im = g * vm + hm[q];
      waves.w[0][q][n] = g * vk + ik;
      waves.w[1][q][n] = g * vm + im;
      u[b] = vk;
      i[b] = ik;
    }
    if (rec)
      for (int r = 0; r < net.n_rec; ++r) rec[(size_t)(n - 1) * net.n_rec + r] = v[rec_node(net, r)];
    if (v_traj) std::copy(v.begin(), v.end(), v_traj + (size_t)n * N);
    if (i_traj) std::copy(i.begin(), i.end(), i_traj + (size_t)n * B);
    if (u_traj) std::copy(u.begin(), u.end(), u_traj + (size_t)n * B);
  }
  return 0;
}

// Sinusoidal steady state of the initial topology (not in the paper: the
// usual start of an EMTP-type run). With every source at one angular
// frequency w, the companion recursion i_n = g u_n + h_n, h_{n+1} = beta i_n
// + gamma u_n, u_n = A^T v_n - e_n has the periodic solution x_n = Re(X z^n)
// with z = exp(j w dt): each branch acts as the discrete admittance
// y = (g z + gamma) / (z - beta), the node phasors solve (A y A^T) V = A y E
// with E_b = E_b exp(j phase_b) on sources, and the state at step 0 is
// v_0 = Re V, u_0 = Re U, i_0 = Re(y U), U = A^T V - E. A network without
// sources rests at zero. Returns 0, 1 (bad input: distributed-parameter
// lines, sources at different frequencies) or 2 (singular).
int steady_state(const OracleNet &net, const double *theta, double dt, double *v0, double *i0, double *Vre,
                 double *Vim) {
  if (!valid(net, dt, 1) || has_lines(net) || has_diodes(net)) return 1;
  const int N = net.n_nodes, B = net.n_branches;
  double w = 0.0;
  bool any = false;
  for (int b = 0; b < B; ++b) {
    if (net.kind[b] != K_SRC) continue;
    if (any && net.omega[b] != w) return 1;
    w = net.omega[b];
    any = true;
  }
  std::vector<cplx> V(N, cplx(0.0, 0.0));
  std::vector<uint8_t> ins(B);
  for (int b = 0; b < B; ++b)
    ins[b] = net.in_service0 ? net.in_service0[b] : (net.kind[b] == K_SWITCH ? 0 : 1);
  Companions<double> c;
  companions(net, theta, dt, ins, c);
  const cplx z = std::polar(1.0, w * dt);
  std::vector<cplx> y(B, cplx(0.0, 0.0)), E(B, cplx(0.0, 0.0));
  std::vector<cplx> yo(B, cplx(0.0, 0.0));  // mutual admittance of coupled groups
  const std::vector<std::vector<int>> groups = group_members(net);
  for (int b = 0; b < B; ++b) {
    if (!ins[b]) continue;
    y[b] = (c.g[b] * z + c.gamma[b]) / (z - c.beta[b]);
    if (net.kind[b] == K_SRC) E[b] = std::polar(net.E[b], net.phase[b]);
  }
  for (const auto &mem : groups)
    for (int b : mem) {
      // per sequence (zero: d + 2o, positive/negative: d - o) the scalar
      // admittance, then back to the circulant's diagonal and off-diagonal
      const cplx y0 = (cplx(c.g[b] + 2 * c.go[b]) * z + (c.gamma[b] + 2 * c.co[b])) /
                      (z - (c.beta[b] + 2 * c.bo[b]));
      const cplx y1 = (cplx(c.g[b] - c.go[b]) * z + (c.gamma[b] - c.co[b])) / (z - (c.beta[b] - c.bo[b]));
      y[b] = (y0 + 2.0 * y1) / 3.0;
      yo[b] = (y0 - y1) / 3.0;
    }
  if (any) {
    std::vector<cplx> Y((size_t)N * N, cplx(0.0, 0.0));
    for (int b = 0; b < B; ++b) {
      const int k = net.k[b], m = net.m[b];
      if (k >= 0) {
        Y[(size_t)k * N + k] += y[b];
        V[k] += y[b] * E[b];
      }
      if (m >= 0) {
        Y[(size_t)m * N + m] += y[b];
        V[m] -= y[b] * E[b];
      }
      if (k >= 0 && m >= 0) {
        Y[(size_t)k * N + m] -= y[b];
        Y[(size_t)m * N + k] -= y[b];
      }
    }
    for (const auto &mem : groups)
      for (int p : mem)
        for (int q : mem) {
          if (p == q) continue;
          const int tp[2] = {net.k[p], net.m[p]}, tq[2] = {net.k[q], net.m[q]};
          for (int a = 0; a < 2; ++a)
            for (int e = 0; e < 2; ++e)
              if (tp[a] >= 0 && tq[e] >= 0) Y[(size_t)tp[a] * N + tq[e]] += (a == e) ? yo[p] : -yo[p];
        }
    DenseLU<cplx> lu;
    lu.by_modulus = true;
    if (!lu.factor(Y, N)) return 2;
    lu.solve(V);
  }
  for (int a = 0; a < N; ++a) {
    if (v0) v0[a] = V[a].real();
    if (Vre) Vre[a] = V[a].real();
    if (Vim) Vim[a] = V[a].imag();
  }
  std::vector<cplx> U(B);
  for (int b = 0; b < B; ++b) {
    const cplx vk = net.k[b] >= 0 ? V[net.k[b]] : cplx(0.0, 0.0);
    const cplx vm = net.m[b] >= 0 ? V[net.m[b]] : cplx(0.0, 0.0);
    U[b] = vk - vm - E[b];
  }
  std::vector<cplx> I(B);
  for (int b = 0; b < B; ++b) I[b] = y[b] * U[b];
  for (const auto &mem : groups) {
    cplx su(0.0, 0.0);
    for (int q : mem) su += U[q];
    for (int p : mem) I[p] += yo[p] * (su - U[p]);
  }
  if (i0)
    for (int b = 0; b < B; ++b) i0[b] = I[b].real();
  return 0;
}

}  // namespace

extern "C" {

// Steady state of the initial topology: v0 [N], i0 [B] (the state at step
// 0 for oracle_run) and the node phasors V (all nullable).
int oracle_steady_state(const OracleNet *net, const double *theta, double dt, double *v0, double *i0,
                        double *V_re, double *V_im) {
  return steady_state(*net, theta, dt, v0, i0, V_re, V_im);
}

// Forward run in double. rec: [T][n_rec]. Trajectories (nullable): [T+1][N]
// node voltages, [T+1][B] branch currents and passive-branch voltages.
int oracle_run(const OracleNet *net, const double *theta, double dt, int64_t T,
               const double *v0, const double *i0, double *rec, double *v_traj,
               double *i_traj, double *u_traj) {
  return forward<double>(*net, theta, dt, T, v0, i0, rec, v_traj, i_traj, u_traj, nullptr,
                         nullptr, nullptr);
}

// Complex-step loss: theta = theta_re + i*theta_im, J = sum_n sum_r
// (v_{n,r} - target_{n,r})^2 evaluated in complex arithmetic.
int oracle_loss_complex(const OracleNet *net, const double *theta_re, const double *theta_im,
                        double dt, int64_t T, const double *target, double *J_re,
                        double *J_im) {
  std::vector<cplx> th(net->n_params);
  for (int p = 0; p < net->n_params; ++p) th[p] = cplx(theta_re[p], theta_im[p]);
  std::vector<cplx> rec((size_t)T * net->n_rec);
  int st = forward<cplx>(*net, th.data(), dt, T, nullptr, nullptr, rec.data(), nullptr,
                         nullptr, nullptr, nullptr, nullptr, nullptr);
  if (st) return st;
  cplx J(0);
  for (size_t q = 0; q < rec.size(); ++q) {
    cplx d = rec[q] - target[q];
    J += d * d;
  }
  *J_re = J.real();
  *J_im = J.imag();
  return 0;
}

// Vector-Jacobian product of the recorded waveform: given dJ/drec [T][n_rec],
// returns dJ/dtheta [n_params] and (nullable) the per-branch adjoints of the
// companion coefficients g, beta, gamma.
int oracle_adjoint(const OracleNet *net, const double *theta, double dt, int64_t T,
                   const double *dJ_drec, double *grad, double *gbar_out,
                   double *betabar_out, double *gammabar_out) {
  if (has_lines(*net) || has_groups(*net) || has_diodes(*net)) return 1;  // forward only
  const int N = net->n_nodes, B = net->n_branches;
  std::vector<double> i_traj((size_t)(T + 1) * B), u_traj((size_t)(T + 1) * B);
  std::vector<int> topo_of_step;
  std::vector<Companions<double>> topos;
  std::vector<DenseLU<double>> lus;
  int st = forward<double>(*net, theta, dt, T, nullptr, nullptr, nullptr, nullptr,
                           i_traj.data(), u_traj.data(), &topo_of_step, &topos, &lus);
  if (st) return st;

  std::vector<double> gbar(B, 0), bbar(B, 0), cbar(B, 0);
  std::vector<double> hbar_next(B, 0), beta_next(B, 0), gamma_next(B, 0);
  std::vector<double> ibar(B), q(B), hbar(B), x(N);
  for (int64_t n = T; n >= 1; --n) {
    const Companions<double> &c = topos[topo_of_step[n]];
    const DenseLU<double> &lu = lus[topo_of_step[n]];
    for (int b = 0; b < B; ++b) {
      const bool on = c.g[b] != 0.0;
      ibar[b] = beta_next[b] * hbar_next[b];
      q[b] = on ? gamma_next[b] * hbar_next[b] + c.g[b] * ibar[b] : 0.0;
    }
    std::fill(x.begin(), x.end(), 0.0);
    for (int r = 0; r < net->n_rec; ++r) x[rec_node(*net, r)] += dJ_drec[(size_t)(n - 1) * net->n_rec + r];
    for (int b = 0; b < B; ++b) {
      if (net->k[b] >= 0) x[net->k[b]] += q[b];
      if (net->m[b] >= 0) x[net->m[b]] -= q[b];
    }
    lu.solve_transposed(x);
    const double *un = &u_traj[(size_t)n * B];
    const double *up = &u_traj[(size_t)(n - 1) * B];
    const double *ip = &i_traj[(size_t)(n - 1) * B];
    for (int b = 0; b < B; ++b) {
      const bool on = c.g[b] != 0.0;
      double wk = net->k[b] >= 0 ? x[net->k[b]] : 0.0;
      double wm = net->m[b] >= 0 ? x[net->m[b]] : 0.0;
      hbar[b] = on ? ibar[b] - (wk - wm) : 0.0;
      gbar[b] += hbar[b] * un[b];
      bbar[b] += hbar[b] * ip[b];
      cbar[b] += hbar[b] * up[b];
      hbar_next[b] = hbar[b];
      beta_next[b] = c.beta[b];
      gamma_next[b] = c.gamma[b];
    }
  }

  // Chain rule to the line parameters.
  if (grad) {
    std::fill(grad, grad + net->n_params, 0.0);
    for (int b = 0; b < B; ++b) {
      const int l = net->line[b];
      if (l < 0) continue;
      double R, L, C;
      branch_values<double>(*net, theta, b, R, L, C);
      if (net->kind[b] == K_RL) {
        const double g0 = 1.0 / (R + 2.0 * L / dt);
        const double g2 = g0 * g0;
        grad[3 * l + 0] += (gbar[b] + cbar[b]) * (-g2) + bbar[b] * (-(4.0 * L / dt) * g2);
        grad[3 * l + 1] += (gbar[b] + cbar[b]) * (-(2.0 / dt) * g2) + bbar[b] * ((4.0 * R / dt) * g2);
      } else if (net->kind[b] == K_C) {
        grad[3 * l + 2] += (gbar[b] - cbar[b]) / dt;
      }
    }
  }
  if (gbar_out) std::copy(gbar.begin(), gbar.end(), gbar_out);
  if (betabar_out) std::copy(bbar.begin(), bbar.end(), betabar_out);
  if (gammabar_out) std::copy(cbar.begin(), cbar.end(), gammabar_out);
  return 0;
}

// Many independent scenarios, OpenMP over scenarios (the CPU baseline for
// batched workloads). thetas: per-scenario pointers (entries may be null);
// recs: per-scenario outputs [T][n_rec]. Returns the first nonzero status.
int oracle_run_batch(const OracleNet *nets, int n_scen, const double *const *thetas,
                     double dt, int64_t T, double *const *recs, int n_threads) {
  int status = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(max : status)
#endif
  for (int s = 0; s < n_scen; ++s) {
    int st = forward<double>(nets[s], thetas ? thetas[s] : nullptr, dt, T, nullptr, nullptr,
                             recs[s], nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    status = std::max(status, st);
  }
  return status;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Test hooks: the dense conductance matrix of a topology, and the LU solver.
int oracle_assemble(const OracleNet *net, const double *theta, double dt,
                    const uint8_t *in_service, double *G_out) {
  std::vector<uint8_t> ins(in_service, in_service + net->n_branches);
  Companions<double> c;
  companions(*net, theta, dt, ins, c);
  std::vector<double> G;
  assemble(*net, c, G);
  std::copy(G.begin(), G.end(), G_out);
  return 0;
}

int oracle_companions(const OracleNet *net, const double *theta, double dt,
                      const uint8_t *in_service, double *g, double *beta, double *gamma) {
  std::vector<uint8_t> ins(in_service, in_service + net->n_branches);
  Companions<double> c;
  companions(*net, theta, dt, ins, c);
  std::copy(c.g.begin(), c.g.end(), g);
  std::copy(c.beta.begin(), c.beta.end(), beta);
  std::copy(c.gamma.begin(), c.gamma.end(), gamma);
  return 0;
}

int oracle_lu_solve(int n, const double *G, const double *b, double *x, int transposed) {
  DenseLU<double> lu;
  std::vector<double> Gv(G, G + (size_t)n * n);
  if (!lu.factor(Gv, n)) return 2;
  std::vector<double> xv(b, b + n);
  if (transposed)
    lu.solve_transposed(xv);
  else
    lu.solve(xv);
  std::copy(xv.begin(), xv.end(), x);
  return 0;
}

}  // extern "C"
