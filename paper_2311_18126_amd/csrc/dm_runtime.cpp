// dm_runtime.cpp -- host runtime of libdmrod: rod/joint construction, topology and DOF
// numbering, stencil tables, banded/border layouts, upload and launch (C ABI of dmrod.h).
//
// Host work happens once per finalize: joint merging, the rest quantities of every edge
// and stencil, the initial reference frames, and the solver layout.  Every Newton
// iteration and time step runs in dm_step_kernel on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <limits>
#include <string>
#include <type_traits>
#include <fstream>
#include <vector>

#include "../../include/dmrod.h"
#include "dm_layout.h"
#include "dm_math.h"

extern "C" hipError_t dm_launch_step(const DmStepArgs* args, int block, size_t lds_bytes, hipStream_t stream);
extern "C" hipError_t dm_launch_adjoint(const DmAdjArgs* args, int block, size_t lds_bytes, hipStream_t stream);
extern "C" hipError_t dm_launch_gather_tips(const double* x, int nn, const int* tip, int n, double* out,
                                            hipStream_t stream);
extern "C" hipError_t dm_launch_fit_loss(const double* tips, const double* target, int n, double* dL, double* loss,
                                         hipStream_t stream);
extern "C" hipError_t dm_launch_axpy(double* y, const double* x, double a, int n, hipStream_t stream);
extern "C" hipError_t dm_launch_stencil_curvature(const DmStepArgs* args, double* out, hipStream_t stream);
extern "C" hipError_t dm_launch_curvature_adjoint(const DmCurvArgs* args, int block, size_t lds_bytes,
                                                  hipStream_t stream);
extern "C" hipError_t dm_launch_predict(const DmStepArgs* args, int block, size_t lds_bytes, double* out,
                                        hipStream_t stream);
extern "C" hipError_t dm_ws_launch_features(const DmDev* D, int rows, const int* cn_chain, const double* nconst,
                                            double* F, hipStream_t st);
extern "C" hipError_t dm_ws_launch_targets(const DmDev* D, int rows, const int* cn_chain, const double* Fprev,
                                           double dt, double* T, hipStream_t st);

namespace {

thread_local std::string g_err;

dm_status fail(dm_status s, const std::string& msg) { g_err = msg; return s; }

#define DM_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return fail(DM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct Rod {
  int n = 0;
  std::vector<double> x0;               // [n][3]
  double h = 0, E = 0, nu = 0, rho = 0;
  std::vector<double> kbar;             // [n-2][2], 1/m
  bool has_kbar = false;
  bool act = false;
  double A = 0, f = 0, phi = 0;
  std::vector<double> force;            // [n][3]
  std::vector<double> moment;           // [n-1]
  std::vector<char> nfix, efix;
};

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
};

}  // namespace

// One captured trajectory segment: len one-step launches, each followed by the tip gather or
// the state save; replayed while the step arguments, length and destinations are the same.
struct SegGraph {
  DmStepArgs args{};
  int len = 0, block = 0;
  size_t lds = 0;
  const double* tips = nullptr;
  const double* states = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct dm_sim {
  dm_config cfg{};
  bool finalized = false;
  std::vector<Rod> rods;
  std::vector<std::array<int, 4>> joints;
  hipStream_t stream = nullptr;
  // layout
  int n_nodes = 0, n_edges = 0, n_st = 0, n_sys = 0, n_chains = 0, n_arms = 0, n_dof = 0;
  int max_nb = 0, max_arms = 0, max_seg = 0, block = 0;
  bool block_auto = false;   // no workgroup size given or tuned: the step's default applies
  // edge-edge self-contact of single-rod systems (dm_set_self_contact)
  int sc_on = 0, sc_max_edges = 0;
  double sc_delta = 0.0, sc_kc = 0.0, sc_mu = 0.0, sc_nu = 1.0;
  std::vector<int> rod_sys;
  std::vector<std::vector<int>> rod_node, rod_edge;   // global ids per rod node / edge
  std::vector<int> rod_st0;                            // global stencil id of rod node 1
  std::vector<DmSystem> sys;
  std::vector<double> h_Vbar, h_kbend, h_ktwist;       // needed for natural-curvature updates
  std::vector<double> h_kbar, h_act, h_kappa_rest;
  std::vector<void*> allocs;
  DmDev dev{};
  double time = 0.0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  float last_kernel_ms = 0.0f;
  // trajectory and adjoint buffers, allocated on first use and grown as needed
  double* ck = nullptr;   size_t ck_n = 0;      // checkpoints of dm_rollout
  double* seg = nullptr;  size_t seg_n = 0;     // states of one recomputed segment + final state
  double* adj = nullptr;  size_t adj_n = 0;     // adjoint arrays
  double* tips_dev = nullptr; size_t tips_n = 0;
  double* dl_dev = nullptr;   size_t dl_n = 0;
  int* tip_nodes = nullptr;
  // warm start: per feature row (rod node) its chain and constants (log10 E, h, mean ebar)
  int ws_rows = 0;
  int* cn_chain = nullptr;
  double* nconst = nullptr;
  double* ws_F = nullptr; size_t ws_F_n = 0;
  dm_mlp* ws_net = nullptr;
  int ws_mode = 0;
  int scheme = DM_BACKWARD_EULER;   // time integrator of dm_step
  int max_halvings = 0;             // adaptive step halving depth of dm_step (0: off)
  // captured step sequences of trajectory segments (dm_rollout, the adjoint's recomputation)
  hipStream_t cap_stream = nullptr;
  std::vector<SegGraph> seg_graphs;
  double* tips_stage = nullptr; size_t tips_stage_n = 0;
  double* tune_ck = nullptr; size_t tune_ck_n = 0;
  // limb curvatures and their gradient (Real2Sim fit): per-stencil curvature, weights, adjoint
  // solution, per-stencil derivatives, and the per-system skip mask of the fit's launches
  double* curv_st = nullptr; size_t curv_st_n = 0;
  double* curv_w = nullptr; size_t curv_w_n = 0;
  double* curv_mu = nullptr; size_t curv_mu_n = 0;
  double* curv_p = nullptr; size_t curv_p_n = 0;
  double* skip_buf = nullptr; size_t skip_n = 0;   // int flags, sized in doubles
  int roll_steps = 0, roll_ckpt = 0;
  double roll_dt = 0.0;
  bool roll_valid = false;
};

namespace {

// Device memory of a simulation: the caller's allocator hook when one is set (dm_config.alloc),
// else hipMalloc; nullptr on failure.
void* dev_malloc(const dm_sim* s, size_t bytes) {
  bytes = std::max<size_t>(bytes, 1);
  if (s->cfg.alloc) return s->cfg.alloc(bytes, s->cfg.alloc_ctx);
  void* p = nullptr;
  return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}

// Release a buffer of dev_malloc once the simulation's stream has drained (a hook's allocator
// may hand the pages out again at once).
void dev_free(const dm_sim* s, void* p) {
  if (!p) return;
  (void)hipStreamSynchronize(s->stream);
  if (s->cfg.alloc) s->cfg.free_(p, s->cfg.alloc_ctx);
  else (void)hipFree(p);
}

template <class T>
dm_status upload(dm_sim* s, const std::vector<T>& h, T** out) {
  size_t bytes = std::max<size_t>(h.size(), 1) * sizeof(T);
  void* p = dev_malloc(s, bytes);
  if (!p) return fail(DM_ERR_OOM, "device allocation failed (" + std::to_string(bytes) + " bytes)");
  s->allocs.push_back(p);
  if (!h.empty()) DM_HIP(hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  *out = static_cast<T*>(p);
  return DM_OK;
}

template <class T>
dm_status alloc(dm_sim* s, size_t n, T** out) {
  size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
  void* p = dev_malloc(s, bytes);
  if (!p) return fail(DM_ERR_OOM, "device allocation failed (" + std::to_string(bytes) + " bytes)");
  s->allocs.push_back(p);
  DM_HIP(hipMemset(p, 0, bytes));
  *out = static_cast<T*>(p);
  return DM_OK;
}

bool finite_all(const double* a, size_t n) {
  for (size_t i = 0; i < n; ++i) if (!std::isfinite(a[i])) return false;
  return true;
}

struct UF {
  std::vector<int> p;
  explicit UF(int n) : p(n) { std::iota(p.begin(), p.end(), 0); }
  int find(int i) { while (p[i] != i) { p[i] = p[p[i]]; i = p[i]; } return i; }
  void join(int a, int b) { a = find(a); b = find(b); if (a != b) p[b] = a; }
};

// Initial reference directors of one rod: d1 of the first edge is z projected off its
// tangent (x when the tangent is within 1e-6 of z), then space-parallel transport along the
// rod, so that a rod's initial shape has zero reference twist.
void initial_frames(const std::vector<v3>& t, std::vector<v3>& d1) {
  d1.resize(t.size());
  v3 z = mk3(0, 0, 1);
  if (std::fabs(dot(t[0], z)) > 1.0 - 1e-6) z = mk3(1, 0, 0);
  v3 d = z - dot(z, t[0]) * t[0];
  d1[0] = (1.0 / std::sqrt(dot(d, d))) * d;
  for (size_t j = 1; j < t.size(); ++j) d1[j] = transport_perp(t[j - 1], t[j], d1[j - 1]);
}

dm_status do_finalize(dm_sim* s) {
  const int nr = (int)s->rods.size();
  if (nr == 0) return fail(DM_ERR_STATE, "dm_finalize: no rods");
  // ---- rod-node keys, joint merging, connected rod sets
  std::vector<int> key0(nr + 1, 0);
  for (int r = 0; r < nr; ++r) key0[r + 1] = key0[r] + s->rods[r].n;
  UF nodes(key0[nr]), rodset(nr);
  for (auto& j : s->joints) {
    nodes.join(key0[j[0]] + j[1], key0[j[2]] + j[3]);
    rodset.join(j[0], j[2]);
  }
  std::map<int, std::vector<int>> comp;
  for (int r = 0; r < nr; ++r) comp[rodset.find(r)].push_back(r);
  std::vector<std::vector<int>> groups;
  for (auto& kv : comp) groups.push_back(kv.second);
  std::sort(groups.begin(), groups.end(), [](const std::vector<int>& a, const std::vector<int>& b) { return a[0] < b[0]; });

  s->rod_sys.assign(nr, -1);
  s->rod_node.assign(nr, {});
  s->rod_edge.assign(nr, {});
  s->rod_st0.assign(nr, -1);
  // host arrays
  std::vector<double> X, mass, radius, force, Ith, ebar, EA, moment;
  std::vector<int> en0, en1;
  std::vector<int> sn0, sn1, sn2, sef, see, ssign, st_rod;
  std::vector<double> Vbar, kbend, ktwist, kbar0, kbar1, tbar, act0, act1, act2, bref;
  std::vector<char> nfix, efix;
  std::vector<DmChain> chains;
  std::vector<DmArm> arms;
  std::vector<int> chain_node, chain_edge, bmap, bsrc, bjst, node_owner;
  std::vector<unsigned char> bfix, cfix;
  std::vector<DmSystem> systems;
  std::vector<std::vector<int>> sys_bst;   // per system: stencils assembled into the dense border
  std::vector<v3> tref, d1ref;
  std::vector<int> node_home_c[3], edge_home;
  int dof_total = 0, fac_total = 0;

  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const std::vector<int>& rods = groups[gi];
    DmSystem S{};
    S.node0 = (int)mass.size();
    S.edge0 = (int)ebar.size();
    S.st0 = (int)Vbar.size();
    S.chain0 = (int)chains.size();
    S.arm0 = (int)arms.size();
    // global node ids: first occurrence in rod order
    std::map<int, int> gid;
    for (int r : rods) {
      s->rod_sys[r] = (int)gi;
      for (int i = 0; i < s->rods[r].n; ++i) {
        int k = nodes.find(key0[r] + i);
        auto it = gid.find(k);
        if (it == gid.end()) {
          int g = (int)mass.size();
          gid[k] = g;
          const double* p = &s->rods[r].x0[3 * i];
          X.push_back(p[0]); X.push_back(p[1]); X.push_back(p[2]);
          mass.push_back(0.0); radius.push_back(0.0);
          force.push_back(0.0); force.push_back(0.0); force.push_back(0.0);
          nfix.push_back(0);
          node_owner.push_back(-1);
          s->rod_node[r].push_back(g);
        } else {
          s->rod_node[r].push_back(it->second);
        }
      }
    }
    // topology check: a single rod, or rods meeting at one shared node (the hub), which is an
    // end node or an interior node of each of them.  A rod joined at an interior node k is
    // solved as two chains, nodes 0..k and k..N-1, that meet at the hub.
    std::map<int, int> mult;
    for (int r : rods) for (int g : s->rod_node[r]) mult[g]++;
    std::vector<int> shared;
    for (auto& kv : mult) if (kv.second > 1) shared.push_back(kv.first);
    int hub = -1;
    struct ChainSpec { int rod, lo, hi; bool hub_at_start; };
    std::vector<ChainSpec> specs;
    if (rods.size() == 1) {
      if (!shared.empty()) return fail(DM_ERR_UNSUPPORTED, "rod " + std::to_string(rods[0]) + " is joined to itself");
      specs.push_back({rods[0], 0, s->rods[rods[0]].n - 1, false});
    } else {
      if (shared.size() != 1) return fail(DM_ERR_UNSUPPORTED, "joined rods must meet at exactly one shared node");
      hub = shared[0];
      for (int r : rods) {
        const auto& rn = s->rod_node[r];
        const int N = (int)rn.size();
        int at = -1, count = 0;
        for (int i = 0; i < N; ++i)
          if (rn[i] == hub) { at = i; ++count; }
        if (count != 1) return fail(DM_ERR_UNSUPPORTED, "rod " + std::to_string(r) + " meets the joint node more than once");
        if (at == 0) specs.push_back({r, 0, N - 1, true});
        else if (at == N - 1) specs.push_back({r, 0, N - 1, false});
        else {
          specs.push_back({r, 0, at, false});
          specs.push_back({r, at, N - 1, true});
        }
      }
      if ((int)specs.size() > DM_MAX_CHAINS)
        return fail(DM_ERR_UNSUPPORTED, "more than 8 rod branches at one joint");
    }
    // edges, masses, rest lengths
    for (int r : rods) {
      const Rod& R = s->rods[r];
      const double Ar = M_PI * R.h * R.h;
      for (int j = 0; j + 1 < R.n; ++j) {
        int a = s->rod_node[r][j], b = s->rod_node[r][j + 1];
        v3 pa = mk3(X[3 * a], X[3 * a + 1], X[3 * a + 2]), pb = mk3(X[3 * b], X[3 * b + 1], X[3 * b + 2]);
        v3 d = pb - pa;
        double L0 = std::sqrt(dot(d, d));
        if (!(L0 > 0.0)) return fail(DM_ERR_INVALID_ARG, "rod " + std::to_string(r) + " has a zero-length edge");
        s->rod_edge[r].push_back((int)ebar.size());
        en0.push_back(a); en1.push_back(b);
        ebar.push_back(L0);
        EA.push_back(R.E * Ar);
        Ith.push_back(R.rho * (M_PI * std::pow(R.h, 4) / 2.0) * L0);
        moment.push_back(R.moment.empty() ? 0.0 : R.moment[j]);
        efix.push_back(R.efix.empty() ? 0 : R.efix[j]);
        mass[a] += 0.5 * R.rho * Ar * L0;
        mass[b] += 0.5 * R.rho * Ar * L0;
        radius[a] = std::max(radius[a], R.h);
        radius[b] = std::max(radius[b], R.h);
        tref.push_back((1.0 / L0) * d);
      }
      for (int i = 0; i < R.n; ++i) {
        int g = s->rod_node[r][i];
        if (!R.force.empty()) for (int c = 0; c < 3; ++c) force[3 * g + c] += R.force[3 * i + c];
        if (!R.nfix.empty() && R.nfix[i]) nfix[g] = 1;
      }
      // initial frames of this rod
      std::vector<v3> t(s->rod_edge[r].size()), d1;
      for (size_t j = 0; j < t.size(); ++j) t[j] = tref[s->rod_edge[r][j]];
      initial_frames(t, d1);
      d1ref.resize(tref.size());
      for (size_t j = 0; j < t.size(); ++j) d1ref[s->rod_edge[r][j]] = d1[j];
    }
    // stencils: rod-interior (chain) stencils, then pairs of edges at the joint
    auto push_st = [&](int p, int c, int n, int f, int e, int sg, int rf, int re, int rodid) {
      sn0.push_back(p); sn1.push_back(c); sn2.push_back(n); sef.push_back(f); see.push_back(e); ssign.push_back(sg);
      st_rod.push_back(rodid);
      double V = 0.5 * (ebar[f] + ebar[e]);
      const Rod& A = s->rods[rf];
      const Rod& B = s->rods[re];
      double EIa = A.E * M_PI * std::pow(A.h, 4) / 4.0, EIb = B.E * M_PI * std::pow(B.h, 4) / 4.0;
      double GJa = A.E / (2.0 * (1.0 + A.nu)) * M_PI * std::pow(A.h, 4) / 2.0;
      double GJb = B.E / (2.0 * (1.0 + B.nu)) * M_PI * std::pow(B.h, 4) / 2.0;
      Vbar.push_back(V);
      kbend.push_back(0.5 * (EIa + EIb) / V);
      ktwist.push_back(0.5 * (GJa + GJb) / V);
      // rest strains of the initial shape (theta = 0), frames in the stencil's orientation
      double sf = (sg & 1) ? -1.0 : 1.0, se = (sg & 2) ? -1.0 : 1.0;
      double k1, k2, b;
      stencil_strains(sf * tref[f], d1ref[f], 0.0, se * tref[e], d1ref[e], 0.0, 0.0, true, &k1, &k2, &b);
      bref.push_back(b);
      s->h_kappa_rest.push_back(k1);
      s->h_kappa_rest.push_back(k2);
      tbar.push_back(rodid >= 0 ? 0.0 : b);
      kbar0.push_back(k1); kbar1.push_back(k2);
      act0.push_back(NAN); act1.push_back(0.0); act2.push_back(0.0);
    };
    for (int r : rods) {
      const Rod& R = s->rods[r];
      s->rod_st0[r] = (int)Vbar.size();
      for (int i = 1; i + 1 < R.n; ++i) {
        push_st(s->rod_node[r][i - 1], s->rod_node[r][i], s->rod_node[r][i + 1], s->rod_edge[r][i - 1],
                s->rod_edge[r][i], 0, r, r, r);
        int st = (int)Vbar.size() - 1;
        if (R.has_kbar) {
          kbar0[st] = R.kbar[2 * (i - 1)] * Vbar[st];
          kbar1[st] = R.kbar[2 * (i - 1) + 1] * Vbar[st];
        }
        if (R.act) { act0[st] = R.A; act1[st] = R.f; act2[st] = R.phi; }
      }
    }
    S.jst0 = (int)Vbar.size();
    std::vector<int> bst;       // stencils of this system assembled into the dense border
    std::vector<int> edge_rod(ebar.size(), -1);
    for (int r : rods) for (int e : s->rod_edge[r]) edge_rod[e] = r;
    if (hub >= 0) {
      // a rod joined at an interior node k keeps its own stencil there (its natural curvature,
      // actuation and stiffness); that stencil couples the two chains and goes to the border
      for (const ChainSpec& cs : specs)
        if (cs.hub_at_start && cs.lo > 0) bst.push_back(s->rod_st0[cs.rod] + cs.lo - 1);
      std::vector<std::pair<int, int>> inc;   // (edge, +1 leaves hub / -1 enters hub), sorted by edge
      for (const ChainSpec& cs : specs) {
        if (cs.hub_at_start) inc.push_back({s->rod_edge[cs.rod][cs.lo], +1});
        else inc.push_back({s->rod_edge[cs.rod][cs.hi - 1], -1});
      }
      std::sort(inc.begin(), inc.end());
      for (size_t p = 0; p < inc.size(); ++p)
        for (size_t q = p + 1; q < inc.size(); ++q) {
          int ja = inc[p].first, da = inc[p].second, jb = inc[q].first, db = inc[q].second;
          int f, e, sfr = 0, ser = 0;
          if (da == -1 && db == +1) { f = ja; e = jb; }
          else if (db == -1 && da == +1) { f = jb; e = ja; }
          else if (da == +1 && db == +1) { f = ja; e = jb; sfr = 1; }
          else { f = ja; e = jb; ser = 1; }
          // the two edges of one rod at an interior joint: that rod's own stencil (kept above)
          if (!sfr && !ser && edge_rod[f] == edge_rod[e] && e == f + 1) continue;
          int np = sfr ? en1[f] : en0[f];
          int nn = ser ? en0[e] : en1[e];
          push_st(np, hub, nn, f, e, sfr | (ser << 1), edge_rod[f], edge_rod[e], -1);
          bst.push_back((int)Vbar.size() - 1);
        }
    }
    S.n_jst = (int)bst.size();
    S.n_nodes = (int)mass.size() - S.node0;
    S.n_edges = (int)ebar.size() - S.edge0;
    S.n_st = (int)Vbar.size() - S.st0;
    // ---- chains, border, arms
    S.n_chains = (int)specs.size();
    S.nb = (hub >= 0) ? 3 + 4 * (int)specs.size() : 0;
    std::vector<std::vector<std::pair<int, int>>> src;   // border index -> (chain, dof)
    int chain_nodes = 0;
    for (size_t a = 0; a < specs.size(); ++a) {
      const ChainSpec& cs = specs[a];
      const int r = cs.rod;
      DmChain C{};
      C.n_nodes = cs.hi - cs.lo + 1;
      C.node_tab = (int)chain_node.size();
      C.edge_tab = (int)chain_edge.size();
      C.st_off = s->rod_st0[r] + cs.lo;     // the stencil of chain node m is the rod's node lo + m
      C.dof_off = dof_total;
      C.global_id = (int)chains.size();
      C.rod = r;
      for (int k = cs.lo; k <= cs.hi; ++k) chain_node.push_back(s->rod_node[r][k]);
      for (int k = cs.lo; k < cs.hi; ++k) chain_edge.push_back(s->rod_edge[r][k]);
      const int n = 4 * C.n_nodes - 1;
      C.bmap_off = (int)bmap.size();
      std::vector<DmArm> ca;
      if (hub < 0) {
        if (n <= 10) {
          C.b_lo = 0; C.b_hi = n;
        } else {
          int m = (n - 10) / 2;
          C.b_lo = m; C.b_hi = m + 10;
          if (m > 0) ca.push_back(DmArm{C.global_id, +1, 0, m, 10, 0});
          if (n - m - 10 > 0) ca.push_back(DmArm{C.global_id, -1, n - 1, n - m - 10, 10, 0});
        }
        S.nb = C.b_hi - C.b_lo;
        src.assign(S.nb, {});
        for (int i = C.b_lo; i < C.b_hi; ++i) { bmap.push_back(i - C.b_lo); src[i - C.b_lo].push_back({C.global_id, i}); }
      } else {
        const bool at_start = cs.hub_at_start;
        if (src.empty()) src.assign(S.nb, {});
        const int base = 3 + 4 * (int)a;
        int map7[7];
        if (at_start) {
          C.b_lo = 0; C.b_hi = std::min(7, n);
          map7[0] = 0; map7[1] = 1; map7[2] = 2; map7[3] = base; map7[4] = base + 1; map7[5] = base + 2; map7[6] = base + 3;
          if (n - 7 > 0) ca.push_back(DmArm{C.global_id, -1, n - 1, n - 7, 7, 0});
          else if (n < 7) return fail(DM_ERR_UNSUPPORTED, "joined rod too short");
        } else {
          C.b_lo = n - 7; C.b_hi = n;
          // chain DOFs n-7..n-1: x_{N-2} (3), theta_{N-2}, x_{N-1} = hub (3)
          map7[0] = base + 1; map7[1] = base + 2; map7[2] = base + 3; map7[3] = base; map7[4] = 0; map7[5] = 1; map7[6] = 2;
          if (n - 7 > 0) ca.push_back(DmArm{C.global_id, +1, 0, n - 7, 7, 0});
        }
        for (int i = 0; i < C.b_hi - C.b_lo; ++i) {
          bmap.push_back(map7[i]);
          src[map7[i]].push_back({C.global_id, C.b_lo + i});
        }
      }
      for (auto& A : ca) {
        A.fac_off = fac_total;
        fac_total += A.count;
        arms.push_back(A);
      }
      // clamps per chain DOF
      for (int k = cs.lo; k <= cs.hi; ++k) {
        int g = s->rod_node[r][k];
        for (int c = 0; c < 3; ++c) cfix.push_back(nfix[g]);
        if (k < cs.hi) cfix.push_back(efix[s->rod_edge[r][k]]);
      }
      for (int k = cs.lo; k <= cs.hi; ++k) {
        const int g = s->rod_node[r][k];
        if (node_owner[g] < 0) node_owner[g] = C.global_id;
      }
      chains.push_back(C);
      dof_total += n;
      chain_nodes += C.n_nodes;
    }
    S.n_arms = (int)arms.size() - S.arm0;
    S.chain_nodes = chain_nodes;
    S.n_dof = dof_total - chains[S.chain0].dof_off;
    S.bsrc_off = (int)bsrc.size() / 2;   // in units of (chain, dof) slots
    for (int b = 0; b < S.nb; ++b) {
      if ((int)src[b].size() > DM_MAX_BSRC) return fail(DM_ERR_UNSUPPORTED, "border source table overflow");
      for (int q = 0; q < DM_MAX_BSRC; ++q) {
        if (q < (int)src[b].size()) { bsrc.push_back(src[b][q].first); bsrc.push_back(src[b][q].second); }
        else { bsrc.push_back(-1); bsrc.push_back(-1); }
      }
    }
    S.bfix_off = (int)bfix.size();
    for (int b = 0; b < S.nb; ++b) {
      auto pr = src[b][0];
      const DmChain& C = chains[pr.first];
      bfix.push_back(cfix[C.dof_off + pr.second]);
    }
    // joint stencils: border index of each local DOF
    S.bjst_off = (int)bjst.size();
    for (int js = 0; js < S.n_jst; ++js) {
      int st = bst[js];
      auto nodeb = [&](int g, int c) -> int {
        if (g == hub) return c;
        for (int a = 0; a < S.n_chains; ++a) {
          const DmChain& C = chains[S.chain0 + a];
          for (int i = C.b_lo; i < C.b_hi; ++i) {
            int k = i >> 2, cc = i & 3;
            if (cc == c && chain_node[C.node_tab + k] == g) return bmap[C.bmap_off + i - C.b_lo];
          }
        }
        return -1;
      };
      auto edgeb = [&](int e) -> int {
        for (int a = 0; a < S.n_chains; ++a) {
          const DmChain& C = chains[S.chain0 + a];
          for (int i = C.b_lo; i < C.b_hi; ++i)
            if ((i & 3) == 3 && chain_edge[C.edge_tab + (i >> 2)] == e) return bmap[C.bmap_off + i - C.b_lo];
        }
        return -1;
      };
      int loc[11];
      for (int c = 0; c < 3; ++c) { loc[c] = nodeb(sn0[st], c); loc[4 + c] = nodeb(sn1[st], c); loc[8 + c] = nodeb(sn2[st], c); }
      loc[3] = edgeb(sef[st]);
      loc[7] = edgeb(see[st]);
      for (int i = 0; i < 11; ++i) {
        if (loc[i] < 0) return fail(DM_ERR_UNSUPPORTED, "joint stencil DOF outside the joint border");
        bjst.push_back(loc[i]);
      }
    }
    s->max_nb = std::max(s->max_nb, S.nb);
    s->max_arms = std::max(s->max_arms, S.n_arms);
    systems.push_back(S);
    sys_bst.push_back(bst);
  }
  // ---- terms of every dense border entry (entry b (nb + 1) + col, col = nb: right-hand side),
  // in the order the assembly sums them: each source chain row's residual and border-column
  // band entries, then the joint stencils' gradient and Hessian terms
  std::vector<int> bent;
  std::vector<DmBItem> bitem;
  const int NST = (int)Vbar.size();      // every stencil is placed by now
  for (size_t si = 0; si < systems.size(); ++si) {
    DmSystem& S = systems[si];
    const int W = S.nb + 1;
    std::vector<std::vector<DmBItem>> ent((size_t)S.nb * W);
    for (int b = 0; b < S.nb; ++b) {
      if (bfix[S.bfix_off + b]) continue;
      for (int q = 0; q < DM_MAX_BSRC; ++q) {
        const int ci = bsrc[2 * (S.bsrc_off + b * DM_MAX_BSRC + q)];
        if (ci < 0) break;
        const int r = bsrc[2 * (S.bsrc_off + b * DM_MAX_BSRC + q) + 1];
        const DmChain& C = chains[ci];
        ent[(size_t)b * W + S.nb].push_back(DmBItem{2, C.dof_off + r, 1.0});
        for (int o = 0; o < DM_NDIAG; ++o) {
          const int col = r - DM_HALF_BAND + o;
          if (col < C.b_lo || col >= C.b_hi) continue;
          const int bc = bmap[C.bmap_off + col - C.b_lo];
          if (bfix[S.bfix_off + bc]) continue;
          ent[(size_t)b * W + bc].push_back(DmBItem{0, (C.bmap_off + r - C.b_lo) * DM_NDIAG + o, 1.0});
        }
      }
    }
    for (int js = 0; js < S.n_jst; ++js) {
      const int* bj = &bjst[S.bjst_off + js * 11];
      const int st = sys_bst[si][js];
      const double sf = (ssign[st] & 1) ? -1.0 : 1.0, se = (ssign[st] & 2) ? -1.0 : 1.0;
      for (int a = 0; a < 11; ++a) {
        const int b = bj[a];
        if (bfix[S.bfix_off + b]) continue;
        int va[2], vc[2];
        double ca[2], cc[2];
        const int na = loc_terms(a, sf, se, va, ca);
        for (int t = 0; t < na; ++t) ent[(size_t)b * W + S.nb].push_back(DmBItem{3, va[t] * NST + st, ca[t]});
        for (int c = 0; c < 11; ++c) {
          const int bc = bj[c];
          if (bc < 0 || bfix[S.bfix_off + bc]) continue;
          const int nc = loc_terms(c, sf, se, vc, cc);
          for (int t = 0; t < na; ++t)
            for (int u = 0; u < nc; ++u)
              ent[(size_t)b * W + bc].push_back(DmBItem{1, (va[t] * 8 + vc[u]) * NST + st, ca[t] * cc[u]});
        }
      }
    }
    // each entry's terms in segments of DM_SEG (the last one padded with zero-pad terms);
    // bent holds the global index of every entry's first segment
    S.bent_off = (int)bent.size();
    S.seg0 = (int)(bitem.size() / DM_SEG);
    S.seg_long = 0;
    for (const auto& e : ent) {
      if (e.size() > DM_SEG) S.seg_long = 1;
      bent.push_back((int)(bitem.size() / DM_SEG));
      for (size_t i = 0; i < e.size(); i += DM_SEG)
        for (size_t j = i; j < i + DM_SEG; ++j) bitem.push_back(j < e.size() ? e[j] : DmBItem{4, 0, 0.0});
    }
    bent.push_back((int)(bitem.size() / DM_SEG));
    S.n_seg = (int)(bitem.size() / DM_SEG) - S.seg0;
    s->max_seg = std::max(s->max_seg, S.n_seg);
  }
  // ---- per arm, the border entry each of its Schur-complement slots adds to: slot i * 10 + j
  // (trailing DOFs i, j) or 100 + i (right-hand side of trailing DOF i)
  std::vector<int> bsch(arms.size() * 110, -1);
  for (const DmSystem& S : systems) {
    if (S.nb > 255) return fail(DM_ERR_UNSUPPORTED, "border larger than 255 DOFs");
    for (int a = S.arm0; a < S.arm0 + S.n_arms; ++a) {
      const DmArm& A = arms[a];
      const DmChain& C = chains[A.chain];
      const int ntr = A.n_trail;
      auto bidx = [&](int i) { return bmap[C.bmap_off + (A.first + A.dir * (A.count + i)) - C.b_lo]; };
      for (int i = 0; i < ntr; ++i) {
        const int bi = bidx(i);
        if (bfix[S.bfix_off + bi]) continue;
        for (int j = 0; j < ntr; ++j) {
          const int bj = bidx(j);
          if (!bfix[S.bfix_off + bj]) bsch[(size_t)a * 110 + i * (ntr + 1) + j] = (bi << 16) | (bj << 8) | (i * 10 + j);
        }
        bsch[(size_t)a * 110 + i * (ntr + 1) + ntr] = (bi << 16) | (S.nb << 8) | (100 + i);
      }
    }
  }
  // ---- homes of every DOF (delta index or border)
  const int NN = (int)mass.size(), NE = (int)ebar.size();
  for (int c = 0; c < 3; ++c) node_home_c[c].assign(NN, 0);
  edge_home.assign(NE, 0);
  for (const DmSystem& S : systems)
    for (int a = 0; a < S.n_chains; ++a) {
      const DmChain& C = chains[S.chain0 + a];
      for (int k = 0; k < C.n_nodes; ++k) {
        for (int c = 0; c < 4; ++c) {
          int r = 4 * k + c;
          if (c == 3 && k == C.n_nodes - 1) break;
          int home = (r >= C.b_lo && r < C.b_hi) ? -1 - bmap[C.bmap_off + r - C.b_lo] : C.dof_off + r;
          if (c < 3) node_home_c[c][chain_node[C.node_tab + k]] = home;
          else edge_home[chain_edge[C.edge_tab + k]] = home;
        }
      }
    }
  // launch order: largest systems first
  std::vector<int> order(systems.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return systems[a].n_dof > systems[b].n_dof; });

  s->n_nodes = NN; s->n_edges = NE; s->n_st = (int)Vbar.size();
  s->n_sys = (int)systems.size(); s->n_chains = (int)chains.size(); s->n_arms = (int)arms.size(); s->n_dof = dof_total;
  s->sys = systems;
  s->h_Vbar = Vbar; s->h_kbend = kbend; s->h_ktwist = ktwist;
  s->h_kbar.resize(2 * s->n_st); s->h_act.resize(3 * s->n_st);
  for (int i = 0; i < s->n_st; ++i) {
    s->h_kbar[i] = kbar0[i]; s->h_kbar[s->n_st + i] = kbar1[i];
    s->h_act[i] = act0[i]; s->h_act[s->n_st + i] = act1[i]; s->h_act[2 * s->n_st + i] = act2[i];
  }
  // ---- SoA packing and upload
  auto soa3 = [](const std::vector<double>& aos) {
    size_t n = aos.size() / 3;
    std::vector<double> o(aos.size());
    for (size_t i = 0; i < n; ++i) for (int c = 0; c < 3; ++c) o[c * n + i] = aos[3 * i + c];
    return o;
  };
  auto soav = [](const std::vector<v3>& a) {
    size_t n = a.size();
    std::vector<double> o(3 * n);
    for (size_t i = 0; i < n; ++i) { o[i] = a[i].x; o[n + i] = a[i].y; o[2 * n + i] = a[i].z; }
    return o;
  };
  std::vector<int> en(2 * NE), sn(3 * s->n_st), se(2 * s->n_st), nh(3 * NN);
  for (int e = 0; e < NE; ++e) { en[e] = en0[e]; en[NE + e] = en1[e]; }
  for (int i = 0; i < s->n_st; ++i) {
    sn[i] = sn0[i]; sn[s->n_st + i] = sn1[i]; sn[2 * s->n_st + i] = sn2[i];
    se[i] = sef[i]; se[s->n_st + i] = see[i];
  }
  for (int c = 0; c < 3; ++c) for (int n = 0; n < NN; ++n) nh[c * NN + n] = node_home_c[c][n];
  // band-assembly masks per chain-node row: clamped and border bits of chain DOFs
  // 4k - 12 .. 4k + 19, and whether the chain owns the node
  std::vector<unsigned> nmask(4 * chain_node.size(), 0u);
  for (const DmChain& C : chains) {
    const int n = 4 * C.n_nodes - 1;
    for (int k = 0; k < C.n_nodes; ++k) {
      unsigned* m = &nmask[4 * (size_t)(C.node_tab + k)];
      for (int i = 0; i < 32; ++i) {
        const int r = 4 * k - 12 + i;
        if (r < 0 || r >= n) continue;
        m[0] |= (unsigned)(cfix[C.dof_off + r] != 0) << i;
        m[1] |= (unsigned)(r >= C.b_lo && r < C.b_hi) << i;
      }
      m[2] = node_owner[chain_node[C.node_tab + k]] == C.global_id ? 1u : 0u;
    }
  }
  DmDev& D = s->dev;
  dm_status st;
  auto up = [&](const auto& vec, auto& field) -> dm_status {
    using T = typename std::remove_reference_t<decltype(vec)>::value_type;
    T* p = nullptr;
    dm_status r = upload(s, vec, &p);
    field = p;
    return r;
  };
#define UP(vec, field) if ((st = up(vec, D.field)) != DM_OK) return st;
  UP(systems, sys) UP(chains, chain) UP(arms, arm) UP(order, order) UP(chain_node, chain_node) UP(chain_edge, chain_edge)
  UP(bmap, bmap) UP(bsrc, bsrc) UP(bjst, bjst) UP(bfix, bfix) UP(cfix, cfix) UP(nmask, nmask)
  UP(bent, bent) UP(bitem, bitem) UP(bsch, bsch)
  UP(mass, mass) UP(radius, radius)
  std::vector<double> forceS = soa3(force);
  UP(forceS, force) UP(node_owner, node_owner) UP(nh, node_home)
  std::vector<double> arc0(ebar.size(), 0.0);
  for (int r = 0; r < nr; ++r) {
    double acc = 0.0;
    for (int e : s->rod_edge[r]) { arc0[e] = acc; acc += ebar[e]; }
  }
  UP(en, en) UP(ebar, ebar) UP(arc0, arc0) UP(EA, EA) UP(Ith, Ith) UP(moment, moment) UP(edge_home, edge_home)
  UP(sn, sn) UP(se, se) UP(ssign, ssign) UP(Vbar, Vbar) UP(kbend, kbend) UP(ktwist, ktwist)
  UP(s->h_kbar, kbar) UP(tbar, tbar) UP(s->h_act, act)
  std::vector<double> XS = soa3(X), trefS = soav(tref), d1S = soav(d1ref);
  UP(XS, x) UP(XS, x0) UP(trefS, tref) UP(d1S, d1ref) UP(bref, bref)
#undef UP
  if ((st = alloc(s, 3 * (size_t)NN, &D.v)) != DM_OK) return st;
  if ((st = alloc(s, 3 * (size_t)NN, &D.vprev)) != DM_OK) return st;
  if ((st = alloc(s, 3 * (size_t)NN, &D.vprev2)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)NE, &D.th)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)NE, &D.th0)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)NE, &D.om)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)s->n_sys, &D.time)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)DM_ST_G * s->n_st, &D.st_g)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)DM_ST_H * s->n_st, &D.st_H)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)DM_ED * NE, &D.ed)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)DM_ND * NN, &D.nd)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)DM_NDIAG * dof_total, &D.band)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)DM_NDIAG * bmap.size(), &D.bpr)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)dof_total, &D.R)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)DM_FAC_STRIDE * std::max(fac_total, 1), &D.fac)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)dof_total, &D.delta)) != DM_OK) return st;
  if ((st = alloc(s, bmap.size(), &D.babs)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)s->n_sys, &D.s_floor_res)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)s->n_sys, &D.s_floor_est)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)16, &D.zpad)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)s->n_sys, &D.s_steps)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)s->n_sys, &D.s_iters)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)s->n_sys, &D.s_status)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)s->n_sys, &D.s_res)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)s->n_sys, &D.s_floor)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)s->n_sys, &D.s_fallback)) != DM_OK) return st;
  if ((st = alloc(s, (size_t)s->n_sys, &D.s_halved)) != DM_OK) return st;
  {
    // warm-start feature rows: one per chain node
    std::vector<int> cnc(chain_node.size());
    std::vector<double> nc(3 * chain_node.size());
    for (const DmChain& C : chains) {
      const Rod& R = s->rods[C.rod];
      for (int k = 0; k < C.n_nodes; ++k) {
        const int i = C.node_tab + k;
        cnc[i] = C.global_id;
        const double el = k == 0 ? ebar[chain_edge[C.edge_tab]]
                        : (k == C.n_nodes - 1 ? ebar[chain_edge[C.edge_tab + k - 1]]
                                              : 0.5 * (ebar[chain_edge[C.edge_tab + k - 1]] + ebar[chain_edge[C.edge_tab + k]]));
        nc[3 * i] = std::log10(R.E);
        nc[3 * i + 1] = R.h;
        nc[3 * i + 2] = el;
      }
    }
    s->ws_rows = (int)chain_node.size();
    if ((st = upload(s, cnc, &s->cn_chain)) != DM_OK) return st;
    if ((st = upload(s, nc, &s->nconst)) != DM_OK) return st;
    D.nconst = s->nconst;
  }
#ifdef DM_PHASE_TIMING
  if ((st = alloc(s, (size_t)s->n_sys * 8, &D.dbg)) != DM_OK) return st;
#else
  D.dbg = nullptr;
#endif
  D.n_nodes_tot = NN; D.n_edges_tot = NE; D.n_st_tot = s->n_st;
  // natural curvature and actuation may be set again later; keep a copy of stencil->rod
  s->finalized = true;
  int blk = s->cfg.block_size;
  s->block_auto = blk <= 0;
  if (blk <= 0) blk = 256;   // four wavefronts: element work in parallel, up to 16 arms per sweep
  s->block = blk;
  return DM_OK;
}

dm_status check_rod(const dm_sim* s, int rod) {
  if (!s) return fail(DM_ERR_INVALID_ARG, "null sim");
  if (rod < 0 || rod >= (int)s->rods.size()) return fail(DM_ERR_INVALID_ARG, "rod index out of range");
  return DM_OK;
}

dm_status upload_kbar(dm_sim* s) {
  DM_HIP(hipMemcpy((void*)s->dev.kbar, s->h_kbar.data(), s->h_kbar.size() * sizeof(double), hipMemcpyHostToDevice));
  DM_HIP(hipMemcpy((void*)s->dev.act, s->h_act.data(), s->h_act.size() * sizeof(double), hipMemcpyHostToDevice));
  return DM_OK;
}

size_t state_doubles(const dm_sim* s) { return 3 * (size_t)s->n_nodes * 3 + 3 * (size_t)s->n_edges + 6 * (size_t)s->n_edges + s->n_st + s->n_sys; }


// Step arguments and LDS size of a launch.
void fill_step_args(const dm_sim* s, double dt, int nsteps, DmStepArgs& A) {
  std::memset(&A, 0, sizeof(A));       // padding too: captured segments are keyed by these bytes
  A.d = s->dev;
  A.midpoint = s->scheme == DM_IMPLICIT_MIDPOINT;
  A.max_halvings = s->max_halvings;
  A.dt = A.midpoint ? 0.5 * dt : dt;
  A.tol = s->cfg.newton_tol;
  A.floor_factor = s->cfg.floor_factor;
  for (int c = 0; c < 3; ++c) A.g[c] = s->cfg.gravity[c];
  A.damping = s->cfg.damping;
  A.floor_on = s->cfg.floor_contact;
  A.floor_z = s->cfg.floor_z; A.delta = s->cfg.delta; A.nu = s->cfg.nu; A.mu = s->cfg.mu; A.kc = s->cfg.k_contact;
  A.max_iter = s->cfg.max_iter;
  A.warm_max_iter = s->cfg.warm_max_iter > 0 ? s->cfg.warm_max_iter : s->cfg.max_iter;
  A.nsteps = nsteps;
  A.line_search = s->cfg.line_search;
  A.n_systems = s->n_sys;
  A.max_nb = std::max(s->max_nb, 1);
  A.max_arms = std::max(s->max_arms, 1);
  A.max_seg = std::max(s->max_seg, 1);
  A.warm = s->ws_mode;
  if (s->ws_mode == 2) dm_mlp_view(s->ws_net, &A.net);
  if (s->sc_on) {
    A.sc_on = 1;
    A.sc_max_edges = std::max(s->sc_max_edges, 1);
    int cap = 64;
    while (cap < 4 * A.sc_max_edges) cap <<= 1;    // pair slots: four per edge, a power of two
    A.sc_cap = cap;
    A.sc_delta = s->sc_delta;
    A.sc_kc = s->sc_kc;
    A.sc_mu = s->sc_mu;
    A.sc_nu = s->sc_nu;
  }
}

// LDS bytes of a step launch; places the network's activations (warm mode 2) after the
// solver's arrays, 16-byte aligned.
size_t step_lds(DmStepArgs& A) {
  size_t base = sizeof(double) * ((size_t)A.max_nb * (A.max_nb + 1) + (size_t)A.max_arms * 110 + A.max_nb +
                                   40 + 2 + (size_t)A.max_seg);
  if (A.sc_on) {
    // self-contact: boxes [6][max edges] floats, pair keys [cap], four ints (pair count,
    // overflow flag, half bandwidth), then the solve's vector and multiplier column
    // [4 max edges + 3] doubles each and its blocked LU's panel and U block, 2 x sc_pb x 144
    // doubles: panels of 16 columns where they fit in 64 KB, else of 8
    A.sc_lds = (int)((base + 15) / 16 * 16);
    base = (size_t)A.sc_lds + 24 * (size_t)A.sc_max_edges + 4 * (size_t)A.sc_cap + 16 +
           2 * sizeof(double) * (4 * (size_t)A.sc_max_edges + 3);
    const size_t net = A.warm == 2 ? 16 + DM_NET_LDS_BYTES : 0;    // the network's area after it
    A.sc_pb = base + sizeof(double) * 2 * 16 * 144 + net <= 65536 ? 16 : 8;
    base += sizeof(double) * 2 * (size_t)A.sc_pb * 144;
  }
  if (A.warm != 2) return base;
  A.net_lds = (int)((base + 15) / 16 * 16);
  return (size_t)A.net_lds + DM_NET_LDS_BYTES;
}

// Device buffer of at least n doubles (contents not kept when it grows).
dm_status grow(dm_sim* s, double** p, size_t* cap, size_t n) {
  if (*cap >= n && *p) return DM_OK;
  if (*p) { dev_free(s, *p); *p = nullptr; *cap = 0; }
  void* q = dev_malloc(s, std::max<size_t>(n, 1) * sizeof(double));
  if (!q) return fail(DM_ERR_OOM, "device allocation failed (" + std::to_string(n * sizeof(double)) + " bytes)");
  *p = static_cast<double*>(q);
  *cap = n;
  return DM_OK;
}

// One stored state: x, v, theta, omega, t_ref, d1_ref, beta_ref, time (the layout the
// adjoint kernel reads).
size_t traj_stride(const dm_sim* s) {
  return 6 * (size_t)s->n_nodes + 8 * (size_t)s->n_edges + (size_t)s->n_st + (size_t)s->n_sys;
}

hipError_t save_state_on(const dm_sim* s, double* dst, hipStream_t q) {
  const size_t NN = s->n_nodes, NE = s->n_edges;
  const hipMemcpyKind k = hipMemcpyDeviceToDevice;
  double* p = dst;
  hipError_t e = hipMemcpyAsync(p, s->dev.x, sizeof(double) * 3 * NN, k, q); p += 3 * NN;
  if (e == hipSuccess) e = hipMemcpyAsync(p, s->dev.v, sizeof(double) * 3 * NN, k, q); p += 3 * NN;
  if (e == hipSuccess) e = hipMemcpyAsync(p, s->dev.th, sizeof(double) * NE, k, q); p += NE;
  if (e == hipSuccess) e = hipMemcpyAsync(p, s->dev.om, sizeof(double) * NE, k, q); p += NE;
  if (e == hipSuccess) e = hipMemcpyAsync(p, s->dev.tref, sizeof(double) * 3 * NE, k, q); p += 3 * NE;
  if (e == hipSuccess) e = hipMemcpyAsync(p, s->dev.d1ref, sizeof(double) * 3 * NE, k, q); p += 3 * NE;
  if (e == hipSuccess) e = hipMemcpyAsync(p, s->dev.bref, sizeof(double) * s->n_st, k, q); p += s->n_st;
  if (e == hipSuccess) e = hipMemcpyAsync(p, s->dev.time, sizeof(double) * s->n_sys, k, q);
  return e;
}

dm_status save_state(dm_sim* s, double* dst) {
  DM_HIP(save_state_on(s, dst, s->stream));
  return DM_OK;
}

dm_status load_state(dm_sim* s, const double* src) {
  const size_t NN = s->n_nodes, NE = s->n_edges;
  const hipMemcpyKind k = hipMemcpyDeviceToDevice;
  const double* p = src;
  DM_HIP(hipMemcpyAsync(s->dev.x, p, sizeof(double) * 3 * NN, k, s->stream));
  DM_HIP(hipMemcpyAsync(s->dev.x0, p, sizeof(double) * 3 * NN, k, s->stream)); p += 3 * NN;
  DM_HIP(hipMemcpyAsync(s->dev.v, p, sizeof(double) * 3 * NN, k, s->stream));
  DM_HIP(hipMemcpyAsync(s->dev.vprev, p, sizeof(double) * 3 * NN, k, s->stream));
  DM_HIP(hipMemcpyAsync(s->dev.vprev2, p, sizeof(double) * 3 * NN, k, s->stream)); p += 3 * NN;
  DM_HIP(hipMemcpyAsync(s->dev.th, p, sizeof(double) * NE, k, s->stream));
  DM_HIP(hipMemcpyAsync(s->dev.th0, p, sizeof(double) * NE, k, s->stream)); p += NE;
  DM_HIP(hipMemcpyAsync(s->dev.om, p, sizeof(double) * NE, k, s->stream)); p += NE;
  DM_HIP(hipMemcpyAsync(s->dev.tref, p, sizeof(double) * 3 * NE, k, s->stream)); p += 3 * NE;
  DM_HIP(hipMemcpyAsync(s->dev.d1ref, p, sizeof(double) * 3 * NE, k, s->stream)); p += 3 * NE;
  DM_HIP(hipMemcpyAsync(s->dev.bref, p, sizeof(double) * s->n_st, k, s->stream)); p += s->n_st;
  DM_HIP(hipMemcpyAsync(s->dev.time, p, sizeof(double) * s->n_sys, k, s->stream));
  return DM_OK;
}

// Runs the enclosing call on the capture stream when graphs are on and the sim has no
// stream (capture needs a stream other than the null stream); device synchronisation fences
// the call against earlier null-stream work, and the stream is drained on exit.
struct CaptureStream {
  dm_sim* s;
  bool swapped = false;
  explicit CaptureStream(dm_sim* s_) : s(s_) {
    if (!s->cfg.use_graphs || s->stream) return;
    if (!s->cap_stream && hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking) != hipSuccess) return;
    (void)hipDeviceSynchronize();
    s->stream = s->cap_stream;
    swapped = true;
  }
  ~CaptureStream() {
    if (!swapped) return;
    (void)hipStreamSynchronize(s->stream);
    s->stream = nullptr;
  }
};

// len one-step launches of A; after step i the rod tips go to tips + 3 i n_rods (if tips) and
// the state to states + (i + 1) W (if states).
hipError_t seg_sequence(dm_sim* s, const DmStepArgs& A, size_t lds, int len, double* tips, double* states) {
  const int nr = (int)s->rods.size();
  const size_t W = traj_stride(s);
  for (int i = 0; i < len; ++i) {
    hipError_t e = dm_launch_step(&A, s->block, lds, s->stream);
    if (e == hipSuccess && tips)
      e = dm_launch_gather_tips(s->dev.x, s->n_nodes, s->tip_nodes, nr, tips + (size_t)i * nr * 3, s->stream);
    if (e == hipSuccess && states) e = save_state_on(s, states + (size_t)(i + 1) * W, s->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// One trajectory segment of len steps (statistics accumulate; a failed system sits out the
// rest).  With graphs on, the sequence is captured once per step configuration, length and
// destination and replayed afterwards.
dm_status run_segment(dm_sim* s, double dt, int len, double* tips, double* states) {
  DmStepArgs A;
  fill_step_args(s, dt, 1, A);
  A.accum = 1;
  const size_t lds = step_lds(A);
  if (!s->cfg.use_graphs) {
    DM_HIP(seg_sequence(s, A, lds, len, tips, states));
    return DM_OK;
  }
  SegGraph* g = nullptr;
  for (SegGraph& c : s->seg_graphs)
    if (c.len == len && c.tips == tips && c.states == states && c.block == s->block && c.lds == lds &&
        std::memcmp(&c.args, &A, sizeof(A)) == 0)
      g = &c;
  if (!g) {
    if (s->seg_graphs.size() >= 8) {
      for (SegGraph& c : s->seg_graphs) { (void)hipGraphExecDestroy(c.exec); (void)hipGraphDestroy(c.graph); }
      s->seg_graphs.clear();
    }
    SegGraph c;
    c.args = A; c.len = len; c.tips = tips; c.states = states; c.block = s->block; c.lds = lds;
    DM_HIP(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    const hipError_t ce = seg_sequence(s, A, lds, len, tips, states);
    const hipError_t ee = hipStreamEndCapture(s->stream, &c.graph);
    if (ce != hipSuccess) {
      if (c.graph) (void)hipGraphDestroy(c.graph);
      DM_HIP(ce);
    }
    DM_HIP(ee);
    const hipError_t ie = hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      (void)hipGraphDestroy(c.graph);
      DM_HIP(ie);
    }
    s->seg_graphs.push_back(c);
    g = &s->seg_graphs.back();
  }
  DM_HIP(hipGraphLaunch(g->exec, s->stream));
  return DM_OK;
}

// Zero the per-system statistics (before accumulating launches).
dm_status zero_stats(dm_sim* s) {
  for (int* p : {s->dev.s_steps, s->dev.s_iters, s->dev.s_status, s->dev.s_floor, s->dev.s_fallback,
                 s->dev.s_halved})
    DM_HIP(hipMemsetAsync(p, 0, sizeof(int) * s->n_sys, s->stream));
  for (double* p : {s->dev.s_floor_res, s->dev.s_floor_est})
    DM_HIP(hipMemsetAsync(p, 0, sizeof(double) * s->n_sys, s->stream));
  return DM_OK;
}

// Worst status over the systems after accumulating launches (DM_OK, DM_NOT_CONVERGED or
// DM_ERR_SINGULAR); synchronises the stream.
dm_status worst_status(dm_sim* s) {
  std::vector<int> status(s->n_sys);
  DM_HIP(hipMemcpyAsync(status.data(), s->dev.s_status, sizeof(int) * s->n_sys, hipMemcpyDeviceToHost, s->stream));
  DM_HIP(hipStreamSynchronize(s->stream));
  dm_status w = DM_OK;
  for (int v : status) {
    if (v == DM_ERR_SINGULAR || v == DM_ERR_UNSUPPORTED) w = DM_ERR_SINGULAR;
    else if (v == DM_NOT_CONVERGED && w == DM_OK) w = DM_NOT_CONVERGED;
  }
  return w;
}

// The adjoint covers independent rods without contact or time-dependent actuation.
dm_status adjoint_supported(const dm_sim* s) {
  if (s->scheme != DM_BACKWARD_EULER) return fail(DM_ERR_UNSUPPORTED, "adjoint: only the backward-Euler step");
  if (s->max_halvings != 0) return fail(DM_ERR_UNSUPPORTED, "adjoint: adaptive time stepping is not supported");
  if (s->cfg.floor_contact) return fail(DM_ERR_UNSUPPORTED, "adjoint: floor contact is not supported");
  if (s->sc_on) return fail(DM_ERR_UNSUPPORTED, "adjoint: self-contact is not supported");
  for (const DmSystem& S : s->sys)
    if (S.n_chains != 1 || S.n_jst != 0) return fail(DM_ERR_UNSUPPORTED, "adjoint: joined rods are not supported");
  for (const Rod& R : s->rods)
    if (R.act) return fail(DM_ERR_UNSUPPORTED, "adjoint: actuated rods are not supported");
  return DM_OK;
}

size_t kbar_total(const dm_sim* s) {
  size_t n = 0;
  for (const Rod& R : s->rods) n += 2 * (size_t)std::max(R.n - 2, 0);
  return n;
}

// ---- limb curvatures of an equilibrium and their gradient (Real2Sim) ----

dm_status curvature_supported(const dm_sim* s, const char* who) {
  if (!s->finalized) return fail(DM_ERR_STATE, std::string(who) + " before dm_finalize");
  if (s->scheme != DM_BACKWARD_EULER) return fail(DM_ERR_UNSUPPORTED, std::string(who) + ": only the backward-Euler step");
  if (s->cfg.floor_contact) return fail(DM_ERR_UNSUPPORTED, std::string(who) + ": floor contact is not supported");
  if (s->sc_on) return fail(DM_ERR_UNSUPPORTED, std::string(who) + ": self-contact is not supported");
  for (const Rod& R : s->rods)
    if (R.act) return fail(DM_ERR_UNSUPPORTED, std::string(who) + ": actuated rods are not supported");
  return DM_OK;
}

// Mean over each rod's interior stencils of kappa1 / Vbar at the committed state (0 for rods of
// fewer than 3 nodes), summed in stencil order.
dm_status read_limb_curvatures(dm_sim* s, std::vector<double>& kappa) {
  dm_status st;
  if ((st = grow(s, &s->curv_st, &s->curv_st_n, (size_t)s->n_st)) != DM_OK) return st;
  DmStepArgs A;
  fill_step_args(s, 1.0, 0, A);
  DM_HIP(dm_launch_stencil_curvature(&A, s->curv_st, s->stream));
  std::vector<double> h(s->n_st);
  DM_HIP(hipMemcpyAsync(h.data(), s->curv_st, sizeof(double) * s->n_st, hipMemcpyDeviceToHost, s->stream));
  DM_HIP(hipStreamSynchronize(s->stream));
  kappa.assign(s->rods.size(), 0.0);
  for (size_t r = 0; r < s->rods.size(); ++r) {
    const int m = s->rods[r].n - 2;
    if (m <= 0) continue;
    double sum = 0.0;
    for (int i = 0; i < m; ++i) sum += h[s->rod_st0[r] + i];
    kappa[r] = sum / m;
  }
  return DM_OK;
}

// d (sum_r w_r kappa_r) / d kbar_r at the committed (settled) state, kbar_r a rod's uniform
// natural curvature (1/m, first component), by the equilibrium adjoint with a step of dt;
// systems whose flag in skip_dev (device ints, or null) is set are left out (their entries 0).
dm_status limb_curvature_gradient(dm_sim* s, double dt, const double* w, std::vector<double>& g, const int* skip_dev) {
  dm_status st;
  const size_t NN = s->n_nodes, NE = s->n_edges, NS = s->n_st;
  std::vector<double> wst(NS, 0.0);
  for (size_t r = 0; r < s->rods.size(); ++r) {
    const int m = s->rods[r].n - 2;
    for (int i = 0; i < m; ++i) {
      const int k = s->rod_st0[r] + i;
      wst[k] = w[r] / (m * s->h_Vbar[k]);
    }
  }
  if ((st = grow(s, &s->curv_w, &s->curv_w_n, NS)) != DM_OK) return st;
  if ((st = grow(s, &s->curv_mu, &s->curv_mu_n, 3 * NN + NE)) != DM_OK) return st;
  if ((st = grow(s, &s->curv_p, &s->curv_p_n, NS)) != DM_OK) return st;
  DM_HIP(hipMemcpyAsync(s->curv_w, wst.data(), sizeof(double) * NS, hipMemcpyHostToDevice, s->stream));
  DM_HIP(hipMemsetAsync(s->curv_p, 0, sizeof(double) * NS, s->stream));
  DmCurvArgs C;
  std::memset(&C, 0, sizeof(C));
  fill_step_args(s, dt, 0, C.s);
  C.s.warm = 0;
  C.c.wst = s->curv_w;
  C.c.mu = s->curv_mu;
  C.c.pst = s->curv_p;
  C.c.skip = skip_dev;
  const size_t lds = step_lds(C.s);
  DM_HIP(dm_launch_curvature_adjoint(&C, s->block, lds, s->stream));
  std::vector<double> p(NS);
  std::vector<int> status(s->n_sys);
  DM_HIP(hipMemcpyAsync(p.data(), s->curv_p, sizeof(double) * NS, hipMemcpyDeviceToHost, s->stream));
  DM_HIP(hipMemcpyAsync(status.data(), s->dev.s_status, sizeof(int) * s->n_sys, hipMemcpyDeviceToHost, s->stream));
  DM_HIP(hipStreamSynchronize(s->stream));
  std::vector<int> skip(s->n_sys, 0);
  if (skip_dev) DM_HIP(hipMemcpy(skip.data(), skip_dev, sizeof(int) * s->n_sys, hipMemcpyDeviceToHost));
  for (int k = 0; k < s->n_sys; ++k)
    if (!skip[k] && status[k] == DM_ERR_SINGULAR)
      return fail(DM_ERR_SINGULAR, "limb curvature gradient: singular Newton matrix in some system");
  g.assign(s->rods.size(), 0.0);
  for (size_t r = 0; r < s->rods.size(); ++r) {
    const int m = s->rods[r].n - 2;
    double sum = 0.0;
    for (int i = 0; i < m; ++i) sum += p[s->rod_st0[r] + i];
    g[r] = sum;
  }
  return DM_OK;
}
}  // namespace

extern "C" {

void dm_config_default(dm_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->gravity[2] = -9.81;
  c->newton_tol = 1e-9;
  c->floor_factor = 1.0;
  c->max_iter = 50;
  c->use_graphs = 1;
  c->delta = 5e-4;
  c->nu = 1e-3;
  c->mu = 0.0;
  c->k_contact = 0.0;
}

dm_status dm_create(const dm_config* cfg, dm_sim** out) {
  if (!cfg || !out) return fail(DM_ERR_INVALID_ARG, "dm_create: null argument");
  if (!(cfg->newton_tol >= 0.0) || !(cfg->floor_factor >= 0.0) || !std::isfinite(cfg->floor_factor) ||
      cfg->max_iter < 1 || cfg->warm_max_iter < 0)
    return fail(DM_ERR_INVALID_ARG, "dm_create: bad Newton settings");
  if (cfg->alloc && !cfg->free_) return fail(DM_ERR_INVALID_ARG, "dm_create: an allocator hook needs free_");
  if (cfg->block_size != 0 && (cfg->block_size < 64 || cfg->block_size > 512 || cfg->block_size % 64))
    return fail(DM_ERR_INVALID_ARG, "dm_create: block_size must be 0 or a multiple of 64 in [64, 512]");
  if (cfg->floor_contact && (!(cfg->delta > 0) || !(cfg->nu > 0) || !(cfg->k_contact >= 0) || !(cfg->mu >= 0)))
    return fail(DM_ERR_INVALID_ARG, "dm_create: bad contact parameters");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(DM_ERR_HIP, "dm_create: no HIP device");
  if (cfg->device < 0 || cfg->device >= ndev) return fail(DM_ERR_INVALID_ARG, "dm_create: device out of range");
  DM_HIP(hipSetDevice(cfg->device));
  dm_sim* s = new dm_sim();
  s->cfg = *cfg;
  s->stream = static_cast<hipStream_t>(cfg->stream);
  *out = s;
  return DM_OK;
}

dm_status dm_add_rod(dm_sim* s, int n, const double* x0, double h, double E, double nu, double rho, int* rod_id) {
  if (!s || !x0) return fail(DM_ERR_INVALID_ARG, "dm_add_rod: null argument");
  if (s->finalized) return fail(DM_ERR_STATE, "dm_add_rod after dm_finalize");
  if (n < 2) return fail(DM_ERR_INVALID_ARG, "dm_add_rod: need at least 2 nodes");
  if (!(h > 0) || !(E > 0) || !(rho > 0) || !(nu > -1.0) || !finite_all(x0, 3 * (size_t)n))
    return fail(DM_ERR_INVALID_ARG, "dm_add_rod: non-positive or non-finite parameter");
  Rod r;
  r.n = n; r.x0.assign(x0, x0 + 3 * n); r.h = h; r.E = E; r.nu = nu; r.rho = rho;
  r.nfix.assign(n, 0); r.efix.assign(n - 1, 0);
  s->rods.push_back(std::move(r));
  if (rod_id) *rod_id = (int)s->rods.size() - 1;
  return DM_OK;
}

dm_status dm_add_joint(dm_sim* s, int ra, int na, int rb, int nb) {
  if (!s) return fail(DM_ERR_INVALID_ARG, "null sim");
  if (s->finalized) return fail(DM_ERR_STATE, "dm_add_joint after dm_finalize");
  dm_status st;
  if ((st = check_rod(s, ra)) != DM_OK || (st = check_rod(s, rb)) != DM_OK) return st;
  if (na < 0 || na >= s->rods[ra].n || nb < 0 || nb >= s->rods[rb].n) return fail(DM_ERR_INVALID_ARG, "dm_add_joint: node index out of range");
  if (ra == rb) return fail(DM_ERR_UNSUPPORTED, "dm_add_joint: a rod joined to itself");
  s->joints.push_back({ra, na, rb, nb});
  return DM_OK;
}

dm_status dm_fix_nodes(dm_sim* s, int rod, const int* nodes, int n) {
  dm_status st;
  if ((st = check_rod(s, rod)) != DM_OK) return st;
  if (s->finalized) return fail(DM_ERR_STATE, "dm_fix_nodes after dm_finalize");
  if (n > 0 && !nodes) return fail(DM_ERR_INVALID_ARG, "dm_fix_nodes: null nodes");
  for (int i = 0; i < n; ++i) if (nodes[i] < 0 || nodes[i] >= s->rods[rod].n) return fail(DM_ERR_INVALID_ARG, "dm_fix_nodes: index out of range");
  for (int i = 0; i < n; ++i) s->rods[rod].nfix[nodes[i]] = 1;
  return DM_OK;
}

dm_status dm_fix_edges(dm_sim* s, int rod, const int* edges, int n) {
  dm_status st;
  if ((st = check_rod(s, rod)) != DM_OK) return st;
  if (s->finalized) return fail(DM_ERR_STATE, "dm_fix_edges after dm_finalize");
  if (n > 0 && !edges) return fail(DM_ERR_INVALID_ARG, "dm_fix_edges: null edges");
  for (int i = 0; i < n; ++i) if (edges[i] < 0 || edges[i] >= s->rods[rod].n - 1) return fail(DM_ERR_INVALID_ARG, "dm_fix_edges: index out of range");
  for (int i = 0; i < n; ++i) s->rods[rod].efix[edges[i]] = 1;
  return DM_OK;
}

dm_status dm_set_natural_curvature(dm_sim* s, int rod, const double* kbar) {
  dm_status st;
  if ((st = check_rod(s, rod)) != DM_OK) return st;
  Rod& R = s->rods[rod];
  if (R.n < 3) return DM_OK;
  if (!kbar) return fail(DM_ERR_INVALID_ARG, "dm_set_natural_curvature: null kbar");
  if (!finite_all(kbar, 2 * (size_t)(R.n - 2))) return fail(DM_ERR_INVALID_ARG, "dm_set_natural_curvature: non-finite value");
  R.kbar.assign(kbar, kbar + 2 * (R.n - 2));
  R.has_kbar = true;
  if (s->finalized) {
    for (int i = 1; i + 1 < R.n; ++i) {
      int st_ = s->rod_st0[rod] + i - 1;
      s->h_kbar[st_] = kbar[2 * (i - 1)] * s->h_Vbar[st_];
      s->h_kbar[s->n_st + st_] = kbar[2 * (i - 1) + 1] * s->h_Vbar[st_];
    }
    return upload_kbar(s);
  }
  return DM_OK;
}

dm_status dm_set_actuation_sine(dm_sim* s, int rod, double A, double f, double phi) {
  dm_status st;
  if ((st = check_rod(s, rod)) != DM_OK) return st;
  if (!std::isfinite(A) || !std::isfinite(f) || !std::isfinite(phi)) return fail(DM_ERR_INVALID_ARG, "dm_set_actuation_sine: non-finite");
  Rod& R = s->rods[rod];
  R.act = true; R.A = A; R.f = f; R.phi = phi;
  if (s->finalized) {
    for (int i = 1; i + 1 < R.n; ++i) {
      int st_ = s->rod_st0[rod] + i - 1;
      s->h_act[st_] = A; s->h_act[s->n_st + st_] = f; s->h_act[2 * s->n_st + st_] = phi;
    }
    return upload_kbar(s);
  }
  return DM_OK;
}

dm_status dm_set_external_load(dm_sim* s, int rod, const double* force, const double* moment) {
  dm_status st;
  if ((st = check_rod(s, rod)) != DM_OK) return st;
  if (s->finalized) return fail(DM_ERR_STATE, "dm_set_external_load after dm_finalize");
  Rod& R = s->rods[rod];
  if (force) {
    if (!finite_all(force, 3 * (size_t)R.n)) return fail(DM_ERR_INVALID_ARG, "dm_set_external_load: non-finite force");
    R.force.assign(force, force + 3 * R.n);
  }
  if (moment) {
    if (!finite_all(moment, (size_t)R.n - 1)) return fail(DM_ERR_INVALID_ARG, "dm_set_external_load: non-finite moment");
    R.moment.assign(moment, moment + R.n - 1);
  }
  return DM_OK;
}

dm_status dm_finalize(dm_sim* s) {
  if (!s) return fail(DM_ERR_INVALID_ARG, "null sim");
  if (s->finalized) return fail(DM_ERR_STATE, "dm_finalize called twice");
  DM_HIP(hipSetDevice(s->cfg.device));
  dm_status st = do_finalize(s);
  if (st != DM_OK) {
    for (void* p : s->allocs) dev_free(s, p);
    s->allocs.clear();
    s->finalized = false;
  }
  return st;
}

dm_status dm_step(dm_sim* s, double dt, int nsteps, dm_stats* stats) {
  if (!s) return fail(DM_ERR_INVALID_ARG, "null sim");
  if (!s->finalized) return fail(DM_ERR_STATE, "dm_step before dm_finalize");
  if (s->sc_on && s->scheme != DM_BACKWARD_EULER)
    return fail(DM_ERR_UNSUPPORTED, "dm_step: self-contact needs the backward-Euler step");
  if (!(dt > 0) || !std::isfinite(dt) || nsteps < 0) return fail(DM_ERR_INVALID_ARG, "dm_step: bad dt or nsteps");
  if (nsteps == 0) return DM_OK;
  DM_HIP(hipSetDevice(s->cfg.device));
  DmStepArgs A;
  fill_step_args(s, dt, nsteps, A);
  const size_t lds = step_lds(A);
  if (!s->ev0) { DM_HIP(hipEventCreate(&s->ev0)); DM_HIP(hipEventCreate(&s->ev1)); }
  // one persistent launch for all steps; a warm start guesses inside it at every step start
  DM_HIP(hipEventRecord(s->ev0, s->stream));
  DM_HIP(dm_launch_step(&A, s->block, lds, s->stream));
  DM_HIP(hipEventRecord(s->ev1, s->stream));
  DM_HIP(hipStreamSynchronize(s->stream));
  DM_HIP(hipEventElapsedTime(&s->last_kernel_ms, s->ev0, s->ev1));
  std::vector<int> steps(s->n_sys), iters(s->n_sys), status(s->n_sys), floors(s->n_sys), falls(s->n_sys),
      halved(s->n_sys);
  DM_HIP(hipMemcpy(falls.data(), s->dev.s_fallback, sizeof(int) * s->n_sys, hipMemcpyDeviceToHost));
  DM_HIP(hipMemcpy(halved.data(), s->dev.s_halved, sizeof(int) * s->n_sys, hipMemcpyDeviceToHost));
  std::vector<double> res(s->n_sys), fres(s->n_sys), fest(s->n_sys);
  DM_HIP(hipMemcpy(fres.data(), s->dev.s_floor_res, sizeof(double) * s->n_sys, hipMemcpyDeviceToHost));
  DM_HIP(hipMemcpy(fest.data(), s->dev.s_floor_est, sizeof(double) * s->n_sys, hipMemcpyDeviceToHost));
  DM_HIP(hipMemcpy(steps.data(), s->dev.s_steps, sizeof(int) * s->n_sys, hipMemcpyDeviceToHost));
  DM_HIP(hipMemcpy(iters.data(), s->dev.s_iters, sizeof(int) * s->n_sys, hipMemcpyDeviceToHost));
  DM_HIP(hipMemcpy(status.data(), s->dev.s_status, sizeof(int) * s->n_sys, hipMemcpyDeviceToHost));
  DM_HIP(hipMemcpy(res.data(), s->dev.s_res, sizeof(double) * s->n_sys, hipMemcpyDeviceToHost));
  DM_HIP(hipMemcpy(floors.data(), s->dev.s_floor, sizeof(int) * s->n_sys, hipMemcpyDeviceToHost));
  dm_status worst = DM_OK;
  for (int i = 0; i < s->n_sys; ++i) {
    if (stats) {
      stats[i].steps_done = steps[i]; stats[i].newton_iters = iters[i]; stats[i].status = status[i];
      stats[i].floor_steps = floors[i]; stats[i].residual = res[i]; stats[i].fallbacks = falls[i];
      stats[i].halvings = halved[i];
      stats[i].floor_residual_max = fres[i]; stats[i].floor_estimate = fest[i];
    }
    if (status[i] == DM_ERR_UNSUPPORTED) worst = DM_ERR_UNSUPPORTED;
    else if (status[i] == DM_ERR_SINGULAR && worst != DM_ERR_UNSUPPORTED) worst = DM_ERR_SINGULAR;
    else if (status[i] == DM_NOT_CONVERGED && worst == DM_OK) worst = DM_NOT_CONVERGED;
  }
  s->time += dt * nsteps;
  if (worst == DM_ERR_UNSUPPORTED)
    return fail(DM_ERR_UNSUPPORTED, "dm_step: more self-contact pairs in some system than its pair list holds");
  if (worst == DM_ERR_SINGULAR) return fail(DM_ERR_SINGULAR, "dm_step: zero or non-finite pivot in some system");
  if (worst == DM_NOT_CONVERGED) { g_err = "dm_step: Newton did not converge in some system"; }
  return worst;
}

dm_status dm_set_natural_curvature_all(dm_sim* s, const double* kbar, int on_device) {
  if (!s || !kbar) return fail(DM_ERR_INVALID_ARG, "dm_set_natural_curvature_all: null argument");
  const size_t n = kbar_total(s);
  std::vector<double> h(n);
  if (on_device) {
    if (!s->finalized) return fail(DM_ERR_STATE, "dm_set_natural_curvature_all: device input before dm_finalize");
    DM_HIP(hipSetDevice(s->cfg.device));
    DM_HIP(hipStreamSynchronize(s->stream));
    if (n) DM_HIP(hipMemcpy(h.data(), kbar, n * sizeof(double), hipMemcpyDeviceToHost));
  } else {
    h.assign(kbar, kbar + n);
  }
  if (!finite_all(h.data(), n)) return fail(DM_ERR_INVALID_ARG, "dm_set_natural_curvature_all: non-finite value");
  size_t off = 0;
  for (size_t r = 0; r < s->rods.size(); ++r) {
    Rod& R = s->rods[r];
    if (R.n < 3) continue;
    R.kbar.assign(h.begin() + off, h.begin() + off + 2 * (R.n - 2));
    R.has_kbar = true;
    if (s->finalized)
      for (int i = 1; i + 1 < R.n; ++i) {
        const int st_ = s->rod_st0[r] + i - 1;
        s->h_kbar[st_] = R.kbar[2 * (i - 1)] * s->h_Vbar[st_];
        s->h_kbar[s->n_st + st_] = R.kbar[2 * (i - 1) + 1] * s->h_Vbar[st_];
      }
    off += 2 * (R.n - 2);
  }
  return s->finalized ? upload_kbar(s) : DM_OK;
}

int dm_ws_rows(const dm_sim* s) { return s && s->finalized ? s->ws_rows : 0; }

dm_status dm_ws_features(dm_sim* s, double* F) {
  if (!s || !F) return fail(DM_ERR_INVALID_ARG, "dm_ws_features: null argument");
  if (!s->finalized) return fail(DM_ERR_STATE, "dm_ws_features before dm_finalize");
  DM_HIP(hipSetDevice(s->cfg.device));
  DM_HIP(dm_ws_launch_features(&s->dev, s->ws_rows, s->cn_chain, s->nconst, F, s->stream));
  DM_HIP(hipStreamSynchronize(s->stream));
  return DM_OK;
}

dm_status dm_ws_targets(dm_sim* s, const double* F_prev, double dt, double* T) {
  if (!s || !F_prev || !T) return fail(DM_ERR_INVALID_ARG, "dm_ws_targets: null argument");
  if (!s->finalized) return fail(DM_ERR_STATE, "dm_ws_targets before dm_finalize");
  DM_HIP(hipSetDevice(s->cfg.device));
  DM_HIP(dm_ws_launch_targets(&s->dev, s->ws_rows, s->cn_chain, F_prev, dt, T, s->stream));
  DM_HIP(hipStreamSynchronize(s->stream));
  return DM_OK;
}

dm_status dm_set_self_contact(dm_sim* s, double delta, double k_c, double mu, double nu) {
  if (!s) return fail(DM_ERR_INVALID_ARG, "dm_set_self_contact: null sim");
  if (!s->finalized) return fail(DM_ERR_STATE, "dm_set_self_contact before dm_finalize");
  if (k_c == 0.0) {
    s->sc_on = 0;
    if (s->block_auto) s->block = 256;
    return DM_OK;
  }
  if (!(delta > 0.0) || !(k_c > 0.0) || !(mu >= 0.0) || !(nu > 0.0) || !std::isfinite(delta) || !std::isfinite(k_c) ||
      !std::isfinite(mu) || !std::isfinite(nu))
    return fail(DM_ERR_INVALID_ARG, "dm_set_self_contact: need delta > 0, k_c > 0, mu >= 0, nu > 0");
  int me = 0;
  for (const DmSystem& S : s->sys) {
    if (S.n_chains != 1) return fail(DM_ERR_UNSUPPORTED, "dm_set_self_contact: joined rods are not supported");
    me = std::max(me, S.n_edges);
  }
  // per rod: its n x n Newton matrix, n doubles, and the pair area (156 doubles per pair slot)
  size_t cap = 64;
  while (cap < 4 * (size_t)std::max(me, 1)) cap <<= 1;
  size_t total = 0;
  std::vector<long long> off;
  for (const DmSystem& S : s->sys) {
    const size_t n = 4 * (size_t)S.n_nodes - 1;
    off.push_back((long long)total);
    total += n * n + n + 156 * cap;
  }
  if (me > 4096) return fail(DM_ERR_UNSUPPORTED, "dm_set_self_contact: rods of more than 4097 nodes");
  if (total * sizeof(double) > ((size_t)32 << 30))
    return fail(DM_ERR_UNSUPPORTED, "dm_set_self_contact: the rods' Newton matrices would exceed 32 GiB");
  if (!s->dev.sc_mat) {
    // one dense Newton matrix per rod (the layout is fixed once finalized)
    dm_status st = alloc(s, total, &s->dev.sc_mat);
    if (st != DM_OK) return st;
    long long* p = nullptr;
    if ((st = upload(s, off, &p)) != DM_OK) return st;
    s->dev.sc_off = p;
  }
  s->sc_on = 1;
  s->sc_max_edges = me;
  s->sc_delta = delta;
  s->sc_kc = k_c;
  s->sc_mu = mu;
  s->sc_nu = nu;
  DmStepArgs A;
  fill_step_args(s, 1.0, 1, A);
  if (step_lds(A) > 65536) {
    s->sc_on = 0;
    return fail(DM_ERR_UNSUPPORTED, "dm_set_self_contact: the pair list of the longest rod does not fit in LDS");
  }
  // eight wavefronts per rod by default: a rod's self-contact solve is bound by the latency of
  // its own stages, which more lanes shorten (256 coils, one per CU: 12.3 ms per step at 512
  // lanes against 16.2 at 256); dm_autotune picks per workload
  if (s->block_auto) s->block = 512;
  return DM_OK;
}

dm_status dm_set_integrator(dm_sim* s, int scheme) {
  if (!s) return fail(DM_ERR_INVALID_ARG, "dm_set_integrator: null sim");
  if (scheme != DM_BACKWARD_EULER && scheme != DM_IMPLICIT_MIDPOINT)
    return fail(DM_ERR_INVALID_ARG, "dm_set_integrator: unknown scheme " + std::to_string(scheme));
  s->scheme = scheme;
  return DM_OK;
}

dm_status dm_set_adaptive(dm_sim* s, int max_halvings) {
  if (!s) return fail(DM_ERR_INVALID_ARG, "dm_set_adaptive: null sim");
  if (max_halvings < 0 || max_halvings > 20)
    return fail(DM_ERR_INVALID_ARG, "dm_set_adaptive: max_halvings must be 0..20");
  s->max_halvings = max_halvings;
  return DM_OK;
}

dm_status dm_set_warm_start(dm_sim* s, dm_mlp* net, int mode) {
  if (!s) return fail(DM_ERR_INVALID_ARG, "null sim");
  if (!s->finalized) return fail(DM_ERR_STATE, "dm_set_warm_start before dm_finalize");
  if (mode < 0 || mode > 4) return fail(DM_ERR_INVALID_ARG, "dm_set_warm_start: mode must be 0 .. 4");
  if (mode == 2 && !net) return fail(DM_ERR_INVALID_ARG, "dm_set_warm_start: mode 2 needs a network");
  const int old_mode = s->ws_mode;
  dm_mlp* const old_net = s->ws_net;
  s->ws_mode = mode;
  s->ws_net = mode == 2 ? net : nullptr;
  if (s->sc_on && mode == 2) {
    DmStepArgs A;
    fill_step_args(s, 1.0, 1, A);
    if (step_lds(A) > 65536) {
      s->ws_mode = old_mode;
      s->ws_net = old_net;
      return fail(DM_ERR_UNSUPPORTED,
                  "dm_set_warm_start: the network's activations and the self-contact arrays do not fit together in LDS");
    }
  }
  return DM_OK;
}

dm_status dm_ws_predict(dm_sim* s, double dt, double* dx, int on_device) {
  if (!s || !dx) return fail(DM_ERR_INVALID_ARG, "dm_ws_predict: null argument");
  if (!s->finalized) return fail(DM_ERR_STATE, "dm_ws_predict before dm_finalize");
  if (s->ws_mode == 0) return fail(DM_ERR_STATE, "dm_ws_predict: no warm start set");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(DM_ERR_INVALID_ARG, "dm_ws_predict: bad dt");
  DM_HIP(hipSetDevice(s->cfg.device));
  DmStepArgs A;
  fill_step_args(s, dt, 0, A);
  const size_t lds = step_lds(A);
  const size_t n = (size_t)s->ws_rows * 3;
  double* out = dx;
  dm_status st;
  if (!on_device) {
    if ((st = grow(s, &s->ws_F, &s->ws_F_n, n)) != DM_OK) return st;
    out = s->ws_F;
  }
  DM_HIP(dm_launch_predict(&A, s->block, lds, out, s->stream));
  if (!on_device) DM_HIP(hipMemcpyAsync(dx, out, sizeof(double) * n, hipMemcpyDeviceToHost, s->stream));
  DM_HIP(hipStreamSynchronize(s->stream));
  return DM_OK;
}

dm_status dm_rollout(dm_sim* s, double dt, int nsteps, int ckpt_every, double* tips, int on_device) {
  if (!s || !tips) return fail(DM_ERR_INVALID_ARG, "dm_rollout: null argument");
  if (!s->finalized) return fail(DM_ERR_STATE, "dm_rollout before dm_finalize");
  if (!(dt > 0) || !std::isfinite(dt) || nsteps <= 0 || ckpt_every <= 0)
    return fail(DM_ERR_INVALID_ARG, "dm_rollout: bad dt, nsteps or ckpt_every");
  dm_status st;
  if ((st = adjoint_supported(s)) != DM_OK) return st;
  DM_HIP(hipSetDevice(s->cfg.device));
  s->roll_valid = false;
  const size_t W = traj_stride(s);
  const int nck = (nsteps + ckpt_every - 1) / ckpt_every;
  const int nr = (int)s->rods.size();
  if ((st = grow(s, &s->ck, &s->ck_n, (size_t)nck * W)) != DM_OK) return st;
  if (!s->tip_nodes) {
    std::vector<int> tn(nr);
    for (int r = 0; r < nr; ++r) tn[r] = s->rod_node[r].back();
    int* p = nullptr;
    if ((st = upload(s, tn, &p)) != DM_OK) return st;
    s->tip_nodes = p;
  }
  double* tdev = tips;
  if (!on_device) {
    if ((st = grow(s, &s->tips_dev, &s->tips_n, (size_t)nsteps * nr * 3)) != DM_OK) return st;
    tdev = s->tips_dev;
  }
  // captured segments gather the tips into a fixed staging buffer, copied out per segment
  if (s->cfg.use_graphs &&
      (st = grow(s, &s->tips_stage, &s->tips_stage_n, (size_t)std::min(ckpt_every, nsteps) * nr * 3)) != DM_OK)
    return st;
  CaptureStream cs(s);
  if ((st = zero_stats(s)) != DM_OK) return st;
  for (int k0 = 0; k0 < nsteps; k0 += ckpt_every) {
    const int len = std::min(ckpt_every, nsteps - k0);
    DM_HIP(save_state_on(s, s->ck + (size_t)(k0 / ckpt_every) * W, s->stream));
    double* out = tdev + (size_t)k0 * nr * 3;
    if ((st = run_segment(s, dt, len, s->cfg.use_graphs ? s->tips_stage : out, nullptr)) != DM_OK) return st;
    if (s->cfg.use_graphs)
      DM_HIP(hipMemcpyAsync(out, s->tips_stage, sizeof(double) * (size_t)len * nr * 3, hipMemcpyDeviceToDevice,
                            s->stream));
  }
  if (!on_device)
    DM_HIP(hipMemcpyAsync(tips, tdev, sizeof(double) * (size_t)nsteps * nr * 3, hipMemcpyDeviceToHost, s->stream));
  st = worst_status(s);
  s->time += dt * nsteps;
  if (st != DM_OK) return fail(st, "dm_rollout: a step failed in some system (state rolled back to that step)");
  s->roll_steps = nsteps;
  s->roll_ckpt = ckpt_every;
  s->roll_dt = dt;
  s->roll_valid = true;
  return DM_OK;
}

dm_status dm_adjoint(dm_sim* s, const double* dL_dtips, int in_on_device, double* dL_dkbar, int out_on_device) {
  if (!s || !dL_dtips || !dL_dkbar) return fail(DM_ERR_INVALID_ARG, "dm_adjoint: null argument");
  if (!s->finalized || !s->roll_valid) return fail(DM_ERR_STATE, "dm_adjoint needs a completed dm_rollout");
  dm_status st;
  if ((st = adjoint_supported(s)) != DM_OK) return st;
  DM_HIP(hipSetDevice(s->cfg.device));
  CaptureStream cs(s);
  const size_t NN = s->n_nodes, NE = s->n_edges, NS = s->n_st, W = traj_stride(s);
  const int T = s->roll_steps, C = s->roll_ckpt, nr = (int)s->rods.size();
  const int nck = (T + C - 1) / C;
  const double dt = s->roll_dt;
  const double* dl = dL_dtips;
  if (!in_on_device) {
    if ((st = grow(s, &s->dl_dev, &s->dl_n, (size_t)T * nr * 3)) != DM_OK) return st;
    DM_HIP(hipMemcpyAsync(s->dl_dev, dL_dtips, sizeof(double) * (size_t)T * nr * 3, hipMemcpyHostToDevice, s->stream));
    dl = s->dl_dev;
  }
  // adjoint arrays: ax, av [3NN]; ath, aom [NE]; atref, ad1 [3NE]; akap [2NS]; lam [3NN+NE];
  // pst [16NS]; pe [3NE]
  const size_t na = 9 * NN + 12 * NE + 18 * NS;
  if ((st = grow(s, &s->adj, &s->adj_n, na)) != DM_OK) return st;
  DM_HIP(hipMemsetAsync(s->adj, 0, sizeof(double) * na, s->stream));
  if ((st = grow(s, &s->seg, &s->seg_n, (size_t)(C + 2) * W)) != DM_OK) return st;
  double* fin = s->seg + (size_t)(C + 1) * W;
  if ((st = save_state(s, fin)) != DM_OK) return st;
  const double t_end = s->time;
  DmAdjArgs P;
  fill_step_args(s, dt, 1, P.s);
  const size_t lds = step_lds(P.s);
  double* q = s->adj;
  P.a = DmAdjDev{};
  P.a.seg = s->seg;
  P.a.dLdtip = dl;
  P.a.ax = q; q += 3 * NN;
  P.a.av = q; q += 3 * NN;
  P.a.ath = q; q += NE;
  P.a.aom = q; q += NE;
  P.a.atref = q; q += 3 * NE;
  P.a.ad1 = q; q += 3 * NE;
  P.a.akap = q; q += 2 * NS;
  P.a.lam = q; q += 3 * NN + NE;
  P.a.pst = q; q += 16 * NS;
  P.a.pe = q;
  P.a.stride = (long long)W;
  P.a.n_rods = nr;
  std::vector<int> status(s->n_sys);
  for (int j = nck - 1; j >= 0; --j) {
    const int g0 = j * C, len = std::min(C, T - g0);
    if ((st = load_state(s, s->ck + (size_t)j * W)) != DM_OK) return st;
    if ((st = save_state(s, s->seg)) != DM_OK) return st;
    if ((st = zero_stats(s)) != DM_OK) return st;
    if ((st = run_segment(s, dt, len, nullptr, s->seg)) != DM_OK) return st;
    if ((st = worst_status(s)) != DM_OK)
      return fail(st, "dm_adjoint: a recomputed step of segment " + std::to_string(j) + " failed");
    P.a.seg_len = len;
    P.a.step0 = g0;
    DM_HIP(dm_launch_adjoint(&P, s->block, lds, s->stream));
    DM_HIP(hipMemcpyAsync(status.data(), s->dev.s_status, sizeof(int) * s->n_sys, hipMemcpyDeviceToHost, s->stream));
    DM_HIP(hipStreamSynchronize(s->stream));
    for (int v : status)
      if (v != 0) return fail(DM_ERR_SINGULAR, "dm_adjoint: zero or non-finite pivot in an adjoint solve");
  }
  if ((st = load_state(s, fin)) != DM_OK) return st;
  s->time = t_end;
  std::vector<double> akap(2 * NS);
  DM_HIP(hipMemcpyAsync(akap.data(), P.a.akap, sizeof(double) * 2 * NS, hipMemcpyDeviceToHost, s->stream));
  DM_HIP(hipStreamSynchronize(s->stream));
  std::vector<double> out(kbar_total(s));
  size_t off = 0;
  for (int r = 0; r < nr; ++r) {
    const int n = s->rods[r].n;
    for (int i = 1; i + 1 < n; ++i) {
      const int st_ = s->rod_st0[r] + i - 1;
      for (int c = 0; c < 2; ++c) out[off + 2 * (i - 1) + c] = akap[c * NS + st_] * s->h_Vbar[st_];
    }
    off += 2 * (size_t)std::max(n - 2, 0);
  }
  if (out_on_device) {
    if (!out.empty()) DM_HIP(hipMemcpy(dL_dkbar, out.data(), sizeof(double) * out.size(), hipMemcpyHostToDevice));
  } else {
    std::copy(out.begin(), out.end(), dL_dkbar);
  }
  return DM_OK;
}

dm_status dm_limb_curvatures(dm_sim* s, double* kappa) {
  if (!s || !kappa) return fail(DM_ERR_INVALID_ARG, "dm_limb_curvatures: null argument");
  if (!s->finalized) return fail(DM_ERR_STATE, "dm_limb_curvatures before dm_finalize");
  DM_HIP(hipSetDevice(s->cfg.device));
  std::vector<double> k;
  dm_status st;
  if ((st = read_limb_curvatures(s, k)) != DM_OK) return st;
  std::copy(k.begin(), k.end(), kappa);
  return DM_OK;
}

dm_status dm_limb_curvature_gradient(dm_sim* s, double dt, const double* w, double* grad) {
  if (!s || !w || !grad) return fail(DM_ERR_INVALID_ARG, "dm_limb_curvature_gradient: null argument");
  dm_status st;
  if ((st = curvature_supported(s, "dm_limb_curvature_gradient")) != DM_OK) return st;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(DM_ERR_INVALID_ARG, "dm_limb_curvature_gradient: bad dt");
  if (!finite_all(w, s->rods.size())) return fail(DM_ERR_INVALID_ARG, "dm_limb_curvature_gradient: non-finite weight");
  DM_HIP(hipSetDevice(s->cfg.device));
  std::vector<double> g;
  if ((st = limb_curvature_gradient(s, dt, w, g, nullptr)) != DM_OK) return st;
  std::copy(g.begin(), g.end(), grad);
  return DM_OK;
}

dm_status dm_fit_limb_curvatures(dm_sim* s, double dt, int n_settle, int n_configs, const double* targets,
                                 double alpha0, double tol, int max_iter, double* kbar_traj, int* steps,
                                 double* losses) {
  if (!s || !targets || !kbar_traj) return fail(DM_ERR_INVALID_ARG, "dm_fit_limb_curvatures: null argument");
  dm_status st;
  if ((st = curvature_supported(s, "dm_fit_limb_curvatures")) != DM_OK) return st;
  if (!(dt > 0) || !std::isfinite(dt) || n_settle < 1 || n_configs < 0 || !(alpha0 > 0) || !std::isfinite(alpha0) ||
      !(tol >= 0) || max_iter < 0)
    return fail(DM_ERR_INVALID_ARG, "dm_fit_limb_curvatures: bad dt, n_settle, n_configs, alpha0, tol or max_iter");
  const int nr = (int)s->rods.size(), ns = s->n_sys;
  if (!finite_all(targets, (size_t)n_configs * nr)) return fail(DM_ERR_INVALID_ARG, "dm_fit_limb_curvatures: non-finite target");
  DM_HIP(hipSetDevice(s->cfg.device));
  if ((st = grow(s, &s->skip_buf, &s->skip_n, ((size_t)ns + 1) / 2)) != DM_OK) return st;
  int* skip_dev = reinterpret_cast<int*>(s->skip_buf);
  std::vector<double> kv(nr, 0.0), kappa, g, w(nr);
  std::vector<int> skip(ns);
  for (int c = 0; c < n_configs; ++c) {
    const double* tgt = targets + (size_t)c * nr;
    std::vector<double> alpha(ns, alpha0), prev(ns, std::numeric_limits<double>::infinity()), lam(ns, 0.0);
    std::vector<int> it(ns, 0), active(ns, 1);
    while (true) {
      // F(kbar): the natural curvature of every rod's interior stencils, then n_settle steps of
      // the systems still fitting
      for (int r = 0; r < nr; ++r) {
        Rod& R = s->rods[r];
        R.kbar.assign(2 * (size_t)std::max(R.n - 2, 0), 0.0);
        R.has_kbar = true;
        for (int i = 0; i + 2 < R.n; ++i) {
          const int k = s->rod_st0[r] + i;
          R.kbar[2 * i] = kv[r];
          s->h_kbar[k] = kv[r] * s->h_Vbar[k];
          s->h_kbar[s->n_st + k] = 0.0;
        }
      }
      if ((st = upload_kbar(s)) != DM_OK) return st;
      for (int k = 0; k < ns; ++k) skip[k] = !active[k];
      DM_HIP(hipMemcpyAsync(skip_dev, skip.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s->stream));
      DmStepArgs A;
      fill_step_args(s, dt, n_settle, A);
      A.skip = skip_dev;
      const size_t lds = step_lds(A);
      DM_HIP(dm_launch_step(&A, s->block, lds, s->stream));
      std::vector<int> status(ns);
      DM_HIP(hipMemcpyAsync(status.data(), s->dev.s_status, sizeof(int) * ns, hipMemcpyDeviceToHost, s->stream));
      DM_HIP(hipStreamSynchronize(s->stream));
      for (int k = 0; k < ns; ++k)
        if (active[k] && status[k] != DM_OK)
          return fail(status[k] == DM_ERR_SINGULAR ? DM_ERR_SINGULAR : DM_NOT_CONVERGED,
                      "dm_fit_limb_curvatures: the quasi-static solve failed in system " + std::to_string(k));
      s->time += dt * n_settle;
      if ((st = read_limb_curvatures(s, kappa)) != DM_OK) return st;
      // Eq. 19 per system, then Alg. 1's stopping test and step-size rule
      std::fill(lam.begin(), lam.end(), 0.0);
      for (int r = 0; r < nr; ++r) lam[s->rod_sys[r]] += std::fabs(tgt[r] - kappa[r]);
      bool any = false;
      for (int k = 0; k < ns; ++k) {
        if (!active[k]) continue;
        if (lam[k] < tol || it[k] >= max_iter) { active[k] = 0; continue; }
        if (lam[k] > prev[k]) alpha[k] *= 0.5;
        prev[k] = lam[k];
        any = true;
      }
      if (!any) break;
      for (int r = 0; r < nr; ++r) {
        const double d = kappa[r] - tgt[r];
        w[r] = active[s->rod_sys[r]] ? (double)((d > 0) - (d < 0)) : 0.0;
      }
      for (int k = 0; k < ns; ++k) skip[k] = !active[k];
      DM_HIP(hipMemcpyAsync(skip_dev, skip.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s->stream));
      if ((st = limb_curvature_gradient(s, dt, w.data(), g, skip_dev)) != DM_OK) return st;
      for (int r = 0; r < nr; ++r) {
        const int k = s->rod_sys[r];
        if (active[k]) kv[r] -= alpha[k] * g[r];
      }
      for (int k = 0; k < ns; ++k) it[k] += active[k];
    }
    for (int r = 0; r < nr; ++r) kbar_traj[(size_t)c * nr + r] = kv[r];
    for (int k = 0; k < ns; ++k) {
      if (steps) steps[(size_t)c * ns + k] = it[k];
      if (losses) losses[(size_t)c * ns + k] = lam[k];
    }
  }
  return DM_OK;
}

dm_status dm_fit_natural_curvature(dm_sim* s, double dt, int nsteps, int ckpt_every, const double* target_tips,
                                   int target_on_device, double alpha0, double tol, int max_iter, double* kbar,
                                   int kbar_on_device, double* losses, int* n_eval) {
  if (!s || !target_tips || !kbar) return fail(DM_ERR_INVALID_ARG, "dm_fit_natural_curvature: null argument");
  if (!s->finalized) return fail(DM_ERR_STATE, "dm_fit_natural_curvature before dm_finalize");
  if (!(alpha0 > 0) || !std::isfinite(alpha0) || !(tol >= 0) || max_iter < 0 || nsteps <= 0 || ckpt_every <= 0)
    return fail(DM_ERR_INVALID_ARG, "dm_fit_natural_curvature: bad alpha0, tol, max_iter, nsteps or ckpt_every");
  dm_status st;
  if ((st = adjoint_supported(s)) != DM_OK) return st;
  DM_HIP(hipSetDevice(s->cfg.device));
  const size_t nk = kbar_total(s), nt = (size_t)nsteps * s->rods.size() * 3, nc = dm_checkpoint_size(s);
  // device work buffers of this call: kbar, its gradient, tips, target, dL/dtips, loss, start state
  std::vector<double*> bufs;
  struct Guard { dm_sim* s; std::vector<double*>& b; ~Guard() { for (double* p : b) dev_free(s, p); } } guard{s, bufs};
  auto get = [&](size_t n, double** p) -> dm_status {
    *p = static_cast<double*>(dev_malloc(s, std::max<size_t>(n, 1) * sizeof(double)));
    if (!*p) return fail(DM_ERR_OOM, "dm_fit_natural_curvature: device allocation failed");
    bufs.push_back(*p);
    return DM_OK;
  };
  double *kb, *g, *tips, *tgt, *dl, *loss, *ck0;
  for (auto pr : {std::make_pair(nk, &kb), std::make_pair(nk, &g), std::make_pair(nt, &tips), std::make_pair(nt, &tgt),
                  std::make_pair(nt, &dl), std::make_pair((size_t)1, &loss), std::make_pair(nc, &ck0)})
    if ((st = get(pr.first, pr.second)) != DM_OK) return st;
  DM_HIP(hipMemcpy(kb, kbar, nk * sizeof(double), kbar_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
  DM_HIP(hipMemcpy(tgt, target_tips, nt * sizeof(double),
                   target_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
  if ((st = dm_save_checkpoint(s, ck0, 1)) != DM_OK) return st;
  double alpha = alpha0, prev = std::numeric_limits<double>::infinity();
  int evals = 0;
  for (int it = 0; it <= max_iter; ++it) {
    if ((st = dm_load_checkpoint(s, ck0, 1)) != DM_OK) return st;
    if ((st = dm_set_natural_curvature_all(s, kb, 1)) != DM_OK) return st;
    if ((st = dm_rollout(s, dt, nsteps, ckpt_every, tips, 1)) != DM_OK) return st;
    DM_HIP(dm_launch_fit_loss(tips, tgt, (int)nt, dl, loss, s->stream));
    double L = 0.0;
    DM_HIP(hipMemcpyAsync(&L, loss, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    DM_HIP(hipStreamSynchronize(s->stream));
    if (losses) losses[evals] = L;
    ++evals;
    if (L < tol || it == max_iter) break;
    if (L > prev) alpha *= 0.5;
    prev = L;
    if ((st = dm_adjoint(s, dl, 1, g, 1)) != DM_OK) return st;
    DM_HIP(dm_launch_axpy(kb, g, -alpha, (int)nk, s->stream));
  }
  // the sim ends at its starting state with the fitted natural curvature
  if ((st = dm_load_checkpoint(s, ck0, 1)) != DM_OK) return st;
  if ((st = dm_set_natural_curvature_all(s, kb, 1)) != DM_OK) return st;
  DM_HIP(hipStreamSynchronize(s->stream));
  DM_HIP(hipMemcpy(kbar, kb, nk * sizeof(double), kbar_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  if (n_eval) *n_eval = evals;
  return DM_OK;
}

dm_status dm_autotune(dm_sim* s, double dt, int trial_steps, const char* cache_path, int* block_out) {
  if (!s) return fail(DM_ERR_INVALID_ARG, "null sim");
  if (!s->finalized) return fail(DM_ERR_STATE, "dm_autotune before dm_finalize");
  if (!(dt > 0) || trial_steps < 1) return fail(DM_ERR_INVALID_ARG, "dm_autotune: bad dt or trial_steps");
  DM_HIP(hipSetDevice(s->cfg.device));
  hipDeviceProp_t prop;
  DM_HIP(hipGetDeviceProperties(&prop, s->cfg.device));
  int max_cn = 0;
  for (const DmSystem& S : s->sys) max_cn = std::max(max_cn, S.chain_nodes);
  char sig[512];
  std::snprintf(sig, sizeof(sig), "dmrod1 %s sys=%d nodes=%d maxcn=%d arms=%d nb=%d dof=%d mode=%d sc=%d", prop.gcnArchName,
                s->n_sys, s->n_nodes, max_cn, s->max_arms, s->max_nb, s->n_dof, s->ws_mode, s->sc_on);
  for (char* c = sig; *c; ++c) if (*c == '\n') *c = ' ';
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      const size_t p = line.rfind(' ');
      if (p != std::string::npos && line.substr(0, p) == sig) {
        const int b = std::atoi(line.c_str() + p + 1);
        if (b >= 64 && b <= 512 && b % 64 == 0) {
          s->block = b;
          s->block_auto = false;
          if (block_out) *block_out = b;
          return DM_OK;
        }
      }
    }
  }
  dm_status st;
  const size_t n = state_doubles(s);
  if ((st = grow(s, &s->tune_ck, &s->tune_ck_n, n)) != DM_OK) return st;
  if ((st = dm_save_checkpoint(s, s->tune_ck, 1)) != DM_OK) return st;
  const double t0 = s->time;
  const int old = s->block;
  int best = old;
  float best_ms = 0.0f;
  for (int b : {64, 128, 256, 512}) {
    if ((st = dm_load_checkpoint(s, s->tune_ck, 1)) != DM_OK) return st;
    s->block = b;
    st = dm_step(s, dt, trial_steps, nullptr);
    if (st == DM_OK && (best_ms == 0.0f || s->last_kernel_ms < best_ms)) { best_ms = s->last_kernel_ms; best = b; }
  }
  if ((st = dm_load_checkpoint(s, s->tune_ck, 1)) != DM_OK) return st;
  s->time = t0;
  s->block = best;
  s->block_auto = false;
  g_err.clear();
  if (cache_path) {
    std::ofstream out(cache_path, std::ios::app);
    if (out) out << sig << ' ' << best << '\n';
  }
  if (block_out) *block_out = best;
  return DM_OK;
}

int dm_num_systems(const dm_sim* s) { return s ? s->n_sys : 0; }
int dm_rod_system(const dm_sim* s, int rod) { return (s && rod >= 0 && rod < (int)s->rod_sys.size()) ? s->rod_sys[rod] : -1; }
int dm_num_rods(const dm_sim* s) { return s ? (int)s->rods.size() : 0; }
int dm_rod_nodes(const dm_sim* s, int rod) { return (s && rod >= 0 && rod < (int)s->rods.size()) ? s->rods[rod].n : -1; }
int dm_num_nodes(const dm_sim* s) { return s ? s->n_nodes : 0; }
int dm_num_edges(const dm_sim* s) { return s ? s->n_edges : 0; }
int dm_node_index(const dm_sim* s, int rod, int node) {
  if (!s || !s->finalized || rod < 0 || rod >= (int)s->rods.size() || node < 0 || node >= s->rods[rod].n) return -1;
  return s->rod_node[rod][node];
}
int dm_edge_index(const dm_sim* s, int rod, int edge) {
  if (!s || !s->finalized || rod < 0 || rod >= (int)s->rods.size() || edge < 0 || edge >= s->rods[rod].n - 1) return -1;
  return s->rod_edge[rod][edge];
}

dm_status dm_get_state(dm_sim* s, double* x, double* th, double* v, double* om, int on_device) {
  if (!s) return fail(DM_ERR_INVALID_ARG, "null sim");
  if (!s->finalized) return fail(DM_ERR_STATE, "dm_get_state before dm_finalize");
  DM_HIP(hipSetDevice(s->cfg.device));
  DM_HIP(hipStreamSynchronize(s->stream));
  const int NN = s->n_nodes, NE = s->n_edges;
  std::vector<double> buf(3 * (size_t)NN);
  auto get3 = [&](const double* src, double* dst) -> dm_status {
    DM_HIP(hipMemcpy(buf.data(), src, sizeof(double) * 3 * NN, hipMemcpyDeviceToHost));
    std::vector<double> aos(3 * (size_t)NN);
    for (int n = 0; n < NN; ++n) for (int c = 0; c < 3; ++c) aos[3 * n + c] = buf[c * NN + n];
    DM_HIP(hipMemcpy(dst, aos.data(), sizeof(double) * 3 * NN, on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
    return DM_OK;
  };
  dm_status st;
  if (x && (st = get3(s->dev.x, x)) != DM_OK) return st;
  if (v && (st = get3(s->dev.v, v)) != DM_OK) return st;
  hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (th) DM_HIP(hipMemcpy(th, s->dev.th, sizeof(double) * NE, k));
  if (om) DM_HIP(hipMemcpy(om, s->dev.om, sizeof(double) * NE, k));
  return DM_OK;
}

dm_status dm_set_state(dm_sim* s, const double* x, const double* th, const double* v, const double* om, int on_device) {
  if (!s) return fail(DM_ERR_INVALID_ARG, "null sim");
  if (!s->finalized) return fail(DM_ERR_STATE, "dm_set_state before dm_finalize");
  DM_HIP(hipSetDevice(s->cfg.device));
  DM_HIP(hipStreamSynchronize(s->stream));
  const int NN = s->n_nodes, NE = s->n_edges;
  auto put3 = [&](const double* src, double* dst, double* dst2, double* dst3) -> dm_status {
    std::vector<double> aos(3 * (size_t)NN), soa(3 * (size_t)NN);
    DM_HIP(hipMemcpy(aos.data(), src, sizeof(double) * 3 * NN, on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
    if (!finite_all(aos.data(), aos.size())) return fail(DM_ERR_INVALID_ARG, "dm_set_state: non-finite value");
    for (int n = 0; n < NN; ++n) for (int c = 0; c < 3; ++c) soa[c * NN + n] = aos[3 * n + c];
    DM_HIP(hipMemcpy(dst, soa.data(), sizeof(double) * 3 * NN, hipMemcpyHostToDevice));
    if (dst2) DM_HIP(hipMemcpy(dst2, soa.data(), sizeof(double) * 3 * NN, hipMemcpyHostToDevice));
    if (dst3) DM_HIP(hipMemcpy(dst3, soa.data(), sizeof(double) * 3 * NN, hipMemcpyHostToDevice));
    return DM_OK;
  };
  dm_status st;
  if (x && (st = put3(x, s->dev.x, s->dev.x0, nullptr)) != DM_OK) return st;
  if (v && (st = put3(v, s->dev.v, s->dev.vprev, s->dev.vprev2)) != DM_OK) return st;
  hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (th) { DM_HIP(hipMemcpy(s->dev.th, th, sizeof(double) * NE, k)); DM_HIP(hipMemcpy(s->dev.th0, th, sizeof(double) * NE, k)); }
  if (om) DM_HIP(hipMemcpy(s->dev.om, om, sizeof(double) * NE, k));
  return DM_OK;
}

dm_status dm_get_rod_state(dm_sim* s, int rod, double* x, double* th, double* v, double* om) {
  dm_status st;
  if ((st = check_rod(s, rod)) != DM_OK) return st;
  if (!s->finalized) return fail(DM_ERR_STATE, "dm_get_rod_state before dm_finalize");
  std::vector<double> X(3 * (size_t)s->n_nodes), V(3 * (size_t)s->n_nodes), T(s->n_edges), O(s->n_edges);
  if ((st = dm_get_state(s, X.data(), T.data(), V.data(), O.data(), 0)) != DM_OK) return st;
  const auto& rn = s->rod_node[rod];
  const auto& re = s->rod_edge[rod];
  for (size_t i = 0; i < rn.size(); ++i) for (int c = 0; c < 3; ++c) {
    if (x) x[3 * i + c] = X[3 * rn[i] + c];
    if (v) v[3 * i + c] = V[3 * rn[i] + c];
  }
  for (size_t j = 0; j < re.size(); ++j) { if (th) th[j] = T[re[j]]; if (om) om[j] = O[re[j]]; }
  return DM_OK;
}

dm_status dm_set_rod_state(dm_sim* s, int rod, const double* x, const double* th, const double* v, const double* om) {
  dm_status st;
  if ((st = check_rod(s, rod)) != DM_OK) return st;
  if (!s->finalized) return fail(DM_ERR_STATE, "dm_set_rod_state before dm_finalize");
  std::vector<double> X(3 * (size_t)s->n_nodes), V(3 * (size_t)s->n_nodes), T(s->n_edges), O(s->n_edges);
  if ((st = dm_get_state(s, X.data(), T.data(), V.data(), O.data(), 0)) != DM_OK) return st;
  const auto& rn = s->rod_node[rod];
  const auto& re = s->rod_edge[rod];
  for (size_t i = 0; i < rn.size(); ++i) for (int c = 0; c < 3; ++c) {
    if (x) X[3 * rn[i] + c] = x[3 * i + c];
    if (v) V[3 * rn[i] + c] = v[3 * i + c];
  }
  for (size_t j = 0; j < re.size(); ++j) { if (th) T[re[j]] = th[j]; if (om) O[re[j]] = om[j]; }
  return dm_set_state(s, X.data(), T.data(), V.data(), O.data(), 0);
}

size_t dm_checkpoint_size(const dm_sim* s) { return s && s->finalized ? state_doubles(s) : 0; }

dm_status dm_save_checkpoint(dm_sim* s, double* buf, int on_device) {
  if (!s || !buf) return fail(DM_ERR_INVALID_ARG, "dm_save_checkpoint: null argument");
  if (!s->finalized) return fail(DM_ERR_STATE, "dm_save_checkpoint before dm_finalize");
  DM_HIP(hipStreamSynchronize(s->stream));
  const size_t NN = s->n_nodes, NE = s->n_edges;
  hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  double* p = buf;
  DM_HIP(hipMemcpy(p, s->dev.x, sizeof(double) * 3 * NN, k)); p += 3 * NN;
  DM_HIP(hipMemcpy(p, s->dev.x0, sizeof(double) * 3 * NN, k)); p += 3 * NN;
  DM_HIP(hipMemcpy(p, s->dev.v, sizeof(double) * 3 * NN, k)); p += 3 * NN;
  DM_HIP(hipMemcpy(p, s->dev.th, sizeof(double) * NE, k)); p += NE;
  DM_HIP(hipMemcpy(p, s->dev.th0, sizeof(double) * NE, k)); p += NE;
  DM_HIP(hipMemcpy(p, s->dev.om, sizeof(double) * NE, k)); p += NE;
  DM_HIP(hipMemcpy(p, s->dev.tref, sizeof(double) * 3 * NE, k)); p += 3 * NE;
  DM_HIP(hipMemcpy(p, s->dev.d1ref, sizeof(double) * 3 * NE, k)); p += 3 * NE;
  DM_HIP(hipMemcpy(p, s->dev.bref, sizeof(double) * s->n_st, k)); p += s->n_st;
  DM_HIP(hipMemcpy(p, s->dev.time, sizeof(double) * s->n_sys, k));
  return DM_OK;
}

dm_status dm_load_checkpoint(dm_sim* s, const double* buf, int on_device) {
  if (!s || !buf) return fail(DM_ERR_INVALID_ARG, "dm_load_checkpoint: null argument");
  if (!s->finalized) return fail(DM_ERR_STATE, "dm_load_checkpoint before dm_finalize");
  DM_HIP(hipStreamSynchronize(s->stream));
  const size_t NN = s->n_nodes, NE = s->n_edges;
  hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const double* p = buf;
  DM_HIP(hipMemcpy(s->dev.x, p, sizeof(double) * 3 * NN, k)); p += 3 * NN;
  DM_HIP(hipMemcpy(s->dev.x0, p, sizeof(double) * 3 * NN, k)); p += 3 * NN;
  DM_HIP(hipMemcpy(s->dev.v, p, sizeof(double) * 3 * NN, k));
  DM_HIP(hipMemcpy(s->dev.vprev, p, sizeof(double) * 3 * NN, k));
  DM_HIP(hipMemcpy(s->dev.vprev2, p, sizeof(double) * 3 * NN, k)); p += 3 * NN;
  DM_HIP(hipMemcpy(s->dev.th, p, sizeof(double) * NE, k)); p += NE;
  DM_HIP(hipMemcpy(s->dev.th0, p, sizeof(double) * NE, k)); p += NE;
  DM_HIP(hipMemcpy(s->dev.om, p, sizeof(double) * NE, k)); p += NE;
  DM_HIP(hipMemcpy(s->dev.tref, p, sizeof(double) * 3 * NE, k)); p += 3 * NE;
  DM_HIP(hipMemcpy(s->dev.d1ref, p, sizeof(double) * 3 * NE, k)); p += 3 * NE;
  DM_HIP(hipMemcpy(s->dev.bref, p, sizeof(double) * s->n_st, k)); p += s->n_st;
  DM_HIP(hipMemcpy(s->dev.time, p, sizeof(double) * s->n_sys, k));
  return DM_OK;
}

double dm_time(const dm_sim* s) { return s ? s->time : 0.0; }

#ifdef DM_PHASE_TIMING
// Diagnosis builds only: per-system phase timers of the last dm_step, [n_systems][8] ticks of
// the 100 MHz wall clock (eval, band, border+norm, sweeps, border solve, back-substitution,
// update, commit).
dm_status dm_debug_phase_times(dm_sim* s, double* out) {
  DM_HIP(hipMemcpy(out, s->dev.dbg, sizeof(double) * 8 * s->n_sys, hipMemcpyDeviceToHost));
  return DM_OK;
}
// Diagnosis builds only: the adjoint arrays after the last dm_adjoint (ax, av, ath, aom,
// atref, ad1, akap, lam, pst, pe in that order); returns their total length.
size_t dm_debug_adjoint_arrays(dm_sim* s, double* out) {
  const size_t na = 9 * (size_t)s->n_nodes + 12 * (size_t)s->n_edges + 18 * (size_t)s->n_st;
  if (out && s->adj) (void)hipMemcpy(out, s->adj, sizeof(double) * na, hipMemcpyDeviceToHost);
  return na;
}
#endif

double dm_last_kernel_ms(const dm_sim* s) { return s ? (double)s->last_kernel_ms : 0.0; }

int dm_block_size(const dm_sim* s) { return s ? s->block : 0; }

const char* dm_last_error(void) { return g_err.c_str(); }

void dm_destroy(dm_sim* s) {
  if (!s) return;
  (void)hipSetDevice(s->cfg.device);
  (void)hipStreamSynchronize(s->stream);
  for (void* p : s->allocs) dev_free(s, p);
  for (double* p : {s->ck, s->seg, s->adj, s->tips_dev, s->dl_dev, s->ws_F, s->tips_stage, s->tune_ck, s->curv_st,
                    s->curv_w, s->curv_mu, s->curv_p, s->skip_buf})
    dev_free(s, p);
  for (SegGraph& c : s->seg_graphs) { (void)hipGraphExecDestroy(c.exec); (void)hipGraphDestroy(c.graph); }
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  if (s->ev0) { (void)hipEventDestroy(s->ev0); (void)hipEventDestroy(s->ev1); }
  delete s;
}

}  // extern "C"
