// dm_kernels.hip -- the implicit DER time step on gfx950, FP64 throughout.
//
// One workgroup advances one system (a rod, or rods joined at a shared end node) for
// `nsteps` backward-Euler steps (Eq. 14-15), each solved by Newton's method (Eq. 16).
// Per Newton iteration:
//   1. element evaluation, one lane per item: bend/twist stencils (Eq. 4-8, exact gradient
//      and Hessian), stretch edges (Eq. 2-3), nodes (inertia, gravity, damping, floor
//      contact Eq. 10-11 and friction Eq. 12-13);
//   2. atomic-free gather assembly: one lane per chain node owns its four band rows and
//      sums the contributions of the elements touching them; border rows are gathered into
//      a small dense matrix in LDS;
//   3. banded LU without pivoting: each arm is eliminated by one wavefront holding an 11x11
//      window, one column per lane (lanes 0..10) plus the right-hand side (lane 11), with
//      the pivot column broadcast by readlane; the arms' Schur complements meet in the dense
//      border, solved with partial pivoting; then each arm back-substitutes;
//   4. q <- q - alpha * delta, with optional step halving (line search).
// After convergence the step is committed: velocity update, reference frames carried to
// the new tangents by time-parallel transport, reference twist recorded for its branch.
#include <hip/hip_runtime.h>
#define DM_KERNEL_TU
#include "dm_layout.h"
#include "dm_math.h"
#include "dm_segment.h"

#ifdef DM_PHASE_TIMING
// Per-phase wall-clock accumulation (100 MHz counter) for diagnosis builds only; every phase
// still runs in full.
#define DM_T0() unsigned long long _t_last = wall_clock64(); unsigned long long _t_acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#define DM_TP(k) do { unsigned long long _n = wall_clock64(); _t_acc[k] += _n - _t_last; _t_last = _n; } while (0)
#define DM_TSAVE(sid) do { if (threadIdx.x == 0 && A.d.dbg) for (int _i = 0; _i < 8; ++_i) A.d.dbg[(sid) * 8 + _i] = (double)_t_acc[_i]; } while (0)
#else
#define DM_T0()
#define DM_TP(k)
#define DM_TSAVE(sid)
#endif

// tangents per stencil task: the stencil Hessian takes 2 x 4 / DM_STENCIL_TANGENTS tasks (one
// tangent per task: the most tasks and the fewest live values per lane)
#ifndef DM_STENCIL_TANGENTS
#define DM_STENCIL_TANGENTS 1
#endif

#define DM_STATUS_OK 0
#define DM_STATUS_NOT_CONVERGED 1
#define DM_STATUS_SINGULAR (-5)
#define DM_STATUS_CONTACT_OVERFLOW (-6)   // more self-contact pairs than the per-system list holds

namespace {

template <class P>
__device__ __forceinline__ v3 ld3(P a, int n, int i) { return mk3(a[i], a[n + i], a[2 * n + i]); }
__device__ __forceinline__ void st3(double DM_G* a, int n, int i, v3 v) { a[i] = v.x; a[n + i] = v.y; a[2 * n + i] = v.z; }

// The step arguments stay in the kernel's argument segment (constant memory) and are reached
// through a pointer that every phase function makes wavefront-uniform, so that their fields
// are scalar loads.
using ArgsP = const DmStepArgs DM_C*;

__device__ __forceinline__ ArgsP uniform(ArgsP p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (ArgsP)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ int uniform(int i) { return __builtin_amdgcn_readfirstlane(i); }

__device__ __forceinline__ double readlane_d(double v, int lane) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ double block_sum(double v, double DM_L* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    red[32] = s;
  }
  __syncthreads();
  return red[32];
}

// ---------------------------------------------------------------------------
// element evaluation
// ---------------------------------------------------------------------------

// One lane-task of a stencil.  rev = 0 evaluates the stencil as stored, rev = 1 with its
// orientation reversed (nodes and edges swapped, edges reversed), which leaves the energy
// unchanged once the second natural-curvature component changes sign, so both run the same
// code; the task seeds NT of the four f-edge variables (e_f.x, e_f.y, e_f.z, theta_f), from
// variable NT * SUB on.  The reversed stencil's f edge is the stored e edge, so its Hessian
// columns are the stored stencil's e-edge columns, reached through the signed permutation
// e_f <-> -e_e, theta_f <-> -theta_e (an even number of sign flips per Hessian entry, so only
// the indices move).  Few tangents per lane keep the pass within the register file.
// WG: the task that seeds the first tangent of the stored orientation also writes the gradient
// (off when a residual pass has already written it).
template <int NT, int SUB, bool WG>
__device__ __forceinline__ void eval_stencil(const DmStepArgs DM_C& A, int s, int rev, double t_end) {
  const DmDev DM_C& D = A.d;
  const int NS = D.n_st_tot, NE = D.n_edges_tot, NN = D.n_nodes_tot;
  int np = D.sn[s], nc = D.sn[NS + s], nn = D.sn[2 * NS + s];
  int ef = D.se[s], ee = D.se[NS + s];
  const int sg = D.ssign[s];
  double sf = (sg & 1) ? -1.0 : 1.0, se = (sg & 2) ? -1.0 : 1.0;
  double k1b = D.kbar[s], k2b = D.kbar[NS + s];
  const double amp = D.act[s];
  if (!isnan(amp)) {   // actuation: kappa1 = A sin(2 pi f t + phi), integrated over Vbar
    k1b = amp * sin(6.283185307179586476925286766559 * D.act[NS + s] * t_end + D.act[2 * NS + s]) * D.Vbar[s];
    k2b = 0.0;
  }
  if (rev) {
    const int tn = np; np = nn; nn = tn;
    const int te = ef; ef = ee; ee = te;
    const double ts = sf; sf = -se; se = -ts;
    k2b = -k2b;
  }
  const v3 xc = ld3(D.x, NN, nc);
  double g8[8], Hf[8][NT];
  stencil_pass_n<NT, NT * SUB>(xc - ld3(D.x, NN, np), ld3(D.x, NN, nn) - xc, sf * D.th[ef], se * D.th[ee],
                             sf * ld3(D.tref, NE, ef), ld3(D.d1ref, NE, ef), se * ld3(D.tref, NE, ee),
                             ld3(D.d1ref, NE, ee), D.bref[s], k1b, k2b, D.tbar[s], D.kbend[s], D.ktwist[s], g8, Hf);
  if (WG && SUB == 0 && !rev) {
#pragma unroll
    for (int a = 0; a < 8; ++a) D.st_g[a * NS + s] = g8[a];
  }
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    // the reversed stencil's variable a is the stored stencil's variable ra
    const int ra = rev ? (a < 3 ? a + 3 : (a < 6 ? a - 3 : 13 - a)) : a;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      const int var = NT * SUB + k;
      const int w = (var < 3 ? var : 6) + (rev ? (var < 3 ? 3 : 1) : 0);
      D.st_H[(ra * 8 + w) * NS + s] = Hf[a][k];
    }
  }
}

// Gradient only of a stencil (the residual pass): the same closed form without tangents.
__device__ __forceinline__ void eval_stencil_grad(const DmStepArgs DM_C& A, int s, double t_end) {
  const DmDev DM_C& D = A.d;
  const int NS = D.n_st_tot, NE = D.n_edges_tot, NN = D.n_nodes_tot;
  const int np = D.sn[s], nc = D.sn[NS + s], nn = D.sn[2 * NS + s];
  const int ef = D.se[s], ee = D.se[NS + s];
  const int sg = D.ssign[s];
  const double sf = (sg & 1) ? -1.0 : 1.0, se = (sg & 2) ? -1.0 : 1.0;
  double k1b = D.kbar[s], k2b = D.kbar[NS + s];
  const double amp = D.act[s];
  if (!isnan(amp)) {   // actuation: kappa1 = A sin(2 pi f t + phi), integrated over Vbar
    k1b = amp * sin(6.283185307179586476925286766559 * D.act[NS + s] * t_end + D.act[2 * NS + s]) * D.Vbar[s];
    k2b = 0.0;
  }
  const v3 xc = ld3(D.x, NN, nc);
  double g8[8];
  stencil_grad_g<double>(tov(xc - ld3(D.x, NN, np)), tov(ld3(D.x, NN, nn) - xc), sf * D.th[ef], se * D.th[ee],
                         tov(sf * ld3(D.tref, NE, ef)), tov(ld3(D.d1ref, NE, ef)), tov(se * ld3(D.tref, NE, ee)),
                         tov(ld3(D.d1ref, NE, ee)), D.bref[s], k1b, k2b, D.tbar[s], D.kbend[s], D.ktwist[s], g8);
#pragma unroll
  for (int a = 0; a < 8; ++a) D.st_g[a * NS + s] = g8[a];
}

// Stretch of one edge (stretch_terms, Eq. 2-3) into the edge scratch.
__device__ __forceinline__ void eval_edge(const DmStepArgs DM_C& A, int e) {
  const DmDev DM_C& D = A.d;
  const int NE = D.n_edges_tot, NN = D.n_nodes_tot;
  double out[9];
  stretch_terms(ld3(D.x, NN, D.en[NE + e]) - ld3(D.x, NN, D.en[e]), D.EA[e], D.ebar[e], out);
#pragma unroll
  for (int k = 0; k < 9; ++k) D.ed[k * NE + e] = out[k];
}

__device__ __forceinline__ double edge_K(const DmDev DM_C& D, int NE, int e, int i, int j) {
  const int a = i < j ? i : j, b = i < j ? j : i;
  const int idx = (a == 0) ? b : (a == 1 ? 2 + b : 5);   // xx xy xz yy yz zz
  return D.ed[(3 + idx) * NE + e];
}

// IMC floor energy profile (Eq. 10): first and second derivative in D, K1 = 15/delta,
// quadratic branch extended below D = 0.
__device__ __forceinline__ void contact_profile(double Dd, double C, double delta, double* e1, double* e2) {
  const double K1 = 15.0 / delta;
  if (Dd <= C - delta) { *e1 = -2.0 * (C - Dd); *e2 = 2.0; }
  else if (Dd < C + delta) {
    double z = K1 * (C - Dd);
    double ez = exp(z);
    double sp = log1p(ez) / K1;
    double sig = ez / (1.0 + ez);
    *e1 = -2.0 * sp * sig;
    *e2 = 2.0 * sig * sig + 2.0 * sp * K1 * sig * (1.0 - sig);
  } else { *e1 = 0.0; *e2 = 0.0; }
}

// gamma(|u|)/|u| of Eq. 12 as a function of s = |u|^2, and its derivative in s; the exact
// limit series is used below s = 1e-8 / K2^2 so that u = 0 is smooth.
__device__ __forceinline__ void friction_ratio(double s, double K2, double* g, double* dg) {
  if (s < 1e-8 / (K2 * K2)) {
    *g = 0.5 * K2 * (1.0 - K2 * K2 * s / 12.0);
    *dg = -K2 * K2 * K2 / 24.0;
  } else {
    double r = sqrt(s);
    double em = exp(-K2 * r);
    double gam = 2.0 / (1.0 + em) - 1.0;
    double gp = 2.0 * K2 * em / ((1.0 + em) * (1.0 + em));
    *g = gam / r;
    *dg = (gp * r - gam) / (2.0 * s * r);
  }
}

// Node terms of the residual (Eq. 15) and Jacobian: inertia, gravity, constant load,
// damping, floor contact (Eq. 10-11) and friction (Eq. 12-13).
__device__ __forceinline__ void eval_node(const DmStepArgs DM_C& A, int n, double dt) {
  const DmDev DM_C& D = A.d;
  const int NN = D.n_nodes_tot;
  const double m = D.mass[n];
  v3 x = ld3(D.x, NN, n), x0 = ld3(D.x0, NN, n), v = ld3(D.v, NN, n), F = ld3(D.force, NN, n);
  const double im = m / (dt * dt);
  double R[3], J[9];
  double xa[3] = {x.x, x.y, x.z}, x0a[3] = {x0.x, x0.y, x0.z}, va[3] = {v.x, v.y, v.z}, Fa[3] = {F.x, F.y, F.z};
  const double jd = im + A.damping * m / dt;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    R[c] = im * (xa[c] - x0a[c] - dt * va[c]) - m * A.g[c] - Fa[c] + A.damping * m * (xa[c] - x0a[c]) / dt;
#pragma unroll
    for (int c2 = 0; c2 < 3; ++c2) J[3 * c + c2] = (c == c2) ? jd : 0.0;
  }
  if (A.floor_on) {
    double e1, e2;
    contact_profile(x.z - A.floor_z, D.radius[n], A.delta, &e1, &e2);
    const double Fn = -A.kc * e1, dFn = -A.kc * e2;     // normal force and d/dz
    R[2] -= Fn;
    J[8] -= dFn;
    if (Fn != 0.0) {
      const double K2 = 15.0 / A.nu;
      double u0 = (x.x - x0.x) / dt, u1 = (x.y - x0.y) / dt;
      double rg, dg;
      friction_ratio(u0 * u0 + u1 * u1, K2, &rg, &dg);
      const double aF = fabs(Fn), sF = Fn > 0.0 ? 1.0 : -1.0;
      const double mu = A.mu;
      // residual gets -F_fr = mu |Fn| ratio u
      R[0] += mu * aF * rg * u0;
      R[1] += mu * aF * rg * u1;
      const double cc = mu * aF / dt;
      J[0] += cc * (rg + 2.0 * dg * u0 * u0);
      J[1] += cc * (2.0 * dg * u0 * u1);
      J[3] += cc * (2.0 * dg * u1 * u0);
      J[4] += cc * (rg + 2.0 * dg * u1 * u1);
      J[2] += mu * sF * dFn * rg * u0;
      J[5] += mu * sF * dFn * rg * u1;
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) D.nd[c * NN + n] = R[c];
#pragma unroll
  for (int k = 0; k < 9; ++k) D.nd[(3 + k) * NN + n] = J[k];
}

// ---------------------------------------------------------------------------
// gather assembly
// ---------------------------------------------------------------------------

// Row L (compile-time local DOF) of a chain stencil's gradient and Hessian, expanded from the
// 8-variable form: local DOF l = sum of coef * variable (loc_terms, orientation +1 in a chain).
// emit(rel0 + b, H_local[L][b]) for b = 0..10; returns g_local[L].  A stencil that does not
// exist (ok false) contributes zero: its loads read stencil 0 (always allocated) and the values
// are dropped by selection, so no load sits behind a branch.
template <int L, class Emit>
__device__ __forceinline__ double stencil_row(const DmDev DM_C& D, int s, bool ok, int rel0, Emit& emit) {
  const int NS = D.n_st_tot;
  s = ok ? s : 0;
  int va[2], vb[2];
  double ca[2], cb[2];
  const int na = loc_terms(L, 1.0, 1.0, va, ca);
  double r8[8];
  double gl = 0.0;
#pragma unroll
  for (int w = 0; w < 8; ++w) r8[w] = 0.0;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    if (t < na) {
      gl += ca[t] * D.st_g[va[t] * NS + s];
#pragma unroll
      for (int w = 0; w < 8; ++w) r8[w] += ca[t] * D.st_H[(va[t] * 8 + w) * NS + s];
    }
  }
#pragma unroll
  for (int b = 0; b < 11; ++b) {
    const int nb = loc_terms(b, 1.0, 1.0, vb, cb);
    double v = cb[0] * r8[vb[0]];
    if (nb > 1) v += cb[1] * r8[vb[1]];
    emit(rel0 + b, ok ? v : 0.0);
  }
  return ok ? gl : 0.0;
}

// Contributions of chain elements to chain row 4k + COMP; emit(rel, value) receives the
// column as rel = column - 4k.  Returns the residual entry.  Every term is loaded (from a valid
// index) and kept or dropped by selection: the terms present depend only on where node k sits
// in its chain and on whether the chain owns the node.
// NE_RES: the residual includes the node and edge terms (off: stencil gradients only).
template <int COMP, bool NE_RES, class Emit>
__device__ __forceinline__ double row_contrib(const DmStepArgs DM_C& A, double dt, const DmChain& ch, int k,
                                              bool own, Emit& emit) {
  const DmDev DM_C& D = A.d;
  const int NE = D.n_edges_tot, NN = D.n_nodes_tot;
  const int N = ch.n_nodes;
  // stencil centred on chain node m (1 <= m <= N-2) is st_off + m - 1
  auto sok = [&](int m) { return (m >= 1) & (m <= N - 2); };
  double Rr = 0.0;
  if (COMP < 3) {
    const int node = D.chain_node[ch.node_tab + k];
    const bool tail = k <= N - 2, head = k >= 1;      // node k is the tail of edge k, head of edge k-1
    const int et = D.chain_edge[ch.edge_tab + (tail ? k : N - 2)];
    const int eh = D.chain_edge[ch.edge_tab + (head ? k - 1 : 0)];
    const double rn = D.nd[COMP * NN + node];
    if (NE_RES) Rr += own ? rn : 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double v = D.nd[(3 + 3 * COMP + c) * NN + node];
      emit(c, own ? v : 0.0);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double Kt = edge_K(D, NE, et, COMP, c), Kh = edge_K(D, NE, eh, COMP, c);
      const double kt = tail ? Kt : 0.0, kh = head ? Kh : 0.0;
      emit(c, kt + kh);
      emit(4 + c, -kt);
      emit(-4 + c, -kh);
    }
    const double ft = D.ed[COMP * NE + et], fh = D.ed[COMP * NE + eh];
    if (NE_RES) Rr += (head ? fh : 0.0) - (tail ? ft : 0.0);
    // stencils centred on nodes k-1, k, k+1 (node k is their next, centre, previous node)
    Rr += stencil_row<8 + COMP>(D, ch.st_off + k - 2, sok(k - 1), -8, emit);
    Rr += stencil_row<4 + COMP>(D, ch.st_off + k - 1, sok(k), -4, emit);
    Rr += stencil_row<COMP>(D, ch.st_off + k, sok(k + 1), 0, emit);
  } else {
    const int e = D.chain_edge[ch.edge_tab + k];
    const double I = D.Ith[e] / (dt * dt);
    emit(3, I);
    if (NE_RES) Rr += I * (D.th[e] - D.th0[e] - dt * D.om[e]) - D.moment[e];
    Rr += stencil_row<7>(D, ch.st_off + k - 1, sok(k), -4, emit);
    Rr += stencil_row<3>(D, ch.st_off + k, sok(k + 1), 0, emit);
  }
  return Rr;
}

// Band row 4k + COMP.  Contributions are summed per diagonal first; clamped columns, and
// border columns of a border row (those couplings live in the dense border), are zeroed
// afterwards.  fixmask / bmask: bit i describes chain DOF 4k - 12 + i.
// MODE 0: matrix row and residual entry; 1: the residual entry only (the element terms not
// read are never loaded); 2: the matrix row only; 3: the residual entry from the stencil
// gradients alone (a right-hand side built from per-stencil vectors in st_g).
template <int COMP, int MODE>
__device__ __forceinline__ double band_row(const DmStepArgs DM_C& A, double dt, const DmChain& ch, int k,
                                           unsigned fixmask, unsigned bmask, bool own) {
  const int r = 4 * k + COMP;
  const bool rowb = (bmask >> (12 + COMP)) & 1u;
  const bool rowfix = (fixmask >> (12 + COMP)) & 1u;
  double acc[DM_NDIAG];
#pragma unroll
  for (int o = 0; o < DM_NDIAG; ++o) acc[o] = 0.0;
  auto emit = [&](int rel, double v) { acc[rel - COMP + 10] += v; };
  double Rr = row_contrib<COMP, MODE != 3>(A, dt, ch, k, own, emit);
  if (MODE != 1 && MODE != 3 && rowb && !rowfix) {
    // the border-block part of a border row goes to the dense border (assemble_border)
    double DM_G* bp = A.d.bpr + (size_t)(ch.bmap_off + r - ch.b_lo) * DM_NDIAG;
#pragma unroll
    for (int o = 0; o < DM_NDIAG; ++o) {
      const unsigned bit = 1u << (COMP + 2 + o);
      bp[o] = ((bmask & bit) && !(fixmask & bit)) ? acc[o] : 0.0;
    }
  }
  const unsigned drop = fixmask | (rowb ? bmask : 0u);
#pragma unroll
  for (int o = 0; o < DM_NDIAG; ++o) {
    // column r - 10 + o is chain DOF 4k - 12 + (COMP + 2 + o)
    if ((drop >> (COMP + 2 + o)) & 1u) acc[o] = 0.0;
  }
  if (rowfix) {
#pragma unroll
    for (int o = 0; o < DM_NDIAG; ++o) acc[o] = (o == 10) ? 1.0 : 0.0;
    Rr = 0.0;
  }
  if (MODE != 1 && MODE != 3) {
    double DM_G* out = A.d.band + (size_t)(ch.dof_off + r) * DM_NDIAG;
#pragma unroll
    for (int o = 0; o < DM_NDIAG; ++o) out[o] = acc[o];
  }
  if (MODE == 2) return 0.0;
  A.d.R[ch.dof_off + r] = Rr;
  return (rowfix || rowb) ? 0.0 : Rr * Rr;
}

// Band rows of chain node k (4 rows; 3 for the last node).  Returns the squared residual of
// its free, non-border rows.
template <int MODE>
__device__ __forceinline__ double band_node(const DmStepArgs DM_C& A, double dt, int ci, int k) {
  const DmDev DM_C& D = A.d;
  const DmChain ch = D.chain[ci];
  const uint4 m = *(const uint4 DM_C*)(D.nmask + 4 * (size_t)(ch.node_tab + k));
  const bool own = m.z & 1u;
  double s = band_row<0, MODE>(A, dt, ch, k, m.x, m.y, own);
  s += band_row<1, MODE>(A, dt, ch, k, m.x, m.y, own);
  s += band_row<2, MODE>(A, dt, ch, k, m.x, m.y, own);
  if (k < ch.n_nodes - 1) s += band_row<3, MODE>(A, dt, ch, k, m.x, m.y, own);
  return s;
}

#include "dm_warm.h"

// Phase drivers: each loops over its items with the whole workgroup, so that the cost of a
// call is paid once per phase.

// Stencil tasks: 64 consecutive stencils per wavefront and task kind (two orientations x
// 4 / DM_STENCIL_TANGENTS tangent groups), so that a wavefront never mixes kinds.
template <bool WG>
__device__ __noinline__ void eval_stencils(ArgsP Ap, int sid, double t_end) {
  const DmStepArgs DM_C& A = *uniform(Ap);
  const DmSystem DM_C& S = A.d.sys[uniform(sid)];
  constexpr int NT = DM_STENCIL_TANGENTS, NSUB = 4 / NT, NTASK = 2 * NSUB;
  for (int i = threadIdx.x; i < 64 * NTASK * ((S.n_st + 63) >> 6); i += blockDim.x) {
    const int st = (i / (64 * NTASK)) * 64 + (i & 63);
    const int p = (i >> 6) % NTASK;      // orientation p / NSUB, tangent group p % NSUB
    if (st < S.n_st) {
      const int rev = p / NSUB, sub = p % NSUB;
      if (NSUB == 1) eval_stencil<NT, 0, WG>(A, S.st0 + st, rev, t_end);
      else if (sub == 0) eval_stencil<NT, 0, WG>(A, S.st0 + st, rev, t_end);
      else if (NSUB == 2 || sub == 1) eval_stencil<NT, (NSUB > 1 ? 1 : 0), WG>(A, S.st0 + st, rev, t_end);
      else if (sub == 2) eval_stencil<NT, (NSUB > 2 ? 2 : 0), WG>(A, S.st0 + st, rev, t_end);
      else eval_stencil<NT, (NSUB > 3 ? 3 : 0), WG>(A, S.st0 + st, rev, t_end);
    }
  }
}

// Stencil gradients only (the residual pass), one lane per stencil.
__device__ __noinline__ void eval_stencil_grads(ArgsP Ap, int sid, double t_end) {
  const DmStepArgs DM_C& A = *uniform(Ap);
  const DmSystem DM_C& S = A.d.sys[uniform(sid)];
  for (int i = threadIdx.x; i < S.n_st; i += blockDim.x) eval_stencil_grad(A, S.st0 + i, t_end);
}


// dt: the Newton step of the (sub)step being solved.
__device__ __noinline__ void eval_edges_nodes(ArgsP Ap, int sid, double dt) {
  const DmStepArgs DM_C& A = *uniform(Ap);
  const DmSystem DM_C& S = A.d.sys[uniform(sid)];
  for (int i = threadIdx.x; i < S.n_edges; i += blockDim.x) eval_edge(A, S.edge0 + i);
  for (int i = threadIdx.x; i < S.n_nodes; i += blockDim.x) eval_node(A, S.node0 + i, dt);
}

// LDS operations of a wavefront stay in program order: this keeps the compiler from moving
// them across (the hardware runs one wavefront's LDS instructions in order).
__device__ __forceinline__ void lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// edge-edge self-contact of a single rod (Contact and Friction subsection: Eq. 10-13 applied
// to pairs of the rod's edges)
// ---------------------------------------------------------------------------

// E_c'(D) and E_c''(D) of Eq. 10 (K1 = 15 / delta).
__device__ __forceinline__ void sc_profile(double D, double C, double delta, double& E1, double& E2) {
  if (D <= C - delta) {
    E1 = -2.0 * (C - D);
    E2 = 2.0;
  } else if (D < C + delta) {
    const double K1 = 15.0 / delta, z = K1 * (C - D);
    const double L = log1p(exp(z)), sg = 1.0 / (1.0 + exp(-z));
    E1 = -2.0 * L * sg / K1;
    E2 = 2.0 * (sg * sg + L * sg * (1.0 - sg));
  } else {
    E1 = E2 = 0.0;
  }
}

__device__ __forceinline__ float sc_down(double v) {
  const float f = (float)v;
  return (double)f > v ? nextafterf(f, -INFINITY) : f;
}
__device__ __forceinline__ float sc_up(double v) {
  const float f = (float)v;
  return (double)f < v ? nextafterf(f, INFINITY) : f;
}

// Blocked LU of the self-contact solve: the widest panel (the launch's sc_pb, 8 or 16, is what
// its LDS holds) and the largest half bandwidth the LDS panel takes
constexpr int SC_PBMAX = 16, SC_WPANEL = 128;

// One pair of a rod's edges at the current iterate: the nodes of its roles (edge i's nodes a, b,
// edge j's nodes c, d), the closest-point parameters (s, t), r = P(s) - Q(t), the edge vectors,
// D, the contact profile's E_c' and E_c'', the inverse of f_zz over the free parameters and, with
// friction, the slip quantities of Eq. 12-13 at (s, t).
struct ScPair {
  int node[4];
  double s, t, r[3], u[3], v[3], Dd, invD, E1, E2, M00, M01, M11;
  bool fric;
  double un, ut[3], vr[3], u0[3], v0[3];
};

__device__ __forceinline__ void sc_pair(const DmDev DM_C& D, const DmChain& ch, int key, double delta, double mu,
                                        ScPair& P) {
  const int NN = D.n_nodes_tot, i = key >> 16, j = key & 0xffff;
  P.node[0] = D.chain_node[ch.node_tab + i];
  P.node[1] = D.chain_node[ch.node_tab + i + 1];
  P.node[2] = D.chain_node[ch.node_tab + j];
  P.node[3] = D.chain_node[ch.node_tab + j + 1];
  const v3 pa = ld3(D.x, NN, P.node[0]), pb = ld3(D.x, NN, P.node[1]);
  const v3 pc = ld3(D.x, NN, P.node[2]), pd = ld3(D.x, NN, P.node[3]);
  const double p1[3] = {pa.x, pa.y, pa.z}, p2[3] = {pc.x, pc.y, pc.z};
  P.u[0] = pb.x - pa.x; P.u[1] = pb.y - pa.y; P.u[2] = pb.z - pa.z;
  P.v[0] = pd.x - pc.x; P.v[1] = pd.y - pc.y; P.v[2] = pd.z - pc.z;
  P.Dd = sqrt(seg_closest(p1, P.u, p2, P.v, P.s, P.t, P.r));
  P.invD = P.Dd > 0.0 ? 1.0 / P.Dd : 0.0;
  sc_profile(P.Dd, D.radius[P.node[0]] + D.radius[P.node[2]], delta, P.E1, P.E2);
  const bool fs = P.s > 0.0 && P.s < 1.0, ft = P.t > 0.0 && P.t < 1.0;
  const double zss = seg_dot(P.u, P.u), ztt = seg_dot(P.v, P.v), zst = -seg_dot(P.u, P.v);
  P.M00 = P.M01 = P.M11 = 0.0;
  if (fs && ft) {
    const double det = zss * ztt - zst * zst;
    P.M00 = ztt / det;
    P.M11 = zss / det;
    P.M01 = -zst / det;
  } else if (fs) {
    P.M00 = 1.0 / zss;
  } else if (ft) {
    P.M11 = 1.0 / ztt;
  }
  P.fric = mu > 0.0 && P.E1 != 0.0 && P.Dd > 0.0;
  P.un = 0.0;
  if (P.fric) {
    const v3 qa = ld3(D.x0, NN, P.node[0]), qb = ld3(D.x0, NN, P.node[1]);
    const v3 qc = ld3(D.x0, NN, P.node[2]), qd = ld3(D.x0, NN, P.node[3]);
    const double pn[3][4] = {{qa.x, qb.x, qc.x, qd.x}, {qa.y, qb.y, qc.y, qd.y}, {qa.z, qb.z, qc.z, qd.z}};
#pragma unroll
    for (int al = 0; al < 3; ++al) {
      const double Pn = pn[al][0] + P.s * (pn[al][1] - pn[al][0]), Qn = pn[al][2] + P.t * (pn[al][3] - pn[al][2]);
      P.vr[al] = P.r[al] - (Pn - Qn);       // the slip over the step; divided by dt where used
      P.u0[al] = pn[al][1] - pn[al][0];     // the edges at the step start
      P.v0[al] = pn[al][3] - pn[al][2];
    }
    const double vn = seg_dot(P.vr, P.r) * P.invD * P.invD;
#pragma unroll
    for (int al = 0; al < 3; ++al) P.ut[al] = P.vr[al] - vn * P.r[al];
    P.un = sqrt(seg_dot(P.ut, P.ut));
  }
}

// Closest-point weight of role k, and this role's block of D_x and of f_xs, f_xt.
__device__ __forceinline__ double sc_role(const ScPair& P, int k, double gD[3], double Gs[3], double Gt[3]) {
  const double w = k == 0 ? 1.0 - P.s : (k == 1 ? P.s : (k == 2 ? -(1.0 - P.t) : -P.t));
#pragma unroll
  for (int al = 0; al < 3; ++al) {
    gD[al] = w * P.r[al] * P.invD;
    Gs[al] = (k == 0 ? -P.r[al] : (k == 1 ? P.r[al] : 0.0)) + w * P.u[al];
    Gt[al] = (k == 2 ? P.r[al] : (k == 3 ? -P.r[al] : 0.0)) - w * P.v[al];
  }
  return w;
}

// Block (rows of role k, columns of role l) of the pair's Jacobian: the contact energy's
// Hessian k_c (E_c'' D_x D_x^T + E_c' D_xx), D_xx = (F_xx - D_x D_x^T) / D with
// F_xx = f_xx - f_xz f_zz^-1 f_zx over the free parameters, and the derivative of the friction
// term: with rho = mu F_n gamma(|u|) u_hat the friction residual of role k is w_k rho,
// F_n = k_c |E_c'|, u = P_t vr / dt (vr here the slip over the step), so at fixed (s, t)
// d(w_k rho)/dx_l = w_k (mu F_n K du/dx_l + mu gamma u_hat dF_n/dx_l), K = d(gamma u_hat)/du,
// du/dx_l = w_l (P_t / dt - (n (P_t vr)^T + (vr.n) P_t) / (D dt)); the closest-point
// parameters move with the nodes, dz/dx_l = -f_zz^-1 f_zx_l over the free ones, which adds
// d(w_k rho)/dz dz/dx_l (D is stationary in z, so F_n is not).
__device__ __forceinline__ void sc_block(const ScPair& P, int k, int l, double kc, double mu, double K2, double dt,
                                         double H[3][3]) {
  double gk[3], sk[3], tk[3], gl[3], sl[3], tl[3];
  const double wk = sc_role(P, k, gk, sk, tk), wl = sc_role(P, l, gl, sl, tl);
#pragma unroll
  for (int al = 0; al < 3; ++al) {
    const double Ws = sk[al] * P.M00 + tk[al] * P.M01, Wt = sk[al] * P.M01 + tk[al] * P.M11;
#pragma unroll
    for (int be = 0; be < 3; ++be) {
      const double fxx = al == be ? wk * wl : 0.0;
      H[al][be] = kc * P.E2 * gk[al] * gl[be] + kc * P.E1 * P.invD * (fxx - (Ws * sl[be] + Wt * tl[be]) - gk[al] * gl[be]);
    }
  }
  if (!P.fric) return;
  const double Fn = kc * fabs(P.E1), idt = 1.0 / dt;
  const double u = P.un * idt;                       // |u|, the tangential slip velocity
  double n[3], uh[3], Kf[3][3], Q[3][3];
#pragma unroll
  for (int al = 0; al < 3; ++al) {
    n[al] = P.r[al] * P.invD;
    uh[al] = u > 0.0 ? P.ut[al] / P.un : 0.0;
  }
  const double z = 0.5 * K2 * u, th = tanh(z);
  const double gam = th;                             // gamma(u) = tanh(K2 u / 2)
  const double gp = 0.5 * K2 * (1.0 - th * th);      // gamma'(u)
  const double gu = u > 0.0 ? th / u : 0.5 * K2;     // gamma(u) / u
  const double vn = seg_dot(P.vr, n) * idt;
  double ptv[3];                                     // P_t vr / dt
#pragma unroll
  for (int al = 0; al < 3; ++al) ptv[al] = P.vr[al] * idt - vn * n[al];
#pragma unroll
  for (int al = 0; al < 3; ++al)
#pragma unroll
    for (int be = 0; be < 3; ++be) {
      const double id = al == be ? 1.0 : 0.0, Pt = id - n[al] * n[be];
      Kf[al][be] = u > 0.0 ? gp * uh[al] * uh[be] + gu * (id - uh[al] * uh[be]) : gu * id;
      Q[al][be] = Pt * idt - (n[al] * ptv[be] + vn * Pt) * P.invD;
    }
  const double c1 = wk * wl * mu * Fn, c2 = -wk * mu * gam * kc * P.E2;
#pragma unroll
  for (int al = 0; al < 3; ++al)
#pragma unroll
    for (int be = 0; be < 3; ++be) {
      const double kq = Kf[al][0] * Q[0][be] + Kf[al][1] * Q[1][be] + Kf[al][2] * Q[2][be];
      H[al][be] += c1 * kq + c2 * uh[al] * gl[be];
    }
  // through (s, t): du/ds and du/dt at fixed nodes
  double du[3], dv[3], nu_ = 0.0, nv_ = 0.0, nu0 = 0.0, nv0 = 0.0;
#pragma unroll
  for (int al = 0; al < 3; ++al) {
    du[al] = P.u[al] - P.u0[al];
    dv[al] = P.v[al] - P.v0[al];
    nu_ += n[al] * P.u[al];
    nv_ += n[al] * P.v[al];
    nu0 += n[al] * du[al];
    nv0 += n[al] * dv[al];
  }
  const double pu = seg_dot(ptv, P.u), pv = seg_dot(ptv, P.v);
  double dus[3], dut[3];
#pragma unroll
  for (int al = 0; al < 3; ++al) {
    dus[al] = (du[al] - n[al] * nu0) * idt - (n[al] * pu + vn * (P.u[al] - n[al] * nu_)) * P.invD;
    dut[al] = -(dv[al] - n[al] * nv0) * idt + (n[al] * pv + vn * (P.v[al] - n[al] * nv_)) * P.invD;
  }
  const double dws = k == 0 ? -1.0 : (k == 1 ? 1.0 : 0.0), dwt = k == 2 ? 1.0 : (k == 3 ? -1.0 : 0.0);
  double dRs[3], dRt[3], dsx[3], dtx[3];
#pragma unroll
  for (int al = 0; al < 3; ++al) {
    const double rho = mu * Fn * gam * uh[al];
    dRs[al] = dws * rho + wk * mu * Fn * (Kf[al][0] * dus[0] + Kf[al][1] * dus[1] + Kf[al][2] * dus[2]);
    dRt[al] = dwt * rho + wk * mu * Fn * (Kf[al][0] * dut[0] + Kf[al][1] * dut[1] + Kf[al][2] * dut[2]);
    dsx[al] = -(P.M00 * sl[al] + P.M01 * tl[al]);
    dtx[al] = -(P.M01 * sl[al] + P.M11 * tl[al]);
  }
#pragma unroll
  for (int al = 0; al < 3; ++al)
#pragma unroll
    for (int be = 0; be < 3; ++be) H[al][be] += dRs[al] * dsx[be] + dRt[al] * dtx[be];
}

// The rod's pair area: after its n x n Newton matrix and n doubles, SC_PAIR doubles per pair
// slot (the residual terms of the pair's four nodes, then its 12 x 12 Jacobian, row-major).
constexpr int SC_PAIR = 12 + 144;
__device__ __forceinline__ double DM_G* sc_pair_area(const DmDev DM_C& D, int sid, int N) {
  const size_t n = 4 * (size_t)N - 1;
  return D.sc_mat + D.sc_off[sid] + n * n + n;
}

// Each node's pairs for the gathers: SC_SLOTS ints per node (pair slot << 2 | role) and then
// a count per node, over the solve's vector and multiplier area (unused until its LU).
constexpr int SC_SLOTS = 14;
__device__ __forceinline__ int DM_L* sc_node_lists(char DM_L* sc_lds, int ME, int cap) {
  return (int DM_L*)(sc_lds + 24 * (size_t)ME + 4 * (size_t)cap + 16);
}

// Self-contact of the rod of system sid at the current iterate.  The pairs of its edges within
// reach, D < h_i + h_j + delta, are found over all pairs i < j by a test of boxes inflated by
// h + delta / 2 (rounded outward to float32 in LDS), the rest-arclength exclusion (edges closer
// than h_i + h_j + delta along the rest rod are never a pair) and the exact segment distance,
// and sorted in LDS; the sorted list stays in LDS for the Newton solve of the same iterate
// (sc_solve).  Each pair's residual terms and 12 x 12 Jacobian are then computed once, one lane
// per pair, into the rod's pair area, and each node's pairs are listed in LDS; each node adds,
// over its pairs, the contact energy's gradient minus the friction force to its residual terms,
// and its own 3 x 3 block of the pair Jacobian to its Jacobian block; sc_solve adds the blocks
// between different nodes.
// LDS (at A.sc_lds): box [6][sc_max_edges] floats, keys [sc_cap] ints, four ints (pair count,
// half bandwidth), then sc_solve's vectors (the node lists until its LU); an overflow sets
// flags[1].
__device__ __noinline__ void self_contact(ArgsP Ap, int sid, double dt, int DM_L* flags) {
  const DmStepArgs DM_C& A = *uniform(Ap);
  extern __shared__ double lds_raw[];
  char DM_L* sc_lds = (char DM_L*)lds_raw + A.sc_lds;
  const DmDev DM_C& D = A.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  const DmChain ch = D.chain[S.chain0];
  const int N = ch.n_nodes, E = N - 1, NN = D.n_nodes_tot, ME = A.sc_max_edges, cap = A.sc_cap;
  float DM_L* box = (float DM_L*)sc_lds;
  int DM_L* keys = (int DM_L*)(box + 6 * ME);
  int DM_L* cnt = keys + cap;
  const double delta = A.sc_delta;
  const int tid = threadIdx.x, bd = blockDim.x;
  if (tid == 0) cnt[0] = 0;
  for (int e = tid; e < E; e += bd) {
    const int a = D.chain_node[ch.node_tab + e], b = D.chain_node[ch.node_tab + e + 1];
    const v3 pa = ld3(D.x, NN, a), pb = ld3(D.x, NN, b);
    const double inf = D.radius[a] + 0.5 * delta;
    box[e] = sc_down(fmin(pa.x, pb.x) - inf);
    box[ME + e] = sc_down(fmin(pa.y, pb.y) - inf);
    box[2 * ME + e] = sc_down(fmin(pa.z, pb.z) - inf);
    box[3 * ME + e] = sc_up(fmax(pa.x, pb.x) + inf);
    box[4 * ME + e] = sc_up(fmax(pa.y, pb.y) + inf);
    box[5 * ME + e] = sc_up(fmax(pa.z, pb.z) + inf);
  }
  __syncthreads();
  for (int p = tid; p < E * E; p += bd) {
    const int i = p / E, j = p - i * E;
    if (j <= i) continue;
    if (box[j] > box[3 * ME + i] || box[i] > box[3 * ME + j] || box[ME + j] > box[4 * ME + i] ||
        box[ME + i] > box[4 * ME + j] || box[2 * ME + j] > box[5 * ME + i] || box[2 * ME + i] > box[5 * ME + j])
      continue;
    const int ei = D.chain_edge[ch.edge_tab + i], ej = D.chain_edge[ch.edge_tab + j];
    const int a = D.chain_node[ch.node_tab + i], c = D.chain_node[ch.node_tab + j];
    const double reach = D.radius[a] + D.radius[c] + delta;
    if (D.arc0[ej] - D.arc0[ei] - D.ebar[ei] < reach) continue;      // near along the rest rod
    const int b = D.chain_node[ch.node_tab + i + 1], d = D.chain_node[ch.node_tab + j + 1];
    const v3 pa = ld3(D.x, NN, a), pb = ld3(D.x, NN, b), pc = ld3(D.x, NN, c), pd = ld3(D.x, NN, d);
    const double p1[3] = {pa.x, pa.y, pa.z}, d1[3] = {pb.x - pa.x, pb.y - pa.y, pb.z - pa.z};
    const double p2[3] = {pc.x, pc.y, pc.z}, d2[3] = {pd.x - pc.x, pd.y - pc.y, pd.z - pc.z};
    double sv, tv, r[3];
    if (seg_closest(p1, d1, p2, d2, sv, tv, r) < reach * reach) {
      const int k = atomicAdd(cnt, 1);
      if (k < cap) keys[k] = (i << 16) | j;
    }
  }
  __syncthreads();
  int np = cnt[0];
  if (np > cap) {
    if (tid == 0) flags[1] = 1;
    np = cap;
  }
  int n2 = 1;
  while (n2 < np) n2 <<= 1;
  for (int k = np + tid; k < n2; k += bd) keys[k] = 0x7fffffff;
  __syncthreads();
  // bitonic sort of the keys (fixed order, so the node sums below do not depend on timing)
  for (int k = 2; k <= n2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < n2; i += bd) {
        const int q = i ^ j;
        if (q > i) {
          const int u = keys[i], w = keys[q];
          if (((i & k) == 0) ? (u > w) : (u < w)) {
            keys[i] = w;
            keys[q] = u;
          }
        }
      }
      __syncthreads();
    }
  // each node's pairs (slot and role, in the list's order) into LDS, for the gathers below
  // and in sc_solve: SC_SLOTS per node, a longer list is walked over all pairs instead
  int DM_L* nl = sc_node_lists(sc_lds, ME, cap);
  int DM_L* ncount = nl + (ME + 1) * SC_SLOTS;
  for (int k = tid; k < N; k += bd) {
    int c = 0;
    for (int q = 0; q < np; ++q) {
      const int key = keys[q], i = key >> 16, j = key & 0xffff;
      const int role = k == i ? 0 : (k == i + 1 ? 1 : (k == j ? 2 : (k == j + 1 ? 3 : -1)));
      if (role < 0) continue;
      if (c < SC_SLOTS) nl[k * SC_SLOTS + c] = (q << 2) | role;
      ++c;
    }
    ncount[k] = c;
  }
  // each pair once, one lane per pair: its residual terms for its four nodes and its 12 x 12
  // Jacobian, to the rod's pair area in HBM (SC_PAIR doubles per pair)
  const double kc = A.sc_kc, mu = A.sc_mu, K2 = 15.0 / A.sc_nu;
  double DM_G* pr = sc_pair_area(D, sid, N);
  for (int q = tid; q < np; q += bd) {
    ScPair P;
    sc_pair(D, ch, keys[q], delta, mu, P);
    double DM_G* o = pr + (size_t)q * SC_PAIR;
    for (int k = 0; k < 4; ++k) {
      double gD[3], Gs[3], Gt[3];
      const double w = sc_role(P, k, gD, Gs, Gt);
      double g[3];
#pragma unroll
      for (int al = 0; al < 3; ++al) g[al] = kc * P.E1 * gD[al];
      if (P.fric && P.un > 0.0) {
        // friction on edge i (Eq. 12-13): u the tangential relative velocity of the closest
        // points over the step at (s, t); edge j takes the opposite force
        const double un = P.un / dt;
        const double gamma = 2.0 / (1.0 + exp(-K2 * un)) - 1.0;
        const double m = -mu * gamma * kc * fabs(P.E1) / un;
#pragma unroll
        for (int al = 0; al < 3; ++al) g[al] -= w * m * (P.ut[al] / dt);      // residual: minus the force
      }
#pragma unroll
      for (int al = 0; al < 3; ++al) o[3 * k + al] = g[al];
      for (int l = 0; l < 4; ++l) {
        double B[3][3];
        sc_block(P, k, l, kc, mu, K2, dt, B);
#pragma unroll
        for (int al = 0; al < 3; ++al)
#pragma unroll
          for (int be = 0; be < 3; ++be) o[12 + (3 * k + al) * 12 + 3 * l + be] = B[al][be];
      }
    }
  }
  __syncthreads();
  // each node sums its pairs' terms in the list's order (so the sums do not depend on timing):
  // the residual terms and its own block
  for (int k = tid; k < N; k += bd) {
    double g[3] = {0.0, 0.0, 0.0}, H[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    const int cnk = ncount[k], walk = cnk <= SC_SLOTS ? cnk : np;
    for (int e = 0; e < walk; ++e) {
      int q, role;
      if (cnk <= SC_SLOTS) {
        q = nl[k * SC_SLOTS + e] >> 2;
        role = nl[k * SC_SLOTS + e] & 3;
      } else {
        const int key = keys[e], i = key >> 16, j = key & 0xffff;
        q = e;
        role = k == i ? 0 : (k == i + 1 ? 1 : (k == j ? 2 : (k == j + 1 ? 3 : -1)));
        if (role < 0) continue;
      }
      const double DM_G* o = pr + (size_t)q * SC_PAIR;
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        g[al] += o[3 * role + al];
#pragma unroll
        for (int be = 0; be < 3; ++be) H[al][be] += o[12 + (3 * role + al) * 12 + 3 * role + be];
      }
    }
    const int n0 = D.chain_node[ch.node_tab + k];
#pragma unroll
    for (int al = 0; al < 3; ++al) {
      D.nd[al * NN + n0] += g[al];
#pragma unroll
      for (int be = 0; be < 3; ++be) D.nd[(3 + 3 * al + be) * NN + n0] += H[al][be];
    }
  }
}

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// LU without pivoting of a panel of b <= SC_PBMAX columns and R <= blockDim.x rows, held in LDS
// column by column (pan[c * RP + i]): thread tid keeps row tid in registers, and a row goes
// back to LDS once it is final, so that pivot q reads row q there; one barrier per pivot.  The
// pivot guard is the band solve's (a pivot below 1e-12 of its assembled diagonal dg, or not
// finite): returns true, in every thread, when a pivot failed it (the later pivots still run,
// on values the caller discards).  Otherwise pan holds the factorised panel, U on and above
// the diagonal and the multipliers below it.  The pivot loop has no early exit, so that it
// unrolls and the row stays in registers.
__device__ __forceinline__ bool sc_panel(double DM_L* pan, const double DM_G* dg, int b, int R, int tid) {
  constexpr int RP = SC_WPANEL + SC_PBMAX;
  const bool mine = tid < R;
  double row[SC_PBMAX], guard[SC_PBMAX];
#pragma unroll
  for (int c = 0; c < SC_PBMAX; ++c) {
    row[c] = mine && c < b ? pan[c * RP + tid] : 0.0;
    guard[c] = c < b ? 1e-12 * fabs(dg[c]) : 0.0;     // loaded once, not after each barrier
  }
  bool bad = false;
#pragma unroll
  for (int q = 0; q < SC_PBMAX; ++q) {
    if (q < b) {
      __syncthreads();                 // row q is final in LDS (row 0 as loaded)
      const double p = pan[q * RP + q];
      bad = bad || !(fabs(p) > guard[q]) || !isfinite(p);
      const double inv = 1.0 / p;
      double pr[SC_PBMAX];
#pragma unroll
      for (int c = q + 1; c < SC_PBMAX; ++c) pr[c] = c < b ? pan[c * RP + q] : 0.0;
      if (mine && tid > q) {
        const double l = row[q] * inv;
        row[q] = l;
#pragma unroll
        for (int c = q + 1; c < SC_PBMAX; ++c) row[c] -= l * pr[c];
        if (tid == q + 1 && tid < b) {
#pragma unroll
          for (int c = 0; c < SC_PBMAX; ++c)
            if (c < b) pan[c * RP + tid] = row[c];
        }
      }
    }
  }
  if (mine && tid >= b) {               // the rows below the panel's top: their multipliers
#pragma unroll
    for (int c = 0; c < SC_PBMAX; ++c)
      if (c < b) pan[c * RP + tid] = row[c];
  }
  __syncthreads();
  return bad;
}

// Newton step of a rod with self-contact.  The rod's Jacobian, its band (the border rows'
// border columns included) plus the blocks between the different nodes of every pair, goes to
// the system's dense n x n matrix over the half bandwidth w the pairs need (at least the
// band's 10); LU without pivoting over that band (the pivot guard of the band solve: a pivot
// below 1e-12 of its assembled diagonal, or not finite, sets the singular flag), forward and
// back substitution, and the step goes to the delta and border-solution slots the update
// reads.  Called by the whole workgroup after the matrix pass of the iterate whose
// pairs self_contact left in LDS.
__device__ __noinline__ void sc_solve(ArgsP Ap, int sid, double dt, double DM_L* xB, int DM_L* flags) {
  const DmStepArgs DM_C& A = *uniform(Ap);
  extern __shared__ double lds_raw[];
  char DM_L* sc_lds = (char DM_L*)lds_raw + A.sc_lds;
  const DmDev DM_C& D = A.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  const DmChain ch = D.chain[S.chain0];
  const int N = ch.n_nodes, n = 4 * N - 1, ME = A.sc_max_edges, cap = A.sc_cap, NN = D.n_nodes_tot;
  int DM_L* keys = (int DM_L*)(sc_lds + 24 * (size_t)ME);
  int DM_L* cnt = keys + cap;
  double DM_L* y = (double DM_L*)(cnt + 4);
  double DM_L* lcol = y + (4 * ME + 3);
  double DM_G* M = D.sc_mat + D.sc_off[uniform(sid)];
  double DM_G* d0 = M + (size_t)n * n;
  const int np = min(cnt[0], cap), tid = threadIdx.x, bd = blockDim.x, lane = tid & 63;
  // half bandwidth: the band's, or the widest coupling of a pair (node i's rows, node j+1's
  // columns)
  if (tid == 0) cnt[2] = 10;
  __syncthreads();
  int wl = 10;
  for (int q = tid; q < np; q += bd) wl = max(wl, 4 * ((keys[q] & 0xffff) + 1 - (keys[q] >> 16)) + 2);
  if (wl > 10) atomicMax(cnt + 2, wl);
  __syncthreads();
  const int w = min(cnt[2], n - 1);
  // the band into the matrix, zeros out to w plus the LU panel's width: the blocked LU reads
  // its panel and U's block row that far from the diagonal (entries that are zero, and stay
  // zero, in a band of half width w), where an earlier iterate's wider band may have left
  // values
  const int wz = min(w + (w <= SC_WPANEL ? A.sc_pb : 0), n - 1), W2 = 2 * wz + 1;
  for (int idx = tid; idx < n * W2; idx += bd) {
    const int r = idx / W2, c = r - wz + (idx - r * W2);
    if (c < 0 || c >= n) continue;
    const int o = c - r + 10;
    double v = 0.0;
    if (o >= 0 && o < DM_NDIAG) {
      v = D.band[(size_t)(ch.dof_off + r) * DM_NDIAG + o];
      const unsigned m = D.nmask[4 * (size_t)(ch.node_tab + (r >> 2)) + 1], bit = 1u << (12 + (r & 3));
      const unsigned f = D.nmask[4 * (size_t)(ch.node_tab + (r >> 2))];
      if ((m & bit) && !(f & bit)) v += D.bpr[(size_t)(ch.bmap_off + r - ch.b_lo) * DM_NDIAG + o];
    }
    M[(size_t)r * n + c] = v;
    if (c == r) d0[r] = v;
  }
  __syncthreads();
  // the pairs' blocks between different nodes, from the pair area self_contact filled at this
  // iterate; each lane owns the rows of its node and adds its pairs in the list's order, each
  // pair's 27 entries loaded before any is stored
  const double DM_G* pr = sc_pair_area(D, sid, N);
  const int DM_L* nl = sc_node_lists(sc_lds, ME, cap);
  const int DM_L* ncount = nl + (ME + 1) * SC_SLOTS;
  for (int k = tid; k < N; k += bd) {
    const unsigned fk = D.nmask[4 * (size_t)(ch.node_tab + k)] >> 12;
    const int cnk = ncount[k], walk = cnk <= SC_SLOTS ? cnk : np;
    for (int e = 0; e < walk; ++e) {
      int q, role;
      if (cnk <= SC_SLOTS) {
        q = nl[k * SC_SLOTS + e] >> 2;
        role = nl[k * SC_SLOTS + e] & 3;
      } else {
        const int key = keys[e], i0 = key >> 16, j0 = key & 0xffff;
        q = e;
        role = k == i0 ? 0 : (k == i0 + 1 ? 1 : (k == j0 ? 2 : (k == j0 + 1 ? 3 : -1)));
        if (role < 0) continue;
      }
      const int key = keys[q], i = key >> 16, j = key & 0xffff;
      const double DM_G* o = pr + (size_t)q * SC_PAIR + 12 + 3 * role * 12;
      double add[3][3][3], cur[3][3][3];
      size_t at[3][3][3];
      bool use[3][3][3];
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const int l = m < role ? m : m + 1;
        const int kl = l == 0 ? i : (l == 1 ? i + 1 : (l == 2 ? j : j + 1));
        const unsigned fl = D.nmask[4 * (size_t)(ch.node_tab + kl)] >> 12;
#pragma unroll
        for (int al = 0; al < 3; ++al)
#pragma unroll
          for (int be = 0; be < 3; ++be) {
            at[m][al][be] = (size_t)(4 * k + al) * n + 4 * kl + be;
            use[m][al][be] = !((fk >> al) & 1u) && !((fl >> be) & 1u);
            add[m][al][be] = o[al * 12 + 3 * l + be];
            cur[m][al][be] = M[at[m][al][be]];
          }
      }
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int al = 0; al < 3; ++al)
#pragma unroll
          for (int be = 0; be < 3; ++be)
            if (use[m][al][be]) M[at[m][al][be]] = cur[m][al][be] + add[m][al][be];
    }
  }
  __syncthreads();
  // LU without pivoting over the band of half width w.  Blocked: sc_pb pivot columns at a time
  // are factorised (the panel of their rows below, staged in LDS, each thread's rows in
  // registers; the block row of U to their right solved per column in registers), the
  // forward substitution passes through the panel, then the trailing band takes one rank-sc_pb
  // update in HBM, each lane loading its entries in batches before any is stored, so the loads
  // overlap (the update streams the band through the caches once per panel: the wider the
  // panel, the less traffic).  A rod whose half bandwidth exceeds the LDS panel takes one
  // pivot at a time and row-by-row substitutions.
  constexpr int SB = 12;
  bool bad = false;
  if (w <= SC_WPANEL) {
    constexpr int RP = SC_WPANEL + SC_PBMAX, TB = 16;
    const int PB = A.sc_pb;
    double DM_L* pan = lcol + (4 * ME + 3);          // [PB][RP]: column q of the panel
    double DM_L* ub = pan + PB * RP;                 // [PB][RP]: row q of U right of the panel
    // the right-hand side: the forward substitution runs inside the LU, a panel at a time
    for (int r = tid; r < n; r += bd) y[r] = D.R[ch.dof_off + r];
    for (int k0 = 0; k0 < n; k0 += PB) {
      const int b = min(PB, n - k0), R = min(n - k0, b + w), C = min(n - k0 - b, w);
      for (int e = tid; e < R * b; e += bd) {        // a row's b entries by consecutive lanes
        const int i = e / b, q = e - i * b;
        pan[q * RP + i] = M[(size_t)(k0 + i) * n + k0 + q];
      }
      for (int e = tid; e < b * C; e += bd) {
        const int q = e / C, c = e - q * C;
        ub[q * RP + c] = M[(size_t)(k0 + q) * n + k0 + b + c];
      }
      __syncthreads();
      if (R <= bd) {
        bad = sc_panel(pan, d0 + k0, b, R, tid);
      } else {
        // a workgroup narrower than the panel: each lane owns rows in LDS, one barrier per pivot
        for (int q = 0; q < b; ++q) {
          const double p = pan[q * RP + q];
          if (!(fabs(p) > 1e-12 * fabs(d0[k0 + q])) || !isfinite(p)) { bad = true; break; }
          const double inv = 1.0 / p;
          for (int i = q + 1 + tid; i < R; i += bd) {
            const double l = pan[q * RP + i] * inv;
            pan[q * RP + i] = l;
            for (int c = q + 1; c < b; ++c) pan[c * RP + i] -= l * pan[c * RP + q];
          }
          __syncthreads();
        }
      }
      if (bad) break;
      // forward substitution through the panel (one wavefront, rows lane + 64 m): the top b
      // rows' values are final here, and each goes out to the rows below by its multipliers
      if (tid < 64) {
        double z[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) z[m] = lane + 64 * m < R ? y[k0 + lane + 64 * m] : 0.0;
#pragma unroll
        for (int q = 0; q < SC_PBMAX; ++q) {
          if (q < b) {
            const double yq = readlane_d(z[0], q);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
              const int i = lane + 64 * m;
              if (i > q && i < R) z[m] -= pan[q * RP + i] * yq;
            }
          }
        }
#pragma unroll
        for (int m = 0; m < 3; ++m)
          if (lane + 64 * m < R) y[k0 + lane + 64 * m] = z[m];
      }
      // U's block row: the unit lower triangle of the panel's top solved per column
      for (int c = tid; c < C; c += bd) {
        double u[SC_PBMAX];
#pragma unroll
        for (int t = 0; t < SC_PBMAX; ++t) u[t] = t < b ? ub[t * RP + c] : 0.0;
#pragma unroll
        for (int t = 1; t < SC_PBMAX; ++t)
          if (t < b) {
            double v = u[t];
#pragma unroll
            for (int q = 0; q < t; ++q) v -= pan[q * RP + t] * u[q];
            u[t] = v;
          }
#pragma unroll
        for (int t = 1; t < SC_PBMAX; ++t)
          if (t < b) ub[t * RP + c] = u[t];
      }
      __syncthreads();
      // the trailing band's rank-b update: one column per lane (its U entries in registers),
      // the lanes of a column group taking every G-th row, TB rows' loads before their stores;
      // then the panel and U block back to HBM
      const int tr = R - b;
      if (C > 0 && tr > 0) {
        const int G = bd >= C ? bd / C : 1;
        for (int c0 = bd >= C ? tid % C : tid, g = bd >= C ? tid / C : 0; g < G && c0 < C; c0 += bd >= C ? C * G : bd) {
          double u[SC_PBMAX];
#pragma unroll
          for (int t = 0; t < SC_PBMAX; ++t) u[t] = t < b ? ub[t * RP + c0] : 0.0;
          for (int i0 = g; i0 < tr; i0 += G * TB) {
            double val[TB];
            size_t at[TB];
#pragma unroll
            for (int q = 0; q < TB; ++q) {
              const int i = min(i0 + q * G, tr - 1);
              at[q] = (size_t)(k0 + b + i) * n + k0 + b + c0;
              val[q] = M[at[q]];
            }
#pragma unroll
            for (int q = 0; q < TB; ++q) {
              const int i = i0 + q * G;
              if (i < tr) {
                double acc = val[q];
#pragma unroll
                for (int t = 0; t < SC_PBMAX; ++t)
                  if (t < b) acc -= pan[t * RP + b + i] * u[t];
                M[at[q]] = acc;
              }
            }
          }
        }
      }
      for (int e = tid; e < R * b; e += bd) {
        const int i = e / b, q = e - i * b;
        M[(size_t)(k0 + i) * n + k0 + q] = pan[q * RP + i];
      }
      for (int e = tid; e < b * C; e += bd) {
        const int q = e / C, c = e - q * C;
        M[(size_t)(k0 + q) * n + k0 + b + c] = ub[q * RP + c];
      }
      __syncthreads();
    }
    // back substitution a block of PB rows at a time from the bottom: the block's rows of U
    // (from the diagonal to w right of it) come to LDS, each loaded while the block before is
    // solved; the part right of the block is summed by 16 lanes per row, then one wavefront
    // solves the block's triangle a column at a time
    if (!bad) {
      constexpr int PF = 12;
      const int nblk = (n + PB - 1) / PB;
      auto blk_entry = [&](int kb, int e, int Wd, bool& ok) -> size_t {
        const int q = e / Wd, c = e - q * Wd;
        ok = c >= q && c - q <= w;
        return (size_t)(kb * PB + q) * n + kb * PB + c;
      };
      {
        const int k0 = (nblk - 1) * PB, b = n - k0, Wd = min(n - k0, b + w);
        double DM_L* buf = ((nblk - 1) & 1) ? ub : pan;
        for (int e0 = tid; e0 < b * Wd; e0 += PF * bd) {
          double v[PF];
#pragma unroll
          for (int j = 0; j < PF; ++j) {
            const int e = min(e0 + j * bd, b * Wd - 1);
            bool ok;
            const size_t at = blk_entry(nblk - 1, e, Wd, ok);
            v[j] = ok ? M[at] : 0.0;
          }
#pragma unroll
          for (int j = 0; j < PF; ++j) {
            const int e = e0 + j * bd;
            if (e < b * Wd) buf[(e / Wd) * RP + e % Wd] = v[j];
          }
        }
      }
      for (int kb = nblk - 1; kb >= 0; --kb) {
        __syncthreads();                             // block kb in LDS, the rows below solved
        const int k0 = kb * PB, b = min(PB, n - k0), Wd = min(n - k0, b + w);
        const double DM_L* buf = (kb & 1) ? ub : pan;
        // the next block's entries: loads issued now, stored after this block's solve
        const int kn = kb - 1, Wn = kn >= 0 ? min(n - kn * PB, PB + w) : 0, tn = kn >= 0 ? PB * Wn : 0;
        double nv[PF];
#pragma unroll
        for (int j = 0; j < PF; ++j) {
          const int e = min(tid + j * bd, max(tn - 1, 0));
          bool ok = false;
          const size_t at = tn > 0 ? blk_entry(kn, e, Wn, ok) : 0;
          nv[j] = ok ? M[at] : 0.0;
        }
        for (int t = tid; t < b * 16; t += bd) {
          const int q = t >> 4, sub = t & 15;
          double acc = 0.0;
          for (int c = b + sub; c < Wd; c += 16) acc += buf[q * RP + c] * y[k0 + c];
          acc += __shfl_xor(acc, 8, 16);
          acc += __shfl_xor(acc, 4, 16);
          acc += __shfl_xor(acc, 2, 16);
          acc += __shfl_xor(acc, 1, 16);
          if (sub == 0) lcol[q] = acc;
        }
        __syncthreads();
        if (tid < 64) {
          double u[SC_PBMAX];
#pragma unroll
          for (int c = 0; c < SC_PBMAX; ++c) u[c] = lane < b && c < b ? buf[lane * RP + c] : 0.0;
          double v = lane < b ? y[k0 + lane] - lcol[lane] : 0.0, mine = 0.0;
#pragma unroll
          for (int c = SC_PBMAX - 1; c >= 0; --c) {
            if (c < b) {
              const double yc = readlane_d(v / u[c], c);
              if (lane == c) mine = yc;
              if (lane < c) v -= u[c] * yc;
            }
          }
          if (lane < b) y[k0 + lane] = mine;
        }
        if (kn >= 0) {
          double DM_L* nb = (kn & 1) ? ub : pan;
#pragma unroll
          for (int j = 0; j < PF; ++j) {
            const int e = tid + j * bd;
            if (e < tn) nb[(e / Wn) * RP + e % Wn] = nv[j];
          }
          for (int e = tid + PF * bd; e < tn; e += bd) {
            bool ok;
            const size_t at = blk_entry(kn, e, Wn, ok);
            nb[(e / Wn) * RP + e % Wn] = ok ? M[at] : 0.0;
          }
        }
      }
    }
  } else {
    for (int k = 0; k < n; ++k) {
      const double p = M[(size_t)k * n + k];
      if (!(fabs(p) > 1e-12 * fabs(d0[k])) || !isfinite(p)) { bad = true; break; }
      const int m = min(w, n - 1 - k);
      if (m == 0) break;
      const double inv = 1.0 / p;
      for (int i = tid; i < m; i += bd) lcol[i] = M[(size_t)(k + 1 + i) * n + k] * inv;
      __syncthreads();
      const double DM_G* rk = M + (size_t)k * n + k;
      const int tot = m * (m + 1);
      for (int b0 = tid; b0 < tot; b0 += SB * bd) {
        double val[SB], lv[SB], uv[SB];
        size_t at[SB];
        unsigned lmask = 0;                  // entries of column k: they take the multiplier
#pragma unroll
        for (int q = 0; q < SB; ++q) {
          const int idx = min(b0 + q * bd, tot - 1);
          const int i = idx / (m + 1), jj = idx - i * (m + 1);
          at[q] = (size_t)(k + 1 + i) * n + k + jj;
          val[q] = M[at[q]];
          lv[q] = lcol[i];
          uv[q] = rk[jj];
          lmask |= (jj == 0 ? 1u : 0u) << q;
        }
#pragma unroll
        for (int q = 0; q < SB; ++q)
          if (b0 + q * bd < tot) M[at[q]] = ((lmask >> q) & 1u) ? lv[q] : val[q] - lv[q] * uv[q];
      }
      __syncthreads();
    }
    // forward and back substitution by one wavefront, a row's sum over the band at a time
    if (!bad && tid < 64) {
      for (int i = 0; i < n; ++i) {
        const double DM_G* row = M + (size_t)i * n;
        double acc = 0.0;
        for (int j = max(0, i - w) + lane; j < i; j += 64) acc += row[j] * y[j];
        acc = wave_sum64(acc);
        if (lane == 0) y[i] = D.R[ch.dof_off + i] - acc;
        lds_order();
      }
      for (int i = n - 1; i >= 0; --i) {
        const double DM_G* row = M + (size_t)i * n;
        double acc = 0.0;
        for (int j = i + 1 + lane; j <= min(n - 1, i + w); j += 64) acc += row[j] * y[j];
        acc = wave_sum64(acc);
        if (lane == 0) y[i] = (y[i] - acc) / row[i];
        lds_order();
      }
    }
  }
  if (bad) {
    if (tid == 0) flags[0] = 1;
    __syncthreads();
    return;
  }
  __syncthreads();
  for (int r = tid; r < n; r += bd) {
    const int k = r >> 2, c = r & 3;
    const int h = c < 3 ? D.node_home[c * NN + D.chain_node[ch.node_tab + k]] : D.edge_home[D.chain_edge[ch.edge_tab + k]];
    if (h >= 0) D.delta[h] = y[r];
    else xB[-1 - h] = y[r];
  }
  __syncthreads();
}

// Band rows of every chain node of the system; returns this lane's share of the squared
// residual of free, non-border rows.
template <int MODE>
__device__ __noinline__ double assemble_band(ArgsP Ap, int sid, double dt) {
  const DmStepArgs DM_C& A = *uniform(Ap);
  const DmDev DM_C& D = A.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  double r2 = 0.0;
  for (int i = threadIdx.x; i < S.chain_nodes; i += blockDim.x) {
    int c = S.chain0, k = i;
    while (k >= D.chain[c].n_nodes) { k -= D.chain[c].n_nodes; ++c; }
    r2 += band_node<MODE>(A, dt, c, k);
  }
  return r2;
}

// FP64 rounding floor of the residual norm of the iterate whose Newton matrix J is assembled
// (band, border rows' band parts and the dense border Bt): a free DOF cannot be placed closer
// than eps |q_k| to the root, so row i cannot be resolved below eps sum_k |J_ik| |q_k|; with
// |q_k| bounded by its kind's magnitude at the (sub)step start (largest |position coordinate|;
// largest |theta| plus pi, the reference twist's range) the floor is
// floor_factor * eps * || |J| s ||_2 over free rows and columns.  Called by the whole
// workgroup, only when a stopping or line-search decision needs it; the same value in every
// lane.
__device__ __noinline__ double residual_floor(ArgsP Ap, int sid, const double DM_L* Bt, int ld, double DM_L* red) {
  const DmStepArgs DM_C& A = *uniform(Ap);
  const DmDev DM_C& D = A.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  const int NN = D.n_nodes_tot, w = threadIdx.x >> 6;
  // magnitudes of the (sub)step start
  double mx = 0.0, mt = 0.0;
  for (int i = threadIdx.x; i < S.n_nodes; i += blockDim.x)
#pragma unroll
    for (int c = 0; c < 3; ++c) mx = fmax(mx, fabs(D.x0[c * NN + S.node0 + i]));
  for (int i = threadIdx.x; i < S.n_edges; i += blockDim.x) mt = fmax(mt, fabs(D.th0[S.edge0 + i]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, o, 64));
    mt = fmax(mt, __shfl_xor(mt, o, 64));
  }
  if ((threadIdx.x & 63) == 0) { red[16 + w] = mx; red[24 + w] = mt; }
  __syncthreads();
  double xs = 0.0, ts = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) { xs = fmax(xs, red[16 + i]); ts = fmax(ts, red[24 + i]); }
  ts += 3.141592653589793238462643383279;
  // band rows: row sums of free rows (a border row's band part goes to babs)
  double f2 = 0.0;
  for (int a = 0; a < S.n_chains; ++a) {
    const DmChain DM_C& C = D.chain[S.chain0 + a];
    const int n = 4 * C.n_nodes - 1;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
      if (D.cfix[C.dof_off + r]) continue;
      const double DM_G* row = D.band + (size_t)(C.dof_off + r) * DM_NDIAG;
      double fa = 0.0;
      for (int o = 0; o < DM_NDIAG; ++o) fa = fma(fabs(row[o]), ((r - DM_HALF_BAND + o) & 3) == 3 ? ts : xs, fa);
      if (r >= C.b_lo && r < C.b_hi) D.babs[C.bmap_off + r - C.b_lo] = fa;
      else f2 = fma(fa, fa, f2);
    }
  }
  __syncthreads();
  // border rows (nb <= 64: wavefront 0): each source chain's band part plus the dense border row
  const int nb = S.nb, b = threadIdx.x;
  if (b < nb && !D.bfix[S.bfix_off + b]) {
    double fa = 0.0;
    for (int q = 0; q < DM_MAX_BSRC; ++q) {
      const int slot = 2 * ((S.bsrc_off + b * DM_MAX_BSRC) + q);
      const int ci = D.bsrc[slot];
      if (ci < 0) break;
      const DmChain DM_C& C = D.chain[ci];
      fa += D.babs[C.bmap_off + D.bsrc[slot + 1] - C.b_lo];
    }
    for (int c = 0; c < nb; ++c) {
      const int r0 = D.bsrc[2 * (S.bsrc_off + c * DM_MAX_BSRC) + 1];     // a chain DOF of border DOF c
      fa = fma(fabs(Bt[b * ld + c]), (r0 & 3) == 3 ? ts : xs, fa);
    }
    f2 = fma(fa, fa, f2);
  }
  f2 = wave_sum(f2);
  if ((threadIdx.x & 63) == 0) red[8 + w] = f2;
  __syncthreads();
  double tot = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) tot += red[8 + i];
  __syncthreads();
  return A.floor_factor * 2.220446049250313080847263336181640625e-16 * sqrt(tot);   // eps = 2^-52
}

// Value of a border term (kind 4: the zero pad).
__device__ __forceinline__ double bterm(const DmDev DM_C& D, const DmBItem& it) {
  const double DM_G* src = it.kind == 0 ? D.bpr
                         : it.kind == 1 ? D.st_H
                         : it.kind == 2 ? D.R
                         : it.kind == 3 ? D.st_g : D.zpad;
  return it.coef * src[it.idx];
}

// Dense border from the entries' term segments of DM_SEG terms (built once at finalize),
// summed in their stored order; a clamped border row is the identity row with a zero
// right-hand side.  When every entry has at most one segment (a rod's separator), one lane per
// entry sums its segment.  Otherwise (a hub's entries have dozens of terms) it takes two
// passes: one lane per segment into segsum (two segments per lane at a time, so that every
// item and value load of both is in flight together), then one lane per entry adds its
// segments in order.  Called by the whole workgroup.  Returns this lane's share of the
// squared residual of free border rows.
// MODE 0: every entry; 1: the right-hand side column only, one lane per row summing its
// segments in the same order; 2: the matrix entries only (the right-hand side column is left
// as the residual pass wrote it).
template <int MODE>
__device__ __noinline__ double assemble_border(ArgsP Ap, int sid, double DM_L* Bt, int ld, double DM_L* segsum) {
  const DmStepArgs DM_C& A = *uniform(Ap);
  const DmDev DM_C& D = A.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  const int nb = S.nb, W = nb + 1, ns = S.n_seg;
  if (MODE == 1) {
    double r2 = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
      const int e = b * W + nb;
      double v = 0.0;
      if (!D.bfix[S.bfix_off + b]) {
        const int s1 = D.bent[S.bent_off + e + 1];
        for (int q = D.bent[S.bent_off + e]; q < s1; ++q) {
          const DmBItem DM_C* p = D.bitem + (size_t)q * DM_SEG;
          DmBItem it[DM_SEG];
          double x[DM_SEG];
#pragma unroll
          for (int j = 0; j < DM_SEG; ++j) it[j] = p[j];
#pragma unroll
          for (int j = 0; j < DM_SEG; ++j) x[j] = bterm(D, it[j]);
          double sg = 0.0;
#pragma unroll
          for (int j = 0; j < DM_SEG; ++j) sg += x[j];
          v += sg;
        }
        r2 += v * v;
      }
      Bt[b * ld + nb] = v;
    }
    return r2;
  }
  if (!S.seg_long) {
    double r2 = 0.0;
    for (int e = threadIdx.x; e < nb * W; e += blockDim.x) {
      const int b = e / W, col = e - b * W;
      if (MODE == 2 && col == nb) continue;
      double v = 0.0;
      if (D.bfix[S.bfix_off + b]) {
        v = col == b ? 1.0 : 0.0;
      } else {
        const int s0 = D.bent[S.bent_off + e];
        if (D.bent[S.bent_off + e + 1] > s0) {
          const DmBItem DM_C* p = D.bitem + (size_t)s0 * DM_SEG;
          DmBItem it[DM_SEG];
          double x[DM_SEG];
#pragma unroll
          for (int j = 0; j < DM_SEG; ++j) it[j] = p[j];
#pragma unroll
          for (int j = 0; j < DM_SEG; ++j) x[j] = bterm(D, it[j]);
#pragma unroll
          for (int j = 0; j < DM_SEG; ++j) v += x[j];
        }
        if (col == nb) r2 += v * v;
      }
      Bt[b * ld + col] = v;
    }
    return r2;
  }
  for (int g = threadIdx.x; g < ns; g += 2 * blockDim.x) {
    const int g2 = g + blockDim.x;
    const bool two = g2 < ns;
    const DmBItem DM_C* p1 = D.bitem + (size_t)(S.seg0 + g) * DM_SEG;
    const DmBItem DM_C* p2 = D.bitem + (size_t)(S.seg0 + (two ? g2 : g)) * DM_SEG;
    DmBItem i1[DM_SEG], i2[DM_SEG];
#pragma unroll
    for (int j = 0; j < DM_SEG; ++j) { i1[j] = p1[j]; i2[j] = p2[j]; }
    double v1 = 0.0, v2 = 0.0, x1[DM_SEG], x2[DM_SEG];
#pragma unroll
    for (int j = 0; j < DM_SEG; ++j) { x1[j] = bterm(D, i1[j]); x2[j] = bterm(D, i2[j]); }
#pragma unroll
    for (int j = 0; j < DM_SEG; ++j) { v1 += x1[j]; v2 += x2[j]; }
    segsum[g] = v1;
    if (two) segsum[g2] = v2;
  }
  __syncthreads();
  double r2 = 0.0;
  for (int e = threadIdx.x; e < nb * W; e += blockDim.x) {
    const int b = e / W, col = e - b * W;
    if (MODE == 2 && col == nb) continue;
    double v = 0.0;
    if (D.bfix[S.bfix_off + b]) {
      v = col == b ? 1.0 : 0.0;
    } else {
      const int s0 = D.bent[S.bent_off + e] - S.seg0, s1 = D.bent[S.bent_off + e + 1] - S.seg0;
      for (int q = s0; q < s1; ++q) v += segsum[q];
      if (col == nb) r2 += v * v;
    }
    Bt[b * ld + col] = v;
  }
  return r2;
}

// ---------------------------------------------------------------------------
// banded elimination of up to four arms by one wavefront, one arm per 16-lane row
// ---------------------------------------------------------------------------

// Lane roles: row = lane / 16 selects the arm (rows beyond the group's arm count mirror its
// last arm: they compute the same values and store them to the same places), l = lane % 16
// the role within the row: l < 11 a window column, l == 11 the right-hand side, l > 11 idle.
// Every value that crosses lanes moves by DPP row broadcasts, which stay inside a row.

// Band, right-hand side and factor records of one arm (per lane: the lane's arm), in
// arm-local numbering: local row l is chain DOF first + dir * l, and lmax local rows exist.
// Band entry (l, l2) sits at band index b0() + d21() * l + dir * (l2 - l).  Out-of-range
// entries are redirected to the chain's first band entry (always valid) and zeroed after the
// load, so a load never sits behind a branch.
struct ArmView {
  const double DM_G* band; const double DM_G* R; double DM_G* fac; const double DM_G* zpad;
  int dof_off, first, dir, count, fac_off, lmax;
  __device__ __forceinline__ int cd(int l) const { return first + dir * l; }
  __device__ __forceinline__ int b0() const { return (dof_off + first) * DM_NDIAG + DM_HALF_BAND; }
  __device__ __forceinline__ int d21() const { return DM_NDIAG * dir; }
};

// The lane's arm within a group of na arms starting at global arm ai0.
__device__ __forceinline__ int lane_arm(int ai0, int na, int lane) {
  const int r = lane >> 4;
  return ai0 + (r < na ? r : na - 1);
}

__device__ __forceinline__ ArmView arm_view(const DmDev DM_C& D, const DmArm& arm) {
  const DmChain ch = D.chain[arm.chain];
  const int n = 4 * ch.n_nodes - 1;
  return ArmView{D.band, D.R, D.fac, D.zpad, ch.dof_off, arm.first, arm.dir, arm.count, arm.fac_off,
                 arm.dir > 0 ? n - arm.first : arm.first + 1};
}

// Smallest and largest arm length of a group (uniform).
__device__ __forceinline__ void group_counts(const DmDev DM_C& D, int ai0, int na, int& cmin, int& cmax) {
  cmin = 0x7fffffff; cmax = 0;
  for (int r = 0; r < na; ++r) {
    const int c = D.arm[ai0 + r].count;
    cmin = c < cmin ? c : cmin;
    cmax = c > cmax ? c : cmax;
  }
}

// Pointer select by bit masks (no branch around the load that follows).
__device__ __forceinline__ const double DM_G* sel_ptr(bool c, const double DM_G* a, const double DM_G* b) {
  const unsigned long long ia = (unsigned long long)a, ib = (unsigned long long)b;
  const unsigned long long m = 0ull - (unsigned long long)c;
  return (const double DM_G*)((ia & ~m) | (ib & m));
}

// Entry of local row r in the column of role s (s < 11: column r + t - 10, the column
// congruent to s mod 11 among r-10 .. r, with t = (s - r - 1) mod 11 given by the caller;
// s == 11: the right-hand side of row r, zero for the border rows r >= count).  One load per
// lane; a missing entry is read from the zero pad, so the loaded value needs no masking
// (which would wait for the load).
__device__ __forceinline__ double row_entry(const ArmView& V, int r, int s, int t) {
  const int rhs = s == DM_WIN;
  const int ok = (rhs & (r < V.count)) | ((r < V.lmax) & (s < DM_WIN));
  const int ib = V.b0() + V.d21() * r + V.dir * (t - DM_HALF_BAND);
  const int ir = V.dof_off + V.cd(r);
  return *sel_ptr(ok, V.zpad, sel_ptr(rhs, V.band + ib, V.R + ir));
}

// (s - T - 1) mod 11 for 0 <= s, T <= 11.
__device__ __forceinline__ int wrap11(int s, int T) {
  const int t = s - T - 1;
  return t < 0 ? t + DM_WIN : t;
}

// Initial window entry of role s: band entry (r, s) for s < 11, the right-hand side of row r
// for s == 11 (r, s <= 10, so the entry is inside the band when both rows exist).
__device__ __forceinline__ double init_entry(const ArmView& V, int r, int s) {
  const int rhs = s == DM_WIN;
  const int ok = (rhs & (r < V.count)) | ((r < V.lmax) & (s < V.lmax) & (s < DM_WIN));
  const int ib = V.b0() + V.d21() * r + V.dir * (s - r);
  const int ir = V.dof_off + V.cd(r);
  return *sel_ptr(ok, V.zpad, sel_ptr(rhs, V.band + ib, V.R + ir));
}

// Window halves: an arm's window rows (slots 0..10, a row's slot being its index mod 11) are
// split over the two 16-lane rows of a row pair, the even row holding slots 0..5 and the odd
// row slots 6..10 (its sixth register unused), so each lane updates half a column per step.
#define DM_HS 6

// The column role s takes over at its pivot step kp = k0 + s, as this lane's half of it:
// slot g = 6h + j holds row kp + i of column kp + 11 with i = (g - s) mod 11 (i = 11, the new
// diagonal, in slot s).  All zero once column kp + 11 is past the chain end (read from the
// zero pad).  Roles >= 11 load role 0's column, which they never take.
__device__ __forceinline__ void load_new_column(double (&col)[DM_HS], int k0, int s, int h, const ArmView& V) {
  const int sr = s < DM_WIN ? s : 0;
  const int kp = k0 + sr;
  const bool ok = kp + DM_WIN < V.lmax;
  // entry (kp + i, kp + 11) at b0 + d21 (kp + i) + dir (11 - i) = x + i * 20 dir
  const double DM_G* p = sel_ptr(ok, V.zpad, V.band + (V.b0() + V.d21() * kp + DM_WIN * V.dir));
  const int st = ok ? V.d21() - V.dir : 0;
#pragma unroll
  for (int j = 0; j < DM_HS; ++j) {
    int i = DM_HS * h + j - sr;
    i += i <= 0 ? DM_WIN : 0;             // 1 .. 11 for the slots 0..10 (slot 11 of the odd row: unused)
    col[j] = p[(i < DM_WIN + 1 ? i : DM_WIN) * st];
  }
}

// The value of the even (odd) row of each row pair, in both rows of the pair
// (v_permlane16_swap_b32).
__device__ __forceinline__ double from_half(double v, int half) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
  const unsigned l32 = half ? lo[1] : lo[0], h32 = half ? hi[1] : hi[0];
  return __longlong_as_double((long long)(((unsigned long long)h32 << 32) | l32));
}

// 1/p from the hardware estimate (about 24 correct bits) refined by one third-order
// correction r (1 + e + e^2), e = 1 - p r, which leaves a relative error of order e^3 (below
// the float64 rounding of the result).
__device__ __forceinline__ double recip(double p) {
  const double r = __builtin_amdgcn_rcp(p);
  const double e = fma(-p, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

// Value of lane T of each 16-lane row, in every lane of that row (v_mov_b64 with DPP
// row_newbcast).
template <int T>
__device__ __forceinline__ double row_bcast(double v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + T, 0xF, 0xF, false);
}

// Eliminate window position k (k % 11 == T).  Role s < 11 holds the column congruent to s
// (mod 11), role 11 the right-hand side; row half h holds slots 6h .. 6h+5.  The pivot row's
// entries (slot T, in half T / 6) reach the other half by one row-pair swap; the pivot column
// is broadcast within each row.  col: this lane's half of the column the pivot role takes
// over; ent: the entry of row k + 11 in this role's column (used by the half owning slot T).
// MASK: rows whose arm ends before k leave their window untouched and park their store in the
// padding of their first record.
// A pivot below this fraction of its row's diagonal in the assembled band marks the system's
// Newton matrix as numerically singular (the elimination does not pivot).
#define DM_PIVOT_TAU 1e-12

template <int T, bool MASK>
__device__ __forceinline__ void elim_step(double (&w)[DM_HS], const double (&col)[DM_HS], double ent, int k, int l,
                                          int h, const ArmView& V, double DM_G* recp, int& bad, double& dg) {
  constexpr int hT = T >= DM_HS ? 1 : 0, tT = T - DM_HS * hT;
  const bool act = MASK ? k < V.count : true;
  const double u = from_half(w[tT], hT);              // row k's entry in this lane's column
  const double piv = row_bcast<T>(u);
  // the lane holding slot T of role T keeps the assembled diagonal of the row it pivots next;
  // a pivot that is zero, subnormal, infinite or NaN, or small against that diagonal, marks
  // the matrix (bitwise logic: no branch on the serial chain)
  const bool dlane = (l == T) & (h == hT);
  const bool small = dlane & !(fabs(piv) >= DM_PIVOT_TAU * fabs(dg));
  bad |= (int)(act & (!__builtin_isnormal(piv) | small));
  dg = dlane ? col[tT] : dg;                          // the diagonal of row k + 11
  const double inv = recip(piv);
  double cv[DM_HS];
#pragma unroll
  for (int j = 0; j < DM_HS; ++j) cv[j] = row_bcast<T>(w[j]);
  const bool piv_lane = (l == T);
  // factor record of row k: [1/pivot, U(k, k+1..k+10), modified rhs]; every lane stores (no
  // branch; both halves store the same values), idle roles into the record's padding
  *recp = piv_lane ? inv : u;
  // the pivot lane's scale is exactly 1, so its own column becomes exactly zero and the new
  // column k + 11 it takes over is added in exactly; a parked row scales by zero
  const double us = !act ? 0.0 : (piv_lane ? 1.0 : u * inv);
  const double take = (act && piv_lane) ? 1.0 : 0.0;
#pragma unroll
  for (int q = 0; q < DM_HS; ++q) w[q] = fma(take, col[q], fma(-cv[q], us, w[q]));
  // slot T now holds row k + 11 (the pivot lane: the new diagonal)
  const double wn = piv_lane ? col[tT] : ent;
  w[tT] = (act && h == hT) ? wn : w[tT];
}

#define DM_UNROLL11(M) M(0) M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10)

// Where role l stores in the factor record of row k (k % 11 == T): slot (l - T) mod 11 of the
// window columns, 11 for the right-hand side, the padding for idle roles and parked rows.
template <int T>
__device__ __forceinline__ double DM_G* rec_ptr(const ArmView& V, int k, int l, bool act) {
  const int j = l < DM_WIN ? (l - T + DM_WIN) % DM_WIN : (l == DM_WIN ? DM_WIN : DM_FAC);
  const int rec = act ? (V.fac_off + k) * DM_FAC_STRIDE + j : V.fac_off * DM_FAC_STRIDE + DM_FAC;
  return V.fac + rec;
}

// Forward elimination of the na (<= 2) arms ai0 .. ai0+na-1, one per row pair; deltas: the
// Schur-complement slots (110 doubles per arm) of arm ai0.  The new columns of a block are
// loaded one block ahead; the entering row of step T is loaded right after step T of the
// previous block, into the register that step has just freed.
__device__ __noinline__ void sweep_arms(ArgsP Ap, int ai0, int na, double DM_L* deltas, int DM_L* bad_flag) {
  const DmStepArgs DM_C& A = *uniform(Ap);
  const DmDev DM_C& D = A.d;
  ai0 = uniform(ai0);
  na = uniform(na);
  const int lane = threadIdx.x & 63, l = lane & 15, h = (lane >> 4) & 1, pr = lane >> 5;
  const int ai = ai0 + (pr < na ? pr : na - 1);
  const DmArm arm = D.arm[ai];
  const ArmView V = arm_view(D, arm);
  int cmin, cmax;
  group_counts(D, ai0, na, cmin, cmax);
  double w[DM_HS], col[DM_HS], ncol[DM_HS], ent[DM_WIN];
  double dg = 0.0;        // role l's next pivot row's assembled diagonal (lane of slot l only)
#pragma unroll
  for (int j = 0; j < DM_HS; ++j) {
    const int g = DM_HS * h + j;
    w[j] = init_entry(V, g < DM_WIN ? g : 0, l);
    dg = (g == l) ? w[j] : dg;
  }
  load_new_column(col, 0, l, h, V);
#pragma unroll
  for (int T = 0; T < DM_WIN; ++T) ent[T] = row_entry(V, T + DM_WIN, l, wrap11(l, T));
  int bad = 0;
  // Deep blocks (k0 + 33 <= every arm's count: the block's rows and the entering rows it loads,
  // k0 + 22 .. k0 + 32, are inside every arm) address by fixed per-lane strides from one
  // pointer per block.  Entering row of step T: the right-hand side role (and the idle roles,
  // which load the same row's right-hand side and never use it) reads R at T dir past the
  // block's base, the column roles read band entry (r, r + t - 10), t = (l - T - 1) mod 11,
  // at 20 dir T past the base plus 11 dir once T >= l.  Record of step T: 15 T past the base
  // for the column roles (16 T for the others) plus 11 once T > l.
  const bool side = l >= DM_WIN;
  const int e_step = side ? V.dir : (DM_NDIAG - 1) * V.dir, e_jump = side ? 0 : DM_WIN * V.dir;
  const int e_adv = DM_WIN * (side ? V.dir : V.d21());
  const int r_step = side ? DM_FAC_STRIDE : DM_FAC_STRIDE - 1;
  const int r_base = l < DM_WIN ? l : (l == DM_WIN ? DM_WIN : DM_FAC);
  const double DM_G* ep = side ? V.R + (V.dof_off + V.cd(2 * DM_WIN)) : V.band + (V.b0() + V.d21() * (2 * DM_WIN) + V.dir * (l - DM_WIN));
  double DM_G* rp = V.fac + (size_t)V.fac_off * DM_FAC_STRIDE + r_base;
  for (int k0 = 0; k0 < cmax; k0 += DM_WIN) {
    load_new_column(ncol, k0 + DM_WIN, l, h, V);
    // a deep block runs unmasked; in the last blocks the rows whose arm has ended are masked
    // per step, the loads of rows past an arm's end read the zero pad, and the group stops
    // on a uniform branch
    if (k0 + 3 * DM_WIN <= cmin) {
#define DM_E(T) \
  elim_step<T, false>(w, col, ent[T], k0 + T, l, h, V, rp + (T * r_step + (T > l && !side ? DM_WIN : 0)), bad, dg); \
  ent[T] = ep[T * e_step + (T >= l ? e_jump : 0)];
      DM_UNROLL11(DM_E)
#undef DM_E
    } else {
#define DM_E(T) \
  if (k0 + T < cmax) elim_step<T, true>(w, col, ent[T], k0 + T, l, h, V, rec_ptr<T>(V, k0 + T, l, k0 + T < V.count), bad, dg); \
  ent[T] = row_entry(V, k0 + T + 2 * DM_WIN, l, wrap11(l, T));
      DM_UNROLL11(DM_E)
#undef DM_E
    }
    ep += e_adv;
    rp += DM_WIN * DM_FAC_STRIDE;
#pragma unroll
    for (int q = 0; q < DM_HS; ++q) col[q] = ncol[q];
  }
  // trailing (border) block of the window = this arm's Schur complement contribution
  double DM_L* dl = deltas + (ai - ai0) * 110;
  const int c0 = arm.count % DM_WIN, nt = arm.n_trail;
  if (l < DM_WIN) {
    const int jc = (l - c0 + DM_WIN) % DM_WIN;
    if (jc < nt) {
#pragma unroll
      for (int q = 0; q < DM_HS; ++q) {
        const int g = DM_HS * h + q;
        const int i = (g - c0 + DM_WIN) % DM_WIN;
        if (g < DM_WIN && i < nt) dl[i * 10 + jc] = w[q];
      }
    }
  } else if (l == DM_WIN) {
#pragma unroll
    for (int q = 0; q < DM_HS; ++q) {
      const int g = DM_HS * h + q;
      const int i = (g - c0 + DM_WIN) % DM_WIN;
      if (g < DM_WIN && i < nt) dl[100 + i] = w[q];
    }
  }
  if (bad) *bad_flag = 1;
}

// Back substitution of one 11-row block.  Role s < 11 of a row holds the factor record of the
// block's row s of its arm; at step T every lane evaluates row k0 + T's equation with its own
// record and the common solution window, role T's value (the one whose record is row k0 + T's)
// is broadcast in the row by DPP, and every lane enters it into its window.  xv: the solution
// window (slots by row mod 11), the same in every lane of a row.  MASK: rows whose arm ends
// below the block's row T keep their window (it holds the trailing border values).
template <int T, bool MASK>
__device__ __forceinline__ void back_step(double (&xv)[DM_WIN], const double (&cur)[DM_FAC], double& xs, int l,
                                          bool act) {
  // y_k - sum_j U(k, k+j) x_{k+j}: the older solutions first, in two interleaved partial sums
  // each ending with its most recent term, and x_{k+1} (solved by the previous step) last
  double s0 = cur[DM_WIN], s1 = 0.0;
#pragma unroll
  for (int j = DM_WIN - 1; j >= 2; --j) {
    if (j & 1) s0 = fma(-cur[j], xv[(T + j) % DM_WIN], s0);
    else s1 = fma(-cur[j], xv[(T + j) % DM_WIN], s1);
  }
  const double xo = fma(-cur[1], xv[(T + 1) % DM_WIN], s0 + s1) * cur[0];
  const double xl = row_bcast<T>(xo);
  xv[T] = (!MASK || act) ? xl : xv[T];
  xs = (l == T) ? xo : xs;             // role T keeps the solution of row k0 + T
}

// Factor records of block rows lb .. lb+10: role s < 11 loads record lb + s (12 doubles from a
// 128-byte aligned record, as six 16-byte loads); missing records read the arm's first record.
__device__ __forceinline__ void load_records(double (&buf)[DM_FAC], const ArmView& V, int lb, int l) {
  const int ok = (lb >= 0) & (l < DM_WIN) & (lb + l < V.count);
  const double2 DM_G* p = (const double2 DM_G*)(V.fac + (size_t)(V.fac_off + ok * (lb + l)) * DM_FAC_STRIDE);
#pragma unroll
  for (int q = 0; q < DM_FAC / 2; ++q) {
    const double2 v = p[q];
    buf[2 * q] = v.x;
    buf[2 * q + 1] = v.y;
  }
}

__device__ __noinline__ void backsub_arms(ArgsP Ap, int ai0, int na, const double DM_L* xB) {
  const DmStepArgs DM_C& A = *uniform(Ap);
  const DmDev DM_C& D = A.d;
  ai0 = uniform(ai0);
  na = uniform(na);
  const int lane = threadIdx.x & 63, l = lane & 15;
  const DmArm arm = D.arm[lane_arm(ai0, na, lane)];
  const DmChain ch = D.chain[arm.chain];
  const ArmView V = arm_view(D, arm);
  int cmin, cmax;
  group_counts(D, ai0, na, cmin, cmax);
  const int c0 = arm.count % DM_WIN;
  double xv[DM_WIN];
#pragma unroll
  for (int q = 0; q < DM_WIN; ++q) {
    const int i = (q - c0 + DM_WIN) % DM_WIN;
    double val = 0.0;
    if (i < arm.n_trail) val = xB[D.bmap[ch.bmap_off + V.cd(arm.count + i) - ch.b_lo]];
    xv[q] = val;
  }
  if (cmax == 0) return;
  double cur[DM_FAC], nxt[DM_FAC];
  int lb = ((cmax - 1) / DM_WIN) * DM_WIN;
  load_records(cur, V, lb, l);
  for (; lb >= 0; lb -= DM_WIN) {
    load_records(nxt, V, lb - DM_WIN, l);
    double xs = 0.0;
    if (lb + DM_WIN <= cmin) {
#define DM_B(T) back_step<10 - T, false>(xv, cur, xs, l, true);
      DM_UNROLL11(DM_B)
#undef DM_B
    } else {
#define DM_B(T) if (lb + (10 - T) < cmax) back_step<10 - T, true>(xv, cur, xs, l, lb + (10 - T) < V.count);
      DM_UNROLL11(DM_B)
#undef DM_B
    }
    if ((l < DM_WIN) & (lb + l < V.count)) D.delta[V.dof_off + V.cd(lb + l)] = xs;
#pragma unroll
    for (int q = 0; q < DM_FAC; ++q) cur[q] = nxt[q];
  }
}

// The sweep takes a system's arms in groups of two (one per row pair), the back-substitution
// in groups of four (one per row), one group per wavefront.
__device__ __forceinline__ void sweep_all(ArgsP Ap, const DmSystem DM_C& S, int wave, int nwaves,
                                          double DM_L* deltas, int DM_L* flags) {
  for (int g = 2 * wave; g < S.n_arms; g += 2 * nwaves)
    sweep_arms(Ap, S.arm0 + g, min(2, S.n_arms - g), deltas + g * 110, flags);
}

__device__ __forceinline__ void backsub_all(ArgsP Ap, const DmSystem DM_C& S, int wave, int nwaves,
                                            const double DM_L* xB) {
  for (int g = 4 * wave; g < S.n_arms; g += 4 * nwaves) backsub_arms(Ap, S.arm0 + g, min(4, S.n_arms - g), xB);
}

// 32-bit halves of a double through a DPP row rotation (row_ror:N), and the partner row's
// value of a row pair (v_permlane16_swap_b32).
template <int N>
__device__ __forceinline__ double row_ror_d(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, 0x120 + N, 0xF, 0xF, false);
  const unsigned hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), 0x120 + N, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int N>
__device__ __forceinline__ int row_ror_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x120 + N, 0xF, 0xF, false); }
__device__ __forceinline__ unsigned partner_row(unsigned v, int odd) {
  const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return odd ? r[0] : r[1];
}

// Largest v over the lanes of each 16-lane row (NBX <= 16) or row pair (NBX <= 32), the
// smallest lane among equals, as (value, lane) in every lane of the row (pair).
__device__ __forceinline__ void argmax_step(double& v, int& i, double ov, int oi) {
  const bool take = (ov > v) | ((ov == v) & (oi < i));
  v = take ? ov : v;
  i = take ? oi : i;
}
template <int NBX>
__device__ __forceinline__ void row_argmax(double& v, int& i) {
  argmax_step(v, i, row_ror_d<8>(v), row_ror_i<8>(i));
  argmax_step(v, i, row_ror_d<4>(v), row_ror_i<4>(i));
  argmax_step(v, i, row_ror_d<2>(v), row_ror_i<2>(i));
  argmax_step(v, i, row_ror_d<1>(v), row_ror_i<1>(i));
  if (NBX > 16) {
    const int odd = (threadIdx.x >> 4) & 1;
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = partner_row((unsigned)b, odd), hi = partner_row((unsigned)(b >> 32), odd);
    const double ov = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    argmax_step(v, i, ov, (int)partner_row((unsigned)i, odd));
  }
}

// Gaussian elimination with partial pivoting of a border of nb <= NBX DOFs held in registers:
// lane i holds row i (columns in r[0..NBX), the right-hand side in rhs).  Rows are not
// exchanged: step p picks the not yet pivotal row with the largest |entry| in column p (the
// first such row among equals), broadcasts it by lane reads, and eliminates column p from the
// other open rows; back substitution runs over the pivots in reverse, every lane keeping its
// row's partial sum.  The solution of border DOF j ends in lane j.
template <int NBX>
__device__ __forceinline__ double border_lu_regs(const double DM_L* Bt, int ld, int nb, int& bad) {
  const int lane = threadIdx.x & 63;
  const bool row = lane < nb;
  const double DM_L* br = Bt + (row ? lane : 0) * ld;
  double r[NBX];
#pragma unroll
  for (int c = 0; c < NBX; ++c) r[c] = (row && c < nb) ? br[c < nb ? c : 0] : 0.0;
  double rhs = row ? br[nb] : 0.0;
  bool open = row;
  int piv[NBX];
  double pinv[NBX];
  // largest assembled entry of the border: a pivot below DM_PIVOT_TAU of it marks the border
  // numerically singular
  double amax = 0.0;
#pragma unroll
  for (int c = 0; c < NBX; ++c) amax = fmax(amax, fabs(r[c]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
#pragma unroll
  for (int p = 0; p < NBX; ++p) {
    piv[p] = 0;
    pinv[p] = 0.0;
    if (p < nb) {
      double v = open ? fabs(r[p]) : -1.0;
      int im = lane;
      row_argmax<NBX>(v, im);
      im = uniform(im);
      const double pv = readlane_d(r[p], im);
      bad |= !(fabs(pv) > 1e-300) | !isfinite(pv) | !(fabs(pv) >= DM_PIVOT_TAU * amax);
      const double inv = 1.0 / pv;
      piv[p] = im;
      pinv[p] = inv;
      open = open && lane != im;
      const double l = open ? r[p] * inv : 0.0;
#pragma unroll
      for (int c = p + 1; c < NBX; ++c) r[c] = fma(-l, readlane_d(r[c], im), r[c]);
      rhs = fma(-l, readlane_d(rhs, im), rhs);
    }
  }
  double x = 0.0;
#pragma unroll
  for (int p = NBX - 1; p >= 0; --p) {
    if (p < nb) {
      const double xp = readlane_d(rhs, piv[p]) * pinv[p];
      rhs = fma(-r[p], xp, rhs);
      x = lane == p ? xp : x;
    }
  }
  return x;
}

// The same elimination on the border in LDS, for borders of more than 32 DOFs: rows are
// exchanged, one lane per candidate row and a butterfly for the maximum; back substitution
// with one lane per column (two for borders of more than 64 DOFs) and a butterfly sum per row.
__device__ __forceinline__ void border_lu_lds(double DM_L* Bt, int ld, int nb, double DM_L* xB, int& bad) {
  const int lane = threadIdx.x;
  double amax = 0.0;           // largest assembled entry (see border_lu_regs)
  for (int q = lane; q < nb * nb; q += 64) amax = fmax(amax, fabs(Bt[(q / nb) * ld + q % nb]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
  for (int p = 0; p < nb; ++p) {
    double vm = (lane >= p && lane < nb) ? fabs(Bt[lane * ld + p]) : -1.0;
    int im = lane;
    for (int p2 = lane + 64; p2 < nb; p2 += 64) {
      const double v2 = fabs(Bt[p2 * ld + p]);
      if (p2 >= p && v2 > vm) { vm = v2; im = p2; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(vm, o, 64);
      const int oi = __shfl_xor(im, o, 64);
      if (ov > vm || (ov == vm && oi < im)) { vm = ov; im = oi; }
    }
    im = uniform(im);
    if (!(vm > 1e-300) || !isfinite(vm) || !(vm >= DM_PIVOT_TAU * amax)) bad = 1;
    if (im != p)
      for (int j = lane; j <= nb; j += 64) {
        const double t = Bt[p * ld + j];
        Bt[p * ld + j] = Bt[im * ld + j];
        Bt[im * ld + j] = t;
      }
    lds_order();
    const double inv = 1.0 / Bt[p * ld + p];
    const int w = nb - p;   // columns p+1 .. nb
    for (int q = lane; q < (nb - p - 1) * w; q += 64) {
      const int i = p + 1 + q / w, j = p + 1 + q % w;
      Bt[i * ld + j] -= Bt[i * ld + p] * inv * Bt[p * ld + j];
    }
    lds_order();
  }
  double x0 = 0.0, x1 = 0.0;      // solutions of columns lane and lane + 64
  for (int i = nb - 1; i >= 0; --i) {
    double part = 0.0;
    if (lane > i && lane < nb) part = Bt[i * ld + lane] * x0;
    if (lane + 64 > i && lane + 64 < nb) part += Bt[i * ld + lane + 64] * x1;
    const double xi = (Bt[i * ld + nb] - wave_sum(part)) / Bt[i * ld + i];
    if (lane == i) x0 = xi;
    if (lane + 64 == i) x1 = xi;
  }
  if (lane < nb) xB[lane] = x0;
  if (lane + 64 < nb) xB[lane + 64] = x1;
}

// Dense border solve by wavefront 0, without workgroup barriers (the workgroup meets once at
// the end): the arms' Schur contributions are added in arm order (each lane adds the slots the
// arm's table assigns it), then Gaussian elimination with partial pivoting.
__device__ __noinline__ void border_solve(ArgsP Ap, int sid, double DM_L* Bt, int ld,
                             const double DM_L* deltas, double DM_L* xB, double DM_L* scal, int DM_L* bad_flag) {
  const DmStepArgs DM_C& A = *uniform(Ap);
  const DmDev DM_C& D = A.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  (void)scal;
  const int nb = S.nb, lane = threadIdx.x, na = S.n_arms;
  if (threadIdx.x < 64) {
    for (int a0 = 0; a0 < na; a0 += 4) {
      int c0[4], c1[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {        // the table entries of four arms, loaded together
        const int* t = D.bsch + (size_t)(S.arm0 + (a0 + q < na ? a0 + q : 0)) * 110;
        c0[q] = t[lane];
        c1[q] = t[lane + 64 < 110 ? lane + 64 : 109];
        c1[q] = lane + 64 < 110 ? c1[q] : -1;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (a0 + q < na) {
          const double DM_L* dl = deltas + (a0 + q) * 110;
          if (c0[q] >= 0) Bt[(c0[q] >> 16) * ld + ((c0[q] >> 8) & 255)] += dl[c0[q] & 255];
          if (c1[q] >= 0) Bt[(c1[q] >> 16) * ld + ((c1[q] >> 8) & 255)] += dl[c1[q] & 255];
          lds_order();
        }
      }
    }
    int bad = 0;
    if (nb <= 32) {
      const double x = nb <= 10 ? border_lu_regs<10>(Bt, ld, nb, bad)
                     : nb <= 16 ? border_lu_regs<16>(Bt, ld, nb, bad) : border_lu_regs<32>(Bt, ld, nb, bad);
      if (lane < nb) xB[lane] = x;
    } else {
      border_lu_lds(Bt, ld, nb, xB, bad);
    }
    if (bad && lane == 0) *bad_flag = 1;
  }
  __syncthreads();
}

// q <- q - alpha delta over the system's nodes and edges.
__device__ __noinline__ void apply_update(ArgsP Ap, int sid, const double DM_L* xB, double alpha) {
  const DmStepArgs DM_C& A = *uniform(Ap);
  const DmDev DM_C& D = A.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  const int NN = D.n_nodes_tot;
  for (int i = threadIdx.x; i < S.n_nodes; i += blockDim.x) {
    const int n = S.node0 + i;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int h = D.node_home[c * NN + n];
      const double d = h >= 0 ? D.delta[h] : xB[-1 - h];
      D.x[c * NN + n] -= alpha * d;
    }
  }
  for (int i = threadIdx.x; i < S.n_edges; i += blockDim.x) {
    const int e = S.edge0 + i;
    const int h = D.edge_home[e];
    const double d = h >= 0 ? D.delta[h] : xB[-1 - h];
    D.th[e] -= alpha * d;
  }
}

__device__ __noinline__ void rollback(ArgsP Ap, int sid) {
  const DmStepArgs DM_C& A = *uniform(Ap);
  const DmDev DM_C& D = A.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  const int NN = D.n_nodes_tot;
  for (int i = threadIdx.x; i < S.n_nodes; i += blockDim.x)
#pragma unroll
    for (int c = 0; c < 3; ++c) D.x[c * NN + S.node0 + i] = D.x0[c * NN + S.node0 + i];
  for (int i = threadIdx.x; i < S.n_edges; i += blockDim.x) D.th[S.edge0 + i] = D.th0[S.edge0 + i];
}

// Velocity update (after Eq. 16) and the step-end reference frames.
// dt: the Newton step of the (sub)step just solved (half of it under midpoint).
__device__ __noinline__ void commit(ArgsP Ap, int sid, double dt) {
  const DmStepArgs DM_C& A = *uniform(Ap);
  const DmDev DM_C& D = A.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  const int NN = D.n_nodes_tot, NE = D.n_edges_tot, NS = D.n_st_tot;
  if (A.midpoint) {
    // implicit midpoint: the Newton solve (a backward-Euler solve over half the step) gave the
    // midpoint state q_m; the step ends at q_{n+1} = 2 q_m - q_n (clamped DOFs stay put)
    for (int i = threadIdx.x; i < S.n_nodes; i += blockDim.x)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int k = c * NN + S.node0 + i;
        D.x[k] = 2.0 * D.x[k] - D.x0[k];
      }
    for (int i = threadIdx.x; i < S.n_edges; i += blockDim.x) D.th[S.edge0 + i] = 2.0 * D.th[S.edge0 + i] - D.th0[S.edge0 + i];
    __syncthreads();
  }
  for (int i = threadIdx.x; i < S.n_st; i += blockDim.x) {
    const int s = S.st0 + i;
    const int np = D.sn[s], nc = D.sn[NS + s], nn = D.sn[2 * NS + s];
    const int ef = D.se[s], ee = D.se[NS + s];
    const int sg = D.ssign[s];
    const double sf = (sg & 1) ? -1.0 : 1.0, se = (sg & 2) ? -1.0 : 1.0;
    v3 a = ld3(D.x, NN, nc) - ld3(D.x, NN, np), b = ld3(D.x, NN, nn) - ld3(D.x, NN, nc);
    v3 tf = (1.0 / sqrt(dot(a, a))) * a, te = (1.0 / sqrt(dot(b, b))) * b;
    v3 d1f = transport_perp(sf * ld3(D.tref, NE, ef), tf, ld3(D.d1ref, NE, ef));
    v3 d1e = transport_perp(se * ld3(D.tref, NE, ee), te, ld3(D.d1ref, NE, ee));
    D.bref[s] = ref_twist(tf, d1f, te, d1e, D.bref[s], false);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < S.n_edges; i += blockDim.x) {
    const int e = S.edge0 + i;
    v3 d = ld3(D.x, NN, D.en[NE + e]) - ld3(D.x, NN, D.en[e]);
    v3 t = (1.0 / sqrt(dot(d, d))) * d;
    v3 d1 = transport_perp(ld3(D.tref, NE, e), t, ld3(D.d1ref, NE, e));
    st3(D.tref, NE, e, t);
    st3(D.d1ref, NE, e, d1);
    // backward Euler: (q_{n+1} - q_n) / dt; midpoint (dt = half the step):
    // 2 (q_{n+1} - q_n) / step - qdot_n
    const double om = (D.th[e] - D.th0[e]) / dt;
    D.om[e] = A.midpoint ? om - D.om[e] : om;
    D.th0[e] = D.th[e];
  }
  for (int i = threadIdx.x; i < S.n_nodes; i += blockDim.x) {
    const int n = S.node0 + i;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double v0 = D.v[c * NN + n], v = (D.x[c * NN + n] - D.x0[c * NN + n]) / dt;
      D.vprev2[c * NN + n] = D.vprev[c * NN + n];
      D.vprev[c * NN + n] = v0;
      D.v[c * NN + n] = A.midpoint ? v - v0 : v;
      D.x0[c * NN + n] = D.x[c * NN + n];
    }
  }
  __syncthreads();
}


// ---------------------------------------------------------------------------
// discrete adjoint of a stored trajectory segment (single-rod systems, no contact)
//
// Backward over step n -> n+1 with the state cotangents of n+1 held in ax, av, ath, aom,
// atref, ad1:
//   commit: v = (x - x_n)/dt, omega = (theta - theta_n)/dt, t_ref' = t(x),
//           d1_ref' = transport(t_ref, t(x), d1_ref) give the cotangent qbar of the Newton
//           root q = (x, theta) and direct cotangents of the step-start state;
//   implicit-function theorem: lambda = J^-1 qbar with J the step's Jacobian at q (symmetric
//           without friction), assembled and factorised by the same phases as the step;
//   every step-start input p of the residual receives -lambda^T dR/dp: inertia and damping
//           in closed form, the step-start frames and the natural curvature through the
//           stencil gradient in dual numbers seeded on those parameters.
// ---------------------------------------------------------------------------
using AdjP = const DmAdjArgs DM_C*;

__device__ __forceinline__ AdjP uniform(AdjP p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (AdjP)(((unsigned long long)hi << 32) | lo);
}

// Working state of step i of the segment: x, theta = q (state i+1); x0, v, theta0, omega,
// frames and reference twist = state i.
__device__ __noinline__ void adj_load_states(AdjP Pp, int sid, int i) {
  const DmAdjArgs DM_C& P = *uniform(Pp);
  const DmDev DM_C& D = P.s.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  const int NN = D.n_nodes_tot, NE = D.n_edges_tot;
  const size_t o_v = 3 * (size_t)NN, o_th = 6 * (size_t)NN, o_om = o_th + NE, o_tr = o_om + NE;
  const size_t o_d1 = o_tr + 3 * (size_t)NE, o_b = o_d1 + 3 * (size_t)NE;
  const double DM_C* s0 = P.a.seg + (size_t)uniform(i) * (size_t)P.a.stride;
  const double DM_C* s1 = s0 + P.a.stride;
  for (int k = threadIdx.x; k < S.n_nodes; k += blockDim.x) {
    const int n = S.node0 + k;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      D.x[c * NN + n] = s1[c * NN + n];
      D.x0[c * NN + n] = s0[c * NN + n];
      D.v[c * NN + n] = s0[o_v + c * NN + n];
    }
  }
  for (int k = threadIdx.x; k < S.n_edges; k += blockDim.x) {
    const int e = S.edge0 + k;
    D.th[e] = s1[o_th + e];
    D.th0[e] = s0[o_th + e];
    D.om[e] = s0[o_om + e];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      D.tref[c * NE + e] = s0[o_tr + c * NE + e];
      D.d1ref[c * NE + e] = s0[o_d1 + c * NE + e];
    }
  }
  for (int k = threadIdx.x; k < S.n_st; k += blockDim.x) D.bref[S.st0 + k] = s0[o_b + S.st0 + k];
}

// Loss gradient of the tip after step g + 1, then the commit's vector-Jacobian product per
// edge: cotangents of t_ref and d1_ref of the step start, and of the new edge vector (pe).
__device__ __noinline__ void adj_commit_vjp(AdjP Pp, int sid, int g) {
  const DmAdjArgs DM_C& P = *uniform(Pp);
  const DmDev DM_C& D = P.s.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  const DmAdjDev DM_C& J = P.a;
  const int NN = D.n_nodes_tot, NE = D.n_edges_tot;
  if (threadIdx.x == 0) {
    const DmChain DM_C& ch = D.chain[S.chain0];
    const int tip = D.chain_node[ch.node_tab + ch.n_nodes - 1];
    const double DM_C* dl = J.dLdtip + ((size_t)uniform(g) * J.n_rods + ch.rod) * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) J.ax[c * NN + tip] += dl[c];
  }
  for (int k = threadIdx.x; k < S.n_edges; k += blockDim.x) {
    const int e = S.edge0 + k;
    const v3 d = ld3(D.x, NN, D.en[NE + e]) - ld3(D.x, NN, D.en[e]);
    const double il = 1.0 / sqrt(dot(d, d));
    const v3 t = il * d;
    // u = v - c (a + b), c = (b.v)/(1 + a.b): a = t_ref, b = t, v = d1_ref
    const v3 a = ld3(D.tref, NE, e), v = ld3(D.d1ref, NE, e), ub = ld3(J.ad1, NE, e);
    const v3 sab = a + t;
    const double iden = 1.0 / (1.0 + dot(a, t));
    const double bv = dot(t, v), c = bv * iden, us = dot(ub, sab);
    const v3 vb = ub - (us * iden) * t;
    const v3 ab = (us * bv * iden * iden) * t - c * ub;
    const v3 bb = (-us) * (iden * v - (bv * iden * iden) * a) - c * ub;
    const v3 tb = ld3(J.atref, NE, e) + bb;
    const v3 eb = il * (tb - dot(t, tb) * t);           // through t = e / |e|
    st3(J.pe, NE, e, eb);
    st3(J.atref, NE, e, ab);
    st3(J.ad1, NE, e, vb);
  }
}

// Right-hand side qbar of the adjoint solve, in the band (R) and the border column of Bt.
__device__ __noinline__ void adj_rhs(AdjP Pp, int sid, double DM_L* Bt, int ld) {
  const DmAdjArgs DM_C& P = *uniform(Pp);
  const DmDev DM_C& D = P.s.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  const DmAdjDev DM_C& J = P.a;
  const int NN = D.n_nodes_tot, NE = D.n_edges_tot;
  const double idt = 1.0 / P.s.dt;
  const DmChain DM_C& ch = D.chain[S.chain0];
  const int n = 4 * ch.n_nodes - 1;
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    const int k = r >> 2, c = r & 3;
    double qb;
    if (c < 3) {
      const int node = D.chain_node[ch.node_tab + k];
      qb = J.ax[c * NN + node] + J.av[c * NN + node] * idt;
      if (k >= 1) qb += J.pe[c * NE + D.chain_edge[ch.edge_tab + k - 1]];
      if (k <= ch.n_nodes - 2) qb -= J.pe[c * NE + D.chain_edge[ch.edge_tab + k]];
    } else {
      const int e = D.chain_edge[ch.edge_tab + k];
      qb = J.ath[e] + J.aom[e] * idt;
    }
    if (D.cfix[ch.dof_off + r]) qb = 0.0;
    if (r >= ch.b_lo && r < ch.b_hi) Bt[D.bmap[ch.bmap_off + r - ch.b_lo] * ld + S.nb] = qb;
    else D.R[ch.dof_off + r] = qb;
  }
}

__device__ __noinline__ void adj_store_lambda(AdjP Pp, int sid, const double DM_L* xB) {
  const DmAdjArgs DM_C& P = *uniform(Pp);
  const DmDev DM_C& D = P.s.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  const int NN = D.n_nodes_tot;
  for (int i = threadIdx.x; i < S.n_nodes; i += blockDim.x) {
    const int n = S.node0 + i;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int h = D.node_home[c * NN + n];
      P.a.lam[c * NN + n] = h >= 0 ? D.delta[h] : xB[-1 - h];
    }
  }
  for (int i = threadIdx.x; i < S.n_edges; i += blockDim.x) {
    const int e = S.edge0 + i;
    const int h = D.edge_home[e];
    P.a.lam[3 * NN + e] = h >= 0 ? D.delta[h] : xB[-1 - h];
  }
}

// Per stencil: derivatives of psi = lambda_loc . g_loc with respect to the step-start frames
// of both edges and the natural curvature, stored as pst[q] for the 16 parameters
// q = (t_f.x, t_f.y, t_f.z, kbar1, d1_f.x, d1_f.y, d1_f.z, kbar2, t_e.x, t_e.y, t_e.z, -,
// d1_e.x, d1_e.y, d1_e.z, -) (the two unused slots hold zero).  One lane-task per stencil and
// parameter, a 1-tangent dual pass seeded on that parameter (seeds selected by value); 64
// consecutive stencils per wavefront and parameter.
__device__ __forceinline__ void adj_stencil_task(const DmAdjArgs DM_C& P, int s, int q) {
  typedef Dual<1> D1;
  const DmDev DM_C& D = P.s.d;
  const int NS = D.n_st_tot, NE = D.n_edges_tot, NN = D.n_nodes_tot;
  if ((q & 3) == 3 && q >= 8) {            // no parameter
    P.a.pst[q * NS + s] = 0.0;
    return;
  }
  const int np = D.sn[s], nc = D.sn[NS + s], nn = D.sn[2 * NS + s];
  const int ef = D.se[s], ee = D.se[NS + s];
  const int sg = D.ssign[s];
  const double sf = (sg & 1) ? -1.0 : 1.0, se = (sg & 2) ? -1.0 : 1.0;
  const v3 xc = ld3(D.x, NN, nc);
  const v3 efv = xc - ld3(D.x, NN, np), eev = ld3(D.x, NN, nn) - xc;
  const v3 lp = ld3(P.a.lam, NN, np), lc = ld3(P.a.lam, NN, nc), ln = ld3(P.a.lam, NN, nn);
  const v3 l0 = lc - lp, l1 = ln - lc;
  const double l8[8] = {l0.x, l0.y, l0.z, l1.x, l1.y, l1.z, sf * P.a.lam[3 * NN + ef], se * P.a.lam[3 * NN + ee]};
  const v3 tnf = sf * ld3(D.tref, NE, ef), d1nf = ld3(D.d1ref, NE, ef);
  const v3 tne = se * ld3(D.tref, NE, ee), d1ne = ld3(D.d1ref, NE, ee);
  auto seed = [&](int p) { return q == p ? 1.0 : 0.0; };
  Vec<D1> TNF = liftv<D1>(tnf), D1NF = liftv<D1>(d1nf), TNE = liftv<D1>(tne), D1NE = liftv<D1>(d1ne);
  D1 K1 = lift<D1>(D.kbar[s]), K2 = lift<D1>(D.kbar[NS + s]);
  TNF.x.d[0] = seed(0); TNF.y.d[0] = seed(1); TNF.z.d[0] = seed(2); K1.d[0] = seed(3);
  D1NF.x.d[0] = seed(4); D1NF.y.d[0] = seed(5); D1NF.z.d[0] = seed(6); K2.d[0] = seed(7);
  TNE.x.d[0] = seed(8); TNE.y.d[0] = seed(9); TNE.z.d[0] = seed(10);
  D1NE.x.d[0] = seed(12); D1NE.y.d[0] = seed(13); D1NE.z.d[0] = seed(14);
  D1 g8[8];
  stencil_grad_g(liftv<D1>(efv), liftv<D1>(eev), lift<D1>(sf * D.th[ef]), lift<D1>(se * D.th[ee]), TNF, D1NF, TNE,
                 D1NE, D.bref[s], K1, K2, D.tbar[s], D.kbend[s], D.ktwist[s], g8);
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < 8; ++a) acc += l8[a] * g8[a].d[0];
  P.a.pst[q * NS + s] = acc;
}

__device__ __noinline__ void adj_stencils(AdjP Pp, int sid) {
  const DmAdjArgs DM_C& P = *uniform(Pp);
  const DmSystem DM_C& S = P.s.d.sys[uniform(sid)];
  for (int i = threadIdx.x; i < 1024 * ((S.n_st + 63) >> 6); i += blockDim.x) {
    const int st = ((i >> 10) << 6) + (i & 63);
    const int q = (i >> 6) & 15;
    if (st < S.n_st) adj_stencil_task(P, S.st0 + st, q);
  }
}

// Cotangents of the step-start state (and the natural-curvature gradient) from lambda.
__device__ __noinline__ void adj_update(AdjP Pp, int sid) {
  const DmAdjArgs DM_C& P = *uniform(Pp);
  const DmDev DM_C& D = P.s.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  const DmAdjDev DM_C& J = P.a;
  const int NS = D.n_st_tot, NE = D.n_edges_tot, NN = D.n_nodes_tot;
  const double dt = P.s.dt, idt = 1.0 / dt, damp = P.s.damping;
  for (int i = threadIdx.x; i < S.n_nodes; i += blockDim.x) {
    const int n = S.node0 + i;
    const double m = D.mass[n];
    const double cx = m * idt * idt + damp * m * idt;     // -dR_x/dx_n
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double lx = J.lam[c * NN + n];
      J.ax[c * NN + n] = -J.av[c * NN + n] * idt + cx * lx;
      J.av[c * NN + n] = m * idt * lx;
    }
  }
  const DmChain DM_C& ch = D.chain[S.chain0];
  const int N = ch.n_nodes;
  for (int k = threadIdx.x; k < N - 1; k += blockDim.x) {
    const int e = D.chain_edge[ch.edge_tab + k];
    const double lt = J.lam[3 * NN + e], I = D.Ith[e];
    J.ath[e] = -J.aom[e] * idt + I * idt * idt * lt;
    J.aom[e] = I * idt * lt;
    v3 tb = ld3(J.atref, NE, e), db = ld3(J.ad1, NE, e);
    if (k + 1 <= N - 2) {          // edge k is the f edge of the stencil centred on node k+1
      const int s = ch.st_off + k;
      const double sf = (D.ssign[s] & 1) ? -1.0 : 1.0;
      tb = tb - sf * mk3(J.pst[0 * NS + s], J.pst[1 * NS + s], J.pst[2 * NS + s]);
      db = db - mk3(J.pst[4 * NS + s], J.pst[5 * NS + s], J.pst[6 * NS + s]);
    }
    if (k >= 1 && k <= N - 2) {    // and the e edge of the stencil centred on node k
      const int s = ch.st_off + k - 1;
      const double se = (D.ssign[s] & 2) ? -1.0 : 1.0;
      tb = tb - se * mk3(J.pst[8 * NS + s], J.pst[9 * NS + s], J.pst[10 * NS + s]);
      db = db - mk3(J.pst[12 * NS + s], J.pst[13 * NS + s], J.pst[14 * NS + s]);
    }
    st3(J.atref, NE, e, tb);
    st3(J.ad1, NE, e, db);
  }
  for (int i = threadIdx.x; i < S.n_st; i += blockDim.x) {
    const int s = S.st0 + i;
    J.akap[s] -= J.pst[3 * NS + s];
    J.akap[NS + s] -= J.pst[7 * NS + s];
  }
}

// ---------------------------------------------------------------------------
// limb curvature of an equilibrium and its gradient with respect to natural curvature
//
// At a settled state (the committed state, its own step start) the residual of one more step
// of dt, R(q; kbar), vanishes; d/dkbar of sum_s w_s kappa1_s (Eq. 5's first curvature) is then
// -mu^T dR/dkbar with J mu = d(sum w kappa1)/dq (J symmetric without friction), and
// dR/dkbar_s (the stencil's natural curvature in 1/m, first component) = -kbend_s Vbar_s
// d kappa1_s / dq, so the derivative is kbend_s Vbar_s mu . d kappa1_s / dq per stencil.
// ---------------------------------------------------------------------------
using CurvP = const DmCurvArgs DM_C*;

__device__ __forceinline__ CurvP uniform(CurvP p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (CurvP)(((unsigned long long)hi << 32) | lo);
}

// d kappa1 / d(e_f, e_e, theta_f, theta_e) of stencil s at the committed state (frames carried
// from the step start, which is the committed state itself).
__device__ __forceinline__ void kappa1_grad(const DmDev DM_C& D, int s, double* g8) {
  const int NS = D.n_st_tot, NE = D.n_edges_tot, NN = D.n_nodes_tot;
  const int np = D.sn[s], nc = D.sn[NS + s], nn = D.sn[2 * NS + s];
  const int ef = D.se[s], ee = D.se[NS + s];
  const int sg = D.ssign[s];
  const double sf = (sg & 1) ? -1.0 : 1.0, se = (sg & 2) ? -1.0 : 1.0;
  const v3 xc = ld3(D.x, NN, nc);
  stencil_kappa1_grad_g<double>(tov(xc - ld3(D.x, NN, np)), tov(ld3(D.x, NN, nn) - xc), sf * D.th[ef],
                                se * D.th[ee], tov(sf * ld3(D.tref, NE, ef)), tov(ld3(D.d1ref, NE, ef)),
                                tov(se * ld3(D.tref, NE, ee)), tov(ld3(D.d1ref, NE, ee)), g8);
}

// Right-hand side vectors: st_g = w_s d kappa1_s / dv (zero where w_s is zero, joint stencils
// included); the unweighted gradient is kept in st_H's first 8 rows for curv_params.
__device__ __noinline__ void curv_rhs(CurvP Cp, int sid) {
  const DmCurvArgs DM_C& C = *uniform(Cp);
  const DmDev DM_C& D = C.s.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  const int NS = D.n_st_tot;
  for (int i = threadIdx.x; i < S.n_st; i += blockDim.x) {
    const int s = S.st0 + i;
    const double w = C.c.wst[s];
    double g8[8];
    kappa1_grad(D, s, g8);
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      D.st_g[a * NS + s] = w * g8[a];
      D.st_H[a * NS + s] = g8[a];
    }
  }
}

// mu of every node position and edge twist from the solve (band rows or the border).
__device__ __noinline__ void curv_store_mu(CurvP Cp, int sid, const double DM_L* xB) {
  const DmCurvArgs DM_C& C = *uniform(Cp);
  const DmDev DM_C& D = C.s.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  const int NN = D.n_nodes_tot;
  for (int i = threadIdx.x; i < S.n_nodes; i += blockDim.x) {
    const int n = S.node0 + i;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int h = D.node_home[c * NN + n];
      C.c.mu[c * NN + n] = h >= 0 ? D.delta[h] : xB[-1 - h];
    }
  }
  for (int i = threadIdx.x; i < S.n_edges; i += blockDim.x) {
    const int e = S.edge0 + i;
    const int h = D.edge_home[e];
    C.c.mu[3 * NN + e] = h >= 0 ? D.delta[h] : xB[-1 - h];
  }
}

// Per stencil: kbend Vbar (mu_loc . d kappa1 / dq_loc), mu_loc mapped to the stencil variables
// (x_c - x_p, x_n - x_c, and the signed twists).
__device__ __noinline__ void curv_params(CurvP Cp, int sid) {
  const DmCurvArgs DM_C& C = *uniform(Cp);
  const DmDev DM_C& D = C.s.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  const int NS = D.n_st_tot, NN = D.n_nodes_tot;
  for (int i = threadIdx.x; i < S.n_st; i += blockDim.x) {
    const int s = S.st0 + i;
    const int np = D.sn[s], nc = D.sn[NS + s], nn = D.sn[2 * NS + s];
    const int ef = D.se[s], ee = D.se[NS + s];
    const int sg = D.ssign[s];
    const double sf = (sg & 1) ? -1.0 : 1.0, se = (sg & 2) ? -1.0 : 1.0;
    const v3 lp = ld3(C.c.mu, NN, np), lc = ld3(C.c.mu, NN, nc), ln = ld3(C.c.mu, NN, nn);
    const v3 l0 = lc - lp, l1 = ln - lc;
    const double l8[8] = {l0.x, l0.y, l0.z, l1.x, l1.y, l1.z, sf * C.c.mu[3 * NN + ef], se * C.c.mu[3 * NN + ee]};
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) acc = fma(l8[a], D.st_H[a * NS + s], acc);
    C.c.pst[s] = D.kbend[s] * D.Vbar[s] * acc;
  }
}

// kappa1 / Vbar of stencil s at the committed state, the frames being the step-start ones.
__device__ __forceinline__ double stencil_curvature(const DmDev DM_C& D, int s) {
  const int NS = D.n_st_tot, NE = D.n_edges_tot;
  const int ef = D.se[s], ee = D.se[NS + s];
  const int sg = D.ssign[s];
  const double sf = (sg & 1) ? -1.0 : 1.0, se = (sg & 2) ? -1.0 : 1.0;
  double k1, k2, b;
  stencil_strains(sf * ld3(D.tref, NE, ef), ld3(D.d1ref, NE, ef), sf * D.th[ef], se * ld3(D.tref, NE, ee),
                  ld3(D.d1ref, NE, ee), se * D.th[ee], D.bref[s], true, &k1, &k2, &b);
  return k1 / D.Vbar[s];
}

}  // namespace

// First curvature over the rest Voronoi length (1/m) of every stencil at the committed state.
__global__ void dm_stencil_curvature_kernel(DmStepArgs, double* out) {
  const ArgsP Ap = (ArgsP)__builtin_amdgcn_kernarg_segment_ptr();   // the by-value argument
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < Ap->d.n_st_tot) out[s] = stencil_curvature(Ap->d, s);
}

extern "C" hipError_t dm_launch_stencil_curvature(const DmStepArgs* args, double* out, hipStream_t stream) {
  const int n = args->d.n_st_tot;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dm_stencil_curvature_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, *args, out);
  return hipGetLastError();
}

// Gradient of sum_s w_s kappa1_s of an equilibrium with respect to the stencils' natural
// curvature; one workgroup per system (systems marked in skip are left alone).
__global__ void __launch_bounds__(512) dm_curvature_adjoint_kernel(DmCurvArgs) {
  extern __shared__ double lds_raw[];
  double DM_L* lds = (double DM_L*)lds_raw;
  const CurvP Cp = (CurvP)__builtin_amdgcn_kernarg_segment_ptr();
  const ArgsP Ap = (ArgsP)__builtin_amdgcn_kernarg_segment_ptr();   // the step arguments lead
  const DmCurvArgs DM_C& C = *Cp;
  const DmStepArgs DM_C& A = C.s;
  const DmDev DM_C& D = A.d;
  const int sid = D.order[blockIdx.x];
  if (C.c.skip && C.c.skip[sid]) return;           // the whole workgroup, before any barrier
  const DmSystem DM_C& S = D.sys[sid];
  const int ld = A.max_nb + 1;
  double DM_L* Bt = lds;
  double DM_L* deltas = Bt + A.max_nb * ld;
  double DM_L* xB = deltas + A.max_arms * 110;
  double DM_L* red = xB + A.max_nb;
  int DM_L* flags = (int DM_L*)(red + 40);
  const int tid = threadIdx.x, wave = tid >> 6, nwaves = blockDim.x >> 6;
  if (tid == 0) flags[0] = 0;
  __syncthreads();
  const double t_end = D.time[sid] + A.dt;
  eval_stencils<true>(Ap, sid, t_end);
  eval_edges_nodes(Ap, sid, A.dt);
  __syncthreads();
  assemble_band<2>(Ap, sid, A.dt);
  __syncthreads();
  assemble_border<2>(Ap, sid, Bt, ld, red + 42);
  __syncthreads();
  curv_rhs(Cp, sid);
  __syncthreads();
  assemble_band<3>(Ap, sid, A.dt);
  __syncthreads();
  assemble_border<1>(Ap, sid, Bt, ld, red + 42);
  __syncthreads();
  sweep_all(Ap, S, wave, nwaves, deltas, flags);
  __syncthreads();
  border_solve(Ap, sid, Bt, ld, deltas, xB, red + 34, flags);
  backsub_all(Ap, S, wave, nwaves, xB);
  __syncthreads();
  const bool bad = flags[0] != 0;
  if (!bad) {
    curv_store_mu(Cp, sid, xB);
    __syncthreads();
    curv_params(Cp, sid);
  }
  if (tid == 0) D.s_status[sid] = bad ? DM_STATUS_SINGULAR : DM_STATUS_OK;
}

extern "C" hipError_t dm_launch_curvature_adjoint(const DmCurvArgs* args, int block, size_t lds_bytes,
                                                  hipStream_t stream) {
  hipLaunchKernelGGL(dm_curvature_adjoint_kernel, dim3(args->s.n_systems), dim3(block), lds_bytes, stream, *args);
  return hipGetLastError();
}

// The step of every system (one workgroup each); SC: the rods' edge-edge self-contact
// (dm_step_sc_kernel), compiled apart so that the plain kernel carries none of its code.
template <bool SC>
__device__ __forceinline__ void step_body() {
  extern __shared__ double lds_raw[];
  double DM_L* lds = (double DM_L*)lds_raw;
  // the by-value argument sits at offset 0 of the argument segment
  const ArgsP Ap = (ArgsP)__builtin_amdgcn_kernarg_segment_ptr();
  const DmStepArgs DM_C& A = *Ap;
  const DmDev DM_C& D = A.d;
  const int sid = D.order[blockIdx.x];
  const DmSystem DM_C& S = D.sys[sid];
  const int ld = A.max_nb + 1;
  double DM_L* Bt = lds;                                   // [max_nb][max_nb + 1]
  double DM_L* deltas = Bt + A.max_nb * ld;                // [max_arms][110]
  double DM_L* xB = deltas + A.max_arms * 110;             // [max_nb]
  double DM_L* red = xB + A.max_nb;                        // [40]
  int DM_L* flags = (int DM_L*)(red + 40);      // [4]; then border term segment sums at red + 42
  unsigned short DM_L* hbuf = (unsigned short DM_L*)((char DM_L*)lds_raw + A.net_lds);   // network (warm == 2)
  const int tid = threadIdx.x, wave = tid >> 6, nwaves = blockDim.x >> 6;
  if (tid == 0) {
    flags[0] = 0;       // singular pivot
    flags[1] = 0;       // more self-contact pairs than the list holds
    red[37] = 0.0;      // largest floor-ended residual of this launch and its floor estimate
    red[38] = 0.0;
  }
  int status = DM_STATUS_OK, iters = 0, steps = 0, floor_hits = 0, fallbacks = 0, halved = 0;
  double res = 0.0;
  double t = D.time[sid];
  // accumulating launches (one step each) leave a system alone once it has failed
  const int nsteps = ((A.accum && D.s_status[sid] != DM_STATUS_OK) || (A.skip && A.skip[sid])) ? 0 : A.nsteps;
  __syncthreads();
  DM_T0();
  for (int step = 0; step < nsteps; ++step) {
    // adaptive halving: substep (lev, idx) covers [idx, idx + 1) dt / 2^lev of the step; a
    // substep whose Newton solve fails is covered by its two halves, down to level
    // A.max_halvings; after a converged substep the next is the following sibling in that
    // binary tree (a right child completes its parent)
    int lev = 0, idx = 0;
    bool failed = false;
    while (true) {
      const double hn = ldexp(A.dt, -lev);        // the substep's Newton step
      const double t_end = t + hn;
      bool conv = false;
      int newton = 0;
      if (A.warm) {
        warm_guess(Ap, sid, hbuf, nullptr, hn);
        __syncthreads();
      }
      // attempt 0 starts from the current positions (the substep start, or a warm-start
      // guess); with a warm start, a failed attempt is repeated from the substep start
      for (int attempt = 0; attempt < (A.warm ? 2 : 1) && !conv; ++attempt) {
        if (attempt == 1) {
          rollback(Ap, sid);
          if (tid == 0) flags[0] = 0;
          ++fallbacks;
          __syncthreads();
        }
        int it = 0, halvings = 0;
        double alpha = 1.0, res_prev = 0.0;
        while (true) {
          // residual pass: stencil gradients, edge and node terms, the residual of every row
          eval_stencil_grads(Ap, sid, t_end);
          eval_edges_nodes(Ap, sid, hn);
          __syncthreads();
          if (SC) {
            self_contact(Ap, sid, hn, flags);
            __syncthreads();
            if (flags[1]) break;        // more pairs than the list holds: the system fails
          }
          DM_TP(0);
          double r2 = assemble_band<1>(Ap, sid, hn);
          __syncthreads();
          r2 += assemble_border<1>(Ap, sid, Bt, ld, red + 42);
          res = sqrt(block_sum(r2, red));
          DM_TP(1);
          if (res <= A.tol) { conv = true; break; }   // (a rise under line search is above tol)
          const bool rise = A.line_search && it > 0 && res >= res_prev;
          const bool stall = it > 0 && res > 0.5 * res_prev && A.floor_factor > 0.0;
          const bool give_up = it >= (A.warm && attempt == 0 ? A.warm_max_iter : A.max_iter) || !isfinite(res);
          if (give_up && !rise && !stall) break;
          // matrix pass, only when a decision or a solve follows: stencil Hessians, the band and
          // the dense border's matrix part
          eval_stencils<false>(Ap, sid, t_end);
          __syncthreads();
          assemble_band<2>(Ap, sid, hn);
          __syncthreads();
          assemble_border<2>(Ap, sid, Bt, ld, red + 42);
          __syncthreads();
          DM_TP(2);
          // the rounding floor is needed only where a decision reads it: a residual that rose
          // under line search, or one that stopped halving above the tolerance
          const double flo = (rise || stall) ? residual_floor(Ap, sid, Bt, ld, red) : 0.0;
          // line search: a step whose residual did not decrease is halved (at most 10 times),
          // unless its residual is within the iterate's rounding floor (noise, not a bad step)
          if (rise && res > flo && halvings < 10) {
            apply_update(Ap, sid, xB, -0.5 * alpha);      // back off to half of the current step
            alpha *= 0.5;
            ++halvings;
            __syncthreads();
            continue;
          }
          if (stall && res <= flo) {
            conv = true;    // the step stopped improving at or below its FP64 rounding floor
            ++floor_hits;
            if (tid == 0 && res > red[37]) { red[37] = res; red[38] = flo; }   // kept in LDS
            break;
          }
          if (give_up) break;
          res_prev = res;
          alpha = 1.0;
          halvings = 0;
          // the arm sweeps, the border solve and the back-substitutions are serial chains on
          // the critical path of the system: their wavefronts take issue priority over the
          // other workgroups' element and assembly work sharing the SIMDs
          if (SC) {
            sc_solve(Ap, sid, hn, xB, flags);     // the rod's Jacobian with its contact pairs
          } else {
            __builtin_amdgcn_s_setprio(3);
            sweep_all(Ap, S, wave, nwaves, deltas, flags);
            __syncthreads();
            DM_TP(3);
            border_solve(Ap, sid, Bt, ld, deltas, xB, red + 34, flags);
            DM_TP(4);
            backsub_all(Ap, S, wave, nwaves, xB);
            __builtin_amdgcn_s_setprio(0);
            __syncthreads();
          }
          DM_TP(5);
          if (flags[0]) break;
          apply_update(Ap, sid, xB, 1.0);
          ++it;
          ++newton;
          __syncthreads();
          DM_TP(6);
        }
      }
      iters += newton;
      if (!conv) {
        const bool singular = flags[0] != 0;
        const bool overflow = SC && flags[1];
        rollback(Ap, sid);
        if (lev < A.max_halvings && !overflow) {
          ++lev;
          idx *= 2;
          ++halved;
          if (tid == 0) flags[0] = 0;
          __syncthreads();
          continue;
        }
        // the system stays at the end of its last converged substep
        status = overflow ? DM_STATUS_CONTACT_OVERFLOW : (singular ? DM_STATUS_SINGULAR : DM_STATUS_NOT_CONVERGED);
        failed = true;
        break;
      }
      commit(Ap, sid, hn);
      DM_TP(7);
      t += A.midpoint ? 2.0 * hn : hn;
      while (lev > 0 && (idx & 1)) { --lev; idx >>= 1; }
      if (lev == 0) break;
      ++idx;
    }
    if (failed) break;
    ++steps;
  }
  DM_TSAVE(sid);
  if (tid == 0 && nsteps > 0) {
    D.time[sid] = t;
    D.s_status[sid] = status;
    D.s_res[sid] = res;
    if (A.accum) {
      D.s_steps[sid] += steps;
      D.s_iters[sid] += iters;
      D.s_floor[sid] += floor_hits;
      D.s_fallback[sid] += fallbacks;
      D.s_halved[sid] += halved;
      if (red[37] > D.s_floor_res[sid]) { D.s_floor_res[sid] = red[37]; D.s_floor_est[sid] = red[38]; }
    } else {
      D.s_steps[sid] = steps;
      D.s_iters[sid] = iters;
      D.s_floor[sid] = floor_hits;
      D.s_fallback[sid] = fallbacks;
      D.s_halved[sid] = halved;
      D.s_floor_res[sid] = red[37];
      D.s_floor_est[sid] = red[38];
    }
  }
}

__global__ void __launch_bounds__(512) dm_step_kernel(DmStepArgs) { step_body<false>(); }
__global__ void __launch_bounds__(512) dm_step_sc_kernel(DmStepArgs) { step_body<true>(); }

extern "C" hipError_t dm_launch_step(const DmStepArgs* args, int block, size_t lds_bytes, hipStream_t stream) {
  if (args->sc_on)
    hipLaunchKernelGGL(dm_step_sc_kernel, dim3(args->n_systems), dim3(block), lds_bytes, stream, *args);
  else
    hipLaunchKernelGGL(dm_step_kernel, dim3(args->n_systems), dim3(block), lds_bytes, stream, *args);
  return hipGetLastError();
}

// Step-start guess of every system without stepping: out[row][3] = predicted displacement of
// each chain-node row for the warm mode in the arguments.  One workgroup per system.
__global__ void __launch_bounds__(512) dm_predict_kernel(DmStepArgs, double* out) {
  extern __shared__ double lds_raw[];
  const ArgsP Ap = (ArgsP)__builtin_amdgcn_kernarg_segment_ptr();
  unsigned short DM_L* hbuf = (unsigned short DM_L*)((char DM_L*)lds_raw + Ap->net_lds);
  warm_guess(Ap, blockIdx.x, hbuf, (double DM_G*)out, Ap->dt);
}

extern "C" hipError_t dm_launch_predict(const DmStepArgs* args, int block, size_t lds_bytes, double* out,
                                        hipStream_t stream) {
  hipLaunchKernelGGL(dm_predict_kernel, dim3(args->n_systems), dim3(block), lds_bytes, stream, *args, out);
  return hipGetLastError();
}

// Backward over the steps of one stored segment, last step first; one workgroup per system.
__global__ void __launch_bounds__(512) dm_adjoint_kernel(DmAdjArgs) {
  extern __shared__ double lds_raw[];
  double DM_L* lds = (double DM_L*)lds_raw;
  const AdjP Pp = (AdjP)__builtin_amdgcn_kernarg_segment_ptr();
  const ArgsP Ap = (ArgsP)__builtin_amdgcn_kernarg_segment_ptr();   // the step arguments lead
  const DmAdjArgs DM_C& P = *Pp;
  const DmStepArgs DM_C& A = P.s;
  const DmDev DM_C& D = A.d;
  const int sid = D.order[blockIdx.x];
  const DmSystem DM_C& S = D.sys[sid];
  const int ld = A.max_nb + 1;
  double DM_L* Bt = lds;
  double DM_L* deltas = Bt + A.max_nb * ld;
  double DM_L* xB = deltas + A.max_arms * 110;
  double DM_L* red = xB + A.max_nb;
  int DM_L* flags = (int DM_L*)(red + 40);
  const int tid = threadIdx.x, wave = tid >> 6, nwaves = blockDim.x >> 6;
  if (tid == 0) flags[0] = 0;
  int status = DM_STATUS_OK;
  __syncthreads();
  for (int i = P.a.seg_len - 1; i >= 0; --i) {
    adj_load_states(Pp, sid, i);
    __syncthreads();
    adj_commit_vjp(Pp, sid, P.a.step0 + i);
    eval_stencils<true>(Ap, sid, 0.0);
    eval_edges_nodes(Ap, sid, A.dt);
    __syncthreads();
    assemble_band<0>(Ap, sid, A.dt);
    __syncthreads();
    assemble_border<0>(Ap, sid, Bt, ld, red + 42);
    __syncthreads();
    adj_rhs(Pp, sid, Bt, ld);
    __syncthreads();
    sweep_all(Ap, S, wave, nwaves, deltas, flags);
    __syncthreads();
    border_solve(Ap, sid, Bt, ld, deltas, xB, red + 34, flags);
    backsub_all(Ap, S, wave, nwaves, xB);
    __syncthreads();
    if (flags[0]) { status = DM_STATUS_SINGULAR; break; }
    adj_store_lambda(Pp, sid, xB);
    __syncthreads();
    adj_stencils(Pp, sid);
    __syncthreads();
    adj_update(Pp, sid);
    __syncthreads();
  }
  if (tid == 0) D.s_status[sid] = status;
}

__global__ void dm_gather_tips_kernel(const double* x, int nn, const int* tip, int n, double* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n)
    for (int c = 0; c < 3; ++c) out[3 * r + c] = x[c * nn + tip[r]];
}

extern "C" hipError_t dm_launch_adjoint(const DmAdjArgs* args, int block, size_t lds_bytes, hipStream_t stream) {
  hipLaunchKernelGGL(dm_adjoint_kernel, dim3(args->s.n_systems), dim3(block), lds_bytes, stream, *args);
  return hipGetLastError();
}

// Tip loss of one fitting iterate: loss = sum over the n entries of (tips - target)^2 and
// dL = 2 (tips - target); one 1024-thread workgroup, summed in a fixed order.
__global__ void __launch_bounds__(1024) dm_fit_loss_kernel(const double* tips, const double* target, int n,
                                                          double* dL, double* loss) {
  __shared__ double part[1024];
  double sum = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double d = tips[i] - target[i];
    dL[i] = 2.0 * d;
    sum = fma(d, d, sum);
  }
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = part[0];
}

// y <- y + a x over n entries.
__global__ void dm_axpy_kernel(double* y, const double* x, double a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = fma(a, x[i], y[i]);
}

extern "C" hipError_t dm_launch_fit_loss(const double* tips, const double* target, int n, double* dL, double* loss,
                                         hipStream_t stream) {
  hipLaunchKernelGGL(dm_fit_loss_kernel, dim3(1), dim3(1024), 0, stream, tips, target, n, dL, loss);
  return hipGetLastError();
}

extern "C" hipError_t dm_launch_axpy(double* y, const double* x, double a, int n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dm_axpy_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, y, x, a, n);
  return hipGetLastError();
}

extern "C" hipError_t dm_launch_gather_tips(const double* x, int nn, const int* tip, int n, double* out,
                                            hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dm_gather_tips_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, x, nn, tip, n, out);
  return hipGetLastError();
}
