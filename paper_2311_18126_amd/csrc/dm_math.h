// dm_math.h -- element math of the implicit DER step in FP64.
//
// Bend/twist stencil (Eq. 4-8) with frames carried from the step-start frames by
// time-parallel transport.  The force is the exact gradient of that energy (Eq. 9)
// and its Jacobian the exact Hessian (Eq. 16):
//   * first derivatives of the strains are closed-form: the classical DER expressions
//     plus, per edge, the time-transport holonomy term  w = -(t_n x t) / ((1 + t_n.t) |e|),
//     which adds (d strain / d theta) w to the edge gradient (rotating the transported
//     director about t is the same as changing theta);
//   * second derivatives come from evaluating those closed forms in forward-mode dual
//     numbers seeded on the 8 stencil variables (two edge vectors, two twist angles), so
//     each dual's tangent is a row of the Hessian.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#define DM_HD __host__ __device__ __forceinline__

// The scalar of the element math: double in every build of the step; a host program that
// counts the method's floating-point operations defines DM_REAL_COUNTED and supplies its own
// counting scalar as dm_real (with the functions used here) before including this header.
#ifndef DM_REAL_COUNTED
typedef double dm_real;
#endif

// ---------------------------------------------------------------------------
// plain double 3-vectors
// ---------------------------------------------------------------------------
struct v3 { dm_real x, y, z; };
DM_HD v3 mk3(dm_real a, dm_real b, dm_real c) { v3 r; r.x = a; r.y = b; r.z = c; return r; }
DM_HD v3 operator+(v3 a, v3 b) { return mk3(a.x + b.x, a.y + b.y, a.z + b.z); }
DM_HD v3 operator-(v3 a, v3 b) { return mk3(a.x - b.x, a.y - b.y, a.z - b.z); }
DM_HD v3 operator*(dm_real s, v3 a) { return mk3(s * a.x, s * a.y, s * a.z); }
DM_HD dm_real dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
DM_HD v3 cross(v3 a, v3 b) { return mk3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }

// Stretch (Eq. 2-3) of an edge with vector d, stiffness EA and rest length eb: the gradient
// EA (|d|/eb - 1) t with respect to the edge vector (out[0..2]) and its Hessian
// (EA/eb) t t^T + EA (1/eb - 1/|d|)(I - t t^T) as xx xy xz yy yz zz (out[3..8]).
DM_HD void stretch_terms(v3 d, dm_real EA, dm_real eb, dm_real* out) {
  dm_real l = sqrt(dot(d, d));
  v3 t = (1.0 / l) * d;
  dm_real f = EA * (l / eb - 1.0);
  dm_real c1 = EA / eb, c2 = EA * (1.0 / eb - 1.0 / l);
  dm_real tt[3] = {t.x, t.y, t.z};
  out[0] = f * t.x;
  out[1] = f * t.y;
  out[2] = f * t.z;
  int k = 3;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) out[k++] = (c1 - c2) * tt[i] * tt[j] + (i == j ? c2 : 0.0);
}

// Parallel transport of v (perpendicular to unit a) onto unit b: the rotation about a x b
// taking a to b, which for v . a = 0 reduces to v - (b.v)/(1 + a.b) (a + b).
DM_HD v3 transport_perp(v3 a, v3 b, v3 v) {
  dm_real c = dot(b, v) / (1.0 + dot(a, b));
  return v - c * (a + b);
}

// Reference twist: signed angle about te from the f director carried onto te by space-parallel
// transport to the e director; the 2 pi branch nearest the step-start value bref.
DM_HD dm_real ref_twist(v3 tf, v3 d1f, v3 te, v3 d1e, dm_real bref, bool raw) {
  v3 u = transport_perp(tf, te, d1f);
  dm_real b = atan2(dot(cross(u, d1e), te), dot(u, d1e));
  if (raw) return b;
  const dm_real two_pi = 6.283185307179586476925286766559;
  return b + two_pi * rint((bref - b) / two_pi);
}

// ---------------------------------------------------------------------------
// forward-mode dual numbers with N tangents, mixing freely with plain doubles
// ---------------------------------------------------------------------------
template <int N> struct Dual { dm_real v; dm_real d[N]; };

template <int N> DM_HD Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int N> DM_HD Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int N> DM_HD Dual<N> operator-(const Dual<N>& a) { Dual<N> r; r.v = -a.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r; }
template <int N> DM_HD Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.v * b.d[i] + a.d[i] * b.v; return r; }
template <int N> DM_HD Dual<N> operator*(dm_real s, const Dual<N>& a) { Dual<N> r; r.v = s * a.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = s * a.d[i]; return r; }
template <int N> DM_HD Dual<N> operator*(const Dual<N>& a, dm_real s) { return s * a; }
template <int N> DM_HD Dual<N> operator+(const Dual<N>& a, dm_real s) { Dual<N> r = a; r.v += s; return r; }
template <int N> DM_HD Dual<N> operator+(dm_real s, const Dual<N>& a) { Dual<N> r = a; r.v += s; return r; }
template <int N> DM_HD Dual<N> operator-(const Dual<N>& a, dm_real s) { Dual<N> r = a; r.v -= s; return r; }
template <int N> DM_HD Dual<N> operator-(dm_real s, const Dual<N>& a) { Dual<N> r = -a; r.v += s; return r; }
// 1/a: on the device the hardware estimate (about 24 correct bits) refined by one third-order
// correction r (1 + e + e^2), e = 1 - a r (relative error of order e^3, below the float64
// rounding of the result; not correctly rounded), in four operations instead of a division.
DM_HD dm_real frcp(dm_real a) {
#ifdef __HIP_DEVICE_COMPILE__
  const dm_real r = __builtin_amdgcn_rcp(a);
  const dm_real e = fma(-a, r, 1.0);
  return fma(r, fma(e, e, e), r);
#else
  return 1.0 / a;
#endif
}
template <int N> DM_HD Dual<N> dinv(const Dual<N>& a) { Dual<N> r; dm_real i = frcp(a.v); dm_real m = -i * i; r.v = i;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = m * a.d[k]; return r; }
template <int N> DM_HD Dual<N> dsqrt(const Dual<N>& a) { Dual<N> r; dm_real s = sqrt(a.v); dm_real h = 0.5 * frcp(s); r.v = s;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = h * a.d[k]; return r; }
template <int N> DM_HD void dsincos(const Dual<N>& a, Dual<N>& s, Dual<N>& c) {
  dm_real sv, cv;
  sincos(a.v, &sv, &cv);      // one argument reduction for both
  s.v = sv; c.v = cv;
#pragma unroll
  for (int k = 0; k < N; ++k) { s.d[k] = cv * a.d[k]; c.d[k] = -sv * a.d[k]; }
}
DM_HD dm_real dinv(dm_real a) { return frcp(a); }
DM_HD dm_real dsqrt(dm_real a) { return sqrt(a); }
DM_HD void dsincos(dm_real a, dm_real& s, dm_real& c) { sincos(a, &s, &c); }
template <int N> DM_HD dm_real val(const Dual<N>& a) { return a.v; }
DM_HD dm_real val(dm_real a) { return a; }

// 3-vectors over any scalar type
template <class S> struct Vec { S x, y, z; };
template <class S> DM_HD Vec<S> mkv(S a, S b, S c) { Vec<S> r; r.x = a; r.y = b; r.z = c; return r; }
template <class A, class B> DM_HD auto vadd(const Vec<A>& a, const Vec<B>& b) { return mkv(a.x + b.x, a.y + b.y, a.z + b.z); }
template <class A, class B> DM_HD auto vsub(const Vec<A>& a, const Vec<B>& b) { return mkv(a.x - b.x, a.y - b.y, a.z - b.z); }
template <class A, class B> DM_HD auto vscale(const A& s, const Vec<B>& v) { return mkv(s * v.x, s * v.y, s * v.z); }
template <class A, class B> DM_HD auto vdot(const Vec<A>& a, const Vec<B>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class A, class B> DM_HD auto vcross(const Vec<A>& a, const Vec<B>& b) {
  return mkv(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
DM_HD Vec<dm_real> tov(v3 a) { return mkv(a.x, a.y, a.z); }
template <class S> DM_HD v3 vval(const Vec<S>& a) { return mk3(val(a.x), val(a.y), val(a.z)); }

// Frame of one stencil edge at its current vector e and twist th: tangent t, inverse length il,
// material directors m1, m2 (from the director d1 transported in time from (tn, d1n)), and the
// holonomy vector w of that transport.  S is double or a dual type.
template <class S> struct EdgeFrame { Vec<S> t, m1, m2, w; S il; v3 d1v; };

template <class S>
DM_HD void edge_frame(const Vec<S>& e, const S& th, v3 tn, v3 d1n, EdgeFrame<S>& F) {
  S l = dsqrt(vdot(e, e));
  F.il = dinv(l);
  F.t = vscale(F.il, e);
  S b = vdot(tov(tn), F.t) + 1.0;
  S ib = dinv(b);
  S c = vdot(tov(d1n), F.t) * ib;
  Vec<S> d1 = vsub(tov(d1n), vscale(c, vadd(F.t, tov(tn))));   // d1n - (t.d1n)/(1 + tn.t) (tn + t)
  Vec<S> d2 = vcross(F.t, d1);
  S sn, cs;
  dsincos(th, sn, cs);
  F.m1 = vadd(vscale(cs, d1), vscale(sn, d2));
  F.m2 = vsub(vscale(cs, d2), vscale(sn, d1));
  F.w = vscale(-(ib * F.il), vcross(tov(tn), F.t));          // w = -(tn x t)/((1 + tn.t) |e|)
  F.d1v = vval(d1);
}

typedef Dual<4> D4;
typedef Dual<2> D2;

// One pass of the bend/twist stencil energy
//   E = kbend/2 |kappa - kappa_bar|^2 + ktwist/2 (tau - tau_bar)^2        (Eq. 4-8)
// with N derivatives seeded on the f-edge variables S0 .. S0+N-1 of (e_f.x, e_f.y, e_f.z,
// theta_f).  Outputs the exact gradient g8 with respect to v = (e_f, e_e, theta_f, theta_e)
// (closed-form strain gradients: classical DER terms plus the holonomy term (d strain/d theta)
// w), whose tangents are the Hessian columns d g8 / d (seeded variables).  Frames are in the
// stencil's orientation.  Returns the reference twist beta.
template <int N, int S0>
DM_HD dm_real stencil_pass_n(v3 ef_v, v3 ee_v, dm_real thf_s, dm_real the_s, v3 tnf, v3 d1nf, v3 tne, v3 d1ne,
                            dm_real bref, dm_real k1bar, dm_real k2bar, dm_real tbar, dm_real kbend, dm_real ktw,
                            dm_real* g8, dm_real (*Hf)[N]) {
  typedef Dual<N> DN;
  DN z;
  z.v = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) z.d[k] = 0.0;
  Vec<DN> ef;
  ef.x = z; ef.y = z; ef.z = z;
  ef.x.v = ef_v.x; ef.y.v = ef_v.y; ef.z.v = ef_v.z;
  DN thf = z;
  thf.v = thf_s;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int var = S0 + k;
    if (var == 0) ef.x.d[k] = 1.0;
    if (var == 1) ef.y.d[k] = 1.0;
    if (var == 2) ef.z.d[k] = 1.0;
    if (var == 3) thf.d[k] = 1.0;
  }
  EdgeFrame<DN> F;
  EdgeFrame<dm_real> G;
  edge_frame(ef, thf, tnf, d1nf, F);
  edge_frame(tov(ee_v), the_s, tne, d1ne, G);
  const dm_real beta = ref_twist(vval(F.t), F.d1v, vval(G.t), G.d1v, bref, false);
  const dm_real tau = the_s - thf_s + beta;                       // Eq. 7
  DN ichi = dinv(vdot(F.t, G.t) + 1.0);
  Vec<DN> kb = vscale(2.0 * ichi, vcross(F.t, G.t));            // Eq. 4
  // c_i = kbend (kappa_i - kappa_bar_i), kappa from Eq. 5; a_f, a_e = sum_i c_i d kappa_i / d theta
  DN k1 = 0.5 * (vdot(kb, F.m2) + vdot(kb, G.m2));
  DN k2 = -0.5 * (vdot(kb, F.m1) + vdot(kb, G.m1));
  DN c1 = kbend * (k1 - k1bar);
  DN c2 = kbend * (k2 - k2bar);
  DN af = -0.5 * (c1 * vdot(kb, F.m1) + c2 * vdot(kb, F.m2));
  DN ae = -0.5 * (c1 * vdot(kb, G.m1) + c2 * vdot(kb, G.m2));
  // ct = ktwist (tau - tau_bar); its tangent is ktwist d tau, with d tau/d e_f = kb/(2|e_f|) - w_f
  // and d tau / d theta_f = -1
  DN ct;
  {
    const v3 gt = 0.5 * val(F.il) * vval(kb) - vval(F.w);
    const dm_real gv[4] = {gt.x, gt.y, gt.z, -1.0};
    ct.v = ktw * (tau - tbar);
#pragma unroll
    for (int k = 0; k < N; ++k) ct.d[k] = ktw * gv[S0 + k];
  }
  // the kappa terms of the edge gradients share M = (c1 (m2f + m2e) - c2 (m1f + m1e)) / chi
  // and c_k = c1 kappa1 + c2 kappa2 (classical DER gradients, grouped)
  DN ck = c1 * k1 + c2 * k2;
  Vec<DN> M = vscale(ichi, vsub(vscale(c1, vadd(F.m2, G.m2)), vscale(c2, vadd(F.m1, G.m1))));
  Vec<DN> V = vadd(vscale(-(ck * ichi), vadd(F.t, G.t)), vscale(0.5 * ct, kb));
  Vec<DN> gf = vadd(vscale(F.il, vadd(vcross(G.t, M), V)), vscale(af - ct, F.w));
  Vec<DN> ge = vadd(vscale(G.il, vsub(V, vcross(F.t, M))), vscale(ae + ct, G.w));
  DN gthf = af - ct;
  DN gthe = ae + ct;
  const DN* out[8] = {&gf.x, &gf.y, &gf.z, &ge.x, &ge.y, &ge.z, &gthf, &gthe};
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    g8[a] = out[a]->v;
#pragma unroll
    for (int k = 0; k < N; ++k) Hf[a][k] = out[a]->d[k];
  }
  return beta;
}

// All four f-edge tangents in one pass.
DM_HD dm_real stencil_pass(v3 ef_v, v3 ee_v, dm_real thf_s, dm_real the_s, v3 tnf, v3 d1nf, v3 tne, v3 d1ne,
                          dm_real bref, dm_real k1bar, dm_real k2bar, dm_real tbar, dm_real kbend, dm_real ktw,
                          dm_real* g8, dm_real (*H8f)[4]) {
  return stencil_pass_n<4, 0>(ef_v, ee_v, thf_s, the_s, tnf, d1nf, tne, d1ne, bref, k1bar, k2bar, tbar, kbend, ktw,
                              g8, H8f);
}

// Local DOF l of a stencil as a signed combination of the 8 stencil variables
// (e_f = x_c - x_p, e_e = x_n - x_c, theta_f, theta_e):
//   x_p (l = 0..2): -e_f;  theta_f (3): sf theta_f;  x_c (4..6): e_f - e_e;  theta_e (7): se theta_e;
//   x_n (8..10): e_e.
DM_HD int loc_terms(int l, dm_real sf, dm_real se, int* var, dm_real* coef) {
  if (l < 3) { var[0] = l; coef[0] = -1.0; return 1; }
  if (l == 3) { var[0] = 6; coef[0] = sf; return 1; }
  if (l < 7) { var[0] = l - 4; coef[0] = 1.0; var[1] = l - 1; coef[1] = -1.0; return 2; }
  if (l == 7) { var[0] = 7; coef[0] = se; return 1; }
  var[0] = l - 5; coef[0] = 1.0; return 1;
}

// Value-only strains of a stencil (setup and reporting): integrated curvature and the raw
// reference twist for frames (t, d1) already in the stencil's orientation.
DM_HD void stencil_strains(v3 tf, v3 d1f, dm_real thf, v3 te, v3 d1e, dm_real the, dm_real bref,
                           bool raw, dm_real* k1, dm_real* k2, dm_real* beta) {
  v3 d2f = cross(tf, d1f), d2e = cross(te, d1e);
  v3 m1f = cos(thf) * d1f + sin(thf) * d2f, m2f = (-sin(thf)) * d1f + cos(thf) * d2f;
  v3 m1e = cos(the) * d1e + sin(the) * d2e, m2e = (-sin(the)) * d1e + cos(the) * d2e;
  v3 kb = (2.0 / (1.0 + dot(tf, te))) * cross(tf, te);
  *k1 = 0.5 * dot(kb, m2f + m2e);
  *k2 = -0.5 * dot(kb, m1f + m1e);
  *beta = ref_twist(tf, d1f, te, d1e, bref, raw);
}

// ---------------------------------------------------------------------------
// Fully generic form of the stencil gradient, for derivatives with respect to the step-start
// frames and the natural curvature (the discrete adjoint).  Every input may carry tangents;
// the reference twist is then evaluated as a dual angle (atan2 derivative
// (x dy - y dx) / (x^2 + y^2)), its 2 pi branch taken from bref as in ref_twist.
// ---------------------------------------------------------------------------
template <int N> DM_HD Dual<N> datan2(const Dual<N>& y, const Dual<N>& x) {
  Dual<N> r;
  r.v = atan2(y.v, x.v);
  const dm_real q = frcp(x.v * x.v + y.v * y.v);
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = (x.v * y.d[k] - y.v * x.d[k]) * q;
  return r;
}
DM_HD dm_real datan2(dm_real y, dm_real x) { return atan2(y, x); }

template <class S> DM_HD S lift(dm_real v) { S r{}; r.v = v; return r; }
template <> DM_HD dm_real lift<dm_real>(dm_real v) { return v; }
template <class S> DM_HD Vec<S> liftv(v3 a) { return mkv(lift<S>(a.x), lift<S>(a.y), lift<S>(a.z)); }

template <class S>
DM_HD void edge_frame_g(const Vec<S>& e, const S& th, const Vec<S>& tn, const Vec<S>& d1n, EdgeFrame<S>& F,
                        Vec<S>& d1) {
  S l = dsqrt(vdot(e, e));
  F.il = dinv(l);
  F.t = vscale(F.il, e);
  S ib = dinv(vdot(tn, F.t) + 1.0);
  S c = vdot(d1n, F.t) * ib;
  d1 = vsub(d1n, vscale(c, vadd(F.t, tn)));
  Vec<S> d2 = vcross(F.t, d1);
  S sn, cs;
  dsincos(th, sn, cs);
  F.m1 = vadd(vscale(cs, d1), vscale(sn, d2));
  F.m2 = vsub(vscale(cs, d2), vscale(sn, d1));
  F.w = vscale(-(ib * F.il), vcross(tn, F.t));
}

// Gradient g8 of the stencil energy with respect to (e_f, e_e, theta_f, theta_e) (the same
// closed forms as stencil_pass), with every argument generic.
template <class S>
DM_HD void stencil_grad_g(const Vec<S>& ef, const Vec<S>& ee, const S& thf, const S& the, const Vec<S>& tnf,
                          const Vec<S>& d1nf, const Vec<S>& tne, const Vec<S>& d1ne, dm_real bref, const S& k1bar,
                          const S& k2bar, dm_real tbar, dm_real kbend, dm_real ktw, S* g8) {
  EdgeFrame<S> F, G;
  Vec<S> d1f, d1e;
  edge_frame_g(ef, thf, tnf, d1nf, F, d1f);
  edge_frame_g(ee, the, tne, d1ne, G, d1e);
  // reference twist (Eq. 7) as a differentiable angle on the branch nearest bref
  Vec<S> u = vsub(d1f, vscale(vdot(G.t, d1f) * dinv(vdot(F.t, G.t) + 1.0), vadd(F.t, G.t)));
  S beta = datan2(vdot(vcross(u, d1e), G.t), vdot(u, d1e));
  const dm_real two_pi = 6.283185307179586476925286766559;
  beta = beta + two_pi * rint((bref - val(beta)) * (1.0 / two_pi));
  S tau = the - thf + beta;
  S ichi = dinv(vdot(F.t, G.t) + 1.0);
  Vec<S> kb = vscale(2.0 * ichi, vcross(F.t, G.t));
  S k1 = 0.5 * (vdot(kb, F.m2) + vdot(kb, G.m2));
  S k2 = -0.5 * (vdot(kb, F.m1) + vdot(kb, G.m1));
  S c1 = kbend * (k1 - k1bar);
  S c2 = kbend * (k2 - k2bar);
  S af = -0.5 * (c1 * vdot(kb, F.m1) + c2 * vdot(kb, F.m2));
  S ae = -0.5 * (c1 * vdot(kb, G.m1) + c2 * vdot(kb, G.m2));
  S ct = ktw * (tau - tbar);
  S ck = c1 * k1 + c2 * k2;
  Vec<S> M = vscale(ichi, vsub(vscale(c1, vadd(F.m2, G.m2)), vscale(c2, vadd(F.m1, G.m1))));
  Vec<S> V = vadd(vscale(-(ck * ichi), vadd(F.t, G.t)), vscale(0.5 * ct, kb));
  Vec<S> gf = vadd(vscale(F.il, vadd(vcross(G.t, M), V)), vscale(af - ct, F.w));
  Vec<S> ge = vadd(vscale(G.il, vsub(V, vcross(F.t, M))), vscale(ae + ct, G.w));
  g8[0] = gf.x; g8[1] = gf.y; g8[2] = gf.z;
  g8[3] = ge.x; g8[4] = ge.y; g8[5] = ge.z;
  g8[6] = af - ct; g8[7] = ae + ct;
}

// Gradient of the first integrated curvature kappa_1 of a stencil (Eq. 5) with respect to
// (e_f, e_e, theta_f, theta_e), frames carried by time-parallel transport from (tn, d1n): the
// bending part of stencil_grad_g's closed form with c1 = 1, c2 = 0 and no twist term.
template <class S>
DM_HD void stencil_kappa1_grad_g(const Vec<S>& ef, const Vec<S>& ee, const S& thf, const S& the, const Vec<S>& tnf,
                                 const Vec<S>& d1nf, const Vec<S>& tne, const Vec<S>& d1ne, S* g8) {
  EdgeFrame<S> F, G;
  Vec<S> d1f, d1e;
  edge_frame_g(ef, thf, tnf, d1nf, F, d1f);
  edge_frame_g(ee, the, tne, d1ne, G, d1e);
  S ichi = dinv(vdot(F.t, G.t) + 1.0);
  Vec<S> kb = vscale(2.0 * ichi, vcross(F.t, G.t));
  S k1 = 0.5 * (vdot(kb, F.m2) + vdot(kb, G.m2));
  S af = -0.5 * vdot(kb, F.m1);
  S ae = -0.5 * vdot(kb, G.m1);
  Vec<S> M = vscale(ichi, vadd(F.m2, G.m2));
  Vec<S> V = vscale(-(k1 * ichi), vadd(F.t, G.t));
  Vec<S> gf = vadd(vscale(F.il, vadd(vcross(G.t, M), V)), vscale(af, F.w));
  Vec<S> ge = vadd(vscale(G.il, vsub(V, vcross(F.t, M))), vscale(ae, G.w));
  g8[0] = gf.x; g8[1] = gf.y; g8[2] = gf.z;
  g8[3] = ge.x; g8[4] = ge.y; g8[5] = ge.z;
  g8[6] = af; g8[7] = ae;
}
