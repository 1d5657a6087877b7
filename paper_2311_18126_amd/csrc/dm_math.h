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

// ---------------------------------------------------------------------------
// plain double 3-vectors
// ---------------------------------------------------------------------------
struct v3 { double x, y, z; };
DM_HD v3 mk3(double a, double b, double c) { v3 r; r.x = a; r.y = b; r.z = c; return r; }
DM_HD v3 operator+(v3 a, v3 b) { return mk3(a.x + b.x, a.y + b.y, a.z + b.z); }
DM_HD v3 operator-(v3 a, v3 b) { return mk3(a.x - b.x, a.y - b.y, a.z - b.z); }
DM_HD v3 operator*(double s, v3 a) { return mk3(s * a.x, s * a.y, s * a.z); }
DM_HD double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
DM_HD v3 cross(v3 a, v3 b) { return mk3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }

// Parallel transport of v (perpendicular to unit a) onto unit b: the rotation about a x b
// taking a to b, which for v . a = 0 reduces to v - (b.v)/(1 + a.b) (a + b).
DM_HD v3 transport_perp(v3 a, v3 b, v3 v) {
  double c = dot(b, v) / (1.0 + dot(a, b));
  return v - c * (a + b);
}

// Reference twist: signed angle about te from the f director carried onto te by space-parallel
// transport to the e director; the 2 pi branch nearest the step-start value bref.
DM_HD double ref_twist(v3 tf, v3 d1f, v3 te, v3 d1e, double bref, bool raw) {
  v3 u = transport_perp(tf, te, d1f);
  double b = atan2(dot(cross(u, d1e), te), dot(u, d1e));
  if (raw) return b;
  const double two_pi = 6.283185307179586476925286766559;
  return b + two_pi * rint((bref - b) / two_pi);
}

// ---------------------------------------------------------------------------
// forward-mode dual numbers with 8 tangents
// ---------------------------------------------------------------------------
struct D8 { double v; double d[8]; };
struct DV { D8 c[3]; };

DM_HD D8 dcst(double a) { D8 r; r.v = a;
#pragma unroll
  for (int i = 0; i < 8; ++i) r.d[i] = 0.0; return r; }
DM_HD D8 operator+(const D8& a, const D8& b) { D8 r; r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < 8; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
DM_HD D8 operator-(const D8& a, const D8& b) { D8 r; r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < 8; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
DM_HD D8 operator-(const D8& a) { D8 r; r.v = -a.v;
#pragma unroll
  for (int i = 0; i < 8; ++i) r.d[i] = -a.d[i]; return r; }
DM_HD D8 operator*(const D8& a, const D8& b) { D8 r; r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < 8; ++i) r.d[i] = a.v * b.d[i] + a.d[i] * b.v; return r; }
DM_HD D8 operator*(double s, const D8& a) { D8 r; r.v = s * a.v;
#pragma unroll
  for (int i = 0; i < 8; ++i) r.d[i] = s * a.d[i]; return r; }
DM_HD D8 operator+(const D8& a, double s) { D8 r = a; r.v += s; return r; }
DM_HD D8 dinv(const D8& a) { D8 r; double i = 1.0 / a.v; double m = -i * i; r.v = i;
#pragma unroll
  for (int k = 0; k < 8; ++k) r.d[k] = m * a.d[k]; return r; }
DM_HD D8 dsqrt(const D8& a) { D8 r; double s = sqrt(a.v); double h = 0.5 / s; r.v = s;
#pragma unroll
  for (int k = 0; k < 8; ++k) r.d[k] = h * a.d[k]; return r; }

DM_HD DV operator+(const DV& a, const DV& b) { DV r; r.c[0] = a.c[0] + b.c[0]; r.c[1] = a.c[1] + b.c[1]; r.c[2] = a.c[2] + b.c[2]; return r; }
DM_HD DV operator-(const DV& a, const DV& b) { DV r; r.c[0] = a.c[0] - b.c[0]; r.c[1] = a.c[1] - b.c[1]; r.c[2] = a.c[2] - b.c[2]; return r; }
DM_HD DV operator*(const D8& s, const DV& a) { DV r; r.c[0] = s * a.c[0]; r.c[1] = s * a.c[1]; r.c[2] = s * a.c[2]; return r; }
DM_HD DV operator*(double s, const DV& a) { DV r; r.c[0] = s * a.c[0]; r.c[1] = s * a.c[1]; r.c[2] = s * a.c[2]; return r; }
DM_HD D8 ddot(const DV& a, const DV& b) { return a.c[0] * b.c[0] + a.c[1] * b.c[1] + a.c[2] * b.c[2]; }
DM_HD D8 ddot(v3 a, const DV& b) { return a.x * b.c[0] + a.y * b.c[1] + a.z * b.c[2]; }
DM_HD DV dcross(const DV& a, const DV& b) {
  DV r;
  r.c[0] = a.c[1] * b.c[2] - a.c[2] * b.c[1];
  r.c[1] = a.c[2] * b.c[0] - a.c[0] * b.c[2];
  r.c[2] = a.c[0] * b.c[1] - a.c[1] * b.c[0];
  return r;
}
DM_HD DV dcross(v3 a, const DV& b) {
  DV r;
  r.c[0] = a.y * b.c[2] - a.z * b.c[1];
  r.c[1] = a.z * b.c[0] - a.x * b.c[2];
  r.c[2] = a.x * b.c[1] - a.y * b.c[0];
  return r;
}
DM_HD DV dadd(const DV& a, v3 b) { DV r = a; r.c[0].v += b.x; r.c[1].v += b.y; r.c[2].v += b.z; return r; }
DM_HD DV dsub_from(v3 a, const DV& b) { DV r; r.c[0] = -b.c[0]; r.c[1] = -b.c[1]; r.c[2] = -b.c[2];
  r.c[0].v += a.x; r.c[1].v += a.y; r.c[2].v += a.z; return r; }
DM_HD v3 dval(const DV& a) { return mk3(a.c[0].v, a.c[1].v, a.c[2].v); }
DM_HD DV dseed(v3 a, int k0) {
  DV r; r.c[0] = dcst(a.x); r.c[1] = dcst(a.y); r.c[2] = dcst(a.z);
  r.c[0].d[k0] = 1.0; r.c[1].d[k0 + 1] = 1.0; r.c[2].d[k0 + 2] = 1.0;
  return r;
}

// Frame of one stencil edge at its current vector e and twist th (both duals):
// tangent t, length l, transported director d1, material directors m1, m2 and the
// holonomy vector w of the time transport from (tn, d1n).
struct EdgeFrame { DV t, d1, m1, m2, w; D8 l, il; };

DM_HD void edge_frame(const DV& e, const D8& th, v3 tn, v3 d1n, EdgeFrame& F) {
  F.l = dsqrt(ddot(e, e));
  F.il = dinv(F.l);
  F.t = F.il * e;
  D8 a = ddot(d1n, F.t);
  D8 b = ddot(tn, F.t) + 1.0;
  D8 ib = dinv(b);
  D8 c = a * ib;
  F.d1 = dsub_from(d1n, c * dadd(F.t, tn));          // d1 = d1n - (t.d1n)/(1 + tn.t) (tn + t)
  DV d2 = dcross(F.t, F.d1);
  double s = sin(th.v), co = cos(th.v);
  D8 S = s * dcst(1.0), C = co * dcst(1.0);
#pragma unroll
  for (int k = 0; k < 8; ++k) { S.d[k] = co * th.d[k]; C.d[k] = -s * th.d[k]; }
  F.m1 = C * F.d1 + S * d2;
  F.m2 = S * (-1.0 * F.d1) + C * d2;
  F.w = (-1.0) * ((ib * F.il) * dcross(tn, F.t));    // w = -(tn x t)/((1 + tn.t) l)
}

// Exact gradient (g: 11 local DOFs) and Hessian (H: upper triangle, 66) of the bend + twist
// energy of one stencil  E = kbend/2 |kappa - kappa_bar|^2 + ktwist/2 (tau - tau_bar)^2.
// Local DOF order: x_prev (0..2), theta_f (3), x_centre (4..6), theta_e (7), x_next (8..10),
// with theta_f, theta_e taken in the stencil's orientation (sf, se = +-1 times the stored
// angle).  tnf/d1nf, tne/d1ne are the step-start frames in the stencil's orientation.
// Returns the reference twist beta of the current configuration.
DM_HD int hidx(int a, int b) { return a <= b ? 10 * a - (a * (a - 1)) / 2 + b : 10 * b - (b * (b - 1)) / 2 + a; }

DM_HD double stencil_eval(v3 xp, v3 xc, v3 xn, double thf_s, double the_s,
                          v3 tnf, v3 d1nf, v3 tne, v3 d1ne, double bref,
                          double k1bar, double k2bar, double tbar, double kbend, double ktw,
                          double sf, double se, double* g, double* H) {
  DV ef = dseed(xc - xp, 0), ee = dseed(xn - xc, 3);
  D8 thf = dcst(thf_s), the = dcst(the_s);
  thf.d[6] = 1.0; the.d[7] = 1.0;
  EdgeFrame F, G;
  edge_frame(ef, thf, tnf, d1nf, F);
  edge_frame(ee, the, tne, d1ne, G);
  D8 chi = ddot(F.t, G.t) + 1.0;
  D8 ichi = dinv(chi);
  DV kb = (2.0 * ichi) * dcross(F.t, G.t);                  // Eq. 4
  DV tt = ichi * (F.t + G.t);
  DV m1s = F.m1 + G.m1, m2s = F.m2 + G.m2;
  D8 k1 = 0.5 * ddot(kb, m2s);                              // Eq. 5
  D8 k2 = -0.5 * ddot(kb, m1s);
  DV m1t = ichi * m1s, m2t = ichi * m2s;
  D8 dk1f = -0.5 * ddot(kb, F.m1), dk1e = -0.5 * ddot(kb, G.m1);   // d kappa / d theta
  D8 dk2f = -0.5 * ddot(kb, F.m2), dk2e = -0.5 * ddot(kb, G.m2);
  // d kappa / d e: classical terms plus holonomy (d kappa / d theta) w
  DV Gk1f = F.il * (dcross(G.t, m2t) - k1 * tt) + dk1f * F.w;
  DV Gk1e = G.il * ((-1.0) * dcross(F.t, m2t) - k1 * tt) + dk1e * G.w;
  DV Gk2f = F.il * ((-1.0) * dcross(G.t, m1t) - k2 * tt) + dk2f * F.w;
  DV Gk2e = G.il * (dcross(F.t, m1t) - k2 * tt) + dk2e * G.w;
  // d tau / d e: kb/(2|e|) plus the holonomy with d tau/d theta_f = -1, d tau/d theta_e = +1
  DV Gtf = (0.5 * F.il) * kb - F.w;
  DV Gte = (0.5 * G.il) * kb + G.w;
  double beta = ref_twist(dval(F.t), dval(F.d1), dval(G.t), dval(G.d1), bref, false);
  double tau = the_s - thf_s + beta;                         // Eq. 7
  D8 c1 = kbend * (k1 + (-k1bar));
  D8 c2 = kbend * (k2 + (-k2bar));
  D8 ct;
  ct.v = ktw * (tau - tbar);
  ct.d[0] = ktw * Gtf.c[0].v; ct.d[1] = ktw * Gtf.c[1].v; ct.d[2] = ktw * Gtf.c[2].v;
  ct.d[3] = ktw * Gte.c[0].v; ct.d[4] = ktw * Gte.c[1].v; ct.d[5] = ktw * Gte.c[2].v;
  ct.d[6] = -ktw; ct.d[7] = ktw;
  D8 g8[8];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    g8[i] = c1 * Gk1f.c[i] + c2 * Gk2f.c[i] + ct * Gtf.c[i];
    g8[3 + i] = c1 * Gk1e.c[i] + c2 * Gk2e.c[i] + ct * Gte.c[i];
  }
  g8[6] = c1 * dk1f + c2 * dk2f - ct;
  g8[7] = c1 * dk1e + c2 * dk2e + ct;
  // symmetric 8 x 8 Hessian in (e_f, e_e, theta_f, theta_e)
  double h8[8][8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) h8[a][b] = 0.5 * (g8[a].d[b] + g8[b].d[a]);
  // local DOF l as a combination of the 8 variables: e_f = x_c - x_p, e_e = x_n - x_c
  // P[l][v]: x_p: -e_f; theta_f: sf; x_c: e_f - e_e; theta_e: se; x_n: e_e
  double P[11][8];
#pragma unroll
  for (int l = 0; l < 11; ++l)
#pragma unroll
    for (int v = 0; v < 8; ++v) P[l][v] = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    P[c][c] = -1.0;
    P[4 + c][c] = 1.0; P[4 + c][3 + c] = -1.0;
    P[8 + c][3 + c] = 1.0;
  }
  P[3][6] = sf; P[7][7] = se;
#pragma unroll
  for (int l = 0; l < 11; ++l) {
    double s = 0.0;
#pragma unroll
    for (int v = 0; v < 8; ++v) s += P[l][v] * g8[v].v;
    g[l] = s;
  }
  double HP[8][11];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int l = 0; l < 11; ++l) {
      double s = 0.0;
#pragma unroll
      for (int v = 0; v < 8; ++v) s += h8[a][v] * P[l][v];
      HP[a][l] = s;
    }
#pragma unroll
  for (int l = 0; l < 11; ++l)
#pragma unroll
    for (int m = l; m < 11; ++m) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < 8; ++a) s += P[l][a] * HP[a][m];
      H[hidx(l, m)] = s;
    }
  return beta;
}

// Value-only strains of a stencil (setup and reporting): integrated curvature and the raw
// reference twist for frames (t, d1) already in the stencil's orientation.
DM_HD void stencil_strains(v3 tf, v3 d1f, double thf, v3 te, v3 d1e, double the, double bref,
                           bool raw, double* k1, double* k2, double* beta) {
  v3 d2f = cross(tf, d1f), d2e = cross(te, d1e);
  v3 m1f = cos(thf) * d1f + sin(thf) * d2f, m2f = (-sin(thf)) * d1f + cos(thf) * d2f;
  v3 m1e = cos(the) * d1e + sin(the) * d2e, m2e = (-sin(the)) * d1e + cos(the) * d2e;
  v3 kb = (2.0 / (1.0 + dot(tf, te))) * cross(tf, te);
  *k1 = 0.5 * dot(kb, m2f + m2e);
  *k2 = -0.5 * dot(kb, m1f + m1e);
  *beta = ref_twist(tf, d1f, te, d1e, bref, raw);
}
