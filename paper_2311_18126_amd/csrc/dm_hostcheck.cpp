// dm_hostcheck.cpp -- host build of the step's element math (dm_math.h) for checks that need no
// GPU: built with AddressSanitizer and UndefinedBehaviorSanitizer by the CPU tests, it runs the
// stencil and stretch closed forms on seeded random stencils and checks
//  * the gradient of the Hessian pass equals the generic-scalar gradient (same closed form);
//  * the Hessian columns (forward-mode tangents) match central differences of that gradient;
//  * the one-tangent passes the kernels run give the four-tangent pass's columns;
//  * the reversed orientation gives the e-edge columns through the signed permutation the
//    kernels use (e_f <-> -e_e, theta_f <-> -theta_e, second curvature component negated);
//  * the stretch gradient and Hessian match central differences of Eq. 3's energy;
//  * parallel transport keeps a director unit and perpendicular to the new tangent;
//  * the closed-form gradient of the first curvature matches central differences of Eq. 5's
//    value (with the frames carried from the step start).
// Prints one summary line and exits non-zero on a failed check.
#include <cmath>
#include <cstdio>
#include <random>

#include "dm_math.h"

namespace {

std::mt19937_64 rng(20231130);
double uni(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }
v3 rnd3(double s) { return mk3(uni(-s, s), uni(-s, s), uni(-s, s)); }
v3 unitv(v3 a) { return (1.0 / std::sqrt(dot(a, a))) * a; }
// a unit director perpendicular to unit t
v3 perp(v3 t) {
  v3 r = rnd3(1.0);
  r = r - dot(r, t) * t;
  return unitv(r);
}

struct Stencil {
  v3 ef, ee, tnf, d1nf, tne, d1ne;
  double thf, the, bref, k1, k2, tbar, kb, kt;
};

Stencil random_stencil() {
  Stencil s;
  const v3 base = unitv(mk3(1.0, uni(-0.3, 0.3), uni(-0.3, 0.3)));
  s.ef = uni(0.005, 0.02) * unitv(base + rnd3(0.3));
  s.ee = uni(0.005, 0.02) * unitv(base + rnd3(0.3));
  // step-start tangents near the current ones, directors perpendicular to them
  s.tnf = unitv(unitv(s.ef) + rnd3(0.05));
  s.tne = unitv(unitv(s.ee) + rnd3(0.05));
  s.d1nf = perp(s.tnf);
  s.d1ne = perp(s.tne);
  s.thf = uni(-0.5, 0.5);
  s.the = uni(-0.5, 0.5);
  s.bref = 0.0;
  s.k1 = uni(-0.1, 0.1);
  s.k2 = uni(-0.1, 0.1);
  s.tbar = uni(-0.05, 0.05);
  s.kb = uni(0.5, 2.0);
  s.kt = uni(0.2, 1.0);
  return s;
}

// gradient of the stencil energy by the generic closed form
void grad(const Stencil& s, v3 ef, v3 ee, double thf, double the, double* g8) {
  stencil_grad_g<double>(tov(ef), tov(ee), thf, the, tov(s.tnf), tov(s.d1nf), tov(s.tne), tov(s.d1ne), s.bref, s.k1,
                         s.k2, s.tbar, s.kb, s.kt, g8);
}

double rel(double a, double b, double scale) { return std::fabs(a - b) / scale; }

}  // namespace

int main() {
  int fail = 0;
  double worst_g = 0.0, worst_fd = 0.0, worst_one = 0.0, worst_rev = 0.0, worst_st = 0.0, worst_tr = 0.0;
  double worst_k = 0.0;
  for (int trial = 0; trial < 400; ++trial) {
    const Stencil s = random_stencil();
    double g8[8], H[8][4];
    stencil_pass_n<4, 0>(s.ef, s.ee, s.thf, s.the, s.tnf, s.d1nf, s.tne, s.d1ne, s.bref, s.k1, s.k2, s.tbar, s.kb, s.kt,
                         g8, H);
    double gg[8];
    grad(s, s.ef, s.ee, s.thf, s.the, gg);
    double gs = 0.0, hs = 0.0;
    for (int a = 0; a < 8; ++a) gs = std::fmax(gs, std::fabs(gg[a]));
    for (int a = 0; a < 8; ++a)
      for (int k = 0; k < 4; ++k) hs = std::fmax(hs, std::fabs(H[a][k]));
    for (int a = 0; a < 8; ++a) worst_g = std::fmax(worst_g, rel(g8[a], gg[a], gs));
    // central differences of the gradient along the f-edge variables
    for (int k = 0; k < 4; ++k) {
      const double h = k < 3 ? 1e-7 * std::sqrt(dot(s.ef, s.ef)) : 1e-6;
      v3 dp = mk3(k == 0 ? h : 0.0, k == 1 ? h : 0.0, k == 2 ? h : 0.0);
      double gp[8], gm[8];
      grad(s, s.ef + dp, s.ee, s.thf + (k == 3 ? h : 0.0), s.the, gp);
      grad(s, s.ef - dp, s.ee, s.thf - (k == 3 ? h : 0.0), s.the, gm);
      for (int a = 0; a < 8; ++a) worst_fd = std::fmax(worst_fd, rel((gp[a] - gm[a]) / (2 * h), H[a][k], hs));
    }
    // one-tangent passes
    double g1[8], H1[8][1];
    stencil_pass_n<1, 2>(s.ef, s.ee, s.thf, s.the, s.tnf, s.d1nf, s.tne, s.d1ne, s.bref, s.k1, s.k2, s.tbar, s.kb,
                         s.kt, g1, H1);
    for (int a = 0; a < 8; ++a) worst_one = std::fmax(worst_one, rel(H1[a][0], H[a][2], hs));
    // the reversed orientation's f-edge columns are the stored stencil's e-edge columns
    double gr[8], Hr[8][4];
    stencil_pass_n<4, 0>(-1.0 * s.ee, -1.0 * s.ef, -s.the, -s.thf, -1.0 * s.tne, s.d1ne, -1.0 * s.tnf, s.d1nf, s.bref,
                         s.k1, -s.k2, s.tbar, s.kb, s.kt, gr, Hr);
    for (int k = 0; k < 4; ++k) {
      const double h = k < 3 ? 1e-7 * std::sqrt(dot(s.ee, s.ee)) : 1e-6;
      v3 dp = mk3(k == 0 ? h : 0.0, k == 1 ? h : 0.0, k == 2 ? h : 0.0);
      double gp[8], gm[8];
      grad(s, s.ef, s.ee + dp, s.thf, s.the + (k == 3 ? h : 0.0), gp);
      grad(s, s.ef, s.ee - dp, s.thf, s.the - (k == 3 ? h : 0.0), gm);
      // stored variable a is the reversed stencil's variable ra; both derivatives flip sign
      for (int a = 0; a < 8; ++a) {
        const int ra = a < 3 ? a + 3 : (a < 6 ? a - 3 : 13 - a);
        worst_rev = std::fmax(worst_rev, rel((gp[a] - gm[a]) / (2 * h), Hr[ra][k], hs));
      }
    }
    // stretch against central differences of 1/2 EA (|d|/eb - 1)^2 eb
    const double EA = uni(10.0, 1000.0), eb = std::sqrt(dot(s.ef, s.ef)) * uni(0.9, 1.1);
    double st[9];
    stretch_terms(s.ef, EA, eb, st);
    auto energy = [&](v3 d) { const double e = std::sqrt(dot(d, d)) / eb - 1.0; return 0.5 * EA * e * e * eb; };
    const double h = 1e-7 * eb;
    const int idx[3][3] = {{3, 4, 5}, {4, 6, 7}, {5, 7, 8}};
    double gsc = 0.0, hsc = 0.0;
    for (int i = 0; i < 3; ++i) gsc = std::fmax(gsc, std::fabs(st[i]));
    for (int i = 3; i < 9; ++i) hsc = std::fmax(hsc, std::fabs(st[i]));
    for (int i = 0; i < 3; ++i) {
      v3 di = mk3(i == 0 ? h : 0.0, i == 1 ? h : 0.0, i == 2 ? h : 0.0);
      worst_st = std::fmax(worst_st, rel((energy(s.ef + di) - energy(s.ef - di)) / (2 * h), st[i], gsc + 1e-30));
      double sp[9], sm[9];
      stretch_terms(s.ef + di, EA, eb, sp);
      stretch_terms(s.ef - di, EA, eb, sm);
      for (int j = 0; j < 3; ++j) worst_st = std::fmax(worst_st, rel((sp[j] - sm[j]) / (2 * h), st[idx[i][j]], hsc));
    }
    // transport of the step-start director onto the current tangent
    const v3 t = unitv(s.ef), d1 = transport_perp(s.tnf, t, s.d1nf);
    worst_tr = std::fmax(worst_tr, std::fmax(std::fabs(dot(d1, d1) - 1.0), std::fabs(dot(d1, t))));
    // first curvature and its closed-form gradient
    auto kappa1 = [&](v3 ef, v3 ee, double thf, double the) {
      const v3 tf = unitv(ef), te = unitv(ee);
      double k1, k2, b;
      stencil_strains(tf, transport_perp(s.tnf, tf, s.d1nf), thf, te, transport_perp(s.tne, te, s.d1ne), the, 0.0, true,
                      &k1, &k2, &b);
      return k1;
    };
    double gk[8];
    stencil_kappa1_grad_g<double>(tov(s.ef), tov(s.ee), s.thf, s.the, tov(s.tnf), tov(s.d1nf), tov(s.tne), tov(s.d1ne),
                                  gk);
    double ks = 0.0;
    for (int a = 0; a < 8; ++a) ks = std::fmax(ks, std::fabs(gk[a]));
    for (int a = 0; a < 8; ++a) {
      const int e = a < 3 ? 0 : (a < 6 ? 1 : (a == 6 ? 2 : 3));
      const int c = a < 6 ? a % 3 : 0;
      const double hh = e < 2 ? 1e-7 * 0.01 : 1e-6;
      v3 dv = mk3(c == 0 ? hh : 0.0, c == 1 ? hh : 0.0, c == 2 ? hh : 0.0);
      const double kp = kappa1(e == 0 ? s.ef + dv : s.ef, e == 1 ? s.ee + dv : s.ee, s.thf + (e == 2 ? hh : 0.0),
                               s.the + (e == 3 ? hh : 0.0));
      const double km = kappa1(e == 0 ? s.ef - dv : s.ef, e == 1 ? s.ee - dv : s.ee, s.thf - (e == 2 ? hh : 0.0),
                               s.the - (e == 3 ? hh : 0.0));
      worst_k = std::fmax(worst_k, rel((kp - km) / (2 * hh), gk[a], ks));
    }
  }
  fail |= !(worst_g < 1e-12) | !(worst_fd < 1e-6) | !(worst_one < 1e-12) | !(worst_rev < 1e-6) |
          !(worst_st < 1e-5) | !(worst_tr < 1e-14) | !(worst_k < 1e-6);
  std::printf("dm_hostcheck: gradient %.2e, Hessian vs differences %.2e, one-tangent %.2e, reversed %.2e, "
              "stretch %.2e, transport %.2e, curvature gradient %.2e: %s\n",
              worst_g, worst_fd, worst_one, worst_rev, worst_st, worst_tr, worst_k, fail ? "FAIL" : "ok");
  return fail ? 1 : 0;
}
