// dm_flops.cpp -- algorithmic floating-point work of one Newton iteration of the implicit DER
// step, per item, as one JSON object on stdout (host program; no GPU).
//
// The element math of the step (dm_math.h: stencil frames, strains, the closed-form gradient
// and its exact Hessian by forward-mode dual numbers, the stretch terms) is compiled here over
// a counting scalar, so its operations are counted exactly as written: every +, -, *, / and
// sqrt counts one, sin and cos one each (sincos two), atan2 one; a sign change and rounding to
// an integer count nothing.  A fused multiply-add in the kernels counts as the two operations
// it replaces.  The stencil's algorithmic form is one gradient pass per orientation with the
// four tangents of its first edge (value once, four Hessian columns), two passes per stencil;
// the kernels run eight one-tangent tasks instead, which repeats the value work.
//
// The remaining items follow the method's operations directly:
//  * node terms without contact (inertia, gravity, loads, damping of Eq. 15 and their
//    Jacobian diagonal) and the twist inertia of an edge;
//  * assembly: the stencil's 8-variable Hessian is mapped to its 11 local DOFs (the centre
//    node is e_f - e_e) and every element entry is added into the band once;
//  * banded LU without pivoting, half-bandwidth 10, right-hand side carried along: per
//    eliminated row one reciprocal, ten multipliers and ten rows of ten entries plus the
//    right-hand side updated by multiply-add; back substitution ten multiply-adds and one
//    multiply per row;
//  * dense LU of a border of nb DOFs with partial pivoting (the same counts over the dense
//    rows; nb = 10 for a rod's separator, 27 for a six-limb hub), the arms' Schur blocks added
//    into it (110 per arm), the update q -= delta and the squared residual norm (two per DOF).
#include <cmath>
#include <cstdio>

namespace {
unsigned long long g_ops = 0;
}

struct CountedReal {
  double v;
  CountedReal() : v(0.0) {}
  CountedReal(double x) : v(x) {}
};
inline CountedReal operator+(CountedReal a, CountedReal b) { ++g_ops; return CountedReal(a.v + b.v); }
inline CountedReal operator-(CountedReal a, CountedReal b) { ++g_ops; return CountedReal(a.v - b.v); }
inline CountedReal operator*(CountedReal a, CountedReal b) { ++g_ops; return CountedReal(a.v * b.v); }
inline CountedReal operator/(CountedReal a, CountedReal b) { ++g_ops; return CountedReal(a.v / b.v); }
inline CountedReal operator-(CountedReal a) { return CountedReal(-a.v); }
inline CountedReal& operator+=(CountedReal& a, CountedReal b) { a = a + b; return a; }
inline CountedReal& operator-=(CountedReal& a, CountedReal b) { a = a - b; return a; }
inline CountedReal sqrt(CountedReal a) { ++g_ops; return CountedReal(std::sqrt(a.v)); }
inline void sincos(CountedReal a, CountedReal* s, CountedReal* c) {
  g_ops += 2;
  *s = CountedReal(std::sin(a.v));
  *c = CountedReal(std::cos(a.v));
}
inline CountedReal sin(CountedReal a) { ++g_ops; return CountedReal(std::sin(a.v)); }
inline CountedReal cos(CountedReal a) { ++g_ops; return CountedReal(std::cos(a.v)); }
inline CountedReal atan2(CountedReal y, CountedReal x) { ++g_ops; return CountedReal(std::atan2(y.v, x.v)); }
inline CountedReal rint(CountedReal a) { return CountedReal(std::rint(a.v)); }

#define DM_REAL_COUNTED
typedef CountedReal dm_real;
#include "dm_math.h"

namespace {

v3 unit(double x, double y, double z) {
  const double n = std::sqrt(x * x + y * y + z * z);
  return mk3(x / n, y / n, z / n);
}

// One stencil pass (one orientation, four tangents) at a generic bent and twisted state.
unsigned long long count_stencil_pass() {
  const v3 ef = mk3(0.011, 0.002, -0.001), ee = mk3(0.009, 0.004, 0.002);
  const v3 tnf = unit(1.0, 0.15, -0.05), tne = unit(1.0, 0.35, 0.1);
  // directors perpendicular to their tangents
  const v3 d1nf = unit(-0.15, 1.0, 0.0), d1ne = unit(-0.35, 1.0, 0.0);
  dm_real g8[8], Hf[8][4];
  g_ops = 0;
  stencil_pass_n<4, 0>(ef, ee, 0.1, -0.2, tnf, d1nf, tne, d1ne, 0.01, 0.3, -0.1, 0.0, 2.0, 1.0, g8, Hf);
  return g_ops;
}

unsigned long long count_stretch() {
  dm_real out[9];
  g_ops = 0;
  stretch_terms(mk3(0.011, 0.002, -0.001), 100.0, 0.0105, out);
  return g_ops;
}

// Local DOF l of a stencil is a combination of na(l) of the 8 variables: expanding the 8 x 8
// Hessian to 11 x 11 takes na(a) na(b) - 1 additions per entry, the gradient na(a) - 1.
unsigned long long count_stencil_expansion() {
  unsigned long long n = 0;
  int v[2];
  dm_real c[2];
  for (int a = 0; a < 11; ++a) {
    const int na = loc_terms(a, 1.0, 1.0, v, c);
    n += na - 1;
    for (int b = 0; b < 11; ++b) n += na * loc_terms(b, 1.0, 1.0, v, c) - 1;
  }
  return n;
}

// Dense Gaussian elimination of nb DOFs with one right-hand side, then back substitution.
unsigned long long count_dense_lu(int nb) {
  unsigned long long n = 0;
  for (int p = 0; p < nb; ++p) {
    const int below = nb - p - 1;
    n += 1;                          // reciprocal of the pivot
    n += below;                      // multipliers
    n += 2ull * below * (below + 1); // multiply-adds over the remaining columns and the rhs
  }
  for (int p = 0; p < nb; ++p) n += 2ull * (nb - p - 1) + 1;   // back substitution
  return n;
}

}  // namespace

int main() {
  const unsigned long long pass = count_stencil_pass();
  const unsigned long long stencil = 2 * pass;
  const unsigned long long stretch = count_stretch();
  // node terms: per component im (x - x0 - dt v) - m g - F + eta m (x - x0)/dt (11), plus
  // im = m / dt^2 (2) and the Jacobian diagonal im + eta m / dt (3)
  const unsigned long long node = 3 * 11 + 2 + 3;
  // twist inertia of an edge: I = Ith / dt^2 (2), I (th - th0 - dt om) - moment (5)
  const unsigned long long edge_inertia = 7;
  const unsigned long long asm_stencil = count_stencil_expansion() + 11 * 11 + 11;
  const unsigned long long asm_edge = 6 * 6 + 6 + 1;   // stretch block and gradient, twist inertia
  const unsigned long long asm_node = 3 * 3 + 3;
  const unsigned long long lu_row = 1 + 10 + 2 * 10 * 11;
  const unsigned long long backsub_row = 2 * 10 + 1;
  const unsigned long long dof = 1 + 2;               // update, squared residual norm
  std::printf("{\"counter\": \"dm_flops\", \"stencil_pass_4_tangents\": %llu, \"stencil\": %llu, "
              "\"stretch\": %llu, \"node\": %llu, \"edge_inertia\": %llu, \"assembly_stencil\": %llu, "
              "\"assembly_edge\": %llu, \"assembly_node\": %llu, \"lu_row\": %llu, \"backsub_row\": %llu, "
              "\"dof\": %llu, \"schur_per_arm\": 110, \"border_lu_10\": %llu, \"border_lu_27\": %llu}\n",
              pass, stencil, stretch, node, edge_inertia, asm_stencil, asm_edge, asm_node, lu_row, backsub_row, dof,
              count_dense_lu(10), count_dense_lu(27));
  return 0;
}
