// dm_contact.hip -- edge-edge contact of the Implicit Contact Model (Contact and Friction
// subsection, Eq. 10-13) on the GPU:
//  * detection, one workgroup per contact group: the group's edges get axis-aligned boxes
//    inflated by radius + delta / 2 (two edges within C + delta = h_i + h_j + delta of each
//    other have overlapping boxes), rounded outward to float32 in LDS; the edges are sorted by
//    the boxes' lower x bound (bitonic sort in LDS) and each edge sweeps forward through the
//    sorted order while the next lower bound is below its upper bound; box overlap in y and z,
//    the rest-shape exclusion of near edges of one rod, and the exact segment distance decide
//    the pair; the pairs found are sorted (by local edge indices) in LDS and written in order;
//  * per pair: the minimum distance D and its closest-point parameters (the clamped
//    closest-point construction for two segments, Ericson, Real-Time Collision Detection, 5.1.9),
//    the energy k_c E_c(D) of Eq. 10, its gradient and its Hessian in closed form, and the
//    friction force of Eq. 12-13.
//
// Hessian of D (x the 12 coordinates of the pair, z = (s, t), r = P(s) - Q(t), f = |r|^2 / 2,
// F(x) = min_z f = D^2 / 2): the gradient is F_x = f_x at the minimiser (envelope theorem), and
// F_xx = f_xx - f_xz f_zz^-1 f_zx over the parameters not clamped at 0 or 1 (implicit
// differentiation of the stationarity f_z = 0); then D_x = F_x / D and
// D_xx = (F_xx - D_x D_x^T) / D.  With c = (1 - s, s, -(1 - t), -t) per node, f_x = c_k r,
// f_xx = c_k c_l I, f_xs = (-r, r, 0, 0) + c_k (b - a), f_xt = (0, 0, r, -r) - c_k (d - c),
// f_zz = [[|b - a|^2, -(b - a).(d - c)], [-(b - a).(d - c), |d - c|^2]].
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <string>
#include <vector>

#include "dmrod.h"
#include "dm_segment.h"

namespace {

constexpr int CT_THREADS = 256;

struct CtTables {
  const int* e0;         // first node of each edge [E]
  const int* e1;         // second node [E]
  const int* rod;        // rod of each edge [E]
  const double* arc0;    // rest arclength of the rod at the edge's first node [E]
  const double* ebar;    // rest length [E]
  const double* rad;     // radius [E]
  const int* gstart;     // first edge of each group [G + 1]
  int n_groups, cap;     // groups; pair slots per group
  double delta;
};

// ---------------------------------------------------------------------------
// segment geometry
// ---------------------------------------------------------------------------

struct V3 {
  double x, y, z;
};
__device__ __forceinline__ V3 ld(const double* p, int n) { return V3{p[3 * n], p[3 * n + 1], p[3 * n + 2]}; }
__device__ __forceinline__ V3 sub(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 axpy(double s, V3 a, V3 b) { return V3{fma(s, a.x, b.x), fma(s, a.y, b.y), fma(s, a.z, b.z)}; }
__device__ __forceinline__ double dotv(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ double clamp01(double v) { return fmin(fmax(v, 0.0), 1.0); }

// Closest points (dm_segment.h) of segments p1 + s d1 and p2 + t d2; returns |P - Q|^2.
__device__ double closest(V3 p1, V3 d1, V3 p2, V3 d2, double& s, double& t) {
  const double a1[3] = {p1.x, p1.y, p1.z}, b1[3] = {d1.x, d1.y, d1.z};
  const double a2[3] = {p2.x, p2.y, p2.z}, b2[3] = {d2.x, d2.y, d2.z};
  double r[3];
  return seg_closest(a1, b1, a2, b2, s, t, r);
}

// Edges i and j of one rod that lie within C + delta of each other in the rest shape (their
// rest arclength gap) are never a pair.
__device__ __forceinline__ bool excluded(const CtTables& T, int i, int j) {
  if (T.rod[i] != T.rod[j]) return false;
  const double gap = T.arc0[i] < T.arc0[j] ? T.arc0[j] - T.arc0[i] - T.ebar[i] : T.arc0[i] - T.arc0[j] - T.ebar[j];
  return gap < T.rad[i] + T.rad[j] + T.delta;
}

// ---------------------------------------------------------------------------
// detection
// ---------------------------------------------------------------------------

constexpr int CT_MAX_EDGES = DM_CONTACT_MAX_GROUP_EDGES;
constexpr int CT_MAX_PAIRS = DM_CONTACT_MAX_PAIRS_PER_GROUP;

// Round a double down / up to a float (the inflated box stays a superset of the exact one).
__device__ __forceinline__ float down(double v) {
  float f = (float)v;
  return (double)f > v ? nextafterf(f, -INFINITY) : f;
}
__device__ __forceinline__ float up(double v) {
  float f = (float)v;
  return (double)f < v ? nextafterf(f, INFINITY) : f;
}

// Bitonic sort of v[0 .. n2) (n2 a power of two) in LDS by less(a, b), by the whole workgroup.
template <class K, class Less>
__device__ void bitonic(K* v, int n2, Less less) {
  for (int k = 2; k <= n2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n2; i += blockDim.x) {
        const int p = i ^ j;
        if (p > i) {
          const K a = v[i], b = v[p];
          const bool up_ = (i & k) == 0;
          if (up_ ? less(b, a) : less(a, b)) {
            v[i] = b;
            v[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(CT_THREADS) ct_find_kernel(CtTables T, const double* __restrict__ x,
                                                           int* __restrict__ pairs, double* __restrict__ dst,
                                                           int* __restrict__ counts) {
  // 60 KB of LDS: float boxes, the sweep order (16-bit local indices), the pair keys
  __shared__ float bmin[3][CT_MAX_EDGES], bmax[3][CT_MAX_EDGES];
  __shared__ short order[CT_MAX_EDGES];
  __shared__ int plist[CT_MAX_PAIRS];
  __shared__ int pcount;
  const int g = blockIdx.x;
  const int e0 = T.gstart[g], n = T.gstart[g + 1] - e0;
  if (threadIdx.x == 0) pcount = 0;
  int n2 = 1;
  while (n2 < n) n2 <<= 1;
  for (int i = threadIdx.x; i < n2; i += blockDim.x) {
    order[i] = (short)(i < n ? i : -1);              // -1: padding, sorted last
    if (i < n) {
      const int e = e0 + i;
      const V3 a = ld(x, T.e0[e]), b = ld(x, T.e1[e]);
      const double inf = T.rad[e] + 0.5 * T.delta;
      bmin[0][i] = down(fmin(a.x, b.x) - inf);
      bmin[1][i] = down(fmin(a.y, b.y) - inf);
      bmin[2][i] = down(fmin(a.z, b.z) - inf);
      bmax[0][i] = up(fmax(a.x, b.x) + inf);
      bmax[1][i] = up(fmax(a.y, b.y) + inf);
      bmax[2][i] = up(fmax(a.z, b.z) + inf);
    }
  }
  __syncthreads();
  // sweep order: lower x bound, then edge index (a total order, so the result is fixed)
  bitonic(order, n2, [&](short a, short b) {
    if (b < 0) return a >= 0;
    if (a < 0) return false;
    const float ka = bmin[0][a], kb = bmin[0][b];
    return ka < kb || (ka == kb && a < b);
  });
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    const int i = order[p];
    const float xi = bmax[0][i];
    const int ei = e0 + i;
    const V3 pa = ld(x, T.e0[ei]), pb = ld(x, T.e1[ei]);
    const V3 di = sub(pb, pa);
    for (int q = p + 1; q < n; ++q) {
      const int j = order[q];
      if (bmin[0][j] > xi) break;
      if (bmin[1][j] > bmax[1][i] || bmin[1][i] > bmax[1][j] || bmin[2][j] > bmax[2][i] || bmin[2][i] > bmax[2][j])
        continue;
      const int ej = e0 + j;
      if (excluded(T, ei, ej)) continue;
      const V3 qa = ld(x, T.e0[ej]), qb = ld(x, T.e1[ej]);
      double s, t;
      const double D2 = closest(pa, di, qa, sub(qb, qa), s, t);
      const double reach = T.rad[ei] + T.rad[ej] + T.delta;
      if (D2 < reach * reach) {
        const int k = atomicAdd(&pcount, 1);
        if (k < CT_MAX_PAIRS) plist[k] = i < j ? (i << 16) | j : (j << 16) | i;
      }
    }
  }
  __syncthreads();
  const int np = pcount, nk = min(np, CT_MAX_PAIRS);
  int m2 = 1;
  while (m2 < nk) m2 <<= 1;
  for (int k = nk + threadIdx.x; k < m2; k += blockDim.x) plist[k] = 0x7fffffff;
  __syncthreads();
  bitonic(plist, m2, [](int a, int b) { return a < b; });
  const int cap = T.cap;
  for (int k = threadIdx.x; k < min(nk, cap); k += blockDim.x) {
    const int i = plist[k] >> 16, j = plist[k] & 0xffff;
    const int ei = e0 + i, ej = e0 + j;
    const V3 pa = ld(x, T.e0[ei]), pb = ld(x, T.e1[ei]), qa = ld(x, T.e0[ej]), qb = ld(x, T.e1[ej]);
    double s, t;
    const double D2 = closest(pa, sub(pb, pa), qa, sub(qb, qa), s, t);
    const size_t slot = (size_t)g * cap + k;
    pairs[2 * slot] = ei;
    pairs[2 * slot + 1] = ej;
    dst[3 * slot] = sqrt(D2);
    dst[3 * slot + 1] = s;
    dst[3 * slot + 2] = t;
  }
  if (threadIdx.x == 0) counts[g] = np;
}

// ---------------------------------------------------------------------------
// energy, gradient, Hessian, friction
// ---------------------------------------------------------------------------

// E_c(D) of Eq. 10 and its first two derivatives in D (K1 = 15 / delta).
__device__ void profile(double D, double C, double delta, double& E, double& E1, double& E2) {
  if (D <= C - delta) {
    E = (C - D) * (C - D);
    E1 = -2.0 * (C - D);
    E2 = 2.0;
  } else if (D < C + delta) {
    const double K1 = 15.0 / delta, z = K1 * (C - D);
    const double L = log1p(exp(z)), sg = 1.0 / (1.0 + exp(-z));
    E = (L / K1) * (L / K1);
    E1 = -2.0 * L * sg / K1;
    E2 = 2.0 * (sg * sg + L * sg * (1.0 - sg));
  } else {
    E = E1 = E2 = 0.0;
  }
}

struct CtTermArgs {
  CtTables T;
  const double* x;
  const double* xprev;   // step start, for friction (may be null)
  const int* pairs;
  const int* counts;
  double dt, kc, mu, nu;
  double* energy;        // [G][cap]
  double* grad;          // [G][12][cap]
  double* hess;          // [G][144][cap] (may be null)
  double* fric;          // [G][12][cap] (may be null)
};

__global__ void __launch_bounds__(CT_THREADS) ct_terms_kernel(CtTermArgs A) {
  const CtTables& T = A.T;
  const int g = blockIdx.x, cap = T.cap;
  const int np = min(A.counts[g], cap);
  for (int k = threadIdx.x; k < np; k += blockDim.x) {
    const size_t slot = (size_t)g * cap + k;
    const int ei = A.pairs[2 * slot], ej = A.pairs[2 * slot + 1];
    const int na = T.e0[ei], nb = T.e1[ei], nc = T.e0[ej], nd = T.e1[ej];
    const V3 pa = ld(A.x, na), pb = ld(A.x, nb), qa = ld(A.x, nc), qb = ld(A.x, nd);
    const V3 u = sub(pb, pa), v = sub(qb, qa);
    double s, t;
    const double D = sqrt(closest(pa, u, qa, v, s, t));
    const V3 r = sub(axpy(s, u, pa), axpy(t, v, qa));
    const double C = T.rad[ei] + T.rad[ej];
    double E, E1, E2;
    profile(D, C, T.delta, E, E1, E2);
    const size_t base = (size_t)g * cap;
    A.energy[slot] = A.kc * E;
    const double cw[4] = {1.0 - s, s, -(1.0 - t), -t};
    const double rv[3] = {r.x, r.y, r.z}, uv[3] = {u.x, u.y, u.z}, vv[3] = {v.x, v.y, v.z};
    // D_x = c_k r / D (zero at D = 0, where the direction is undefined)
    const double invD = D > 0.0 ? 1.0 / D : 0.0;
    double gD[12];
#pragma unroll
    for (int a = 0; a < 12; ++a) gD[a] = cw[a / 3] * rv[a % 3] * invD;
#pragma unroll
    for (int a = 0; a < 12; ++a) A.grad[(base * 12) + (size_t)a * cap + k] = A.kc * E1 * gD[a];
    if (A.hess) {
      // f_xz columns and f_zz restricted to the unclamped parameters
      double Gs[12], Gt[12];
#pragma unroll
      for (int a = 0; a < 12; ++a) {
        const int nk = a / 3, al = a % 3;
        Gs[a] = (nk == 0 ? -rv[al] : (nk == 1 ? rv[al] : 0.0)) + cw[nk] * uv[al];
        Gt[a] = (nk == 2 ? rv[al] : (nk == 3 ? -rv[al] : 0.0)) - cw[nk] * vv[al];
      }
      const bool fs = s > 0.0 && s < 1.0, ft = t > 0.0 && t < 1.0;
      const double zss = dotv(u, u), ztt = dotv(v, v), zst = -dotv(u, v);
      double M00 = 0.0, M01 = 0.0, M11 = 0.0;          // f_zz^-1 on the free block
      if (fs && ft) {
        const double det = zss * ztt - zst * zst;
        M00 = ztt / det;
        M11 = zss / det;
        M01 = -zst / det;
      } else if (fs) {
        M00 = 1.0 / zss;
      } else if (ft) {
        M11 = 1.0 / ztt;
      }
      double Ws[12], Wt[12];
#pragma unroll
      for (int a = 0; a < 12; ++a) {
        Ws[a] = Gs[a] * M00 + Gt[a] * M01;
        Wt[a] = Gs[a] * M01 + Gt[a] * M11;
      }
      // H = k_c (E'' D_x D_x^T + E' D_xx), D_xx = (f_xx - W G^T - D_x D_x^T) / D
      const double c1 = A.kc * E2, c2 = A.kc * E1 * invD;
      double* H = A.hess + base * 144;
#pragma unroll
      for (int a = 0; a < 12; ++a) {
#pragma unroll
        for (int b = 0; b < 12; ++b) {
          const double fxx = (a % 3 == b % 3) ? cw[a / 3] * cw[b / 3] : 0.0;
          const double Dxx = fxx - (Ws[a] * Gs[b] + Wt[a] * Gt[b]) - gD[a] * gD[b];
          H[(size_t)(12 * a + b) * cap + k] = c1 * gD[a] * gD[b] + c2 * Dxx;
        }
      }
    }
    if (A.fric) {
      double f[3] = {0.0, 0.0, 0.0};
      if (A.xprev && D > 0.0 && E1 != 0.0) {
        const V3 ppa = ld(A.xprev, na), ppb = ld(A.xprev, nb), pqa = ld(A.xprev, nc), pqb = ld(A.xprev, nd);
        // relative velocity of the closest points over the step, at fixed (s, t)
        const V3 dP = sub(axpy(s, u, pa), axpy(s, sub(ppb, ppa), ppa));
        const V3 dQ = sub(axpy(t, v, qa), axpy(t, sub(pqb, pqa), pqa));
        const V3 w = sub(dP, dQ);
        const double idt = 1.0 / A.dt;
        const V3 vr = V3{w.x * idt, w.y * idt, w.z * idt};
        const double vn = dotv(vr, r) * invD * invD;        // (v_rel . n) / D, n = r / D
        const V3 ut = V3{vr.x - vn * r.x, vr.y - vn * r.y, vr.z - vn * r.z};
        const double un = sqrt(dotv(ut, ut));
        if (un > 0.0) {
          const double K2 = 15.0 / A.nu;
          const double gamma = 2.0 / (1.0 + exp(-K2 * un)) - 1.0;
          const double m = -A.mu * gamma * A.kc * fabs(E1) / un;
          f[0] = m * ut.x;
          f[1] = m * ut.y;
          f[2] = m * ut.z;
        }
      }
      const double wgt[4] = {1.0 - s, s, -(1.0 - t), -t};
      double* Fo = A.fric + base * 12;
#pragma unroll
      for (int a = 0; a < 12; ++a) Fo[(size_t)a * cap + k] = wgt[a / 3] * f[a % 3];
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

thread_local std::string g_ct_err;
dm_status cfail(dm_status s, const std::string& m) {
  g_ct_err = m;
  return s;
}
#define CH(call)                                                                                        \
  do {                                                                                                  \
    hipError_t e_ = (call);                                                                             \
    if (e_ != hipSuccess) return cfail(DM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

struct dm_contact {
  int device = 0;
  hipStream_t stream = nullptr;
  int n_nodes = 0, n_edges = 0, n_groups = 0, cap = 0;
  double delta = 0.0;
  std::vector<void*> bufs;
  CtTables T{};
  float ms_find = 0.0f, ms_terms = 0.0f;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace {
template <class V>
dm_status upload(dm_contact* c, const std::vector<V>& h, const V** out) {
  void* p = nullptr;
  CH(hipMalloc(&p, std::max<size_t>(h.size(), 1) * sizeof(V)));
  c->bufs.push_back(p);
  if (!h.empty()) CH(hipMemcpy(p, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice));
  *out = static_cast<const V*>(p);
  return DM_OK;
}
bool is_fin(double v) { return std::isfinite(v); }
}  // namespace

extern "C" {

const char* dm_contact_last_error(void) { return g_ct_err.c_str(); }

void dm_contact_destroy(dm_contact* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  for (hipEvent_t e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (void* p : c->bufs) (void)hipFree(p);
  delete c;
}

dm_status dm_contact_create(int device, void* stream, int n_nodes, int n_edges, const int* edges, const int* rod,
                            const double* arc0, const double* ebar, const double* radius, int n_groups,
                            const int* group_start, double delta, int pair_capacity, dm_contact** out) {
  if (!out) return cfail(DM_ERR_INVALID_ARG, "dm_contact_create: null output");
  *out = nullptr;
  if (n_nodes < 0 || n_edges < 0 || n_groups < 0 || (n_edges > 0 && (!edges || !rod || !arc0 || !ebar || !radius)) ||
      !group_start)
    return cfail(DM_ERR_INVALID_ARG, "dm_contact_create: bad size or null table");
  if (!(delta > 0.0) || !is_fin(delta)) return cfail(DM_ERR_INVALID_ARG, "dm_contact_create: delta must be > 0");
  if (pair_capacity < 1 || pair_capacity > DM_CONTACT_MAX_PAIRS_PER_GROUP)
    return cfail(DM_ERR_INVALID_ARG, "dm_contact_create: pair_capacity must be in 1 .. " +
                                         std::to_string(DM_CONTACT_MAX_PAIRS_PER_GROUP));
  if (group_start[0] != 0 || group_start[n_groups] != n_edges)
    return cfail(DM_ERR_INVALID_ARG, "dm_contact_create: group_start must run from 0 to n_edges");
  for (int g = 0; g < n_groups; ++g) {
    const int ne = group_start[g + 1] - group_start[g];
    if (ne < 0 || ne > DM_CONTACT_MAX_GROUP_EDGES)
      return cfail(DM_ERR_INVALID_ARG, "dm_contact_create: group " + std::to_string(g) + " has " + std::to_string(ne) +
                                           " edges (0 .. " + std::to_string(DM_CONTACT_MAX_GROUP_EDGES) + ")");
  }
  std::vector<int> e0(n_edges), e1(n_edges), rd(rod, rod + n_edges);
  std::vector<double> a0(arc0, arc0 + n_edges), eb(ebar, ebar + n_edges), ra(radius, radius + n_edges);
  for (int e = 0; e < n_edges; ++e) {
    e0[e] = edges[2 * e];
    e1[e] = edges[2 * e + 1];
    if (e0[e] < 0 || e0[e] >= n_nodes || e1[e] < 0 || e1[e] >= n_nodes || e0[e] == e1[e])
      return cfail(DM_ERR_INVALID_ARG, "dm_contact_create: edge " + std::to_string(e) + " has a bad node index");
    if (!(ra[e] > 0.0) || !is_fin(ra[e]) || !(eb[e] > 0.0) || !is_fin(eb[e]) || !is_fin(a0[e]))
      return cfail(DM_ERR_INVALID_ARG, "dm_contact_create: edge " + std::to_string(e) + " has a bad radius, length or arclength");
  }
  auto* c = new dm_contact();
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  c->n_nodes = n_nodes;
  c->n_edges = n_edges;
  c->n_groups = n_groups;
  c->cap = pair_capacity;
  c->delta = delta;
  dm_status st = DM_OK;
  auto run = [&]() -> dm_status {
    CH(hipSetDevice(device));
    std::vector<int> gs(group_start, group_start + n_groups + 1);
    dm_status s;
    if ((s = upload(c, e0, &c->T.e0)) != DM_OK) return s;
    if ((s = upload(c, e1, &c->T.e1)) != DM_OK) return s;
    if ((s = upload(c, rd, &c->T.rod)) != DM_OK) return s;
    if ((s = upload(c, a0, &c->T.arc0)) != DM_OK) return s;
    if ((s = upload(c, eb, &c->T.ebar)) != DM_OK) return s;
    if ((s = upload(c, ra, &c->T.rad)) != DM_OK) return s;
    if ((s = upload(c, gs, &c->T.gstart)) != DM_OK) return s;
    for (hipEvent_t& e : c->ev) CH(hipEventCreate(&e));
    return DM_OK;
  };
  if ((st = run()) != DM_OK) {
    dm_contact_destroy(c);
    return st;
  }
  c->T.n_groups = n_groups;
  c->T.cap = pair_capacity;
  c->T.delta = delta;
  *out = c;
  return DM_OK;
}

dm_status dm_contact_find(dm_contact* c, const double* x, int* pairs, double* dst, int* counts, int* total) {
  if (!c || !x || !pairs || !dst || !counts) return cfail(DM_ERR_INVALID_ARG, "dm_contact_find: null argument");
  CH(hipSetDevice(c->device));
  if (c->n_groups > 0) {
    CH(hipEventRecord(c->ev[0], c->stream));
    hipLaunchKernelGGL(ct_find_kernel, dim3(c->n_groups), dim3(CT_THREADS), 0, c->stream, c->T, x, pairs, dst, counts);
    CH(hipGetLastError());
    CH(hipEventRecord(c->ev[1], c->stream));
  }
  CH(hipStreamSynchronize(c->stream));
  if (c->n_groups > 0) CH(hipEventElapsedTime(&c->ms_find, c->ev[0], c->ev[1]));
  std::vector<int> h(c->n_groups);
  if (c->n_groups > 0) CH(hipMemcpy(h.data(), counts, sizeof(int) * c->n_groups, hipMemcpyDeviceToHost));
  long long tot = 0;
  int worst = -1;
  for (int g = 0; g < c->n_groups; ++g) {
    tot += h[g];
    if (h[g] > c->cap && (worst < 0 || h[g] > h[worst])) worst = g;
  }
  if (total) *total = (int)std::min<long long>(tot, 0x7fffffff);
  if (worst >= 0)
    return cfail(DM_ERR_INVALID_ARG, "dm_contact_find: group " + std::to_string(worst) + " has " +
                                         std::to_string(h[worst]) + " pairs, above the capacity of " +
                                         std::to_string(c->cap) + " (the counts are exact; the slots hold a subset)");
  return DM_OK;
}

dm_status dm_contact_terms(dm_contact* c, const double* x, const double* x_prev, double dt, double k_c, double mu,
                           double nu, const int* pairs, const int* counts, double* energy, double* grad, double* hess,
                           double* friction) {
  if (!c || !x || !pairs || !counts || !energy || !grad) return cfail(DM_ERR_INVALID_ARG, "dm_contact_terms: null argument");
  if (!(k_c >= 0.0) || !is_fin(k_c)) return cfail(DM_ERR_INVALID_ARG, "dm_contact_terms: k_c must be >= 0");
  if (friction && x_prev && (!(dt > 0.0) || !is_fin(dt) || !(mu >= 0.0) || !is_fin(mu) || !(nu > 0.0) || !is_fin(nu)))
    return cfail(DM_ERR_INVALID_ARG, "dm_contact_terms: friction needs dt > 0, mu >= 0, nu > 0");
  CH(hipSetDevice(c->device));
  CtTermArgs A{c->T, x, x_prev, pairs, counts, dt, k_c, mu, nu, energy, grad, hess, friction};
  if (c->n_groups > 0) {
    CH(hipEventRecord(c->ev[2], c->stream));
    hipLaunchKernelGGL(ct_terms_kernel, dim3(c->n_groups), dim3(CT_THREADS), 0, c->stream, A);
    CH(hipGetLastError());
    CH(hipEventRecord(c->ev[3], c->stream));
  }
  CH(hipStreamSynchronize(c->stream));
  if (c->n_groups > 0) CH(hipEventElapsedTime(&c->ms_terms, c->ev[2], c->ev[3]));
  return DM_OK;
}

double dm_contact_last_ms(const dm_contact* c, int which) {
  if (!c) return 0.0;
  return which == 0 ? c->ms_find : c->ms_terms;
}

}  // extern "C"
