"""Edge-edge contact of the Implicit Contact Model (oracle).

TEST INFRASTRUCTURE ONLY: used by tests/ to check the HIP path; never imported by the product
path.

The paper's contact model (Contact and Friction subsection) puts an artificial energy E_c(D)
(Eq. 10, stiffness K1 = 15 / delta) on the minimum distance D between two edges, with C the
centreline distance at which contact begins (2h for self-contact).  The contact force is
-dE_c/dD dD/dq (Eq. 11); friction on an edge is -mu gamma u_hat |F_con| with
gamma = 2 / (1 + exp(-K2 |u|)) - 1, K2 = 15 / nu, u the tangential relative velocity of the two
bodies (Eq. 12-13).  The Newton solve uses the contact energy's Hessian (Eq. 16).

Definitions and readings (the paper leaves them open):

* D(a, b, c, d) = min over s, t in [0, 1] of |a + s (b - a) - c - t (d - c)| for edge (a, b)
  and edge (c, d).  The function on the square is convex, so its minimum is the stationary
  point of the two lines when that lies inside the square, and otherwise lies on the square's
  boundary, where it is the distance from an end point to the other segment;
* C = h_i + h_j (2h for two edges of one rod), and the pair's energy is k_c E_c(D), as for the
  floor (Eq. 10 has no stiffness of its own);
* candidate pairs: every pair of edges except two edges of one rod whose rest arclength gap
  (the summed rest lengths of the edges strictly between them) is below C + delta: they would
  be "in contact" in the rest shape (adjacent edges have gap 0); edges of different rods are
  always candidates;
* the contact set is the candidates with D < C + delta (the support of Eq. 10);
* friction: P(s) and Q(t) the closest points, n = (P - Q)/D; the relative velocity of the two
  points over the step, v_rel = (P - P_n - Q + Q_n)/dt at fixed (s, t); u = v_rel - (v_rel.n) n;
  |F_con| on either edge is k_c |dE_c/dD|; edge i gets F_fr = -mu gamma u_hat |F_con|, spread to
  its nodes with weights (1 - s, s), and edge j the opposite force with weights (1 - t, t).

Pinned by tests/test_oracle_contact.py: the distance against a brute-force minimum over a
dense parameter grid refined by a bounded 2-D minimiser, closed-form configurations
(perpendicular skew segments, parallel offset segments, end point to end point), symmetry and
rigid-motion invariance, the gradient against the envelope-theorem closed form and central
differences, the Hessian against central differences of the gradient, the pair list against a
double loop with the exclusion rule written out, and the friction force against Eq. 12-13 in
a configuration where u is known.
"""
from __future__ import annotations

import math

import torch

from . import der

DT = torch.float64


def _val(t):
    """Plain float of a tensor for a branch decision (no derivative flows through it)."""
    return float(t.detach()) if hasattr(t, "detach") else float(t)


# ---------------------------------------------------------------------------
# segment-segment distance
# ---------------------------------------------------------------------------

def point_segment(p, a, b):
    """Distance from point p to segment (a, b) and the clamped parameter of the foot point."""
    ab = b - a
    L2 = torch.dot(ab, ab)
    t = torch.clamp(torch.dot(p - a, ab) / L2, 0.0, 1.0)
    return torch.linalg.norm(p - (a + t * ab)), t


def segment_distance(a, b, c, d):
    """D = min over s, t in [0, 1] of |a + s (b - a) - (c + t (d - c))| and the minimising
    (s, t).  Candidates: the stationary point of the two lines (when the lines are not
    parallel and it lies inside the square), and the four end-point-to-segment distances (the
    square's edges).  The smallest candidate is the minimum; its branch carries the derivative."""
    u, v, w = b - a, d - c, a - c
    A, B, Cc = torch.dot(u, u), torch.dot(u, v), torch.dot(v, v)
    Dd, E = torch.dot(u, w), torch.dot(v, w)
    den = A * Cc - B * B
    cands = []
    if _val(den) > 1e-14 * _val(A * Cc):
        s = (B * E - Cc * Dd) / den
        t = (A * E - B * Dd) / den
        if 0.0 < _val(s) < 1.0 and 0.0 < _val(t) < 1.0:
            cands.append((torch.linalg.norm(w + s * u - t * v), s, t))
    dist, t = point_segment(a, c, d)
    cands.append((dist, torch.zeros_like(dist), t))
    dist, t = point_segment(b, c, d)
    cands.append((dist, torch.ones_like(dist), t))
    dist, s = point_segment(c, a, b)
    cands.append((dist, s, torch.zeros_like(dist)))
    dist, s = point_segment(d, a, b)
    cands.append((dist, s, torch.ones_like(dist)))
    k = min(range(len(cands)), key=lambda i: _val(cands[i][0]))
    return cands[k]


def branch_of(x12):
    """Which candidate of `segment_distance` attains the minimum at the coordinates x12
    (0: the stationary point inside the square, 1..4: end point a, b, c or d against the
    other segment), decided on plain values."""
    a, b, c, d = x12[0:3], x12[3:6], x12[6:9], x12[9:12]
    D, s, t = segment_distance(a, b, c, d)
    sv, tv = _val(s), _val(t)
    if 0.0 < sv < 1.0 and 0.0 < tv < 1.0:
        return 0
    cands = [(_val(point_segment(a, c, d)[0]), 1), (_val(point_segment(b, c, d)[0]), 2),
             (_val(point_segment(c, a, b)[0]), 3), (_val(point_segment(d, a, b)[0]), 4)]
    return min(cands)[1]


def closest_on_branch(x12, k):
    """(D, s, t) by the formula of candidate k alone: no decision on values, so it can be
    differentiated (and vectorised) at coordinates where k is the minimising candidate."""
    a, b, c, d = x12[0:3], x12[3:6], x12[6:9], x12[9:12]
    if k == 0:
        u, v, w = b - a, d - c, a - c
        A, B, Cc = torch.dot(u, u), torch.dot(u, v), torch.dot(v, v)
        Dd, E = torch.dot(u, w), torch.dot(v, w)
        den = A * Cc - B * B
        s = (B * E - Cc * Dd) / den
        t = (A * E - B * Dd) / den
        return torch.linalg.norm(w + s * u - t * v), s, t
    if k == 1:
        D, t = point_segment(a, c, d)
        return D, torch.zeros_like(D), t
    if k == 2:
        D, t = point_segment(b, c, d)
        return D, torch.ones_like(D), t
    if k == 3:
        D, s = point_segment(c, a, b)
        return D, s, torch.zeros_like(D)
    D, s = point_segment(d, a, b)
    return D, s, torch.ones_like(D)


def distance_of(x12):
    """D as a function of the 12 stacked coordinates (a, b, c, d)."""
    a, b, c, d = x12[0:3], x12[3:6], x12[6:9], x12[9:12]
    return segment_distance(a, b, c, d)[0]


def distance_gradient(x12):
    return torch.func.grad(distance_of)(x12)


def distance_hessian(x12):
    return torch.func.jacfwd(torch.func.grad(distance_of))(x12)


# ---------------------------------------------------------------------------
# pairs
# ---------------------------------------------------------------------------

class EdgeSet:
    """The edges of a set of rods: node positions are indexed through `edges` (E, 2);
    `rod` (E,) the rod of each edge, `pos` (E,) its index along the rod, `radius` (E,),
    `ebar` (E,) rest lengths."""

    def __init__(self, edges, rod, pos, radius, ebar):
        self.edges = torch.as_tensor(edges, dtype=torch.long)
        self.rod = torch.as_tensor(rod, dtype=torch.long)
        self.pos = torch.as_tensor(pos, dtype=torch.long)
        self.radius = torch.as_tensor(radius, dtype=DT)
        self.ebar = torch.as_tensor(ebar, dtype=DT)
        E = self.edges.shape[0]
        # cumulative rest length along each rod at the start of every edge
        self.arc0 = torch.zeros(E, dtype=DT)
        for r in torch.unique(self.rod).tolist():
            idx = torch.nonzero(self.rod == r).flatten()
            idx = idx[torch.argsort(self.pos[idx])]
            acc = 0.0
            for i in idx.tolist():
                self.arc0[i] = acc
                acc += float(self.ebar[i])

    @staticmethod
    def from_rods(rods):
        """rods: list of (N_k, 3) rest node arrays and radii [(x0, h), ...]; nodes numbered
        rod after rod.  Returns the EdgeSet and the total node count."""
        edges, rod, pos, rad, eb = [], [], [], [], []
        off = 0
        for k, (x0, h) in enumerate(rods):
            x0 = torch.as_tensor(x0, dtype=DT)
            n = x0.shape[0]
            for j in range(n - 1):
                edges.append((off + j, off + j + 1))
                rod.append(k)
                pos.append(j)
                rad.append(h)
                eb.append(float(torch.linalg.norm(x0[j + 1] - x0[j])))
            off += n
        return EdgeSet(edges, rod, pos, rad, eb), off

    def gap(self, i, j):
        """Rest arclength strictly between edges i and j of one rod (inf for two rods)."""
        if int(self.rod[i]) != int(self.rod[j]):
            return math.inf
        if int(self.pos[i]) > int(self.pos[j]):
            i, j = j, i
        return float(self.arc0[j] - self.arc0[i] - self.ebar[i])

    def contact_distance(self, i, j):
        return float(self.radius[i] + self.radius[j])

    def excluded(self, i, j, delta):
        return self.gap(i, j) < self.contact_distance(i, j) + delta


def pair_coords(es, x, i, j):
    a, b = es.edges[i].tolist()
    c, d = es.edges[j].tolist()
    return torch.cat([x[a], x[b], x[c], x[d]])


def contact_pairs(es, x, delta):
    """Every non-excluded pair i < j with D < C + delta, by a double loop: [(i, j, D, s, t)]."""
    x = torch.as_tensor(x, dtype=DT)
    out = []
    E = es.edges.shape[0]
    for i in range(E):
        for j in range(i + 1, E):
            if es.excluded(i, j, delta):
                continue
            a, b = es.edges[i].tolist()
            c, d = es.edges[j].tolist()
            D, s, t = segment_distance(x[a], x[b], x[c], x[d])
            if float(D) < es.contact_distance(i, j) + delta:
                out.append((i, j, float(D), float(s), float(t)))
    return out


# ---------------------------------------------------------------------------
# energy, forces, Hessian
# ---------------------------------------------------------------------------

def pair_energy(x12, C, delta, k_c):
    """k_c E_c(D) of one pair (Eq. 10 through the oracle's floor profile)."""
    return k_c * der.contact_energy_profile(distance_of(x12), C, delta)


def pair_terms(x12, C, delta, k_c):
    """Energy, gradient (12) and Hessian (12 x 12) of one pair's contact energy."""
    f = lambda q: pair_energy(q, C, delta, k_c)
    return f(x12), torch.func.grad(f)(x12), torch.func.jacfwd(torch.func.grad(f))(x12)


def contact_energy(es, x, pairs, delta, k_c):
    """Total contact energy of the given pairs as a function of all node positions x (n, 3)."""
    tot = torch.zeros((), dtype=DT)
    for (i, j, *_) in pairs:
        tot = tot + pair_energy(pair_coords(es, x, i, j), es.contact_distance(i, j), delta, k_c)
    return tot


def contact_force(es, x, pairs, delta, k_c):
    """F_con = -dE/dx over the pairs (Eq. 11), (n, 3)."""
    x = torch.as_tensor(x, dtype=DT)
    return -torch.func.grad(lambda xx: contact_energy(es, xx, pairs, delta, k_c))(x)


def friction_force(es, x, x_n, dt, pairs, delta, k_c, mu, nu):
    """Friction of Eq. 12-13 on every pair (forces (n, 3)), u per the module's reading."""
    x = torch.as_tensor(x, dtype=DT)
    x_n = torch.as_tensor(x_n, dtype=DT)
    K2 = 15.0 / nu
    F = torch.zeros_like(x)
    for (i, j, *_) in pairs:
        a, b = es.edges[i].tolist()
        c, d = es.edges[j].tolist()
        D, s, t = segment_distance(x[a], x[b], x[c], x[d])
        P = x[a] + s * (x[b] - x[a])
        Q = x[c] + t * (x[d] - x[c])
        n = (P - Q) / D
        Pn = x_n[a] + s * (x_n[b] - x_n[a])
        Qn = x_n[c] + t * (x_n[d] - x_n[c])
        vrel = (P - Pn - Q + Qn) / dt
        u = vrel - torch.dot(vrel, n) * n
        C = es.contact_distance(i, j)
        dEdD = torch.func.grad(lambda dd: der.contact_energy_profile(dd, C, delta))(D)
        fcon = k_c * torch.abs(dEdD)
        un = torch.linalg.norm(u)
        if float(un) == 0.0 or float(fcon) == 0.0:
            continue
        gamma = 2.0 / (1.0 + torch.exp(-K2 * un)) - 1.0
        f = -mu * gamma * fcon * u / un                         # on edge i (Eq. 13)
        F[a] += (1.0 - s) * f
        F[b] += s * f
        F[c] -= (1.0 - t) * f
        F[d] -= t * f
    return F
