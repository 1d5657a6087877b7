"""Plain fp64 CPU oracle of the fully implicit Discrete Elastic Rods (DER) step.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this package.  The product path never
imports it, and it shares no code with the HIP path: only the seeded input
descriptions of `workloads` serve both sides.

What it computes, in the paper's order and notation (DisMech, Methodology):

* DOFs (Eq. 1): N node positions q_i and one twist angle theta^i per edge.
  Here q is stored as [x (n_nodes*3), theta (n_edges)]; the order of DOFs
  does not change the method.
* Frames (Methodology, first paragraph): each edge carries a reference frame
  {d1, d2, t} and a material frame {m1, m2, t}, the latter the reference frame
  rotated by theta about t.  The reference frame is carried from the start of
  the step to the current tangent by time-parallel transport.
* Energies: stretch (Eq. 2-3), curvature binormal (Eq. 4), integrated curvature
  (Eq. 5), bending (Eq. 6), twist with reference twist beta (Eq. 7-8).
* Elastic force (Eq. 9) = minus the gradient of the energy, taken here by
  automatic differentiation of the energy exactly as written above.
* Contact (Eq. 10-11) against a flat floor, smooth Coulomb friction (Eq. 12-13),
  gravity and optional viscous damping (miscellaneous forces).
* Edge-edge self-contact of a rod (the same Eq. 10-13 on pairs of its edges, with the
  distance and pairing of `oracle/contact.py`): the contact energy joins the elastic energy
  and its friction the external force; the pairs, and which closest-point candidate each
  takes, are found at every Newton iterate.
* Backward Euler (Eq. 14-15) solved by Newton's method; the Jacobian (Eq. 16)
  is the automatic Jacobian of the residual.  Velocity update after Eq. 16.
* Adaptive time stepping (named as an option in the same subsection): a step whose Newton
  solve fails is covered by two half steps, recursively.
* Implicit midpoint (named as the alternative implicit scheme in the time-stepping
  subsection, without formulas): the textbook rule for M qddot = F,
  q_{n+1} = q_n + dt (qdot_n + qdot_{n+1}) / 2 and M (qdot_{n+1} - qdot_n) = dt F(q_m)
  at q_m = (q_n + q_{n+1}) / 2, solved by Newton's method for q_{n+1}.
* Elastic joints (Elastic Joints subsection): nodes shared by several rods;
  bend and twist for every pair of edges meeting at the joint.
* Actuation through natural curvature (Actuation subsection).

Readings of points the paper leaves open are listed in the repository's design
notes and restated next to the code that takes them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

DT = torch.float64
TWO_PI = 2.0 * math.pi


# ---------------------------------------------------------------------------
# small vector helpers
# ---------------------------------------------------------------------------

def _dot(a, b):
    return (a * b).sum(-1)


def _cross(a, b):
    return torch.linalg.cross(a, b, dim=-1)


def transport(a, b, v):
    """Parallel transport: rotate v by the rotation about a x b that takes the unit
    vector a onto the unit vector b (Rodrigues' formula written with w = a x b,
    c = a.b:  R = I + [w]x + [w]x^2 / (1 + c)).  Defined for a != -b."""
    w = _cross(a, b)
    c = _dot(a, b)
    return v + _cross(w, v) + _cross(w, _cross(w, v)) / (1.0 + c)[..., None]


def signed_angle(u, v, n):
    """Signed angle from u to v about the axis n."""
    return torch.atan2(_dot(_cross(u, v), n), _dot(u, v))


# ---------------------------------------------------------------------------
# system description
# ---------------------------------------------------------------------------

@dataclass
class System:
    n_nodes: int
    n_edges: int
    edge_nodes: torch.Tensor        # (n_edges, 2) global node ids (tail, head)
    ebar: torch.Tensor              # rest edge length
    EA: torch.Tensor                # stretch stiffness per edge
    Itheta: torch.Tensor            # twist inertia per edge
    st_nodes: torch.Tensor          # (n_st, 3) previous, centre, next node
    st_edges: torch.Tensor          # (n_st, 2) edge f (into the centre), edge e (out of it)
    st_sign: torch.Tensor           # (n_st, 2) +1 if the stored edge has the stencil's orientation
    Vbar: torch.Tensor              # rest Voronoi length per stencil
    EI: torch.Tensor
    GJ: torch.Tensor
    kappa_rest: torch.Tensor        # (n_st, 2) integrated natural curvature used when no input given
    tau_rest: torch.Tensor          # (n_st,)
    st_rod: torch.Tensor            # rod id of a rod-interior stencil, -1 for joint stencils
    st_index: torch.Tensor          # interior node index within its rod (1..N-2), -1 for joints
    st_act: torch.Tensor            # (n_st, 3) actuation A, f, phi (nan if none)
    mass: torch.Tensor              # lumped node mass
    radius_node: torch.Tensor       # contact radius per node
    fixed: torch.Tensor             # bool over DOFs
    force: torch.Tensor             # (n_nodes, 3) constant external force
    moment: torch.Tensor            # (n_edges,) constant external twisting moment on theta
    gravity: torch.Tensor
    floor: dict | None
    damping: float
    rod_nodes: list = field(default_factory=list)   # per rod: global node id of each rod node
    rod_edges: list = field(default_factory=list)   # per rod: global edge id of each rod edge
    kbar_user: list = field(default_factory=list)   # per rod: (N-2, 2) in 1/m or None
    self_contact: dict | None = None                # {"delta", "k_c", "mu", "nu"} or None
    contact_sets: list = field(default_factory=list)  # per rod: its edges (contact.EdgeSet)

    @property
    def n_dof(self):
        return 3 * self.n_nodes + self.n_edges


@dataclass
class State:
    x: torch.Tensor        # (n_nodes, 3)
    theta: torch.Tensor    # (n_edges,)
    v: torch.Tensor        # (n_nodes, 3)
    omega: torch.Tensor    # (n_edges,)
    t_ref: torch.Tensor    # (n_edges, 3) tangents at the start of the step
    d1_ref: torch.Tensor   # (n_edges, 3) reference directors at the start of the step
    beta_ref: torch.Tensor  # (n_st,) reference twist at the start of the step (branch only)
    time: float = 0.0

    def clone(self):
        return State(self.x.clone(), self.theta.clone(), self.v.clone(), self.omega.clone(),
                     self.t_ref.clone(), self.d1_ref.clone(), self.beta_ref.clone(), self.time)


def _t(a):
    return torch.as_tensor(np.asarray(a), dtype=DT)


def components(desc):
    """Groups of rod indices connected by joints (each group is stepped on its own)."""
    n = len(desc["rods"])
    parent = list(range(n))

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i
    for (ra, _, rb, _) in desc["joints"]:
        parent[find(ra)] = find(rb)
    groups = {}
    for i in range(n):
        groups.setdefault(find(i), []).append(i)
    return list(groups.values())


def initial_directors(t):
    """Reference directors of one rod at t = 0 (the paper initialises them arbitrarily).
    Reading: d1 of the first edge is z projected off its tangent (x if the tangent is
    within 1e-6 of z), and each following edge gets the previous director parallel
    transported in space, so the reference twist of the initial shape is zero."""
    z = torch.tensor([0.0, 0.0, 1.0], dtype=DT)
    if abs(float(t[0] @ z)) > 1.0 - 1e-6:
        z = torch.tensor([1.0, 0.0, 0.0], dtype=DT)
    d = z - (z @ t[0]) * t[0]
    d1 = [d / torch.linalg.norm(d)]
    for j in range(1, t.shape[0]):
        d1.append(transport(t[j - 1], t[j], d1[-1]))
    return torch.stack(d1)


def build(desc, rod_ids=None):
    """Build the System and initial State of the rods `rod_ids` (default: all rods;
    they must be closed under joints)."""
    rods = desc["rods"]
    rod_ids = list(range(len(rods))) if rod_ids is None else list(rod_ids)
    local = {r: k for k, r in enumerate(rod_ids)}
    # --- global node numbering, joints merge node_b of rod_b into node_a of rod_a
    key = {}
    for r in rod_ids:
        for i in range(rods[r]["x0"].shape[0]):
            key[(r, i)] = (r, i)

    def find(k):
        while key[k] != k:
            key[k] = key[key[k]]
            k = key[k]
        return k
    for (ra, na, rb, nb) in desc["joints"]:
        if ra in local and rb in local:
            key[find((rb, nb))] = find((ra, na))
    gid, rod_nodes, X = {}, [], []
    for r in rod_ids:
        ids = []
        for i in range(rods[r]["x0"].shape[0]):
            k = find((r, i))
            if k not in gid:
                gid[k] = len(X)
                X.append(rods[k[0]]["x0"][k[1]])
            ids.append(gid[k])
        rod_nodes.append(torch.tensor(ids))
    X = _t(np.array(X))
    n_nodes = X.shape[0]
    # --- edges and their rest data
    edge_nodes, ebar, EA, Ith, rod_edges, edge_rod = [], [], [], [], [], []
    mass = torch.zeros(n_nodes, dtype=DT)
    radius_node = torch.zeros(n_nodes, dtype=DT)
    for k, r in enumerate(rod_ids):
        rd = rods[r]
        h, rho = rd["radius"], rd["density"]
        A = math.pi * h * h
        ids = rod_nodes[k]
        eids = []
        for j in range(len(ids) - 1):
            a, b = int(ids[j]), int(ids[j + 1])
            L0 = float(torch.linalg.norm(X[b] - X[a]))
            eids.append(len(edge_nodes))
            edge_nodes.append((a, b))
            ebar.append(L0)
            EA.append(rd["E"] * A)
            # twist inertia of the edge: rho * J * ebar with J = pi h^4 / 2
            Ith.append(rho * (math.pi * h ** 4 / 2.0) * L0)
            edge_rod.append(k)
            # lumped mass: each node gets half of every incident edge's mass
            mass[a] += 0.5 * rho * A * L0
            mass[b] += 0.5 * rho * A * L0
            radius_node[a] = max(float(radius_node[a]), h)
            radius_node[b] = max(float(radius_node[b]), h)
        rod_edges.append(torch.tensor(eids, dtype=torch.long))
    edge_nodes = torch.tensor(edge_nodes, dtype=torch.long).reshape(-1, 2)
    ebar = _t(ebar)
    n_edges = edge_nodes.shape[0]
    # --- stencils: interior nodes of each rod, then every pair of edges at joint nodes
    st_nodes, st_edges, st_sign, st_rod, st_idx, st_mat = [], [], [], [], [], []
    for k, r in enumerate(rod_ids):
        ids, eids = rod_nodes[k], rod_edges[k]
        for i in range(1, len(ids) - 1):
            st_nodes.append((int(ids[i - 1]), int(ids[i]), int(ids[i + 1])))
            st_edges.append((int(eids[i - 1]), int(eids[i])))
            st_sign.append((1.0, 1.0))
            st_rod.append(k)
            st_idx.append(i)
            st_mat.append((k, k))
    rod_pairs = {(a, b) for (a, b) in st_edges}
    incident = [[] for _ in range(n_nodes)]
    for j in range(n_edges):
        incident[int(edge_nodes[j, 0])].append((j, +1))   # edge leaves the node
        incident[int(edge_nodes[j, 1])].append((j, -1))   # edge enters the node
    for nd in range(n_nodes):
        inc = sorted(incident[nd])
        for p in range(len(inc)):
            for q in range(p + 1, len(inc)):
                ja, da = inc[p]
                jb, db = inc[q]
                # orientation: edge f points into the joint node, edge e out of it
                if da == -1 and db == +1:
                    f, sf, e, se = ja, 1.0, jb, 1.0
                elif db == -1 and da == +1:
                    f, sf, e, se = jb, 1.0, ja, 1.0
                elif da == +1 and db == +1:
                    f, sf, e, se = ja, -1.0, jb, 1.0
                else:
                    f, sf, e, se = ja, 1.0, jb, -1.0
                if sf == 1.0 and se == 1.0 and (f, e) in rod_pairs:
                    continue   # an interior stencil of a rod, already listed
                n_prev = int(edge_nodes[f, 0]) if sf > 0 else int(edge_nodes[f, 1])
                n_next = int(edge_nodes[e, 1]) if se > 0 else int(edge_nodes[e, 0])
                st_nodes.append((n_prev, nd, n_next))
                st_edges.append((f, e))
                st_sign.append((sf, se))
                st_rod.append(-1)
                st_idx.append(-1)
                st_mat.append((edge_rod[f], edge_rod[e]))
    st_nodes = torch.tensor(st_nodes, dtype=torch.long).reshape(-1, 3)
    st_edges = torch.tensor(st_edges, dtype=torch.long).reshape(-1, 2)
    st_sign = _t(st_sign).reshape(-1, 2)
    n_st = st_nodes.shape[0]
    Vbar = 0.5 * (ebar[st_edges[:, 0]] + ebar[st_edges[:, 1]])
    EI, GJ, act = [], [], []
    for s in range(n_st):
        ka, kb = st_mat[s]
        vals = []
        for k in (ka, kb):
            rd = rods[rod_ids[k]]
            h = rd["radius"]
            G = rd["E"] / (2.0 * (1.0 + rd["poisson"]))
            vals.append((rd["E"] * math.pi * h ** 4 / 4.0, G * math.pi * h ** 4 / 2.0))
        # joint stencils joining two rods use the mean of the two rods' stiffnesses
        EI.append(0.5 * (vals[0][0] + vals[1][0]))
        GJ.append(0.5 * (vals[0][1] + vals[1][1]))
        a_ = rods[rod_ids[ka]].get("actuation") if st_rod[s] >= 0 else None
        act.append(a_ if a_ is not None else (float("nan"),) * 3)
    # --- clamps
    fixed = torch.zeros(3 * n_nodes + n_edges, dtype=torch.bool)
    for k, r in enumerate(rod_ids):
        for i in rods[r]["fixed_nodes"]:
            g = int(rod_nodes[k][i])
            fixed[3 * g:3 * g + 3] = True
        for j in rods[r]["fixed_edges"]:
            fixed[3 * n_nodes + int(rod_edges[k][j])] = True
    force = torch.zeros(n_nodes, 3, dtype=DT)
    for k, r in enumerate(rod_ids):
        if rods[r].get("force") is not None:
            force[rod_nodes[k]] += _t(rods[r]["force"])
    moment = torch.zeros(n_edges, dtype=DT)
    for k, r in enumerate(rod_ids):
        if rods[r].get("moment") is not None:
            moment[rod_edges[k]] += _t(rods[r]["moment"])
    sys = System(n_nodes, n_edges, edge_nodes, ebar, _t(EA), _t(Ith), st_nodes, st_edges, st_sign,
                 Vbar, _t(EI), _t(GJ), torch.zeros(n_st, 2, dtype=DT), torch.zeros(n_st, dtype=DT),
                 torch.tensor(st_rod), torch.tensor(st_idx), _t(act).reshape(-1, 3), mass, radius_node,
                 fixed, force, moment, _t(desc["gravity"]), desc.get("floor"), float(desc.get("damping", 0.0)),
                 rod_nodes, rod_edges, [rods[r].get("kbar") for r in rod_ids])
    if desc.get("self_contact"):
        from . import contact as _contact
        if any(ra in local or rb in local for (ra, na, rb, nb) in desc["joints"]):
            raise NotImplementedError("self-contact of joined rods")
        sys.self_contact = dict(desc["self_contact"])
        for k, r in enumerate(rod_ids):
            eids = rod_edges[k]
            sys.contact_sets.append(_contact.EdgeSet(edge_nodes[eids].tolist(), [0] * len(eids),
                                                     list(range(len(eids))), [rods[r]["radius"]] * len(eids),
                                                     ebar[eids].tolist()))
    # --- initial frames, rest curvature and twist of the initial shape
    e = X[edge_nodes[:, 1]] - X[edge_nodes[:, 0]]
    t = e / torch.linalg.norm(e, dim=1, keepdim=True)
    d1 = torch.zeros_like(t)
    for k in range(len(rod_ids)):
        d1[rod_edges[k]] = initial_directors(t[rod_edges[k]])
    theta = torch.zeros(n_edges, dtype=DT)
    beta0 = torch.zeros(n_st, dtype=DT)
    st0 = State(X.clone(), theta, torch.zeros_like(X), torch.zeros_like(theta), t, d1, beta0, 0.0)
    kap, tau, beta = strains(sys, X, theta, st0, raw_beta=True)
    st0.beta_ref = beta.detach().clone()
    sys.kappa_rest = kap.detach().clone()
    # rod-interior stencils start twist-free (space-parallel directors); joint stencils keep
    # the twist of the initial shape as their rest twist, so a joint is stress free at rest
    sys.tau_rest = torch.where(sys.st_rod >= 0, torch.zeros_like(tau), tau.detach())
    if "initial_tip_velocity" in desc:
        for k in range(len(rod_ids)):
            st0.v[rod_nodes[k][-1]] = _t(desc["initial_tip_velocity"])
    return sys, st0


# ---------------------------------------------------------------------------
# kinematics and energies
# ---------------------------------------------------------------------------

def frames(sys, x, theta, st):
    """Tangent, length, reference and material frames of every edge at positions x,
    the reference director being transported in time from the step-start frame."""
    e = x[sys.edge_nodes[:, 1]] - x[sys.edge_nodes[:, 0]]
    ell = torch.linalg.norm(e, dim=1)
    t = e / ell[:, None]
    d1 = transport(st.t_ref, t, st.d1_ref)
    d2 = _cross(t, d1)
    c, s = torch.cos(theta)[:, None], torch.sin(theta)[:, None]
    m1 = c * d1 + s * d2
    m2 = -s * d1 + c * d2
    return t, ell, d1, d2, m1, m2


def strains(sys, x, theta, st, raw_beta=False):
    """Integrated curvature kappa (Eq. 4-5) and twist tau (Eq. 7) of every stencil.
    A stencil whose stored edge runs against its orientation sees that edge reversed:
    tangent and theta change sign, d1 is kept (so d2 and m2 change sign, m1 is kept)."""
    t, ell, d1, d2, m1, m2 = frames(sys, x, theta, st)
    f, e = sys.st_edges[:, 0], sys.st_edges[:, 1]
    sf, se = sys.st_sign[:, 0:1], sys.st_sign[:, 1:2]
    tf, te = sf * t[f], se * t[e]
    kb = 2.0 * _cross(tf, te) / (1.0 + _dot(tf, te))[:, None]                  # Eq. 4
    m1f, m2f = m1[f], sf * m2[f]
    m1e, m2e = m1[e], se * m2[e]
    kappa1 = 0.5 * _dot(kb, m2f + m2e)                                          # Eq. 5
    kappa2 = -0.5 * _dot(kb, m1f + m1e)
    # reference twist: signed angle about t^e from the f director carried onto t^e by
    # space-parallel transport to the e director; branch nearest the step-start value
    u = transport(tf, te, d1[f])
    raw = signed_angle(u, d1[e], te)
    if raw_beta:
        beta = raw
    else:
        beta = raw + TWO_PI * torch.round((st.beta_ref - raw) / TWO_PI)
    tau = se[:, 0] * theta[e] - sf[:, 0] * theta[f] + beta                      # Eq. 7
    return torch.stack([kappa1, kappa2], dim=1), tau, beta


def natural_curvature(sys, time, kbar_rods=None):
    """Integrated natural curvature per stencil at the given time.  A rod's input natural
    curvature (1/m) is multiplied by the rest Voronoi length; actuated rods use
    A sin(2 pi f t + phi) in the first component; otherwise the initial shape's curvature."""
    kap = sys.kappa_rest.clone()
    users = kbar_rods if kbar_rods is not None else sys.kbar_user
    rows, vals = [], []
    for k, kb in enumerate(users):
        if kb is None:
            continue
        sel = torch.nonzero(sys.st_rod == k).flatten()
        idx = sys.st_index[sel] - 1
        kbt = kb if torch.is_tensor(kb) else _t(kb)
        rows.append(sel)
        vals.append(kbt[idx] * sys.Vbar[sel][:, None])
    if rows:
        rows = torch.cat(rows)
        kap = kap.index_put((rows,), torch.cat(vals))
    act = torch.isfinite(sys.st_act[:, 0])
    if bool(act.any()):
        A, f, ph = sys.st_act[:, 0], sys.st_act[:, 1], sys.st_act[:, 2]
        k1 = A * torch.sin(TWO_PI * f * time + ph) * sys.Vbar
        kap = torch.stack([torch.where(act, k1, kap[:, 0]), torch.where(act, torch.zeros_like(k1), kap[:, 1])], 1)
    return kap


def elastic_energy(sys, x, theta, st, kappa_bar, tau_bar=None):
    """E_s + E_b + E_t (Eq. 3, 6, 8) with rest Voronoi lengths."""
    e = x[sys.edge_nodes[:, 1]] - x[sys.edge_nodes[:, 0]]
    eps = torch.linalg.norm(e, dim=1) / sys.ebar - 1.0                          # Eq. 2
    Es = 0.5 * (sys.EA * eps * eps * sys.ebar).sum()                            # Eq. 3
    kap, tau, _ = strains(sys, x, theta, st)
    dk = kap - kappa_bar
    Eb = 0.5 * (sys.EI * (dk * dk).sum(1) / sys.Vbar).sum()                     # Eq. 6
    tb = sys.tau_rest if tau_bar is None else tau_bar
    Et = 0.5 * (sys.GJ * (tau - tb) ** 2 / sys.Vbar).sum()                      # Eq. 8
    return Es + Eb + Et


def contact_energy_profile(D, C, delta):
    """IMC energy of Eq. 10 (without stiffness), K1 = 15/delta.  The quadratic branch is
    extended below D = 0 (a node under the floor)."""
    K1 = 15.0 / delta
    z = torch.clamp(K1 * (C - D), max=60.0)          # the clamp only touches the quadratic region
    soft = (torch.log1p(torch.exp(z)) / K1) ** 2
    quad = (C - D) ** 2
    return torch.where(D <= C - delta, quad, torch.where(D < C + delta, soft, torch.zeros_like(D)))


def friction_ratio(s, K2):
    """gamma(|u|)/|u| with gamma = 2/(1 + exp(-K2 |u|)) - 1 (Eq. 12), as a function of
    s = |u|^2.  At tiny speeds the exact limit series K2/2 (1 - K2^2 s / 12) is used so
    that the ratio and its derivatives stay finite at u = 0."""
    small = s < 1e-8 / (K2 * K2)
    r = torch.sqrt(torch.where(small, torch.ones_like(s), s))
    gam = 2.0 / (1.0 + torch.exp(-K2 * r)) - 1.0
    return torch.where(small, 0.5 * K2 * (1.0 - K2 * K2 * s / 12.0), gam / r)


def external_force(sys, x, st, dt):
    """F_ext = F_con + F_fr + F_misc on the node positions (Eq. 10-13 and the text after)."""
    F = sys.mass[:, None] * sys.gravity[None, :] + sys.force
    if sys.damping > 0.0:
        F = F - sys.damping * sys.mass[:, None] * (x - st.x) / dt
    fl = sys.floor
    if fl is not None:
        D = x[:, 2] - fl["z"]
        C = sys.radius_node
        # contact force = -k_c dE_c/dD dD/dq (Eq. 11); dD/dq = z-hat
        dEdD = torch.func.grad(lambda d: contact_energy_profile(d, C, fl["delta"]).sum())(D)
        Fn = -fl["k_c"] * dEdD
        F = F + torch.stack([torch.zeros_like(Fn), torch.zeros_like(Fn), Fn], 1)
        # friction (Eq. 12-13): u = tangential (horizontal) velocity of the node over the step
        u = (x[:, :2] - st.x[:, :2]) / dt
        K2 = 15.0 / fl["nu"]
        ratio = friction_ratio((u * u).sum(1), K2)
        Ffr = -fl["mu"] * torch.abs(Fn)[:, None] * ratio[:, None] * u
        F = F + torch.cat([Ffr, torch.zeros_like(Fn)[:, None]], 1)
    return F


def unpack(sys, q):
    return q[:3 * sys.n_nodes].reshape(sys.n_nodes, 3), q[3 * sys.n_nodes:]


def pack(x, theta):
    return torch.cat([x.reshape(-1), theta])


def contact_list(sys, q):
    """The self-contact pairs at q and the closest-point candidate each takes there:
    [(a, b, c, d, C, branch)] with global node ids of edge (a, b) and edge (c, d)."""
    if not sys.self_contact:
        return None
    from . import contact as _contact
    x, _ = unpack(sys, q.detach())
    out = []
    for es in sys.contact_sets:
        for (i, j, D, s_, t_) in _contact.contact_pairs(es, x, sys.self_contact["delta"]):
            a, b = es.edges[i].tolist()
            c, d = es.edges[j].tolist()
            br = _contact.branch_of(torch.cat([x[a], x[b], x[c], x[d]]))
            out.append((a, b, c, d, es.contact_distance(i, j), br))
    return out


def self_contact_energy(sys, x, pairs):
    """Sum over the pairs of k_c E_c(D) (Eq. 10), D by each pair's fixed candidate."""
    from . import contact as _contact
    sc = sys.self_contact
    tot = torch.zeros((), dtype=DT)
    for (a, b, c, d, C, br) in pairs:
        D, _, _ = _contact.closest_on_branch(torch.cat([x[a], x[b], x[c], x[d]]), br)
        tot = tot + sc["k_c"] * contact_energy_profile(D, C, sc["delta"])
    return tot


def self_contact_friction(sys, x, st, dt, pairs):
    """Friction (Eq. 12-13) of every pair: u the tangential relative velocity of the closest
    points over the step at the closest-point parameters of x, |F_con| = k_c |dE_c/dD|; edge
    (a, b) gets -mu gamma u_hat |F_con| spread by (1 - s, s), edge (c, d) the opposite."""
    from . import contact as _contact
    sc = sys.self_contact
    K2 = 15.0 / sc["nu"]
    F = torch.zeros_like(x)
    for (a, b, c, d, C, br) in pairs:
        D, s, t = _contact.closest_on_branch(torch.cat([x[a], x[b], x[c], x[d]]), br)
        P, Q = x[a] + s * (x[b] - x[a]), x[c] + t * (x[d] - x[c])
        Pn, Qn = st.x[a] + s * (st.x[b] - st.x[a]), st.x[c] + t * (st.x[d] - st.x[c])
        n = (P - Q) / D
        vrel = (P - Pn - Q + Qn) / dt
        u = vrel - torch.dot(vrel, n) * n
        dEdD = torch.func.grad(lambda dd: contact_energy_profile(dd, C, sc["delta"]))(D)
        ratio = friction_ratio(torch.dot(u, u), K2)          # gamma / |u|, smooth at u = 0
        f = -sc["mu"] * sc["k_c"] * torch.abs(dEdD) * ratio * u
        F = F.index_add(0, torch.tensor([a, b, c, d]), torch.stack([(1 - s) * f, s * f, -(1 - t) * f, -t * f]))
    return F


def residual(sys, q, st, dt, kappa_bar, contact=None):
    """Backward-Euler residual (Eq. 15):  M/dt^2 (q - q_n - dt qdot_n) + dE/dq - F_ext, with
    the self-contact pairs `contact` (contact_list) in the energy and the external force."""
    def energy(qq):
        xx, tt = unpack(sys, qq)
        e = elastic_energy(sys, xx, tt, st, kappa_bar)
        if contact:
            e = e + self_contact_energy(sys, xx, contact)
        return e
    gE = torch.func.grad(energy)(q)
    x, theta = unpack(sys, q)
    Mx = sys.mass[:, None] * (x - st.x - dt * st.v) / (dt * dt)
    Mt = sys.Itheta * (theta - st.theta - dt * st.omega) / (dt * dt)
    F = external_force(sys, x, st, dt)
    if contact and sys.self_contact.get("mu", 0.0) > 0.0:
        F = F + self_contact_friction(sys, x, st, dt, contact)
    return pack(Mx - F, Mt - sys.moment) + gE


def residual_midpoint(sys, q, st, dt, kappa_bar):
    """Implicit-midpoint residual in the unknown q = q_{n+1}: eliminating qdot_{n+1} =
    2 (q_{n+1} - q_n) / dt - qdot_n from M (qdot_{n+1} - qdot_n) = dt F(q_m) gives
        2 M / dt^2 (q_{n+1} - q_n - dt qdot_n) + dE/dq (q_m) - F_ext(q_m) = 0,
    q_m = (q_n + q_{n+1}) / 2.  The elastic energy at q_m uses frames carried by time-parallel
    transport from the step-start frames to q_m; damping and friction see the midpoint
    velocity (q_{n+1} - q_n) / dt = (x_m - x_n) / (dt / 2)."""
    qn = pack(st.x, st.theta)
    qm = 0.5 * (qn + q)

    def energy(qq):
        xx, tt = unpack(sys, qq)
        return elastic_energy(sys, xx, tt, st, kappa_bar)
    gE = torch.func.grad(energy)(qm)
    x1, th1 = unpack(sys, q)
    xm, _ = unpack(sys, qm)
    Mx = 2.0 * sys.mass[:, None] * (x1 - st.x - dt * st.v) / (dt * dt)
    Mt = 2.0 * sys.Itheta * (th1 - st.theta - dt * st.omega) / (dt * dt)
    F = external_force(sys, xm, st, 0.5 * dt)
    return pack(Mx - F, Mt - sys.moment) + gE


@dataclass
class StepInfo:
    iters: int
    residual: float
    converged: bool
    history: list
    at_floor: bool = False       # ended by the rounding-floor rule, not the tolerance
    floor: float = 0.0           # rounding-floor estimate of the last iterate


EPS = 2.0 ** -52


def floor_scales(sys, st):
    """Magnitude of each DOF kind at the step start: the largest |coordinate| of the node
    positions for position DOFs, the largest |theta| plus pi for twist DOFs (the reference
    twist in (-pi, pi] enters every twist strain)."""
    s = torch.empty(sys.n_dof, dtype=DT)
    s[:3 * sys.n_nodes] = float(st.x.abs().max())
    s[3 * sys.n_nodes:] = (float(st.theta.abs().max()) if sys.n_edges else 0.0) + math.pi
    return s


def rounding_floor(J_ff, s_f, factor):
    """Estimate of the FP64 rounding floor of the residual norm: a free DOF cannot be placed
    closer than eps |q_k| to the root, so row i of the residual cannot be resolved below
    eps sum_k |J_ik| |q_k|; with |q_k| bounded by its kind's step-start magnitude the floor is
    factor * eps * || |J| s ||_2 over free rows and columns."""
    return factor * EPS * float(torch.linalg.norm(J_ff.abs() @ s_f))


def newton_solve(sys, st, dt, kappa_bar, tol=1e-9, max_iter=50, q0=None, polish=0, line_search=False,
                 floor_factor=1.0, res=residual, floor_jac_scale=1.0):
    """Newton's method on the residual.  Initial guess q_n unless q0 is given.
    Stops when the 2-norm of the residual over free DOFs is <= tol, or, after at least one
    Newton step, when the residual is at or below its computed rounding floor
    (`rounding_floor`, floor_factor 0 turns the rule off) and the last step failed to halve
    it: the FP64 floor of a stiff rod can lie above tol.  `polish` extra iterations may follow
    the tolerance (used to reach the rounding floor in tests); the last one is returned.
    With line_search (the paper's optional globalisation), the Newton step is halved (at most
    10 times) until the residual norm decreases, unless the trial's residual lies within its
    own rounding floor (a rise there is rounding noise) and is kept.  `res` is the scheme's
    residual; floor_jac_scale multiplies the Jacobian in the floor estimate (2 when the
    unknown is the step end but the rounding acts on the midpoint state)."""
    free = ~sys.fixed
    q = pack(st.x, st.theta).clone() if q0 is None else q0.clone()
    if sys.self_contact and res is not residual:
        raise NotImplementedError("self-contact under the implicit-midpoint rule")
    # with self-contact the pairs (and their closest-point candidates) are those of the
    # iterate being evaluated; the Jacobian at q takes q's pairs
    res_plain = res

    def res(sys_, qq, st_, dt_, kb_):
        if not sys_.self_contact:
            return res_plain(sys_, qq, st_, dt_, kb_)
        return res_plain(sys_, qq, st_, dt_, kb_, contact_list(sys_, qq))

    def jac(qq):
        cl = contact_list(sys, qq)
        if cl is None:
            return torch.func.jacfwd(lambda z: res_plain(sys, z, st, dt, kappa_bar))(qq)
        return torch.func.jacfwd(lambda z: res_plain(sys, z, st, dt, kappa_bar, cl))(qq)
    sc = floor_scales(sys, st)[free]
    hist = []
    it = 0
    extra = 0
    R = res(sys, q, st, dt, kappa_bar)
    J = jac(q)
    while True:
        r = float(torch.linalg.norm(R[free]))
        Jff = J[free][:, free]
        fl = rounding_floor(floor_jac_scale * Jff, sc, floor_factor)
        hist.append(r)
        if r <= tol or extra > 0:
            # converged; polishing iterations (at the rounding floor, where the residual is
            # noise and may sit a hair above tol) end after their count whatever it reads
            if extra >= polish:
                return q, StepInfo(it, r, True, hist, False, fl)
            extra += 1
        elif it > 0 and r <= fl and r > 0.5 * hist[-2]:
            return q, StepInfo(it, r, True, hist, True, fl)
        if it >= max_iter + polish:
            return q, StepInfo(it, r, False, hist, False, fl)
        dq = torch.linalg.solve(Jff, R[free])
        alpha = 1.0
        Jn = None
        for _ in range(11 if line_search else 1):
            qn = q.clone()
            qn[free] = q[free] - alpha * dq
            Rn = res(sys, qn, st, dt, kappa_bar)
            Jn = None
            if not line_search or float(torch.linalg.norm(Rn[free])) < r:
                break
            Jn = jac(qn)
            if float(torch.linalg.norm(Rn[free])) <= rounding_floor(floor_jac_scale * Jn[free][:, free], sc,
                                                                     floor_factor):
                break           # a rise within the trial's own rounding floor is noise, not a bad step
            alpha *= 0.5
        q, R = qn, Rn
        J = Jn if Jn is not None else jac(q)
        it += 1


def commit(sys, st, q, dt):
    """Velocity update (after Eq. 16) and the step-end frames for the next step."""
    x, theta = unpack(sys, q)
    t, ell, d1, d2, m1, m2 = frames(sys, x, theta, st)
    _, _, beta = strains(sys, x, theta, st)
    return State(x.clone(), theta.clone(), (x - st.x) / dt, (theta - st.theta) / dt,
                 t.clone(), d1.clone(), beta.clone(), st.time + dt)


def commit_midpoint(sys, st, q, dt):
    """Implicit-midpoint velocity update qdot_{n+1} = 2 (q_{n+1} - q_n) / dt - qdot_n and the
    step-end frames for the next step."""
    x, theta = unpack(sys, q)
    t, ell, d1, d2, m1, m2 = frames(sys, x, theta, st)
    _, _, beta = strains(sys, x, theta, st)
    return State(x.clone(), theta.clone(), 2.0 * (x - st.x) / dt - st.v, 2.0 * (theta - st.theta) / dt - st.omega,
                 t.clone(), d1.clone(), beta.clone(), st.time + dt)


def step(sys, st, dt, tol=1e-9, max_iter=50, kbar_rods=None, polish=0, q0=None, line_search=False,
         scheme="euler"):
    """One time step: backward Euler ("euler", natural curvature at the end-of-step time) or
    implicit midpoint ("midpoint", natural curvature at the midpoint time t + dt / 2)."""
    if scheme == "midpoint":
        kap = natural_curvature(sys, st.time + 0.5 * dt, kbar_rods)
        q, info = newton_solve(sys, st, dt, kap, tol, max_iter, q0=q0, polish=polish, line_search=line_search,
                               res=residual_midpoint, floor_jac_scale=2.0)
        return (commit_midpoint(sys, st, q, dt) if info.converged else st), info
    kap = natural_curvature(sys, st.time + dt, kbar_rods)
    q, info = newton_solve(sys, st, dt, kap, tol, max_iter, q0=q0, polish=polish, line_search=line_search)
    if not info.converged:
        return st, info
    return commit(sys, st, q, dt), info


def step_adaptive(sys, st, dt, tol=1e-9, max_iter=50, max_halvings=0, polish=0, line_search=False,
                  scheme="euler"):
    """One time step with adaptive step halving (the paper offers adaptive time stepping as an
    option without stating a rule; this is the plain recursive one): try the step; if Newton
    does not converge, cover the same interval by two steps of half the size, each of them
    adaptive in the same way, down to dt / 2^max_halvings.  Returns the new state, whether it
    succeeded, the Newton iterations spent (failed attempts included) and the halvings made."""
    tot = {"iters": 0, "halvings": 0}

    def advance(s, h, level):
        s1, info = step(sys, s, h, tol, max_iter, polish=polish, line_search=line_search, scheme=scheme)
        tot["iters"] += info.iters
        if info.converged:
            return s1, True
        if level == max_halvings:
            return s, False
        tot["halvings"] += 1
        sm, ok = advance(s, 0.5 * h, level + 1)
        if not ok:
            return s, False
        return advance(sm, 0.5 * h, level + 1)
    out, ok = advance(st, dt, 0)
    return out, ok, tot["iters"], tot["halvings"]


def simulate(desc, steps=None, rod_ids=None, tol=None, polish=0, record=False, line_search=None, scheme="euler"):
    """Step the rods `rod_ids` (closed under joints) for `steps` steps."""
    sys, st = build(desc, rod_ids)
    n = desc["steps"] if steps is None else steps
    tol = desc["tol"] if tol is None else tol
    ls = desc.get("line_search", False) if line_search is None else line_search
    traj, infos = [], []
    for _ in range(n):
        st, info = step(sys, st, desc["dt"], tol, desc["max_iter"], polish=polish, line_search=ls, scheme=scheme)
        infos.append(info)
        if not info.converged:
            break
        if record:
            traj.append(st.clone())
    return sys, st, infos, traj


def rod_positions(sys, st, k):
    """Positions of rod k's nodes in rod order."""
    return st.x[sys.rod_nodes[k]]


def rod_thetas(sys, st, k):
    return st.theta[sys.rod_edges[k]]
