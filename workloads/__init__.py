"""Seeded synthetic rod workloads.

This module is shared by the CPU oracle tests and the HIP path.  It only
describes *inputs*: node positions, materials, clamps, natural-curvature
inputs in 1/m, contact and actuation parameters.  It holds none of the
method's arithmetic (no frames, strains, masses, energies or solves); each
side turns a description into its own data structures.

A description is a plain dict:

    {"rods":   [ {"x0": (N,3) float64, "radius", "E", "poisson", "density",
                  "kbar": (N-2, 2) curvature in 1/m or None (rest = initial shape),
                  "fixed_nodes": [...], "fixed_edges": [...],
                  "actuation": None or (A [1/m], f [Hz], phi [rad]),
                  "force": None or (N,3) constant external nodal force [N],
                  "moment": None or (N-1,) constant external twisting moment per edge [N m]} ],
     "joints": [(rod_a, node_a, rod_b, node_b), ...],   # node_b merged into node_a
     "gravity": (gx, gy, gz), "dt", "steps", "tol", "max_iter",
     "floor": None or {"z", "delta", "nu", "mu", "k_c"},
     "damping": eta [1/s], "line_search": bool (optional, default False)}

All randomness is NumPy PCG64 with the seeds stated per workload.
"""
from __future__ import annotations

import math

import numpy as np

G_EARTH = (0.0, 0.0, -9.81)


def straight_nodes(n: int, length: float, origin=(0.0, 0.0, 0.0), direction=(1.0, 0.0, 0.0)) -> np.ndarray:
    """n equally spaced nodes on a straight segment of the given length."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    s = np.linspace(0.0, length, n)
    return np.asarray(origin, dtype=np.float64)[None, :] + s[:, None] * d[None, :]


def helix_nodes(n: int, radius: float, pitch: float, contour: float) -> np.ndarray:
    """n nodes equally spaced in arc length along a helix hanging down from the origin."""
    per_turn = math.hypot(2.0 * math.pi * radius, pitch)
    turns = contour / per_turn
    phi = np.linspace(0.0, 2.0 * math.pi * turns, n)
    return np.stack([radius * np.cos(phi) - radius, radius * np.sin(phi),
                     -pitch * phi / (2.0 * math.pi)], axis=1)


def _rod(x0, radius, E, poisson=0.5, density=1000.0, kbar=None, fixed_nodes=(0, 1),
         fixed_edges=(0,), actuation=None, force=None, moment=None):
    return {"x0": np.ascontiguousarray(x0, dtype=np.float64), "radius": float(radius), "E": float(E),
            "poisson": float(poisson), "density": float(density),
            "kbar": None if kbar is None else np.ascontiguousarray(kbar, dtype=np.float64),
            "fixed_nodes": list(fixed_nodes), "fixed_edges": list(fixed_edges),
            "actuation": actuation, "force": force, "moment": moment}


def rod(x0, radius, E, poisson=0.5, density=1000.0, **kw):
    """One rod entry (clamped at nodes 0, 1 and edge 0 unless told otherwise)."""
    return _rod(x0, radius, E, poisson, density, **kw)


def desc(rods, dt, steps, **kw):
    """A description from rod entries (see module docstring for the keys)."""
    return _desc(rods, dt, steps, **kw)


def _desc(rods, dt, steps, gravity=G_EARTH, joints=(), floor=None, damping=0.0, tol=1e-9, max_iter=50):
    return {"rods": list(rods), "joints": list(joints), "gravity": tuple(float(g) for g in gravity),
            "dt": float(dt), "steps": int(steps), "tol": float(tol), "max_iter": int(max_iter),
            "floor": floor, "damping": float(damping)}


# ---------------------------------------------------------------------------
# The five benchmark workloads
# ---------------------------------------------------------------------------

def cantilever(n_nodes: int = 51, steps: int = 100) -> dict:
    """Single clamped cantilever: 51 nodes, L = 1 m, h = 1 mm, E = 1e7 Pa, nu = 0.5,
    rho = 1000, first two nodes and the first twist clamped, gravity -9.81 z, dt = 1e-2 s."""
    rod = _rod(straight_nodes(n_nodes, 1.0), 1e-3, 1e7, 0.5, 1000.0)
    return _desc([rod], dt=1e-2, steps=steps)


def rod_batch(n_rods: int = 1024, seed: int = 0, nmin: int = 20, nmax: int = 400, steps: int = 1000,
              kbar_sigma: float = 2.0) -> dict:
    """Independent clamped rods of uneven size.  N ~ U{nmin..nmax}, L ~ U(0.5, 2) m,
    h ~ U(1e-3, 5e-3) m, E = 10**U(6, 8) Pa, nu = 0.5, rho = 1000, natural curvature
    per interior node and component ~ N(0, kbar_sigma**2) 1/m, dt = 1e-3 s (seeded PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rods = []
    for _ in range(n_rods):
        n = int(rng.integers(nmin, nmax + 1))
        length = float(rng.uniform(0.5, 2.0))
        h = float(rng.uniform(1e-3, 5e-3))
        E = float(10.0 ** rng.uniform(6.0, 8.0))
        kbar = rng.normal(0.0, kbar_sigma, size=(n - 2, 2))
        rods.append(_rod(straight_nodes(n, length), h, E, 0.5, 1000.0, kbar=kbar))
    return _desc(rods, dt=1e-3, steps=steps)


def star_robots(n_instances: int = 4096, seed: int = 1, limbs: int = 6, limb_nodes: int = 30,
                limb_length: float = 0.2, steps: int = 2000) -> dict:
    """Six-limb soft robots on a floor.  Each instance: a hub at (0, 0, h) and `limbs` rods of
    limb_nodes+1 nodes (node 0 at the hub, joined there) radiating at equal angles in the plane
    z = h; h = 5 mm, rho = 1240, E = 1.793 MPa, nu = 0.5.  Limb natural curvature
    kappa1(t) = A sin(2 pi f t + phi), A ~ U(0, 10) 1/m, f ~ U(0.5, 2) Hz, phi ~ U(0, 2 pi) per
    limb; kappa2 = 0.  Floor z = 0 with delta = 5e-4 m, nu = 1e-3 m/s, mu = 0.5; the contact
    stiffness is chosen so that a limb node's weight compresses the contact by about delta/2.
    Instances are offset along x so that they never interact.  dt = 1e-3 s."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h, rho, E = 5e-3, 1240.0, 1.793e6
    node_weight = rho * math.pi * h * h * (limb_length / limb_nodes) * 9.81
    delta = 5e-4
    rods, joints = [], []
    for k in range(n_instances):
        origin = np.array([1.0 * k, 0.0, h])
        base = len(rods)
        for a in range(limbs):
            ang = 2.0 * math.pi * a / limbs
            x0 = straight_nodes(limb_nodes + 1, limb_length, origin, (math.cos(ang), math.sin(ang), 0.0))
            act = (float(rng.uniform(0.0, 10.0)), float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.0, 2 * math.pi)))
            rods.append(_rod(x0, h, E, 0.5, rho, kbar=None, fixed_nodes=(), fixed_edges=(), actuation=act))
            if a > 0:
                joints.append((base, 0, base + a, 0))
    floor = {"z": 0.0, "delta": delta, "nu": 1e-3, "mu": 0.5, "k_c": node_weight / delta}
    d = _desc(rods, dt=1e-3, steps=steps, joints=joints, floor=floor)
    d["line_search"] = True
    return d


def warm_start_eval(n_rods: int = 1024, seed: int = 3, steps: int = 1000) -> dict:
    """Fresh rods for the learned warm start: as rod_batch but N ~ U{50..400}, seed 3."""
    return rod_batch(n_rods, seed=seed, nmin=50, nmax=400, steps=steps)


def adjoint_rods(n_rods: int = 256, n_nodes: int = 100, seed: int = 2, steps: int = 200) -> dict:
    """256 clamped rods of 100 nodes, L = 1 m, h = 1 mm, E = 1e7, rho = 1000, dt = 1e-3 s.
    Returns the description (natural curvature zero) and the seeded target natural curvature
    kbar* ~ N(0, 2**2) 1/m of shape (n_rods, n_nodes - 2, 2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rods = [_rod(straight_nodes(n_nodes, 1.0), 1e-3, 1e7, 0.5, 1000.0, kbar=np.zeros((n_nodes - 2, 2)))
            for _ in range(n_rods)]
    target = rng.normal(0.0, 2.0, size=(n_rods, n_nodes - 2, 2))
    return _desc(rods, dt=1e-3, steps=steps), target


def two_limb_manipulator(n_robots: int = 1, limb_nodes: int = 12, limb_length: float = 0.076,
                         radius: float = 0.1, spacing: float = 1.0) -> dict:
    """The real2sim dual soft limb manipulator (Real2Sim section): per robot two limbs of
    silicone (rho = 1240, E = 1.793 MPa, Poisson 0.5, the printed rod radius of 10 cm by
    default), each `limb_nodes` nodes over `limb_length` (76 mm, the limbs' length), joined
    end to start by an elastic joint and hanging from a base clamped at its first two nodes
    and first twist, along -z under gravity -9.8 z.  Rods 2r and 2r + 1 are robot r's limbs;
    robots are offset along x.  The limbs' natural curvature is set by the caller.  dt = 1e4 s,
    one step with line search: a quasi-static configuration is one implicit step so long that
    inertia is negligible."""
    rods, joints = [], []
    for k in range(n_robots):
        o = np.array([spacing * k, 0.0, 0.0])
        a = _rod(straight_nodes(limb_nodes, limb_length, o, (0.0, 0.0, -1.0)), radius, 1.793e6, 0.5, 1240.0,
                 kbar=np.zeros((limb_nodes - 2, 2)))
        b = _rod(straight_nodes(limb_nodes, limb_length, o + np.array([0.0, 0.0, -limb_length]), (0.0, 0.0, -1.0)),
                 radius, 1.793e6, 0.5, 1240.0, kbar=np.zeros((limb_nodes - 2, 2)), fixed_nodes=(), fixed_edges=())
        rods += [a, b]
        joints.append((2 * k, limb_nodes - 1, 2 * k + 1, 0))
    d = _desc(rods, dt=1e4, steps=1, gravity=(0.0, 0.0, -9.8), joints=joints)
    d["line_search"] = True
    return d


def limb_curvature_targets(n_configs: int = 8, seed: int = 5, n_robots: int = 1, scale: float = 1.0) -> np.ndarray:
    """Natural curvatures (1/m, first material direction) of a sequence of quasi-static
    configurations of two-limb robots, (n_configs, n_robots, 2): a slow seeded drift per robot
    and limb, as a hardware actuation sweep would give.  The target curvatures of the fit are
    the curvatures the simulated robot shows at these natural curvatures."""
    rng = np.random.Generator(np.random.PCG64(seed))
    start = rng.uniform(-2.0, 2.0, size=(n_robots, 2))
    drift = rng.uniform(-1.0, 1.0, size=(n_robots, 2))
    s = np.arange(n_configs)[:, None, None]
    return scale * (start[None] + drift[None] * s + 0.3 * np.sin(0.9 * s + rng.uniform(0, 6.3, size=(n_robots, 2))[None]))


# ---------------------------------------------------------------------------
# Paper-shape workloads (validation section parameters)
# ---------------------------------------------------------------------------

def paper_cantilever(E: float = 1e5, dt: float = 0.5, steps: int = 200, n_nodes: int = 201,
                     tip_speed: float = 5e-3) -> dict:
    """Dynamic cantilever: N = 201, h = 2 cm, rho = 500, L = 1 m, no gravity, initial tip
    velocity 5 mm/s in z (applied to the tip node only)."""
    rod = _rod(straight_nodes(n_nodes, 1.0), 0.02, E, 0.5, 500.0)
    d = _desc([rod], dt=dt, steps=steps, gravity=(0.0, 0.0, 0.0))
    d["initial_tip_velocity"] = (0.0, 0.0, tip_speed)
    return d


def paper_helix(E: float = 1e7, h: float = 5e-3, dt: float = 6e-3, steps: int = 100, n_nodes: int = 100) -> dict:
    """Oscillating helix under gravity: rho = 1273.52, helix radius 2 cm, pitch 5 cm,
    contour length 0.5 m, N = 100, clamped at the top (first two nodes and first twist),
    rest shape = initial helix, g = 9.8."""
    rod = _rod(helix_nodes(n_nodes, 0.02, 0.05, 0.5), h, E, 0.5, 1273.52, kbar=None)
    return _desc([rod], dt=dt, steps=steps, gravity=(0.0, 0.0, -9.8))


def paper_friction(push: float = 5.0, dt: float = 5e-3, steps: int = 300, n_nodes: int = 26) -> dict:
    """Axial friction: h = 2.5 cm, rho = 509.3, L = 1, E = 1e5, N = 26, resting on the floor
    (centerline at z = h), mu = 0.4, delta = 5e-4 m, nu = 1e-3 m/s, g = 9.8, and a total push
    force `push` [N] along +x spread over the nodes in proportion to their rest edge share
    (end nodes get half)."""
    h, rho, L = 0.025, 509.3, 1.0
    x0 = straight_nodes(n_nodes, L, (0.0, 0.0, h))
    share = np.full(n_nodes, 1.0)
    share[0] = share[-1] = 0.5
    share /= share.sum()
    force = np.zeros((n_nodes, 3))
    force[:, 0] = push * share
    node_weight = rho * math.pi * h * h * (L / (n_nodes - 1)) * 9.8
    rod = _rod(x0, h, 1e5, 0.5, rho, fixed_nodes=(), fixed_edges=(), force=force)
    floor = {"z": 0.0, "delta": 5e-4, "nu": 1e-3, "mu": 0.4, "k_c": node_weight / 5e-4}
    d = _desc([rod], dt=dt, steps=steps, gravity=(0.0, 0.0, -9.8), floor=floor)
    d["line_search"] = True
    return d


def contact_tangle(n_scenes: int = 4096, seed: int = 7, fingers: int = 5, n_nodes: int = 60,
                   length: float = 0.3, radius: float = 5e-3, density: float = 1200.0) -> dict:
    """Scenes of the validation section's entanglement gripper (five fingers of L = 0.3 m,
    h = 5 mm, rho = 1200, N = 60; delta = 5e-4 m, nu = 1e-3 m/s, mu = 0.5) in a coiled, tangled
    state: finger k of a scene is a helix about the scene's vertical axis, hanging from height
    0, pitch ~ U(15, 30) mm, phase 2 pi k / fingers + U(-0.3, 0.3), on nested cylinders whose
    radii start at U(20, 25) mm and grow by U(9.6, 10.4) mm from finger to finger (so the coils
    of neighbouring fingers touch where they cross), with N(0, 0.3 mm) jitter on every node;
    scenes are 1 m apart along x.  The state one
    step (dt = 1e-3 s) earlier, x_prev, differs by N(0, 1 cm/s) velocities per node.  Contact
    stiffness k_c = (node mass) g / delta, the floor's choice.  Returns {"rods": [(x (N, 3),
    radius), ...] scene after scene, "groups": [fingers] * n_scenes, "x_prev": (total nodes, 3),
    "delta", "nu", "mu", "k_c", "dt"}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rods, prev = [], []
    for sc in range(n_scenes):
        R = rng.uniform(0.020, 0.025)
        for k in range(fingers):
            if k > 0:
                R += rng.uniform(0.0096, 0.0104)
            p = rng.uniform(0.015, 0.030)
            ph = 2.0 * math.pi * k / fingers + rng.uniform(-0.3, 0.3)
            per_turn = math.hypot(2.0 * math.pi * R, p)
            phi = ph + np.linspace(0.0, 2.0 * math.pi * length / per_turn, n_nodes)
            x = np.stack([R * np.cos(phi) + 1.0 * sc, R * np.sin(phi), -p * (phi - ph) / (2.0 * math.pi)], 1)
            x = x + rng.normal(0.0, 3e-4, size=x.shape)
            rods.append((x, radius))
            prev.append(x - 1e-3 * rng.normal(0.0, 0.01, size=x.shape))
    delta = 5e-4
    m_node = density * math.pi * radius ** 2 * length / (n_nodes - 1)
    return {"rods": rods, "groups": [fingers] * n_scenes, "x_prev": np.concatenate(prev), "delta": delta,
            "nu": 1e-3, "mu": 0.5, "k_c": m_node * 9.8 / delta, "dt": 1e-3}


def coiled_springs(n_rods: int = 4, seed: int = 13, nmin: int = 40, nmax: int = 80, radius: float = 4e-3,
                   steps: int = 10, mu: float = 0.3, kc_nodes=None) -> dict:
    """Coiled rods standing on their clamped first nodes (a helix rising along +z about a
    vertical axis), N ~ U{nmin..nmax} nodes over 3 to 4 turns, helix radius U(14, 18) mm, pitch
    U(8.1, 8.4) mm (the turns sit just inside the contact reach 2h + delta = 8.5 mm of their
    radius h = 4 mm), E = 10^U(5.5, 6.5) Pa, rho = 1200; gravity -9.81 z presses the turns
    together; rods 1 m apart along x.  Self-contact: delta = 5e-4 m, k_c = (first rod's mass) g
    / delta, so that a contact carries the whole coil's weight at a compression of about delta
    (kc_nodes = m: m node weights instead), mu as given, nu = 1e-3 m/s; dt = 1e-3 s; line
    search on."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rods = []
    m0 = None
    for k in range(n_rods):
        n = int(rng.integers(nmin, nmax + 1))
        R = rng.uniform(0.014, 0.018)
        p = rng.uniform(0.0081, 0.0084)
        turns = rng.uniform(3.0, 4.0)
        phi = np.linspace(0.0, 2.0 * math.pi * turns, n)
        x0 = np.stack([R * np.cos(phi) + 1.0 * k, R * np.sin(phi), p * phi / (2.0 * math.pi)], 1)
        E = 10.0 ** rng.uniform(5.5, 6.5)
        rods.append(_rod(x0, radius, E, 0.5, 1200.0))
        if m0 is None:
            m0 = 1200.0 * math.pi * radius ** 2 * float(np.linalg.norm(x0[1] - x0[0]))
            n0 = n - 1
    d = _desc(rods, dt=1e-3, steps=steps)
    delta = 5e-4
    weights = n0 if kc_nodes is None else kc_nodes
    d["self_contact"] = {"delta": delta, "k_c": weights * m0 * 9.81 / delta, "mu": float(mu), "nu": 1e-3}
    # the regularised friction's stick-slip transitions make Newton cycle without it (as on the
    # floor)
    d["line_search"] = True
    return d


def subset(desc: dict, rod_ids) -> dict:
    """A description restricted to the given rods (joints dropped; use for independent rods)."""
    out = dict(desc)
    out["rods"] = [desc["rods"][i] for i in rod_ids]
    out["joints"] = []
    return out
