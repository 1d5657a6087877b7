"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula.  They check closed forms the paper
prints (kappa = 2 tan(phi/2), the friction kinetic-energy law Eq. 18), textbook
beam statics derived for the discrete rod, invariants (rigid motion, momentum),
finite differences of the energy and residual, an independent rotation routine
(scipy), and the classical discrete-elastic-rods gradient at the step start.
Together they fail on a dropped term, a wrong sign or index, or a transposed
operand anywhere in the oracle's frames, strains, energies, forces or solve.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import workloads as W
from oracle import der

RNG = np.random.Generator(np.random.PCG64(1234))


def unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def T(a):
    return torch.as_tensor(np.asarray(a), dtype=torch.float64)


# ---------------------------------------------------------------------------
# P1 parallel transport (Methodology: time-parallel transport of the reference frame)
# ---------------------------------------------------------------------------

def test_transport_matches_axis_angle_rotation():
    a = unit(RNG.normal(size=(64, 3)))
    b = unit(RNG.normal(size=(64, 3)))
    v = RNG.normal(size=(64, 3))
    got = der.transport(T(a), T(b), T(v)).numpy()
    axis = unit(np.cross(a, b))
    ang = np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), (a * b).sum(1))
    want = Rotation.from_rotvec(axis * ang[:, None]).apply(v)
    assert np.allclose(got, want, rtol=0, atol=1e-13)
    # takes a onto b, preserves length, composes to the identity, identity for a == b
    assert np.allclose(der.transport(T(a), T(b), T(a)).numpy(), b, atol=1e-14)
    assert np.allclose(np.linalg.norm(got, axis=1), np.linalg.norm(v, axis=1), rtol=1e-14)
    back = der.transport(T(b), T(a), T(got)).numpy()
    assert np.allclose(back, v, atol=1e-13)
    assert np.allclose(der.transport(T(a), T(a), T(v)).numpy(), v, atol=1e-15)


# ---------------------------------------------------------------------------
# P5 curvature convention: kappa = 2 tan(phi / 2) (text after Eq. 5)
# ---------------------------------------------------------------------------

def polygon(n, phi, plane_normal_turn):
    """Nodes of a polygon starting along +x that turns by phi at every node toward the
    direction `plane_normal_turn` (a unit vector perpendicular to x)."""
    pts = [np.zeros(3)]
    d = np.array([1.0, 0.0, 0.0])
    w = np.asarray(plane_normal_turn, dtype=np.float64)
    for i in range(n - 1):
        ang = i * phi
        step = math.cos(ang) * d + math.sin(ang) * w
        pts.append(pts[-1] + 0.1 * step)
    return np.array(pts)


@pytest.mark.parametrize("phi", [0.05, 0.4, 1.2])
def test_kappa_equals_two_tan_half_turning_angle(phi):
    # the first edge runs along x, so its first material director starts at +z and
    # the second at -y (right-handed material frame m1 x m2 = t)
    for toward, comp in (([0.0, 0.0, 1.0], 0), ([0.0, -1.0, 0.0], 1)):
        d = W.desc([W.rod(polygon(7, phi, toward), 1e-3, 1e7)], dt=1e-3, steps=1)
        sys, st = der.build(d)
        kap, tau, _ = der.strains(sys, st.x, st.theta, st)
        assert np.allclose(kap[:, comp].numpy(), 2 * math.tan(phi / 2), rtol=1e-13)
        assert np.allclose(kap[:, 1 - comp].numpy(), 0.0, atol=1e-13)
        assert np.allclose(tau.numpy(), 0.0, atol=1e-13)


# ---------------------------------------------------------------------------
# P2 / P3 gradients and Jacobians (Eq. 9, Eq. 15-16)
# ---------------------------------------------------------------------------

def deformed_pair(seed=0, n=8):
    """A step-start state (frames from a curved rod) and a different current q."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x0 = W.helix_nodes(n, 0.05, 0.08, 0.4)
    kb = rng.normal(0.0, 3.0, size=(n - 2, 2))
    d = W.desc([W.rod(x0, 2e-3, 1e6, kbar=kb, fixed_nodes=(), fixed_edges=())], dt=1e-3, steps=1)
    sys, st = der.build(d)
    # move the step start away from the rest shape, with its own transported frames
    q1 = der.pack(st.x + T(rng.normal(0, 0.01, size=(n, 3))), T(rng.normal(0, 0.3, size=n - 1)))
    st = der.commit(sys, st, q1, 1e-3)
    q = der.pack(st.x + T(rng.normal(0, 0.01, size=(n, 3))), st.theta + T(rng.normal(0, 0.3, size=n - 1)))
    kap = der.natural_curvature(sys, st.time)
    return sys, st, q, kap


def energy_fn(sys, st, kap):
    def f(q):
        x, th = der.unpack(sys, q)
        return der.elastic_energy(sys, x, th, st, kap)
    return f


def test_gradient_matches_central_differences():
    sys, st, q, kap = deformed_pair()
    f = energy_fn(sys, st, kap)
    g = torch.func.grad(f)(q)
    h = 1e-6
    fd = torch.zeros_like(q)
    for i in range(q.numel()):
        e = torch.zeros_like(q)
        e[i] = h
        fd[i] = (f(q + e) - f(q - e)) / (2 * h)
    assert torch.allclose(g, fd, rtol=1e-6, atol=1e-8 * float(g.abs().max()))


def test_jacobian_matches_differences_and_is_symmetric():
    sys, st, q, kap = deformed_pair(seed=1)
    dt = 1e-3
    R = lambda qq: der.residual(sys, qq, st, dt, kap)
    J = torch.func.jacfwd(R)(q)
    h = 1e-7
    fd = torch.zeros_like(J)
    for i in range(q.numel()):
        e = torch.zeros_like(q)
        e[i] = h
        fd[:, i] = (R(q + e) - R(q - e)) / (2 * h)
    scale = float(J.abs().max())
    assert float((J - fd).abs().max()) < 1e-6 * scale
    # without friction the Jacobian is a Hessian plus a diagonal: symmetric
    assert float((J - J.T).abs().max()) < 1e-11 * scale


def classical_bend_gradient(tf, te, m1f, m2f, m1e, m2e, lf, le):
    """Classical discrete-elastic-rods gradients of the integrated curvature with respect
    to the two edge vectors (Bergou et al. 2008, frames varied without twist)."""
    chi = 1 + tf @ te
    tt = (tf + te) / chi
    kb = 2 * np.cross(tf, te) / chi
    k1 = 0.5 * kb @ (m2f + m2e)
    k2 = -0.5 * kb @ (m1f + m1e)
    m1t = (m1f + m1e) / chi
    m2t = (m2f + m2e) / chi
    dk1_f = (-k1 * tt + np.cross(te, m2t)) / lf
    dk1_e = (-k1 * tt - np.cross(tf, m2t)) / le
    dk2_f = (-k2 * tt - np.cross(te, m1t)) / lf
    dk2_e = (-k2 * tt + np.cross(tf, m1t)) / le
    return k1, k2, (dk1_f, dk1_e), (dk2_f, dk2_e), kb


def test_step_start_gradient_equals_classical_formula():
    """At q = q_n the exact gradient of the transported-frame energy reduces to the classical
    discrete-elastic-rods expressions (the time-transport holonomy vanishes there)."""
    sys, st, q, kap = deformed_pair(seed=2)
    qn = der.pack(st.x, st.theta)
    f = energy_fn(sys, st, kap)
    g = torch.func.grad(f)(qn).numpy()
    x, th = st.x.numpy(), st.theta.numpy()
    t, ell, d1, d2, m1, m2 = [a.numpy() for a in der.frames(sys, st.x, st.theta, st)]
    kapv, tau, _ = der.strains(sys, st.x, st.theta, st)
    want = np.zeros_like(g)
    n = sys.n_nodes
    for s in range(sys.st_nodes.shape[0]):
        a, b, c = [int(i) for i in sys.st_nodes[s]]
        f_, e_ = [int(i) for i in sys.st_edges[s]]
        k1, k2, dk1, dk2, kb = classical_bend_gradient(t[f_], t[e_], m1[f_], m2[f_], m1[e_], m2[e_], ell[f_], ell[e_])
        EI, GJ, V = float(sys.EI[s]), float(sys.GJ[s]), float(sys.Vbar[s])
        c1 = EI / V * (k1 - float(kap[s, 0]))
        c2 = EI / V * (k2 - float(kap[s, 1]))
        ct = GJ / V * (float(tau[s]) - float(sys.tau_rest[s]))
        gf = c1 * dk1[0] + c2 * dk2[0] + ct * kb / (2 * ell[f_])
        ge = c1 * dk1[1] + c2 * dk2[1] + ct * kb / (2 * ell[e_])
        want[3 * a:3 * a + 3] -= gf
        want[3 * b:3 * b + 3] += gf - ge
        want[3 * c:3 * c + 3] += ge
        # theta derivatives: d kappa1/d theta = -kb.m1 / 2, d kappa2/d theta = -kb.m2 / 2
        for j, sgn in ((f_, -1.0), (e_, 1.0)):
            want[3 * n + j] += c1 * (-0.5 * kb @ m1[j]) + c2 * (-0.5 * kb @ m2[j]) + ct * sgn
    # stretch
    for j in range(sys.n_edges):
        a, b = [int(i) for i in sys.edge_nodes[j]]
        eps = ell[j] / float(sys.ebar[j]) - 1
        ge = float(sys.EA[j]) * eps * t[j]
        want[3 * a:3 * a + 3] -= ge
        want[3 * b:3 * b + 3] += ge
    assert np.allclose(g, want, rtol=1e-10, atol=1e-10 * np.abs(g).max())


def test_newton_converges_quadratically():
    d = W.cantilever(steps=1)
    sys, st = der.build(d)
    _, info = der.step(sys, st, d["dt"], 1e-12, 50)
    h = info.history
    assert info.converged
    # once in the asymptotic regime, r_{k+1} <= C r_k^2
    pairs = [(h[k], h[k + 1]) for k in range(len(h) - 1) if h[k] < 1e-5 and h[k + 1] > 1e-11]
    assert pairs, h
    for r0, r1 in pairs:
        assert r1 <= 1e4 * r0 * r0, h


# ---------------------------------------------------------------------------
# P4 rigid motion
# ---------------------------------------------------------------------------

def test_rigid_motion_invariance():
    sys, st, q, kap = deformed_pair(seed=3)
    f = energy_fn(sys, st, kap)
    E0 = float(f(q))
    R = T(Rotation.from_rotvec([0.3, -0.7, 0.4]).as_matrix())
    c = T([0.5, -1.0, 2.0])
    x, th = der.unpack(sys, q)
    st2 = st.clone()
    st2.t_ref = st.t_ref @ R.T
    st2.d1_ref = st.d1_ref @ R.T
    E1 = float(der.elastic_energy(sys, x @ R.T + c, th, st2, kap))
    assert abs(E1 - E0) <= 1e-13 * abs(E0)
    # translation invariance: the elastic forces sum to zero at any q
    g = torch.func.grad(f)(q)
    gx = g[:3 * sys.n_nodes].reshape(-1, 3)
    assert float(gx.sum(0).abs().max()) < 1e-12 * float(gx.abs().max())
    # rotation invariance at the step start: sum x_i x F_i + sum_j M_j t_j = 0
    qn = der.pack(st.x, st.theta)
    g = torch.func.grad(f)(qn)
    gx, gt = g[:3 * sys.n_nodes].reshape(-1, 3), g[3 * sys.n_nodes:]
    t = der.frames(sys, st.x, st.theta, st)[0]
    torque = torch.linalg.cross(st.x, gx).sum(0) + (gt[:, None] * t).sum(0)
    assert float(torque.abs().max()) < 1e-11 * float(g.abs().max())


# ---------------------------------------------------------------------------
# P7 - P10 statics (backward Euler with a huge step is a static solve)
# ---------------------------------------------------------------------------

def static_solve(d, iters=10):
    sys, st = der.build(d)
    kap = der.natural_curvature(sys, 1e6)
    q, _ = der.newton_solve(sys, st, 1e6, kap, tol=0.0, max_iter=iters)
    x, th = der.unpack(sys, q)
    return sys, st, x, th


def test_static_axial_load_gives_uniform_strain():
    n, L, h, E, P = 21, 1.0, 0.01, 1e7, 3.0
    force = np.zeros((n, 3))
    force[-1, 0] = P
    d = W.desc([W.rod(W.straight_nodes(n, L), h, E, force=force)], dt=1e6, steps=1, gravity=(0, 0, 0))
    sys, st, x, th = static_solve(d)
    EA = E * math.pi * h * h
    ell = torch.linalg.norm(x[1:] - x[:-1], dim=1).numpy()
    eps = ell / (L / (n - 1)) - 1
    assert np.allclose(eps[1:], P / EA, rtol=1e-9)
    assert abs(eps[0]) < 1e-15
    tip = float(x[-1, 0]) - L
    assert abs(tip - (L - L / (n - 1)) * P / EA) < 1e-9 * (L * P / EA)


def test_static_twisting_moment_gives_linear_twist():
    n, L, h, E, Tq = 21, 1.0, 0.01, 1e7, 2e-3
    mom = np.zeros(n - 1)
    mom[-1] = Tq
    d = W.desc([W.rod(W.straight_nodes(n, L), h, E, moment=mom)], dt=1e6, steps=1, gravity=(0, 0, 0))
    sys, st, x, th = static_solve(d)
    GJ = E / 3.0 * math.pi * h ** 4 / 2
    dl = L / (n - 1)
    tau = (th[1:] - th[:-1]).numpy()
    assert np.allclose(tau, Tq * dl / GJ, rtol=1e-9)
    assert abs(float(th[-1]) - Tq * (L - dl) / GJ) < 1e-9 * Tq * L / GJ
    assert float((x - st.x).abs().max()) < 1e-12


@pytest.mark.parametrize("n", [11, 51])
def test_cantilever_tip_point_load(n):
    L, h, E = 1.0, 0.01, 1e7
    EI = E * math.pi * h ** 4 / 4
    P = 3 * EI * 1e-4 / L ** 3           # continuum deflection L / 10^4
    force = np.zeros((n, 3))
    force[-1, 2] = -P
    d = W.desc([W.rod(W.straight_nodes(n, L), h, E, force=force)], dt=1e6, steps=1, gravity=(0, 0, 0))
    sys, st, x, th = static_solve(d)
    m = n - 1
    ebar = L / m
    want = P * ebar ** 3 / EI * sum(k * k for k in range(1, m))
    assert abs(-float(x[-1, 2]) - want) < 2e-6 * want


@pytest.mark.parametrize("n", [11, 51])
def test_cantilever_under_gravity(n):
    L, h, E, rho, g = 1.0, 0.01, 1e12, 1000.0, 9.81
    EI = E * math.pi * h ** 4 / 4
    q = rho * math.pi * h * h * g
    d = W.desc([W.rod(W.straight_nodes(n, L), h, E, density=rho)], dt=1e6, steps=1, gravity=(0, 0, -g))
    sys, st, x, th = static_solve(d)
    m = n - 1
    want = q * L ** 4 / (8 * EI) * (1 - 1 / m) ** 2
    assert want < 1e-3 * L
    assert abs(-float(x[-1, 2]) - want) < 2e-5 * want


def test_natural_curvature_gives_stress_free_polygon():
    n, L, h, E = 15, 0.5, 2e-3, 1e6
    k = 4.0   # 1/m, first component
    kb = np.zeros((n - 2, 2))
    kb[:, 0] = k
    d = W.desc([W.rod(W.straight_nodes(n, L), h, E, kbar=kb)], dt=1e6, steps=1, gravity=(0, 0, 0))
    sys, st, x, th = static_solve(d, iters=30)
    e = (x[1:] - x[:-1]).numpy()
    ell = np.linalg.norm(e, axis=1)
    assert np.allclose(ell, L / (n - 1), rtol=1e-10)
    t = e / ell[:, None]
    turn = np.arccos(np.clip((t[:-1] * t[1:]).sum(1), -1, 1))
    want = 2 * math.atan(k * L / (n - 1) / 2)
    assert np.allclose(turn, want, rtol=1e-8)
    # kappa1 > 0 bends toward the first material director, +z for a rod laid along x
    assert float(x[-1, 2]) > 0 and abs(float(x[:, 1].abs().max())) < 1e-12


# ---------------------------------------------------------------------------
# P6 joints, P11 momentum, P12 friction law
# ---------------------------------------------------------------------------

def test_two_rods_joined_end_to_start_equal_one_rod():
    n, L = 21, 1.0
    x = W.straight_nodes(n, L)
    one = W.desc([W.rod(x, 1e-3, 1e7)], dt=1e-2, steps=3)
    a = W.rod(x[:11], 1e-3, 1e7)
    b = W.rod(x[10:], 1e-3, 1e7, fixed_nodes=(), fixed_edges=())
    two = W.desc([a, b], dt=1e-2, steps=3, joints=[(0, 10, 1, 0)])
    _, s1, _, _ = der.simulate(one, polish=1)
    sys2, s2, _, _ = der.simulate(two, polish=1)
    x2 = torch.cat([der.rod_positions(sys2, s2, 0), der.rod_positions(sys2, s2, 1)[1:]])
    assert float((x2 - s1.x).abs().max()) < 1e-12
    # the same with rod B stored reversed (joined at its last node)
    brev = W.rod(x[10:][::-1].copy(), 1e-3, 1e7, fixed_nodes=(), fixed_edges=())
    rev = W.desc([a, brev], dt=1e-2, steps=3, joints=[(0, 10, 1, 10)])
    sys3, s3, _, _ = der.simulate(rev, polish=1)
    x3 = torch.cat([der.rod_positions(sys3, s3, 0), der.rod_positions(sys3, s3, 1).flip(0)[1:]])
    assert float((x3 - s1.x).abs().max()) < 1e-12


def test_linear_momentum_is_conserved_without_external_forces():
    rng = np.random.Generator(np.random.PCG64(5))
    n = 12
    kb = rng.normal(0, 3.0, size=(n - 2, 2))
    d = W.desc([W.rod(W.helix_nodes(n, 0.05, 0.05, 0.5), 2e-3, 1e6, kbar=kb, fixed_nodes=(), fixed_edges=())],
               dt=1e-3, steps=1, gravity=(0, 0, 0))
    sys, st = der.build(d)
    st.v = T(rng.normal(0, 0.5, size=(n, 3)))
    st.omega = T(rng.normal(0, 5.0, size=n - 1))
    p0 = (sys.mass[:, None] * st.v).sum(0)
    for _ in range(5):
        st, info = der.step(sys, st, d["dt"], 1e-9, 50)
        assert info.converged
        p1 = (sys.mass[:, None] * st.v).sum(0)
        assert float((p1 - p0).abs().max()) <= d["dt"] * math.sqrt(3 * n) * 1e-9
        p0 = p1


@pytest.mark.parametrize("push", [2.0, 8.0])
def test_axial_friction_kinetic_energy_law(push):
    """Eq. 18: a rod resting on the floor under a uniform push F gains kinetic energy
    t^2/(2m) (F - mu m g)^2 once F exceeds mu m g, and none below it."""
    steps = 60
    d = W.paper_friction(push=push, steps=steps)
    sys, st = der.build(d)
    for _ in range(steps):
        st, info = der.step(sys, st, d["dt"], 1e-9, 50, line_search=True)
        assert info.converged
    m = float(sys.mass.sum())
    Ek = 0.5 * float((sys.mass[:, None] * st.v[:, :2] ** 2).sum())
    t = steps * d["dt"]
    mu, g = d["floor"]["mu"], 9.8
    want = t * t / (2 * m) * max(push - mu * m * g, 0.0) ** 2
    if want > 0:
        assert abs(Ek - want) < 0.02 * want
    else:
        # stiction: only creep within the slipping tolerance nu
        assert Ek < 0.5 * m * (d["floor"]["nu"]) ** 2
