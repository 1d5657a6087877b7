"""Pins of the oracle's actuation branch (Actuation subsection) and of its joint stencils
(Elastic Joints subsection) beyond the end-to-start joints of the main pin file.

* Sine actuation: with the frequency at zero the natural curvature is the constant
  A sin(phi), so a free rod without gravity must settle to the stress-free polygon whose
  turning angle is 2 atan(A sin(phi) V / 2) (the closed form kappa = 2 tan(phi/2) after
  Eq. 5), bent toward the first material director.  One actuated step must equal one step
  with the static natural curvature A sin(2 pi f t_{n+1} + phi) in the first component and
  zero in the second: the path that takes static curvature is itself pinned by the
  stress-free polygon of the main pin file.
* Both edges leaving the joint: a rod cut at an interior node and stored as two rods that
  both start at the cut (so the joint stencil has its first edge reversed) must move exactly
  as the uncut rod under a 3-D tip load and a twisting moment.
* A six-limb star (a joint of degree six): zero residual at rest, rigid-motion invariance of
  the energy, zero net elastic force and zero net torque.

Each pin is also run against a deliberately broken oracle (the mistake planted in the test,
on the CPU) to show that it catches that mistake.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import workloads as W
from oracle import der


def T(a):
    return torch.as_tensor(np.asarray(a), dtype=torch.float64)


# ---------------------------------------------------------------------------
# sine actuation
# ---------------------------------------------------------------------------

def actuated_rod(A, f, phi, n=15, L=0.5, h=2e-3, E=1e6, clamp=True):
    kw = {} if clamp else {"fixed_nodes": (), "fixed_edges": ()}
    return W.rod(W.straight_nodes(n, L), h, E, actuation=(A, f, phi), **kw)


def polygon_error(A, phi, n=15, L=0.5):
    """Largest deviation of the static actuated shape (f = 0) from the stress-free polygon."""
    d = W.desc([actuated_rod(A, 0.0, phi, n, L)], dt=1e6, steps=1, gravity=(0, 0, 0))
    sys, st = der.build(d)
    st1, info = der.step(sys, st, 1e6, tol=1e-12, max_iter=40)
    if not info.converged:
        return math.inf, False
    x = st1.x
    e = (x[1:] - x[:-1]).numpy()
    ell = np.linalg.norm(e, axis=1)
    t = e / ell[:, None]
    turn = np.arccos(np.clip((t[:-1] * t[1:]).sum(1), -1, 1))
    k = A * math.sin(phi)
    want = 2 * math.atan(abs(k) * (L / (n - 1)) / 2)
    err_turn = float(np.abs(turn - want).max()) / want
    # positive curvature bends toward +m1 (+z for a rod laid along x), negative toward -z
    side_ok = math.copysign(1.0, float(x[-1, 2])) == math.copysign(1.0, k)
    return max(err_turn, float(np.abs(ell - L / (n - 1)).max()) / (L / (n - 1))), side_ok


def test_constant_actuation_settles_to_stress_free_polygon():
    for A, phi in ((4.0, 1.1), (7.0, 4.0)):
        err, side_ok = polygon_error(A, phi)
        assert err < 1e-8 and side_ok, (A, phi, err, side_ok)


def step_pair(A, f, phi, dt=2e-3, nsteps=3):
    """Final positions of (a) an actuated rod and (b) the same rod whose natural curvature is
    set, before every step, to the static value A sin(2 pi f t_{n+1} + phi) in the first
    component (in 1/m), starting from a moving state so that the step has work to do."""
    n = 12
    rng = np.random.Generator(np.random.PCG64(11))
    da = W.desc([actuated_rod(A, f, phi, n)], dt=dt, steps=nsteps)
    sys_a, st_a = der.build(da)
    db = W.desc([W.rod(W.straight_nodes(n, 0.5), 2e-3, 1e6, kbar=np.zeros((n - 2, 2)))], dt=dt, steps=nsteps)
    sys_b, st_b = der.build(db)
    v0 = T(rng.normal(0, 0.05, size=(n, 3)))
    v0[:2] = 0.0
    st_a.v, st_b.v = v0.clone(), v0.clone()
    st_a.time = st_b.time = 0.37
    for _ in range(nsteps):
        st_a, ia = der.step(sys_a, st_a, dt, tol=1e-12, max_iter=40, polish=1)
        kb = np.zeros((n - 2, 2))
        kb[:, 0] = A * math.sin(2 * math.pi * f * (st_b.time + dt) + phi)
        st_b, ib = der.step(sys_b, st_b, dt, tol=1e-12, max_iter=40, polish=1, kbar_rods=[kb])
        assert ia.converged and ib.converged
    return st_a, st_b


def actuation_step_error(A=6.0, f=1.7, phi=0.9):
    """Largest position difference relative to the largest displacement, and the largest
    twist difference, between the actuated rod and the static-curvature rod."""
    st_a, st_b = step_pair(A, f, phi)
    disp = float((st_b.x - T(W.straight_nodes(12, 0.5))).abs().max())
    assert disp > 1e-4
    return float((st_a.x - st_b.x).abs().max()) / disp, float((st_a.theta - st_b.theta).abs().max())


def test_actuated_step_equals_static_curvature_at_step_end():
    ex, et = actuation_step_error()
    assert ex < 1e-13 and et < 1e-12, (ex, et)


def _planted(monkeypatch, kind):
    """Plant one mistake in the oracle's natural curvature (test-side wrapper)."""
    orig = der.natural_curvature

    def wrong(sys, time, kbar_rods=None):
        act = torch.isfinite(sys.st_act[:, 0])
        if kind == "time":                       # evaluated at the step start, not its end
            return orig(sys, time - 2e-3, kbar_rods)
        kap = orig(sys, time, kbar_rods)
        if kind == "no_vbar":                    # the 1/m value used as the integrated one
            kap = kap.clone()
            kap[act, 0] = kap[act, 0] / sys.Vbar[act]
        elif kind == "component":                # the second material direction
            kap = kap.clone()
            kap[act] = kap[act].flip(1)
        elif kind == "sign":
            kap = kap.clone()
            kap[act, 0] = -kap[act, 0]
        return kap
    monkeypatch.setattr(der, "natural_curvature", wrong)


@pytest.mark.parametrize("kind", ["time", "no_vbar", "component", "sign"])
def test_actuation_pins_catch_planted_mistakes(monkeypatch, kind):
    _planted(monkeypatch, kind)
    st_err = None
    if kind != "time":
        err, side_ok = polygon_error(4.0, 1.1)
        st_err = err
        caught_static = err > 1e-4 or not side_ok
    else:
        caught_static = False
    # the step pin compares against the unbroken static-curvature path: run it with the
    # broken actuation but restore the static path's own natural curvature
    broken = der.natural_curvature
    monkeypatch.undo()
    orig = der.natural_curvature

    def mixed(sys, time, kbar_rods=None):
        return broken(sys, time, kbar_rods) if bool(torch.isfinite(sys.st_act[:, 0]).any()) else orig(sys, time, kbar_rods)
    monkeypatch.setattr(der, "natural_curvature", mixed)
    ex, et = actuation_step_error()
    caught_step = ex > 1e-9 or et > 1e-9
    assert caught_static or caught_step, (kind, st_err, ex, et)
    if kind == "time":
        assert caught_step


# ---------------------------------------------------------------------------
# joint stencil with both edges leaving the joint
# ---------------------------------------------------------------------------

def cut_rod_descs(n=21, cut=10, steps=3):
    L, h, E = 1.0, 2e-3, 2e6
    x = W.straight_nodes(n, L)
    force = np.zeros((n, 3))
    force[-1] = (0.0, 2e-3, -3e-3)
    mom = np.zeros(n - 1)
    mom[-1] = 4e-5
    one = W.desc([W.rod(x, h, E, force=force, moment=mom)], dt=1e-2, steps=steps)
    # rod A: nodes cut .. 0 (starts at the cut, clamped at its far end), rod B: nodes cut .. n-1
    xa = x[:cut + 1][::-1].copy()
    a = W.rod(xa, h, E, fixed_nodes=(cut - 1, cut), fixed_edges=(cut - 1,))
    fb = force[cut:].copy()
    b = W.rod(x[cut:].copy(), h, E, fixed_nodes=(), fixed_edges=(), force=fb, moment=mom[cut:].copy())
    two = W.desc([a, b], dt=1e-2, steps=steps, joints=[(0, 0, 1, 0)])
    return one, two


def cut_rod_error(two_sys_hook=None):
    one, two = cut_rod_descs()
    _, s1, i1, _ = der.simulate(one, polish=1)
    sys2, st2 = der.build(two)
    if two_sys_hook is not None:
        two_sys_hook(sys2)
    for _ in range(two["steps"]):
        st2, info = der.step(sys2, st2, two["dt"], two["tol"], two["max_iter"], polish=1)
        assert info.converged
    xa = der.rod_positions(sys2, st2, 0).flip(0)
    xb = der.rod_positions(sys2, st2, 1)
    x2 = torch.cat([xa, xb[1:]])
    ta = -der.rod_thetas(sys2, st2, 0).flip(0)        # a reversed edge has the opposite twist
    tb = der.rod_thetas(sys2, st2, 1)
    t2 = torch.cat([ta, tb])
    return float((x2 - s1.x).abs().max()), float((t2 - s1.theta).abs().max()), float((s1.x - T(one["rods"][0]["x0"])).abs().max()), float(s1.theta.abs().max())


def test_rod_cut_into_two_rods_leaving_the_cut_equals_one_rod():
    one, two = cut_rod_descs()
    sys2, _ = der.build(two)
    js = torch.nonzero(sys2.st_rod < 0).flatten()
    assert js.numel() == 1 and sys2.st_sign[js[0]].tolist() == [-1.0, 1.0]   # the (+1, +1) branch
    ex, et, disp, twist = cut_rod_error()
    assert disp > 1e-4 and twist > 1e-4            # the load bends and twists the rod
    assert ex < 1e-12 and et < 1e-10, (ex, et)


@pytest.mark.parametrize("plant", ["f_not_reversed", "e_reversed"])
def test_cut_rod_pin_catches_wrong_joint_orientation(plant):
    def hook(sys):
        js = torch.nonzero(sys.st_rod < 0).flatten()
        if plant == "f_not_reversed":
            sys.st_sign[js, 0] = 1.0
        else:
            sys.st_sign[js, 1] = -1.0
    try:
        ex, et, _, _ = cut_rod_error(hook)
    except (AssertionError, RuntimeError):
        return                                   # the broken joint does not even converge
    assert ex > 1e-6 or et > 1e-6, (ex, et)


# ---------------------------------------------------------------------------
# a joint of degree six
# ---------------------------------------------------------------------------

def star_system(gravity=(0, 0, 0)):
    d = W.star_robots(n_instances=1, steps=1)
    d["gravity"] = gravity
    d["floor"] = None
    for r in d["rods"]:
        r["actuation"] = None
    return d, *der.build(d)


def test_six_limb_star_rest_state_has_zero_residual():
    d, sys, st = star_system()
    assert int((sys.st_rod < 0).sum()) == 15          # every pair of the six hub edges
    kap = der.natural_curvature(sys, st.time + 1e-3)
    R = der.residual(sys, der.pack(st.x, st.theta), st, 1e-3, kap)
    assert float(R.abs().max()) == 0.0


def deformed_star(seed=4):
    d, sys, st = star_system()
    rng = np.random.Generator(np.random.PCG64(seed))
    q1 = der.pack(st.x + T(rng.normal(0, 2e-3, size=st.x.shape)), T(rng.normal(0, 0.2, size=st.theta.shape)))
    st = der.commit(sys, st, q1, 1e-3)          # a step start away from rest, with its frames
    q = der.pack(st.x + T(rng.normal(0, 2e-3, size=st.x.shape)), st.theta + T(rng.normal(0, 0.2, size=st.theta.shape)))
    return sys, st, q, der.natural_curvature(sys, st.time)


def test_six_limb_star_energy_is_invariant_under_rigid_motion():
    sys, st, q, kap = deformed_star()
    x, th = der.unpack(sys, q)
    E0 = float(der.elastic_energy(sys, x, th, st, kap))
    R = T(Rotation.from_rotvec([-0.4, 0.9, 0.25]).as_matrix())
    c = T([0.3, 2.0, -1.5])
    st2 = st.clone()
    st2.t_ref = st.t_ref @ R.T
    st2.d1_ref = st.d1_ref @ R.T
    E1 = float(der.elastic_energy(sys, x @ R.T + c, th, st2, kap))
    assert E0 > 0 and abs(E1 - E0) <= 1e-13 * E0, (E0, E1)


def test_six_limb_star_net_force_and_torque_vanish():
    sys, st, q, kap = deformed_star(seed=5)

    def energy(qq):
        xx, tt = der.unpack(sys, qq)
        return der.elastic_energy(sys, xx, tt, st, kap)
    g = torch.func.grad(energy)(q)
    gx = g[:3 * sys.n_nodes].reshape(-1, 3)
    assert float(gx.sum(0).abs().max()) < 1e-12 * float(gx.abs().max())
    # at the step start the holonomy term vanishes and the forces are torque free
    qn = der.pack(st.x, st.theta)
    g = torch.func.grad(energy)(qn)
    gx, gt = g[:3 * sys.n_nodes].reshape(-1, 3), g[3 * sys.n_nodes:]
    t = der.frames(sys, st.x, st.theta, st)[0]
    torque = torch.linalg.cross(st.x, gx).sum(0) + (gt[:, None] * t).sum(0)
    assert float(torque.abs().max()) < 1e-11 * float(g.abs().max())


def symmetric_star_step(drop_one=False):
    """One step of a free star pushed down at its hub (gravity off): the six-fold symmetry
    must leave the hub moving straight down and every limb tip at the same height."""
    d, _, _ = star_system()
    force = np.zeros((31, 3))
    force[0, 2] = -0.02
    d["rods"][0]["force"] = force
    sys, st = der.build(d)
    if drop_one:
        js = torch.nonzero(sys.st_rod < 0).flatten()
        keep = torch.ones(sys.st_nodes.shape[0], dtype=torch.bool)
        keep[js[0]] = False
        for name in ("st_nodes", "st_edges", "st_sign", "Vbar", "EI", "GJ", "kappa_rest", "tau_rest", "st_rod",
                     "st_index", "st_act"):
            setattr(sys, name, getattr(sys, name)[keep])
        st.beta_ref = st.beta_ref[keep]
    st1, info = der.step(sys, st, 1e-2, 1e-12, 40, polish=1)
    assert info.converged
    hub = int(sys.rod_nodes[0][0])
    tips = torch.stack([st1.x[int(sys.rod_nodes[a][-1])] for a in range(6)])
    drop = float(st.x[hub, 2] - st1.x[hub, 2])
    return float(st1.x[hub, :2].abs().max()) / drop, float((tips[:, 2] - tips[0, 2]).abs().max()) / drop


def test_six_limb_star_moves_symmetrically_under_a_hub_load():
    hub_side, tip_spread = symmetric_star_step()
    assert hub_side < 1e-12 and tip_spread < 1e-12, (hub_side, tip_spread)


def test_symmetric_star_pin_catches_a_dropped_hub_stencil():
    hub_side, tip_spread = symmetric_star_step(drop_one=True)
    assert hub_side > 1e-8 or tip_spread > 1e-8, (hub_side, tip_spread)
