"""Pins of the oracle's self-contact inside the step (Eq. 10-13 on pairs of a rod's edges,
with the contact energy in the residual of Eq. 15 and its Hessian in the Jacobian of Eq. 16).

* The contact forces of a pair are internal: on a free coil without gravity, loads or
  friction, the contact forces sum to zero and a step conserves linear momentum.
* The Jacobian the oracle's Newton uses (pairs and closest-point candidates fixed at the
  iterate) is the derivative of its residual: central differences of the residual.
* Switched on, contact changes a step where the turns touch and changes nothing where no pair
  is within reach (a straight rod)."""
import numpy as np
import torch

import workloads as W
from oracle import der


def coil(free=False, mu=0.0, squeeze=1.0):
    d = W.coiled_springs(1, seed=21, nmin=34, nmax=34, mu=mu, kc_nodes=1)
    d["rods"][0]["x0"][:, 2] *= squeeze          # squeeze < 1 presses the turns into each other
    if free:
        d["rods"][0]["fixed_nodes"] = []
        d["rods"][0]["fixed_edges"] = []
        d["gravity"] = (0.0, 0.0, 0.0)
    return d


def test_contact_forces_are_internal_and_conserve_momentum():
    d = coil(free=True, squeeze=0.9)
    sys_, st = der.build(d)
    q = der.pack(st.x, st.theta)
    pairs = der.contact_list(sys_, q)
    assert len(pairs) > 20
    x = st.x.clone()
    F = -torch.func.grad(lambda xx: der.self_contact_energy(sys_, xx, pairs))(x)
    assert float(F.abs().max()) > 0
    assert float(F.sum(0).abs().max()) < 1e-12 * float(F.abs().max())
    # the same force as the pinned pair energy of the contact oracle on its own pair list
    from oracle import contact as OC
    es = sys_.contact_sets[0]
    ref = OC.contact_force(es, x, OC.contact_pairs(es, x, d["self_contact"]["delta"]), d["self_contact"]["delta"],
                           d["self_contact"]["k_c"])
    assert float((F - ref).abs().max()) <= 1e-12 * float(F.abs().max())
    # a step from rest with the contact forces only: total momentum stays zero
    st.v = torch.zeros_like(st.v)
    st1, info = der.step(sys_, st, d["dt"], 1e-11, 50)
    assert info.converged
    p = (sys_.mass[:, None] * st1.v).sum(0)
    assert float(p.abs().max()) < 1e-10 * float((sys_.mass[:, None] * st1.v.abs()).sum())


def test_friction_is_internal_and_matches_the_pair_friction_of_the_contact_oracle():
    """With friction and slipping turns (random start velocities) a free coil still conserves
    linear momentum, and the step's friction equals contact.friction_force on the same pairs."""
    from oracle import contact as OC
    d = coil(free=True, mu=0.4, squeeze=0.9)
    sys_, st = der.build(d)
    rng = np.random.Generator(np.random.PCG64(8))
    st.v = torch.tensor(rng.normal(0.0, 0.02, st.v.shape))
    x = st.x + d["dt"] * st.v            # a trial end state: slip over the step
    q = der.pack(x, st.theta)
    pairs = der.contact_list(sys_, q)
    F = der.self_contact_friction(sys_, x, st, d["dt"], pairs)
    es = sys_.contact_sets[0]
    ref_pairs = OC.contact_pairs(es, x, d["self_contact"]["delta"])
    sc = d["self_contact"]
    Fref = OC.friction_force(es, x, st.x, d["dt"], ref_pairs, sc["delta"], sc["k_c"], sc["mu"], sc["nu"])
    assert float(F.abs().max()) > 0
    assert float((F - Fref).abs().max()) <= 1e-10 * float(F.abs().max())
    assert float(F.sum(0).abs().max()) <= 1e-12 * float(F.abs().max())
    st1, info = der.step(sys_, st, d["dt"], 1e-11, 50, line_search=True)   # slipping turns need it
    assert info.converged
    p0, p1 = (sys_.mass[:, None] * st.v).sum(0), (sys_.mass[:, None] * st1.v).sum(0)
    assert float((p1 - p0).abs().max()) < 1e-10 * float((sys_.mass[:, None] * st1.v.abs()).sum())


def test_jacobian_is_the_derivative_of_the_residual_with_contact_and_friction():
    d = coil(mu=0.4)
    sys_, st = der.build(d)
    kap = der.natural_curvature(sys_, st.time + d["dt"])
    rng = np.random.Generator(np.random.PCG64(3))
    q = der.pack(st.x, st.theta) + torch.tensor(rng.normal(0, 1e-5, sys_.n_dof))
    pairs = der.contact_list(sys_, q)
    assert len(pairs) > 20
    R = lambda qq: der.residual(sys_, qq, st, d["dt"], kap, pairs)
    J = torch.func.jacfwd(R)(q)
    h = 1e-7
    for k in rng.choice(sys_.n_dof, 12, replace=False):
        e = torch.zeros(sys_.n_dof, dtype=torch.float64)
        e[k] = h
        fd = (R(q + e) - R(q - e)) / (2 * h)
        assert float((fd - J[:, k]).abs().max()) <= 1e-5 * float(J.abs().max())


def test_contact_acts_only_where_turns_touch():
    d = coil(squeeze=0.9)
    sys_, st = der.build(d)
    with_c, _ = der.step(sys_, st, d["dt"])
    d0 = coil(squeeze=0.9)
    d0.pop("self_contact")
    sys0, st0 = der.build(d0)
    without, _ = der.step(sys0, st0, d0["dt"])
    assert float((with_c.x - without.x).abs().max()) > 1e-9
    s = W.straight_nodes(30, 0.3)
    ds = W.desc([W.rod(s, 4e-3, 1e6)], dt=1e-3, steps=1)
    ds["self_contact"] = d["self_contact"]
    sa, sta = der.build(ds)
    ds.pop("self_contact")
    sb, stb = der.build(ds)
    a, _ = der.step(sa, sta, ds["dt"])
    b, _ = der.step(sb, stb, ds["dt"])
    assert torch.equal(a.x, b.x)
