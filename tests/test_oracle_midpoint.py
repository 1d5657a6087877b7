"""Pins of the oracle's implicit-midpoint step (the alternative implicit scheme of the
time-stepping subsection) against what the mathematics fixes.

A rod of one edge moving along its own axis is a linear oscillator (the stretch energy of
Eq. 2-3 is quadratic in the edge length), so the midpoint rule reduces to the trapezoidal
rule of the linear system, whose one-step map is a 2 x 2 linear solve written here from the
rule itself (with damping and a constant axial load it stays affine).  On a free bent rod the
rule conserves linear momentum, and on a bent rod under gravity its error is second order in
dt.  A dropped factor, the force taken at the end instead of the midpoint, or the
backward-Euler velocity update each fail one of these.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import der


def T(a):
    return torch.as_tensor(np.asarray(a), dtype=torch.float64)


@pytest.mark.parametrize("eta,g", [(0.0, 0.0), (3.0, 4.0)])
def test_axial_oscillator_follows_the_trapezoidal_map(eta, g):
    L, dt = 0.05, 2e-4
    d = W.desc([W.rod(W.straight_nodes(2, L), 1e-3, 1e7, fixed_nodes=(0,), fixed_edges=(0,))],
               dt=dt, steps=1, gravity=(g, 0.0, 0.0), damping=eta)
    sys, st = der.build(d)
    u0, v0 = 2e-4, -0.3
    st.x[1, 0] = L + u0
    st.v[1, 0] = v0
    k = float(sys.EA[0] / sys.ebar[0])
    m = float(sys.mass[1])
    # u'' = -(k/m) u - eta u' + g as z' = A z + b, z = (u, u'); trapezoidal rule:
    # (I - dt A / 2) z_{n+1} = (I + dt A / 2) z_n + dt b
    A = np.array([[0.0, 1.0], [-k / m, -eta]])
    b = np.array([0.0, g])
    P, Q = np.eye(2) - 0.5 * dt * A, np.eye(2) + 0.5 * dt * A
    z = np.array([u0, v0])
    period = 2 * math.pi / math.sqrt(k / m)
    for n in range(int(1.5 * period / dt)):
        st, info = der.step(sys, st, dt, 1e-12, 50, polish=1, scheme="midpoint")
        assert info.converged
        z = np.linalg.solve(P, Q @ z + dt * b)
        assert abs(float(st.x[1, 0]) - L - z[0]) <= 1e-12 * L, n
        assert abs(float(st.v[1, 0]) - z[1]) <= 1e-9 * abs(v0) + 1e-12, n
        assert float(st.x[1, 1:].abs().max()) == 0.0 and float(st.theta.abs().max()) == 0.0


def test_trapezoidal_energy_of_the_undamped_oscillator_is_exact():
    """Without damping or load the discrete energy m v^2 / 2 + k u^2 / 2 is conserved (the map
    above is a Cayley transform of a skew matrix in energy coordinates), while backward Euler
    loses energy every step."""
    L, dt = 0.05, 5e-4
    d = W.desc([W.rod(W.straight_nodes(2, L), 1e-3, 1e7, fixed_nodes=(0,), fixed_edges=(0,))],
               dt=dt, steps=1, gravity=(0.0, 0.0, 0.0))
    sys, st0 = der.build(d)
    st0.x[1, 0] = L + 3e-4
    k = float(sys.EA[0] / sys.ebar[0])
    m = float(sys.mass[1])

    def energy(s):
        return 0.5 * m * float(s.v[1, 0]) ** 2 + 0.5 * k * (float(s.x[1, 0]) - L) ** 2
    e0 = energy(st0)
    for scheme in ("midpoint", "euler"):
        st = st0.clone()
        for _ in range(40):
            st, info = der.step(sys, st, dt, 1e-12, 50, polish=1, scheme=scheme)
            assert info.converged
        rel = abs(energy(st) - e0) / e0
        if scheme == "midpoint":
            assert rel < 1e-9, rel
        else:
            assert energy(st) < 0.99 * e0


def test_midpoint_conserves_linear_momentum_of_a_free_bent_rod():
    rng = np.random.Generator(np.random.PCG64(7))
    n = 12
    kb = rng.normal(0, 3.0, size=(n - 2, 2))
    d = W.desc([W.rod(W.helix_nodes(n, 0.05, 0.05, 0.5), 2e-3, 1e6, kbar=kb, fixed_nodes=(), fixed_edges=())],
               dt=1e-3, steps=1, gravity=(0, 0, 0))
    sys, st = der.build(d)
    st.v = T(rng.normal(0, 0.5, size=(n, 3)))
    st.omega = T(rng.normal(0, 5.0, size=n - 1))
    p0 = (sys.mass[:, None] * st.v).sum(0)
    for _ in range(5):
        st, info = der.step(sys, st, d["dt"], 1e-9, 50, scheme="midpoint")
        assert info.converged
        p1 = (sys.mass[:, None] * st.v).sum(0)
        assert float((p1 - p0).abs().max()) <= d["dt"] * math.sqrt(3 * n) * 1e-9
        p0 = p1


def test_midpoint_is_second_order_on_a_bent_rod():
    """On a clamped, bent rod under gravity the end-state error against a fine midpoint run
    falls about four times per halving of dt (second order); backward Euler's falls about twice.
    (The step is not exactly time-symmetric: the frames' time-parallel transport starts from
    the step-start tangents, so the elastic force's dependence on the tangent differs between a
    step and its reverse even where their midpoint frames agree.)"""
    rng = np.random.Generator(np.random.PCG64(8))
    n = 12
    kb = rng.normal(0, 2.0, size=(n - 2, 2))
    d = W.desc([W.rod(W.straight_nodes(n, 0.4), 2e-3, 2e6, kbar=kb)], dt=2e-3, steps=1)
    t_end = 0.016

    def run(k, scheme):
        sys, st = der.build(d)
        for _ in range(k):
            st, info = der.step(sys, st, t_end / k, 1e-12, 50, polish=1, scheme=scheme)
            assert info.converged
        return st.x.numpy().copy()
    ref = run(128, "midpoint")
    e = [float(np.abs(run(k, "midpoint") - ref).max()) for k in (8, 16, 32)]
    assert e[0] / e[1] > 3.2 and e[1] / e[2] > 3.2, e
    eb = [float(np.abs(run(k, "euler") - ref).max()) for k in (8, 16)]
    assert 1.6 < eb[0] / eb[1] < 2.4, eb
