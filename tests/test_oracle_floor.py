"""Pins of the oracle's rounding-floor rule (Newton on Eq. 15 with the Jacobian of Eq. 16).

The FP64 residual of a stiff rod cannot be driven to 1e-9: a free position can only be
placed to within eps |x| of the root, and the stretch stiffness EA / ebar amplifies that.
The oracle estimates that floor as eps || |J| s ||_2 (s: the step-start magnitude of each
DOF kind) and accepts a step that has stopped improving at or below it.  These tests check
that the estimate really is a floor (the iteration cannot get under it and does not move
once there), that it is not used where the tolerance is reachable, and that it follows the
rod's distance from the origin, as rounding does."""
import numpy as np
import torch

import workloads as W
from oracle import der


def stiff_rod(offset=0.0, n=400, E=1e8, h=5e-3):
    x = W.straight_nodes(n, 0.5, origin=(offset, 0.0, 0.0))
    rng = np.random.Generator(np.random.PCG64(7))
    kb = rng.normal(0.0, 2.0, size=(n - 2, 2))
    return W.desc([W.rod(x, h, E, kbar=kb)], dt=1e-3, steps=1)


def newton_history(d, iters=14):
    """Residual norms of plain Newton iterations (no stopping rule) and the floor estimate."""
    sys, st = der.build(d)
    kap = der.natural_curvature(sys, st.time + d["dt"])
    free = ~sys.fixed
    jac = torch.func.jacfwd(lambda qq: der.residual(sys, qq, st, d["dt"], kap))
    q = der.pack(st.x, st.theta).clone()
    sc = der.floor_scales(sys, st)[free]
    hist, fl = [], []
    for _ in range(iters):
        R = der.residual(sys, q, st, d["dt"], kap)
        J = jac(q)[free][:, free]
        hist.append(float(torch.linalg.norm(R[free])))
        fl.append(der.rounding_floor(J, sc, 1.0))
        q[free] = q[free] - torch.linalg.solve(J, R[free])
    return hist, fl


def test_stiff_rod_cannot_reach_tolerance_and_ends_at_its_floor():
    d = stiff_rod()
    hist, fl = newton_history(d)
    tail = hist[6:]
    assert min(tail) > 1e-9                      # the tolerance is below the rounding floor
    assert max(tail) < 4 * min(tail)             # the iteration no longer moves
    assert all(h <= f for h, f in zip(tail, fl[6:]))   # and stays under the estimate
    sys, st = der.build(d)
    st1, info = der.step(sys, st, d["dt"], d["tol"], d["max_iter"])
    assert info.converged and info.at_floor and info.residual <= info.floor
    assert info.residual > 1e-9 and info.iters <= 8


def test_floor_rule_is_idle_where_the_tolerance_is_reachable():
    d = stiff_rod(n=40, E=1e6, h=1e-3)
    hist, fl = newton_history(d, iters=8)
    assert fl[-1] < 1e-11 and min(hist) < 1e-11
    sys, st = der.build(d)
    _, info = der.step(sys, st, d["dt"], d["tol"], d["max_iter"])
    assert info.converged and not info.at_floor and info.residual <= 1e-9


def test_floor_follows_distance_from_origin():
    near = stiff_rod(n=120)
    far = stiff_rod(offset=1000.0, n=120)
    hn, fn = newton_history(near, iters=10)
    hf, ff = newton_history(far, iters=10)
    # positions near 1000 m round 1000 / 0.5 times coarser than positions within 0.5 m
    assert 1000 < ff[-1] / fn[-1] < 3000
    assert min(hf[5:]) > 10 * min(hn[5:])
    sys, st = der.build(far)
    _, info = der.step(sys, st, far["dt"], far["tol"], far["max_iter"])
    assert info.converged and info.at_floor and info.residual <= info.floor


def test_floor_rule_off_leaves_stiff_rod_unconverged():
    d = stiff_rod()
    sys, st = der.build(d)
    q, info = der.newton_solve(sys, st, d["dt"], der.natural_curvature(sys, d["dt"]), d["tol"], 12,
                               floor_factor=0.0)
    assert not info.converged
