"""Pins of the oracle's Real2Sim fit (Real2Sim section: Alg. 1, Eq. 19-21) on the joined
two-limb manipulator: the equilibrium gradient against central differences of re-settled
configurations (the paper's finite-difference route of Eq. 20, made central), the stress-free
case without gravity (a limb's curvature by Eq. 5 is then exactly its natural curvature), and
the recovery of known natural curvatures from the target curvatures they produce."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import der
from oracle import real2sim as RS


@pytest.fixture(autouse=True)
def _threads():
    torch.set_num_threads(4)


def manipulator(gravity=True, limb_nodes=8, radius=0.01):
    d = W.two_limb_manipulator(limb_nodes=limb_nodes, radius=radius)
    if not gravity:
        d["gravity"] = (0.0, 0.0, 0.0)
    return d


def test_gradient_matches_central_differences_of_resettled_equilibria():
    d = manipulator()
    sys_, st = der.build(d)
    kv = torch.tensor([1.7, -0.8], dtype=der.DT)
    st = RS.settle(sys_, st, kv, d["dt"], d["steps"])
    for w in ([1.0, 0.0], [0.0, 1.0], [-1.0, 1.0]):
        g = RS.curvature_gradient(sys_, st, kv, torch.tensor(w, dtype=der.DT), d["dt"]).numpy()
        fd = np.zeros(2)
        h = 1e-5
        for k in range(2):
            e = torch.zeros(2, dtype=der.DT)
            e[k] = h
            kp = RS.limb_curvatures(sys_, *(lambda s: (s.x, s.theta, s))(RS.settle(sys_, st, kv + e, d["dt"], 1, tol=1e-13)))
            km = RS.limb_curvatures(sys_, *(lambda s: (s.x, s.theta, s))(RS.settle(sys_, st, kv - e, d["dt"], 1, tol=1e-13)))
            fd[k] = float((torch.tensor(w, dtype=der.DT) * (kp - km)).sum()) / (2 * h)
        assert np.abs(g - fd).max() <= 1e-7 * np.abs(fd).max(), (w, g, fd)
    # gravity couples the limbs: the upper limb's curvature moves with the lower limb's kbar
    g = RS.curvature_gradient(sys_, st, kv, torch.tensor([1.0, 0.0], dtype=der.DT), d["dt"]).numpy()
    assert 0.5 < g[0] < 1.0 and abs(g[1]) > 1e-3


def test_without_gravity_limb_curvature_equals_natural_curvature():
    """Stress-free: every limb stencil sits at its natural curvature and the joint stencil at
    its straight rest shape, so Eq. 5's curvature over the Voronoi length is kbar exactly."""
    d = manipulator(gravity=False)
    sys_, st = der.build(d)
    kv = torch.tensor([2.5, -1.5], dtype=der.DT)
    st = RS.settle(sys_, st, kv, d["dt"], d["steps"], tol=1e-12)
    kap = RS.limb_curvatures(sys_, st.x, st.theta, st)
    assert torch.allclose(kap, kv, rtol=0, atol=1e-9), kap
    # the fit to stress-free targets lands on them
    targets = np.array([[0.4, -0.3], [0.55, -0.1]])
    traj, losses, steps, _ = RS.solve_natural_curvatures(d, targets, tol=1e-4, max_iter=100)
    assert losses[-1] < 1e-4 and np.abs(traj.numpy() - targets).max() < 1e-4
    # alpha = 0.1 with |grad| = 1 per limb moves kbar by 0.1 per step before the first overshoot
    assert steps[0] >= 4


def test_fit_recovers_the_natural_curvatures_that_produced_the_targets():
    d = manipulator()
    kstar = np.array([[0.6, -0.4], [0.75, -0.25], [0.8, 0.0]])
    targets = RS.curvatures_at(d, kstar).numpy()
    # gravity makes the targets differ from the natural curvatures that produced them
    assert np.abs(targets - kstar).max() > 1e-2
    traj, losses, steps, _ = RS.solve_natural_curvatures(d, targets, tol=1e-5, max_iter=150)
    assert all(s < 150 for s in steps), steps
    # the loss is below the tolerance at the end of every configuration, and the slope of the
    # curvature in kbar (about 0.9, from the gradient test) bounds the distance to kstar
    assert np.abs(traj.numpy() - kstar).max() < 3e-5, traj
