"""Pins of the oracle's discrete adjoint: brute-force central differences of the oracle's
forward trajectory for every natural-curvature parameter of tiny rods (the forward pass
shares no code with the adjoint algebra), plus the exact zero at the target."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint as AD


def _fd_all(desc, k0, tgt, h=1e-6):
    fd = np.zeros_like(k0[0])
    for i in range(fd.shape[0]):
        for c in range(2):
            kp = [k0[0].copy()]
            kp[0][i, c] += h
            km = [k0[0].copy()]
            km[0][i, c] -= h
            Lp = AD.tip_loss(AD.rollout(desc, kp)[2], tgt)[0]
            Lm = AD.tip_loss(AD.rollout(desc, km)[2], tgt)[0]
            fd[i, c] = (Lp - Lm) / (2 * h)
    return fd


@pytest.fixture(autouse=True)
def _threads():
    torch.set_num_threads(4)


def test_adjoint_matches_central_differences_clamped_rod_under_gravity():
    rng = np.random.Generator(np.random.PCG64(5))
    n = 6
    d = W.desc([W.rod(W.straight_nodes(n, 0.2), 1e-3, 1e6, kbar=np.zeros((n - 2, 2)))], dt=2e-3, steps=10)
    _, _, tgt = AD.rollout(d, [rng.normal(0, 2.0, size=(n - 2, 2))])
    k0 = [rng.normal(0, 1.0, size=(n - 2, 2))]
    L, g, _ = AD.loss_and_grad(d, k0, tgt)
    assert L > 0
    fd = _fd_all(d, k0, tgt)
    assert np.abs(g[0].numpy() - fd).max() <= 1e-6 * np.abs(fd).max()


def test_adjoint_matches_central_differences_free_helix_with_damping():
    """Twist-bend coupling (helical rest shape, nonzero reference twist), damping, a free
    end moving fast enough that the frames turn appreciably over the steps."""
    rng = np.random.Generator(np.random.PCG64(6))
    n = 7
    r = W.rod(W.helix_nodes(n, 0.02, 0.04, 0.15), 1e-3, 2e5, kbar=np.zeros((n - 2, 2)),
              fixed_nodes=(0, 1), fixed_edges=(0,))
    d = W.desc([r], dt=4e-3, steps=8, damping=2.0)
    _, _, tgt = AD.rollout(d, [rng.normal(0, 3.0, size=(n - 2, 2))])
    k0 = [rng.normal(0, 3.0, size=(n - 2, 2))]
    L, g, _ = AD.loss_and_grad(d, k0, tgt)
    fd = _fd_all(d, k0, tgt)
    assert np.abs(g[0].numpy() - fd).max() <= 1e-6 * np.abs(fd).max()
    # every parameter matters here, so a dropped term would show
    assert (np.abs(fd) > 1e-4 * np.abs(fd).max()).sum() >= fd.size - 2


def test_adjoint_gradient_vanishes_at_the_target():
    rng = np.random.Generator(np.random.PCG64(7))
    n = 6
    d = W.desc([W.rod(W.straight_nodes(n, 0.2), 1e-3, 1e6, kbar=np.zeros((n - 2, 2)))], dt=2e-3, steps=4)
    ks = [rng.normal(0, 2.0, size=(n - 2, 2))]
    _, _, tgt = AD.rollout(d, ks)
    L, g, _ = AD.loss_and_grad(d, ks, tgt)
    assert L == 0.0
    assert float(g[0].abs().max()) == 0.0
