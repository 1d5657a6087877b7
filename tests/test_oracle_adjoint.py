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


# ---------------------------------------------------------------------------
# Real2Sim-style fit (Alg. 1 control flow with the adjoint gradient)
# ---------------------------------------------------------------------------

def test_fit_stops_at_once_on_the_target_and_halves_the_step_after_a_rise():
    d, kstar = W.adjoint_rods(n_rods=1, n_nodes=8, steps=6)
    _, _, target = AD.rollout(d, [kstar[0]])
    ks, losses, alphas = AD.fit_natural_curvature(d, target.numpy(), [kstar[0]], 1.0, 1e-20, 5)
    assert losses == [0.0] and alphas == [] and len(ks) == 1
    # an oversized first step overshoots: the loss rises and the step size halves from then on
    k0 = [np.zeros((6, 2))]
    ks, losses, alphas = AD.fit_natural_curvature(d, target.numpy(), k0, 2.5e10, 0.0, 6)
    assert len(losses) == 7 and len(alphas) == 6
    assert alphas[0] == 2.5e10
    for i in range(1, 6):
        assert alphas[i] == alphas[i - 1] * (0.5 if losses[i] > losses[i - 1] else 1.0)
    assert any(losses[i] > losses[i - 1] for i in range(1, 6))
    # every step is kbar <- kbar - alpha grad at the evaluated iterate
    for i in range(6):
        _, g, _ = AD.loss_and_grad(d, ks[i], target.numpy())
        assert np.allclose(ks[i + 1][0].numpy(), ks[i][0].numpy() - alphas[i] * g[0].numpy(), rtol=0, atol=1e-12)
