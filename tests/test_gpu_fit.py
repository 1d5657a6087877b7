"""GPU Real2Sim-style fit (dm_fit_natural_curvature: Alg. 1 control flow with the adjoint
gradient) against the oracle's fit stored by tests/golden/make_golden.py: the losses of every
iterate (1e-8 relative) and the fitted natural curvature (1e-6 relative) on two 20-node rods
over 30 steps from zero curvature; afterwards the sim is back at its starting state."""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def dm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2311_18126_amd as m
    assert os.path.exists(m.LIB_PATH), "libdmrod.so is not built"
    return m


def test_fit_matches_the_oracle_fit(dm):
    g = np.load(os.path.join(GOLD, "fit.npz"))
    d, _ = W.adjoint_rods(n_rods=2, n_nodes=20, steps=30)
    print("case: fit, 2 rods x 20 nodes x 30 steps, 4 gradient steps", flush=True)
    sim = dm.sim_from_description(d)
    x_start = sim.state()[0].copy()
    iters = int(g["iters"])
    kb, losses = sim.fit_natural_curvature(d["dt"], d["steps"], g["target_tips"], alpha0=float(g["alpha"]),
                                           tol=1e-12, max_iter=iters, ckpt_every=10)
    ref_losses = g["losses"]
    assert losses.shape == ref_losses.shape
    assert np.all(np.abs(losses - ref_losses) <= 1e-8 * ref_losses), (losses, ref_losses)
    assert losses[-1] < 0.5 * losses[0]
    ref_k = g[f"kbar_{iters}"].reshape(-1)
    assert np.linalg.norm(kb - ref_k) <= 1e-6 * np.linalg.norm(ref_k)
    assert np.array_equal(sim.state()[0], x_start)


def test_fit_rejects_bad_arguments(dm):
    d, _ = W.adjoint_rods(n_rods=1, n_nodes=8, steps=3)
    sim = dm.sim_from_description(d)
    with pytest.raises(dm.DmError):
        sim.fit_natural_curvature(d["dt"], 3, np.zeros((3, 1, 3)), alpha0=-1.0)
    sim.set_integrator("midpoint")
    with pytest.raises(dm.DmError):
        sim.fit_natural_curvature(d["dt"], 3, np.zeros((3, 1, 3)))
