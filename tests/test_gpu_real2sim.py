"""GPU Real2Sim fit (Real2Sim section: Alg. 1, Eq. 19-21) against the oracle's
(tests/golden/real2sim.npz, written by the oracle only): the limb curvature readout (Eq. 5) and
its equilibrium gradient on a joined two-limb manipulator, and the whole fit (per-configuration
step-size control, stopping, kbar carried over) for one robot inside a batch of robots fitted at
once.  Tolerances: the quasi-static solve stops at a Newton residual of 1e-9, so curvatures agree
to ~1e-10 and gradients to ~1e-9; the fit's decisions have margins above 3e-7 in the golden."""
import os

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def dm():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2311_18126_amd as m
    assert os.path.exists(m.LIB_PATH), "libdmrod.so is not built"
    return m


def set_limb_kbar(sim, d, kv):
    """Uniform natural curvature kv[r] (first component) on every interior stencil of rod r."""
    sim.set_natural_curvature_all(np.concatenate(
        [np.stack([np.full(r["x0"].shape[0] - 2, k), np.zeros(r["x0"].shape[0] - 2)], 1).reshape(-1)
         for r, k in zip(d["rods"], kv)]))


def test_limb_curvature_and_gradient_match_oracle(dm):
    g = np.load(os.path.join(GOLD, "real2sim.npz"))
    d = W.two_limb_manipulator(limb_nodes=8, radius=0.01)
    print("case: two-limb manipulator settled at kbar (1.7, -0.8)", flush=True)
    sim = dm.sim_from_description(d, line_search=True)
    set_limb_kbar(sim, d, g["settled_kbar"])
    st = sim.step(d["dt"], d["steps"])
    assert st["status"][0] == 0
    kap = sim.limb_curvatures()
    assert np.abs(kap - g["settled_kappa"]).max() < 1e-9 * np.abs(g["settled_kappa"]).max(), (kap, g["settled_kappa"])
    for i, w in enumerate(([1.0, 0.0], [0.0, 1.0])):
        grad = sim.limb_curvature_gradient(d["dt"], np.array(w))
        ref = g[f"grad_{i}"]
        assert np.abs(grad - ref).max() < 1e-7 * np.abs(ref).max(), (i, grad, ref)


def test_fit_matches_oracle_fit_inside_a_batch(dm):
    """64 robots fitted at once, robot 0 on the golden's targets and the others on perturbed
    ones (each system keeps its own step size and stopping): robot 0's fitted natural
    curvatures, gradient-step counts and last losses against the oracle's fit."""
    g = np.load(os.path.join(GOLD, "real2sim.npz"))
    n_rob = 64
    d = W.two_limb_manipulator(n_robots=n_rob, limb_nodes=8, radius=0.01)
    rng = np.random.Generator(np.random.PCG64(17))
    tg = np.repeat(g["targets"][:, None, :], n_rob, axis=1)
    tg[:, 1:, :] += rng.normal(0.0, 0.05, size=(tg.shape[0], n_rob - 1, 2))
    print(f"case: Real2Sim fit, {n_rob} robots, {tg.shape[0]} configurations", flush=True)
    sim = dm.sim_from_description(d, line_search=True)
    assert sim.num_systems == n_rob
    traj, steps, losses = sim.fit_limb_curvatures(d["dt"], d["steps"], tg.reshape(tg.shape[0], -1),
                                                  tol=float(g["tol"]), max_iter=int(g["max_iter"]))
    assert np.array_equal(steps[:, 0], g["steps"]), (steps[:, 0], g["steps"])
    assert np.abs(traj[:, :2] - g["traj"]).max() < 1e-8, (traj[:, :2], g["traj"])
    # the loss that ended each configuration (the oracle's evaluations, configuration by configuration)
    ends = np.cumsum(g["steps"] + 1) - 1
    assert np.abs(losses[:, 0] - g["losses"][ends]).max() < 1e-10
    # every robot reached the tolerance or the iteration cap; most reach the tolerance
    assert ((losses < float(g["tol"])) | (steps == int(g["max_iter"]))).all()
    assert (losses < float(g["tol"])).mean() > 0.9


def test_fit_rejects_unsupported_setups(dm):
    d = W.two_limb_manipulator(limb_nodes=8, radius=0.01)
    d["rods"][0]["actuation"] = (1.0, 1.0, 0.0)
    sim = dm.sim_from_description(d, line_search=True)
    with pytest.raises(dm.DmError) as e:
        sim.limb_curvature_gradient(d["dt"], np.array([1.0, 0.0]))
    assert e.value.status == dm.DM_ERR_UNSUPPORTED
    with pytest.raises(ValueError):
        sim.fit_limb_curvatures(d["dt"], 1, np.zeros((2, 3)))
