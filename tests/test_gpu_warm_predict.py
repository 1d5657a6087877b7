"""The step-start guess computed inside the step kernel (dm_ws_predict, the same device code
the step runs at every step start) against the oracle's features and network, and against
the library's own batch network kernels on the same features.

Tolerances: the analytic predictors are a few float64 operations (1e-13 relative).  The
network part follows the oracle to the bfloat16 tolerance of tests/test_gpu_mlp.py (1e-3
relative in norm), and the batch kernels bit for bit up to the float64 scaling of the output
(1e-12 relative): both run the same matrix-core products in the same order."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import mlp as OM

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2311_18126_amd as m
    assert os.path.exists(m.LIB_PATH), "libdmrod.so is not built"
    return m


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def case(dm):
    """Rods of 3..70 nodes (rows spanning several 16-row tiles and ragged tails) after four
    steps, with the velocities before the last two steps kept for the oracle's features."""
    d = W.rod_batch(7, seed=5, nmin=3, nmax=70)
    sim = dm.sim_from_description(d)
    sim.step(d["dt"], 2)
    vprev2 = [sim.rod_state(r)[2] for r in range(len(d["rods"]))]
    sim.step(d["dt"], 1)
    vprev = [sim.rod_state(r)[2] for r in range(len(d["rods"]))]
    sim.step(d["dt"], 1)
    feats, base = [], {1: [], 3: [], 4: []}
    for r, rd in enumerate(d["rods"]):
        x, _, v, _ = sim.rod_state(r)
        eb = np.linalg.norm(np.diff(rd["x0"], axis=0), axis=1)
        feats.append(OM.rod_features(x, v, vprev[r], vprev2[r], rd["kbar"], rd["E"], rd["radius"], eb))
        a, a_prev = v - vprev[r], vprev[r] - vprev2[r]
        base[1].append(d["dt"] * v)
        base[3].append(d["dt"] * (v + a))
        base[4].append(d["dt"] * (v + a + (a - a_prev)))
    return d, sim, np.concatenate(feats), {k: np.concatenate(b) for k, b in base.items()}


@pytest.mark.parametrize("mode", [1, 3, 4])
def test_analytic_predictors(dm, case, mode):
    d, sim, _, base = case
    sim.set_warm_start(None, mode)
    dx = sim.ws_predict(d["dt"])
    ref = base[mode]
    say(f"mode {mode}: {dx.shape[0]} rows")
    assert dx.shape == ref.shape
    assert np.allclose(dx, ref, rtol=1e-13, atol=1e-18)


def test_network_guess_matches_oracle_and_batch_kernels(dm, case):
    import torch
    d, sim, F, base = case
    b4 = base[4]
    p = OM.init_params(21)
    p["b1"][:] = np.random.Generator(np.random.PCG64(4)).normal(0, 0.1, 256)
    flat = np.concatenate([p[k].reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")]).astype(np.float32)
    mean, std = F.mean(0), F.std(0) + 1e-3
    scale = np.array([2e-5, 1e-5, 3e-5])
    net = dm.Mlp(max_rows=F.shape[0])
    net.set_params(flat)
    net.set_normalisation(mean, std, scale)
    sim.set_warm_start(net, 2)
    dx = sim.ws_predict(d["dt"])
    y_dev = (dx - b4) / scale
    y_ref, _ = OM.forward(p, OM.standardise(F, mean, std))
    rel = np.linalg.norm(y_dev - y_ref) / np.linalg.norm(y_ref)
    say(f"network guess vs oracle: relative error {rel:.2e} over {F.shape[0]} rows")
    assert rel < 1e-3
    # the batch kernels on the oracle's features: the same products in the same order
    Y = torch.empty((F.shape[0], 3), dtype=torch.float32, device="cuda")
    yb = net.forward(torch.tensor(F, device="cuda"), Y).cpu().numpy().astype(np.float64)
    assert np.abs((dx - b4) - scale * yb).max() <= 1e-12 * np.abs(dx).max()
    sim.set_warm_start(None, 0)


def test_midpoint_guess_is_of_the_midpoint_state(dm, case):
    """Under the implicit-midpoint integrator the Newton unknown is the midpoint state: the
    analytic part is taken over half the step, and so is the network's whole-step correction."""
    d, sim, F, base = case
    p = OM.init_params(22)
    flat = np.concatenate([p[k].reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")]).astype(np.float32)
    mean, std = F.mean(0), F.std(0) + 1e-3
    scale = np.array([2e-5, 1e-5, 3e-5])
    net = dm.Mlp(max_rows=F.shape[0])
    net.set_params(flat)
    net.set_normalisation(mean, std, scale)
    y_ref, _ = OM.forward(p, OM.standardise(F, mean, std))
    sim.set_integrator("midpoint")
    try:
        sim.set_warm_start(None, 4)
        assert np.allclose(sim.ws_predict(d["dt"]), 0.5 * base[4], rtol=1e-13, atol=1e-18)
        sim.set_warm_start(net, 2)
        dx = sim.ws_predict(d["dt"])
        y_dev = (dx - 0.5 * base[4]) / (0.5 * scale)
        rel = np.linalg.norm(y_dev - y_ref) / np.linalg.norm(y_ref)
        say(f"midpoint network guess vs oracle: relative error {rel:.2e}")
        assert rel < 1e-3
    finally:
        sim.set_integrator("euler")
        sim.set_warm_start(None, 0)


def test_predict_needs_a_warm_mode(dm, case):
    d, sim, _, _ = case
    sim.set_warm_start(None, 0)
    with pytest.raises(dm.DmError):
        sim.ws_predict(d["dt"])
