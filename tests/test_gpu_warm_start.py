"""The learned warm start on the GPU: trained by the library's own kernels on trajectories the
solver generates, then used as the Newton initial guess on fresh rods.  The plain Newton
solve stays the convergence judge (same 1e-9 residual) and the fallback.

Solutions reached from different initial guesses agree to the Newton tolerance: a residual
of 1e-9 N leaves a position error of at most ~1e-9 / (m / dt^2) ~ 1e-10 m here, so positions
are compared to 1e-8 relative."""
import os

import numpy as np
import pytest

import workloads as W

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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run(dm, d, steps, net=None, mode=0):
    sim = dm.sim_from_description(d)
    sim.set_warm_start(net, mode)
    st = sim.step(d["dt"], steps)
    assert (st["status"] == 0).all() and (st["steps"] == steps).all()
    return sim.state()[0], st


@pytest.fixture(scope="module")
def trained(dm):
    """A network trained on 200 steps (every second one) of 96 rods of the 1024-rod training
    batch (seed 0)."""
    from paper_2311_18126_amd import warm_start as WS
    d = W.subset(W.rod_batch(1024), list(range(96)))
    sim = dm.sim_from_description(d)
    F, T = WS.collect(sim, d["dt"], 200, every=2)
    net = dm.Mlp(max_rows=200_000)
    net.set_params(WS.init_params(0))
    hist = WS.train(net, F, T, epochs=6, batch=4096, lr=1e-3)
    hist += WS.train(net, F, T, epochs=4, batch=4096, lr=3e-4)
    say(f"training loss per epoch: {[f'{h:.3e}' for h in hist]}")
    assert hist[-1] < 0.8 * hist[0]
    return net


def test_explicit_predictor_gives_the_same_solution(dm):
    d = W.warm_start_eval(32, steps=10)
    x0, s0 = run(dm, d, 10)
    x1, s1 = run(dm, d, 10, mode=1)
    assert rel(x1, x0) < 1e-8
    say(f"iterations plain {s0['iters'].sum()} explicit predictor {s1['iters'].sum()}")


@pytest.fixture(scope="module")
def iterations(dm, trained):
    """Fresh rods (N ~ U{50..400}, seed 3), 60 steps from rest: Newton iterations per step of
    the plain step, the analytic predictors and the network on top of the third-order
    extrapolation, all at the same residual."""
    d = W.warm_start_eval(64, steps=60)
    x0, s0 = run(dm, d, 60)
    out = {"plain": s0}
    for name, mode in (("explicit", 1), ("second_order", 3), ("third_order", 4)):
        out[name] = run(dm, d, 60, mode=mode)[1]
    x2, out["network"] = run(dm, d, 60, net=trained, mode=2)
    assert rel(x2, x0) < 1e-8
    it = {k: s["iters"].sum() / s["iters"].size / 60 for k, s in out.items()}
    say("Newton iterations per step: " + ", ".join(f"{k} {v:.3f}" for k, v in it.items())
        + f"; network fallbacks {out['network']['fallbacks'].sum()}")
    return it, out


def test_trained_network_cuts_newton_iterations_on_fresh_rods(dm, iterations):
    it, out = iterations
    assert it["network"] < 0.95 * it["plain"]
    assert out["network"]["fallbacks"].sum() == 0


@pytest.mark.xfail(strict=False, reason=(
    "measured on MI355X: the network and the analytic extrapolations take the same Newton "
    "iterations per step (1024 fresh rods, 1000 steps, network trained streamed on 1.0e6 "
    "rod-steps of the rod batch: second order 2.199, third order 2.197, network 2.204, plain "
    "3.021); in the oracle even the exact end-of-step positions as the guess leave 2 "
    "iterations, so a position guess cannot cut the count by 10 %"))
def test_network_beats_the_extrapolation_by_a_tenth(dm, iterations):
    it, _ = iterations
    assert it["network"] <= 0.9 * it["second_order"]


def test_a_failing_guess_falls_back_to_the_plain_solve(dm):
    """A guess metres off the solution, with the warm-started attempt allowed two Newton
    iterations: every warm-started solve fails, and every step must still reach the plain
    solution through the fallback."""
    from paper_2311_18126_amd import warm_start as WS
    net = dm.Mlp(max_rows=20_000)
    net.set_params(WS.init_params(1))     # untrained: metre-scale, node-to-node random guesses
    net.set_normalisation(np.zeros(dm.NET_IN), np.ones(dm.NET_IN), np.full(3, 1.0))
    d = W.warm_start_eval(8, steps=3)
    x0, _ = run(dm, d, 3)
    sim = dm.sim_from_description(d, warm_max_iter=2)
    sim.set_warm_start(net, 2)
    st = sim.step(d["dt"], 3)
    assert (st["status"] == 0).all()
    say(f"fallbacks {st['fallbacks'].sum()} of {st.size * 3} steps")
    assert (st["fallbacks"] == 3).all()
    assert rel(sim.state()[0], x0) < 1e-8
