"""Batching machinery on the GPU: the captured per-step graph of warm-started stepping
(checked replay by replay against eager launches, with the program's own work and
synchronisation between replays) and the workgroup-size autotuner."""
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


def trajectories(dm, d, use_graphs, mode, net=None, stream=None, calls=(3, 1, 4)):
    sim = dm.sim_from_description(d, use_graphs=use_graphs, stream=stream)
    sim.set_warm_start(net, mode)
    out = []
    for k in calls:
        st = sim.step(d["dt"], k)
        assert (st["status"] == 0).all()
        out.append((sim.state(), st["iters"].copy(), st["fallbacks"].copy()))
        x, th, v, om = sim.state()            # eager work between replays
        sim.set_state(x=x, theta=th, v=v, theta_dot=om)
    return out


@pytest.mark.parametrize("mode", [1, 3])
def test_graph_replays_match_eager_launches(dm, mode):
    d = W.warm_start_eval(24, steps=8)
    say(f"case: warm mode {mode}, 24 rods, 3 calls")
    a = trajectories(dm, d, False, mode)
    b = trajectories(dm, d, True, mode)
    for (sa, ia, fa), (sb, ib, fb) in zip(a, b):
        for u, w in zip(sa, sb):
            assert np.array_equal(u, w)
        assert np.array_equal(ia, ib) and np.array_equal(fa, fb)


def test_graph_with_the_network_on_a_torch_stream(dm):
    import torch
    from paper_2311_18126_amd import warm_start as WS
    d = W.warm_start_eval(16, steps=6)
    net = dm.Mlp(max_rows=10_000)
    net.set_params(WS.init_params(3) * np.float32(1e-3))     # small corrections
    net.set_normalisation(np.zeros(20), np.ones(20), np.full(3, 1e-6))
    s = torch.cuda.Stream()
    a = trajectories(dm, d, False, 2, net=net, stream=s.cuda_stream)
    b = trajectories(dm, d, True, 2, net=net, stream=s.cuda_stream)
    for (sa, ia, _), (sb, ib, _) in zip(a, b):
        for u, w in zip(sa, sb):
            assert np.array_equal(u, w)
        assert np.array_equal(ia, ib)


def test_autotuner_picks_a_size_restores_the_state_and_caches(dm, tmp_path):
    d = W.rod_batch(64, seed=6, nmax=200)
    sim = dm.sim_from_description(d)
    sim.step(d["dt"], 2)
    before = sim.state()
    cache = str(tmp_path / "tune.txt")
    b = sim.autotune(d["dt"], trial_steps=2, cache=cache)
    say(f"autotuned block size {b}")
    assert b in (64, 128, 256, 512) and sim.block_size == b
    after = sim.state()
    for u, w in zip(before, after):
        assert np.array_equal(u, w)
    with open(cache) as f:
        lines = f.read().splitlines()
    assert len(lines) == 1 and lines[0].endswith(f" {b}")
    sim2 = dm.sim_from_description(d)
    assert sim2.autotune(d["dt"], trial_steps=2, cache=cache) == b    # served from the cache
    with open(cache) as f:
        assert len(f.read().splitlines()) == 1
    # stepping after tuning reaches the untuned trajectory to the Newton tolerance (the
    # workgroup size changes the summation order of the residual norm, nothing else)
    sim.step(d["dt"], 3)
    ref = dm.sim_from_description(d)
    ref.step(d["dt"], 5)
    x, xr = sim.state()[0], ref.state()[0]
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)
