"""Batching machinery on the GPU: trajectory segments captured as HIP graphs (rollout and the
adjoint's recomputation; checked replay by replay against eager launches, with the program's
own work and synchronisation between replays) and the workgroup-size autotuner."""
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


def rollouts(dm, d, use_graphs, mode=0, net=None, stream=None, calls=((7, 3), (5, 5), (6, 4))):
    """Rollouts (nsteps, ckpt_every) in a row from the same sim; each returns its tips and the
    state after it, with the program's own eager work (a state round trip) in between."""
    sim = dm.sim_from_description(d, use_graphs=use_graphs, stream=stream)
    sim.set_warm_start(net, mode)
    out = []
    for n, c in calls:
        tips = sim.rollout(d["dt"], n, ckpt_every=c)
        out.append((tips.copy(), sim.state()))
        x, th, v, om = sim.state()            # eager work between replays
        sim.set_state(x=x, theta=th, v=v, theta_dot=om)
    return out


@pytest.mark.parametrize("mode", [0, 3])
def test_captured_segments_match_eager_launches(dm, mode):
    """Rollout segments replayed from captured graphs (each segment length captured once and
    replayed for every later segment of that length) against eager launches, bit for bit."""
    d = W.adjoint_rods(12, 30, steps=20)[0]
    say(f"case: rollout segments, warm mode {mode}, 12 rods")
    a = rollouts(dm, d, False, mode)
    b = rollouts(dm, d, True, mode)
    for (ta, sa), (tb, sb) in zip(a, b):
        assert np.array_equal(ta, tb)
        for u, w in zip(sa, sb):
            assert np.array_equal(u, w)


def test_captured_segments_with_the_network_on_a_torch_stream(dm):
    import torch
    from paper_2311_18126_amd import warm_start as WS
    d = W.adjoint_rods(8, 40, steps=12)[0]
    net = dm.Mlp(max_rows=64)
    net.set_params(WS.init_params(3) * np.float32(1e-3))     # small corrections
    net.set_normalisation(np.zeros(dm.NET_IN), np.ones(dm.NET_IN), np.full(3, 1e-6))
    s = torch.cuda.Stream()
    a = rollouts(dm, d, False, 2, net=net, stream=s.cuda_stream)
    b = rollouts(dm, d, True, 2, net=net, stream=s.cuda_stream)
    for (ta, sa), (tb, sb) in zip(a, b):
        assert np.array_equal(ta, tb)
        for u, w in zip(sa, sb):
            assert np.array_equal(u, w)


def test_adjoint_recomputation_from_captured_segments_matches_eager(dm):
    d, kstar = W.adjoint_rods(6, 30, steps=25)
    grads = []
    for graphs in (False, True):
        sim = dm.sim_from_description(d, use_graphs=graphs)
        tips = sim.rollout(d["dt"], 25, ckpt_every=10)
        g1 = sim.adjoint(2.0 * tips)
        g2 = sim.adjoint(2.0 * tips)             # second pass replays the captured segments
        assert np.array_equal(g1, g2)
        grads.append(g1)
    assert np.array_equal(grads[0], grads[1])


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
