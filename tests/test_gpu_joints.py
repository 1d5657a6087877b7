"""GPU parity for rods joined at an interior node (Elastic Joints subsection: a joint is a node
along a rod with other rods attached).  The library solves a rod joined at its interior node
k as two chains, nodes 0..k and k..N-1, meeting at the hub; the rod's own stencil at k keeps
its natural curvature, actuation and stiffness and is assembled into the hub's dense border
with the joint stencils of every other pair of hub edges.  The oracle builds the same joints
from the description alone (merged nodes, every pair of edges at the joint except a rod's own
consecutive edges).  Tolerances as for the stars: 1e-9 of the positions after one step, 1e-6
of the positions and of the displacement after ten."""
import numpy as np
import pytest

import workloads as W
from oracle import der
from parity import assert_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dm():
    import os
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2311_18126_amd as m
    assert os.path.exists(m.LIB_PATH), "libdmrod.so is not built"
    return m


def say(msg):
    print(msg, flush=True)


def along(n, length, origin, direction):
    return W.straight_nodes(n, length, origin, direction)


def tee(kbar=False, actuated=False):
    """Rod 0 along x (21 nodes, 0.4 m, clamped at its start); rod 1 (11 nodes, 0.2 m) leaves
    rod 0's node 10 along +y, and rod 2 (9 nodes) arrives at the same node from -z: a joint of
    degree four with rod 0 passing through it."""
    rng = np.random.Generator(np.random.PCG64(17))
    a = along(21, 0.4, (0.0, 0.0, 0.0), (1.0, 0.0, 0.0))
    hub = a[10]
    b = along(11, 0.2, hub, (0.0, 1.0, 0.0))
    c = along(9, 0.15, hub + np.array([0.0, 0.0, -0.15]), (0.0, 0.0, 1.0))
    r0 = W.rod(a, 3e-3, 2e6, density=1100.0, kbar=rng.normal(0.0, 2.0, (19, 2)) if kbar else None,
               actuation=(3.0, 1.5, 0.4) if actuated else None)
    r1 = W.rod(b, 2e-3, 5e6, density=1200.0, fixed_nodes=(), fixed_edges=())
    r2 = W.rod(c, 2.5e-3, 1e6, density=900.0, fixed_nodes=(), fixed_edges=())
    return W.desc([r0, r1, r2], dt=2e-3, steps=10, joints=[(0, 10, 1, 0), (0, 10, 2, 8)])


def cross():
    """Two rods crossing at their middle nodes (both joined at an interior node: four chains),
    the first clamped at its start, under gravity."""
    a = along(17, 0.32, (0.0, 0.0, 0.0), (1.0, 0.0, 0.0))
    b = along(17, 0.32, a[8] - np.array([0.0, 0.16, 0.0]), (0.0, 1.0, 0.0))
    r0 = W.rod(a, 2e-3, 3e6)
    r1 = W.rod(b, 2e-3, 3e6, fixed_nodes=(), fixed_edges=())
    return W.desc([r0, r1], dt=2e-3, steps=10, joints=[(0, 8, 1, 8)])


def positions(sim, n_rods):
    return np.concatenate([sim.rod_state(r)[0] for r in range(n_rods)])


def oracle_positions(sys_, st):
    return np.concatenate([der.rod_positions(sys_, st, k).numpy() for k in range(len(sys_.rod_nodes))])


@pytest.mark.parametrize("name,make", [("tee", lambda: tee()), ("tee with natural curvature", lambda: tee(kbar=True)),
                                       ("tee with actuation", lambda: tee(actuated=True)), ("cross", cross)])
def test_interior_joint_matches_live_oracle(dm, name, make):
    d = make()
    say(f"case: {name}")
    sim = dm.sim_from_description(d)
    assert sim.num_systems == 1
    sys_, st = der.build(d)
    x0 = oracle_positions(sys_, st)
    done = 0
    for k in (1, 10):
        for _ in range(k - done):
            st, info = der.step(sys_, st, d["dt"], d["tol"], d["max_iter"])
            assert info.converged
        s = sim.step(d["dt"], k - done)
        done = k
        assert s["status"][0] == 0
        assert_parity(positions(sim, len(d["rods"])), oracle_positions(sys_, st), x0,
                      1e-9 if k == 1 else 1e-6, 1e-6, f"{name} step {k}")
    # the joined nodes stay one node on the GPU side
    xs = [sim.rod_state(r)[0] for r in range(len(d["rods"]))]
    for (ra, na, rb, nb) in d["joints"]:
        assert np.array_equal(xs[ra][na], xs[rb][nb])


def test_two_joint_nodes_in_one_system_are_rejected(dm):
    """A chain of three rods joined at two different nodes would need a dense coupling between
    two borders: DM_ERR_UNSUPPORTED."""
    sim = dm.Sim()
    a = sim.add_rod(W.straight_nodes(5, 1.0), 1e-3, 1e7)
    b = sim.add_rod(W.straight_nodes(5, 1.0, (1.0, 0.0, 0.0)), 1e-3, 1e7)
    c = sim.add_rod(W.straight_nodes(5, 1.0, (2.0, 0.0, 0.0)), 1e-3, 1e7)
    sim.add_joint(a, 4, b, 0)
    sim.add_joint(b, 4, c, 0)
    with pytest.raises(dm.DmError) as e:
        sim.finalize()
    assert e.value.status == dm.DM_ERR_UNSUPPORTED
