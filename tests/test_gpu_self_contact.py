"""Edge-edge self-contact inside the GPU step (dm_set_self_contact) against the oracle's
step with self-contact (oracle/der.py, pinned in tests/test_oracle_self_contact.py).

The GPU's Newton matrix is the rod's band plus every pair's blocks with the friction derivative
taken at fixed closest-point parameters, the oracle's is its exact autodiff Jacobian, so the two
stop at different points within the Newton tolerance (1e-9 N of residual): positions agree to
1e-9 relative and the step's displacement to 1e-6 after one step, and to 1e-6 after three and
after ten steps.  The coils run with line search (their friction needs it)."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import der
from parity import assert_parity

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def dm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2311_18126_amd as m
    assert os.path.exists(m.LIB_PATH), "libdmrod.so is not built"
    return m


def say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_coils_match_live_oracle(dm, mu):
    d = W.coiled_springs(2, seed=13, nmin=36, nmax=44, mu=mu)
    say(f"case: two coils with self-contact, mu {mu}")
    sim = dm.sim_from_description(d)
    iters_gpu = 0
    oracles = []
    for r in range(2):
        sub = W.subset(d, [r])
        sub["self_contact"] = d["self_contact"]
        oracles.append(list(der.build(sub)))
    x0 = [sim.rod_state(r)[0].copy() for r in range(2)]
    done = 0
    for k in (1, 3):
        st = sim.step(d["dt"], k - done)
        assert (st["status"] == 0).all()
        iters_gpu += int(st["iters"].sum())
        for r in range(2):
            sys_, s_ = oracles[r]
            for _ in range(k - done):
                s_, info = der.step(sys_, s_, d["dt"], d["tol"], d["max_iter"], line_search=True)
                assert info.converged
            oracles[r][1] = s_
            n_pairs = len(der.contact_list(sys_, der.pack(s_.x, s_.theta)))
            assert n_pairs > 40
            assert_parity(sim.rod_state(r)[0], s_.x.numpy(), x0[r], 1e-9 if k == 1 else 1e-6, 1e-6,
                          f"coil {r} step {k} ({n_pairs} pairs)")
        done = k
    say(f"GPU Newton iterations over 3 steps of 2 coils: {iters_gpu}")


def test_full_batch_sampled_coils_match_golden(dm):
    """The 256-coil batch stepped as bench.py steps it (one launch for all coils, adaptive
    halving on) against the oracle's steps of two of its coils (tests/golden/coils.npz, written
    by tests/golden/make_golden.py from the oracle alone): 1e-9 of the positions and 1e-6 of the
    displacement after one step, 1e-6 of both after three and five."""
    g = np.load(os.path.join(GOLD, "coils.npz"))
    d = W.coiled_springs(256, steps=5)
    sim = dm.sim_from_description(d)
    sim.set_adaptive(3)
    done = 0
    for k in (1, 3, 5):
        st = sim.step(d["dt"], k - done)
        done = k
        assert (st["status"] == 0).all()
        for j, r in enumerate(g["rods"]):
            r = int(r)
            assert st["halvings"][sim.rod_system(r)] == 0, (r, k)
            assert_parity(sim.rod_state(r)[0], g[f"x_{k}_0_r{j}"], g[f"x0_r{j}"], 1e-9 if k == 1 else 1e-6, 1e-6,
                          f"coil {r} step {k}")
    say(f"sampled coils {g['rods'].tolist()}: oracle Newton iterations {[g[f'iters_r{j}'].tolist() for j in range(len(g['rods']))]}")


def test_coil_with_friction_over_ten_steps(dm):
    """One coil (36 nodes) with friction over 10 steps as the turns settle on each other: the
    friction between touching turns couples nodes a turn apart with a stiffness well above the
    inertia's, which the step solves with the pairs' blocks in its matrix; line search on both
    sides (the stick-slip transitions make plain Newton cycle)."""
    d = W.coiled_springs(1, seed=13, nmin=36, nmax=36, mu=0.3)
    say("case: one coil with friction, 10 steps")
    sim = dm.sim_from_description(d)
    sys_, s_ = der.build(d)
    x0 = s_.x.numpy().copy()
    st = sim.step(d["dt"], 10)
    assert st["status"][0] == 0
    iters = 0
    for _ in range(10):
        s_, info = der.step(sys_, s_, d["dt"], d["tol"], d["max_iter"], line_search=True)
        assert info.converged
        iters += info.iters
    say(f"Newton iterations over 10 steps: GPU {int(st['iters'][0])}, oracle {iters}")
    assert st["iters"][0] <= 2 * iters
    assert_parity(sim.rod_state(0)[0], s_.x.numpy(), x0, 1e-6, 1e-6, "coil step 10")


def test_batch_of_coils_converges(dm):
    """256 coils over 30 steps with friction, line search and adaptive halving (up to three
    levels): every system converges.  Without halving one coil's step 11 does not converge
    within 50 line-searched Newton iterations, on the oracle as here."""
    d = W.coiled_springs(256, steps=30)
    sim = dm.sim_from_description(d)
    sim.set_adaptive(3)
    st = sim.step(d["dt"], 30)
    assert (st["status"] == 0).all()
    per_step = st["iters"] / 30.0
    say(f"256 coils, 30 steps: Newton iterations per step mean {per_step.mean():.2f}, max {per_step.max():.2f}; "
        f"halved steps {int(st['halvings'].sum())}")
    assert per_step.mean() < 10.0


def test_wide_and_long_rods_match_the_band_solve_when_contact_is_negligible(dm):
    """The solve's other paths against the plain band solve, with a contact stiffness so small
    (1e-12) that the step is the plain one to within rounding while the pairs, and so the
    matrix's half bandwidth, are those of the coils: a 60-node coil (half bandwidth 70), a
    150-node coil (166: above the LDS panel, one pivot at a time) and a straight 300-node rod,
    whose length leaves LDS for 8-column panels only, for the whole launch."""
    c60 = W.coiled_springs(1, seed=13, nmin=60, nmax=60, mu=0.0)["rods"][0]
    c150 = W.coiled_springs(1, seed=13, nmin=150, nmax=150, mu=0.0)["rods"][0]
    c150 = dict(c150, x0=c150["x0"] + np.array([1.0, 0.0, 0.0]))
    line = W.rod(W.straight_nodes(300, 1.5, (2.0, 0.0, 0.1)), 2e-3, 1e6)
    d = W.desc([c60, c150, line], dt=1e-3, steps=3)
    plain = dm.sim_from_description(d)
    sc = dm.sim_from_description(d)
    sc.set_self_contact(5e-4, 1e-12)
    x0 = plain.state()[0].copy()
    a = plain.step(d["dt"], 3)
    b = sc.step(d["dt"], 3)
    assert (a["status"] == 0).all() and (b["status"] == 0).all()
    say(f"Newton iterations: band {a['iters'].tolist()}, with the pairs' matrix {b['iters'].tolist()}")
    assert_parity(sc.state()[0], plain.state()[0], x0, 1e-9, 1e-6, "negligible contact vs plain")


@pytest.mark.parametrize("block", [64, 128, 512])
def test_workgroup_sizes_agree(dm, block):
    """The LU's panel keeps each row in a thread's registers where the workgroup has a lane per
    panel row (up to 144 rows), else in LDS (64 and 128 lanes): four coils with friction over
    three steps take the same Newton iterations at 64, 128 and 512 lanes as at 256, and agree
    to 1e-9 relative in position and 1e-6 in displacement."""
    d = W.coiled_springs(4, seed=13, nmin=60, nmax=80)
    say(f"case: four coils, workgroup of {block} lanes against 256")
    if block == 512:
        assert dm.sim_from_description(d).block_size == 512      # the default with self-contact
    ref = dm.sim_from_description(d, block_size=256)
    small = dm.sim_from_description(d, block_size=block)
    x0 = ref.state()[0].copy()
    a = ref.step(d["dt"], 3)
    b = small.step(d["dt"], 3)
    assert (a["status"] == 0).all() and (b["status"] == 0).all()
    say(f"Newton iterations: 256 lanes {a['iters'].tolist()}, {block} lanes {b['iters'].tolist()}")
    assert a["iters"].tolist() == b["iters"].tolist()
    assert_parity(small.state()[0], ref.state()[0], x0, 1e-9, 1e-6, f"{block} lanes vs 256")


def test_autotuner_with_self_contact(dm, tmp_path):
    """dm_autotune times the self-contact step at each workgroup size, restores the state, and
    files its choice under a key of its own: the same rods without self-contact get another
    cache line, and a second simulation with self-contact is served from the file."""
    d = W.coiled_springs(16, seed=13, nmin=40, nmax=60)
    cache = str(tmp_path / "tune.txt")
    plain = dict(d)
    plain.pop("self_contact")
    p = dm.sim_from_description(plain)
    p.autotune(d["dt"], trial_steps=1, cache=cache)
    sim = dm.sim_from_description(d)
    assert sim.block_size == 512                    # the default with self-contact on
    sim.step(d["dt"], 1)
    before = sim.state()
    b = sim.autotune(d["dt"], trial_steps=1, cache=cache)
    say(f"autotuned block size with self-contact {b}")
    assert b in (64, 128, 256, 512) and sim.block_size == b
    for u, w in zip(before, sim.state()):
        assert np.array_equal(u, w)
    with open(cache) as f:
        lines = f.read().splitlines()
    assert len(lines) == 2 and lines[0].rsplit(" ", 1)[0] != lines[1].rsplit(" ", 1)[0]
    again = dm.sim_from_description(d)
    assert again.autotune(d["dt"], trial_steps=1, cache=cache) == b
    with open(cache) as f:
        assert len(f.read().splitlines()) == 2
    st = sim.step(d["dt"], 2)
    assert (st["status"] == 0).all()


def test_runs_are_bitwise_deterministic(dm):
    """Pairs are found with an LDS atomic counter but sorted before any sum, and every node sums
    its pairs in the list's order: two runs of 32 coils with friction agree bit for bit."""
    d = W.coiled_springs(32, seed=5)
    out = []
    for _ in range(2):
        sim = dm.sim_from_description(d)
        sim.set_adaptive(3)
        st = sim.step(d["dt"], 10)
        assert (st["status"] == 0).all()
        out.append(sim.state())
        sim.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_an_earlier_wider_band_leaves_no_trace(dm):
    """A straight 151-node rod wound for one step into a three-turn helix whose turns touch
    (50 nodes a turn: half bandwidth 210, the solve's one-pivot path writes the matrix far from
    its diagonal), then the straight rod's checkpoint restored (no pairs: half bandwidth 10,
    the blocked LU, whose panels reach 16 columns further): the next steps are bit for bit
    those of a simulation that never held the helix."""
    import math
    n, L, h = 151, 1.5, 4e-3
    d = W.desc([W.rod(W.straight_nodes(n, L), h, 1e6)], dt=1e-3, steps=3)
    phi = np.arange(n) * 2.0 * math.pi / 50
    R = 50 * (L / (n - 1)) / (2.0 * math.pi)
    helix = np.stack([R * np.cos(phi), R * np.sin(phi), 7.5e-3 * phi / (2.0 * math.pi)], 1)
    runs = []
    for wind in (False, True):
        sim = dm.sim_from_description(d)
        sim.set_self_contact(5e-4, 10.0)
        start = sim.checkpoint()
        if wind:
            sim.set_rod_state(0, x=helix)
            st = sim.step(d["dt"], 1, allow_failure=True)
            assert st["iters"][0] >= 1          # the wide matrix was factorised
            sim.restore(start)
        st = sim.step(d["dt"], 3)
        assert (st["status"] == 0).all()
        runs.append((sim.state()[0].copy(), int(st["iters"][0])))
        sim.close()
    say(f"Newton iterations: fresh {runs[0][1]}, after the helix {runs[1][1]}")
    assert runs[0][1] == runs[1][1]
    assert np.array_equal(runs[0][0], runs[1][0])


def test_off_is_the_plain_step_bit_for_bit(dm):
    d = W.coiled_springs(2, seed=13, nmin=36, nmax=44)
    plain = dict(d)
    plain.pop("self_contact")
    a = dm.sim_from_description(plain)
    b = dm.sim_from_description(d)
    b.set_self_contact(0.0, 0.0)
    assert b.block_size == a.block_size == 256     # off again: the plain step's workgroup
    a.step(d["dt"], 3)
    b.step(d["dt"], 3)
    assert np.array_equal(a.state()[0], b.state()[0])
    c = dm.sim_from_description(d)
    c.step(d["dt"], 3)
    assert not np.array_equal(a.state()[0], c.state()[0])


def test_pair_list_overflow_is_reported(dm):
    """An accordion-folded rod (pleats of four 5 mm edges, 3 mm apart) puts every edge within
    reach of edges of several pleats: more than four pairs per edge, DM_ERR_UNSUPPORTED, and
    the rod stays at the step start."""
    pts = []
    for p in range(15):
        xs = np.linspace(0.0, 0.02, 5) if p % 2 == 0 else np.linspace(0.02, 0.0, 5)
        pts += [(x, 0.003 * p, 0.0) for j, x in enumerate(xs) if p == 0 or j > 0]
    x0 = np.array(pts)
    d = W.desc([W.rod(x0, 4e-3, 1e6)], dt=1e-3, steps=1, gravity=(0.0, 0.0, 0.0))
    sim = dm.sim_from_description(d)
    sim.set_self_contact(5e-4, 10.0)
    before = sim.state()[0].copy()
    with pytest.raises(dm.DmError) as e:
        sim.step(d["dt"], 1)
    assert e.value.status == dm.DM_ERR_UNSUPPORTED and "pair list" in str(e.value)
    assert np.array_equal(sim.state()[0], before)


def test_unsupported_setups(dm):
    star = W.star_robots(n_instances=1, steps=1)
    sim = dm.sim_from_description(star)
    with pytest.raises(dm.DmError) as e:
        sim.set_self_contact(5e-4, 10.0)
    assert e.value.status == dm.DM_ERR_UNSUPPORTED
    d = W.coiled_springs(1, seed=13, nmin=36, nmax=36)
    sim = dm.sim_from_description(d)
    with pytest.raises(dm.DmError):
        sim.set_self_contact(-1.0, 10.0)
    sim.set_integrator("midpoint")
    with pytest.raises(dm.DmError) as e:
        sim.step(d["dt"], 1)
    assert e.value.status == dm.DM_ERR_UNSUPPORTED
    sim.set_integrator("euler")
    # the network's activations do not fit in LDS beside a 36-node rod's self-contact arrays:
    # refused, and the analytic warm starts stay available
    net = dm.Mlp(max_rows=64)
    with pytest.raises(dm.DmError) as e:
        sim.set_warm_start(net, 2)
    assert e.value.status == dm.DM_ERR_UNSUPPORTED and "LDS" in str(e.value)
    sim.set_warm_start(None, 4)
    assert (sim.step(d["dt"], 2)["status"] == 0).all()
