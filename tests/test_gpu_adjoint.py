"""GPU discrete adjoint (dm_rollout / dm_adjoint and the torch.autograd.Function over them):
against the oracle's adjoint gradient (tests/golden/adjoint.npz, written by the oracle only),
against central differences of the GPU's own forward trajectory at the full 256-rod,
100-node, 200-step size, and through torch autograd.

Tolerances: the GPU forward stops at a Newton residual of 1e-9, which leaves node positions
~1e-9 relative to the oracle's; the gradient inherits errors of that relative order times the
conditioning of the loss, so the oracle comparison uses 1e-7 relative (2-norm over every
parameter; 1.3e-8 observed).  The central differences run both sides to the FP64 rounding floor of the
residual (newton_tol 1e-13 with the stagnation rule), so their error is O(h^2) plus rounding
of the loss over 2h."""
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


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def golden_desc():
    """The adjoint golden's workload: the 100-node adjoint rods' material, shortened to the
    golden's node and step counts (read from the stored arrays)."""
    g = np.load(os.path.join(GOLD, "adjoint.npz"))
    T, R, _ = g["target_tips"].shape
    n = g["kbar0_0"].shape[1] + 2
    d, _ = W.adjoint_rods(n_rods=R, n_nodes=n, steps=T)
    return d, T


@pytest.mark.parametrize("case", [0, 1])
def test_adjoint_matches_oracle_gradient(dm, golden_desc, case):
    g = np.load(os.path.join(GOLD, "adjoint.npz"))
    d, T = golden_desc
    say(f"case: adjoint golden {case}, 2 rods x 20 nodes, {T} steps, checkpoint every 10")
    sim = dm.sim_from_description(d)
    sim.set_natural_curvature_all(g[f"kbar0_{case}"].reshape(-1))
    tips = sim.rollout(d["dt"], T, ckpt_every=10)
    assert np.linalg.norm(tips - g[f"tips_{case}"]) <= 1e-9 * np.linalg.norm(g[f"tips_{case}"])
    grad = sim.adjoint(2.0 * (tips - g["target_tips"]))
    ref = g[f"grad_{case}"].reshape(-1)
    rel = np.linalg.norm(grad - ref) / np.linalg.norm(ref)
    say(f"  relative gradient error vs oracle {rel:.3e}")
    assert rel < 1e-7
    # the sim is back at the rollout's final state
    x, _, _, _ = sim.rod_state(1)
    assert np.allclose(x[-1], tips[-1, 1], rtol=0, atol=0)


def test_full_size_adjoint_matches_oracle_gradient(dm):
    """The adjoint workload at its full size in one launch (256 rods of 100 nodes, 200 steps,
    checkpoints every 20), from zero natural curvature toward the seeded target: the gradients
    of its first two rods against the oracle's adjoint of the same two rods (rods do not
    interact, so the oracle runs them alone), 1e-7 relative."""
    g = np.load(os.path.join(GOLD, "adjoint_full.npz"))
    d, kstar = W.adjoint_rods()
    T = d["steps"]
    say(f"case: full adjoint workload, 256 rods x 100 nodes, {T} steps, checkpoint every 20")
    sim = dm.sim_from_description(d)
    sim.set_natural_curvature_all(kstar.reshape(-1))
    target = sim.rollout(d["dt"], T, ckpt_every=20)
    assert np.linalg.norm(target[:, :2] - g["target_tips"]) <= 1e-9 * np.linalg.norm(g["target_tips"])
    sim.close()
    sim = dm.sim_from_description(d)
    tips = sim.rollout(d["dt"], T, ckpt_every=20)
    assert np.linalg.norm(tips[:, :2] - g["tips"]) <= 1e-9 * np.linalg.norm(g["tips"])
    grad = sim.adjoint(2.0 * (tips - target)).reshape(256, -1)
    for r in range(2):
        ref = g["grad"][r].reshape(-1)
        rel = np.linalg.norm(grad[r] - ref) / np.linalg.norm(ref)
        say(f"  rod {r}: relative gradient error vs oracle {rel:.3e}")
        assert rel < 1e-7


def test_adjoint_checkpoint_interval_does_not_change_the_gradient(dm, golden_desc):
    g = np.load(os.path.join(GOLD, "adjoint.npz"))
    d, T = golden_desc
    out = []
    for ck in (1, 7, T):
        sim = dm.sim_from_description(d)
        sim.set_natural_curvature_all(g["kbar0_1"].reshape(-1))
        tips = sim.rollout(d["dt"], T, ckpt_every=ck)
        out.append(sim.adjoint(2.0 * (tips - g["target_tips"])))
        sim.close()
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def test_adjoint_matches_central_differences_full_size(dm):
    """256 rods x 100 nodes x 200 steps, checkpoint every 20; 16 seeded parameters, each
    perturbed in every rod at once (rods are independent, so per-rod losses separate)."""
    import torch
    d, kstar = W.adjoint_rods()
    T = d["steps"]
    say("case: adjoint full size, 256 rods x 100 nodes x 200 steps")
    stream = torch.cuda.current_stream().cuda_stream
    sim = dm.sim_from_description(d, newton_tol=1e-13, stream=stream)
    start = sim.checkpoint_torch()
    sim.set_natural_curvature_all(kstar.reshape(-1))
    target = sim.rollout(d["dt"], T, ckpt_every=20)
    rng = np.random.Generator(np.random.PCG64(12))
    k0 = 0.5 * rng.normal(size=kstar.shape)

    def tips_at(k):
        sim.restore(start)
        sim.set_natural_curvature_all(k.reshape(-1))
        return sim.rollout(d["dt"], T, ckpt_every=20)

    tips = tips_at(k0)
    grad = sim.adjoint(2.0 * (tips - target)).reshape(kstar.shape)
    h = 1e-6
    params = rng.choice(kstar.shape[1] * 2, 16, replace=False)
    worst = 0.0
    for p in params:
        i, c = divmod(int(p), 2)
        kp, km = k0.copy(), k0.copy()
        kp[:, i, c] += h
        km[:, i, c] -= h
        Lp = ((tips_at(kp) - target) ** 2).sum(axis=(0, 2))
        Lm = ((tips_at(km) - target) ** 2).sum(axis=(0, 2))
        fd = (Lp - Lm) / (2 * h)
        scale = np.abs(grad).max(axis=(1, 2))
        err = np.abs(grad[:, i, c] - fd) / scale
        worst = max(worst, float(err.max()))
    say(f"  worst FD mismatch relative to each rod's largest gradient entry: {worst:.3e}")
    assert worst < 1e-5


def test_autograd_function_and_a_descent_step(dm, golden_desc):
    import torch
    g = np.load(os.path.join(GOLD, "adjoint.npz"))
    d, T = golden_desc
    stream = torch.cuda.current_stream().cuda_stream
    sim = dm.sim_from_description(d, stream=stream)
    start = sim.checkpoint_torch()
    target = torch.tensor(g["target_tips"], device="cuda")
    k = torch.tensor(g["kbar0_1"].reshape(-1), device="cuda", requires_grad=True)
    tips = dm.tip_trajectory(k, sim, start, d["dt"], T, ckpt_every=10)
    loss = ((tips - target) ** 2).sum()
    loss.backward()
    ref = g["grad_1"].reshape(-1)
    got = k.grad.cpu().numpy()
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-6
    # one gradient step along -grad lowers the loss
    with torch.no_grad():
        k2 = k - (0.1 * loss.item() / (k.grad ** 2).sum().item()) * k.grad
    loss2 = ((dm.tip_trajectory(k2, sim, start, d["dt"], T, ckpt_every=10) - target) ** 2).sum()
    assert loss2.item() < loss.item()


def test_adjoint_rejects_unsupported_and_out_of_order_calls(dm):
    sim = dm.sim_from_description(W.rod_batch(2, nmax=30))
    with pytest.raises(dm.DmError) as e:
        sim.adjoint(np.zeros((1, 2, 3)))
    assert e.value.status == dm.DM_ERR_STATE
    star = dm.sim_from_description(W.star_robots(n_instances=1, steps=1))
    with pytest.raises(dm.DmError) as e:
        star.rollout(1e-3, 2)
    assert e.value.status == dm.DM_ERR_UNSUPPORTED
