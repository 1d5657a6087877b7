"""Write the oracle reference trajectories used by the GPU parity tests.

Calls only the CPU oracle (oracle/) and the seeded input descriptions (workloads/).
Run from the repository root:  python tests/golden/make_golden.py [name ...]
Each output is a small .npz holding positions and twists of the listed rods after the
listed step counts, plus the Newton iteration counts.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import adjoint as AD  # noqa: E402
from oracle import der  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))

# rods of the 1024-rod batch compared one by one: the longest, the shortest and six seeded picks
BATCH_SAMPLE_SEED = 11


def batch_sample_ids(desc):
    ns = np.array([r["x0"].shape[0] for r in desc["rods"]])
    rng = np.random.Generator(np.random.PCG64(BATCH_SAMPLE_SEED))
    pick = [int(np.argmax(ns)), int(np.argmin(ns))] + [int(i) for i in rng.choice(len(ns), 6, replace=False)]
    return sorted(set(pick))


def run(desc, rod_ids, checkpoints, polish=1, scheme="euler"):
    """Step the system holding rod_ids and record rod states at the given step counts."""
    sys_, st = der.build(desc, rod_ids)
    out, iters = {}, []
    n = max(checkpoints)
    ls = desc.get("line_search", False)
    for k in range(1, n + 1):
        st, info = der.step(sys_, st, desc["dt"], desc["tol"], desc["max_iter"], polish=polish, line_search=ls,
                            scheme=scheme)
        if not info.converged:
            raise RuntimeError(f"oracle did not converge at step {k}: {info.history}")
        iters.append(info.iters)
        if k in checkpoints:
            for j in range(len(rod_ids)):
                out[f"x_{k}_{j}"] = der.rod_positions(sys_, st, j).numpy()
                out[f"th_{k}_{j}"] = der.rod_thetas(sys_, st, j).numpy()
    out["iters"] = np.array(iters)
    out["rods"] = np.array(rod_ids)
    out["steps"] = np.array(sorted(checkpoints))
    return out


def golden_cantilever():
    d = W.cantilever()
    return run(d, [0], {1, 10, 100})


def golden_cantilever_midpoint():
    # the undamped swing of this soft cantilever at dt = 1e-2 stays within reach of Newton for
    # about 90 steps under the midpoint rule (its step 94 already needs 36 iterations and step
    # 95 does not converge, with or without line search); the record ends at step 50
    d = W.cantilever()
    return run(d, [0], {1, 10, 50}, scheme="midpoint")


def golden_star_midpoint():
    d = W.star_robots(n_instances=1, steps=5)
    return run(d, list(range(6)), {1, 5}, scheme="midpoint")


def golden_batch():
    d = W.rod_batch(1024)
    ids = batch_sample_ids(d)
    outs = {}
    for j, r in enumerate(ids):
        o = run(d, [r], {1, 2})
        for k, v in o.items():
            outs[f"{k}_r{j}"] = v
    outs["rods"] = np.array(ids)
    return outs


def golden_batch100():
    """The sampled batch rods (the longest, N = 400, included) over 100 steps, with their
    initial shapes, for displacement-relative parity at steps 1, 10 and 100."""
    d = W.rod_batch(1024)
    ids = batch_sample_ids(d)
    outs = {}
    for j, r in enumerate(ids):
        o = run(d, [r], {1, 10, 100})
        for k, v in o.items():
            outs[f"{k}_r{j}"] = v
        outs[f"x0_r{j}"] = d["rods"][r]["x0"]
        print(f"  batch100: rod {r} done", flush=True)
    outs["rods"] = np.array(ids)
    return outs


def golden_star100():
    d = W.star_robots(n_instances=1, steps=100)
    out = run(d, list(range(6)), {1, 10, 100})
    for a in range(6):
        out[f"x0_{a}"] = d["rods"][a]["x0"]
    return out


def golden_coils():
    """Two coils of the 256-coil self-contact batch (the one of most nodes and a seeded pick),
    each with its own self-contact and friction, over 5 steps, with their initial shapes."""
    d = W.coiled_springs(256, steps=5)
    ns = np.array([r["x0"].shape[0] for r in d["rods"]])
    rng = np.random.Generator(np.random.PCG64(BATCH_SAMPLE_SEED))
    ids = sorted({int(np.argmax(ns)), int(rng.integers(0, len(ns)))})
    outs = {}
    for j, r in enumerate(ids):
        o = run(d, [r], {1, 3, 5})
        for k, v in o.items():
            outs[f"{k}_r{j}"] = v
        outs[f"x0_r{j}"] = d["rods"][r]["x0"]
        print(f"  coils: coil {r} (N {ns[r]}) done", flush=True)
    outs["rods"] = np.array(ids)
    return outs


# the adjoint workload at its full rod size and length (100 nodes, 200 steps, checkpoints every
# 20), for its first two rods, from zero natural curvature toward the seeded target
ADJ_FULL_RODS = 2


def golden_adjoint_full():
    d, target_kbar = W.adjoint_rods(n_rods=ADJ_FULL_RODS)
    kstar = [target_kbar[r] for r in range(ADJ_FULL_RODS)]
    _, _, target = AD.rollout(d, kstar)
    n = d["rods"][0]["x0"].shape[0]
    k0 = [np.zeros((n - 2, 2)) for _ in range(ADJ_FULL_RODS)]
    L, g, tips = AD.loss_and_grad(d, k0, target)
    return {"target_tips": target.numpy(), "loss": np.array(L), "grad": np.stack([gi.numpy() for gi in g]),
            "tips": tips.numpy()}


# Real2Sim fit (Alg. 1, Eq. 19-21) of the two-limb manipulator (1 cm radius, so that gravity
# bends the limbs visibly), three target configurations produced by known natural curvatures
R2S_KSTAR = [[0.6, -0.4], [0.75, -0.25], [0.8, 0.0]]
R2S_TOL, R2S_MAXIT = 1e-5, 150


def golden_real2sim():
    from oracle import real2sim as RS
    import torch
    d = W.two_limb_manipulator(limb_nodes=8, radius=0.01)
    sys_, st = der.build(d)
    kv = torch.tensor([1.7, -0.8], dtype=der.DT)
    st = RS.settle(sys_, st, kv, d["dt"], d["steps"])
    out = {"settled_kbar": kv.numpy(), "settled_kappa": RS.limb_curvatures(sys_, st.x, st.theta, st).numpy()}
    for i, w in enumerate(([1.0, 0.0], [0.0, 1.0])):
        out[f"grad_{i}"] = RS.curvature_gradient(sys_, st, kv, torch.tensor(w, dtype=der.DT), d["dt"]).numpy()
    targets = RS.curvatures_at(d, np.array(R2S_KSTAR)).numpy()
    traj, losses, steps, _ = RS.solve_natural_curvatures(d, targets, tol=R2S_TOL, max_iter=R2S_MAXIT)
    out.update({"targets": targets, "kstar": np.array(R2S_KSTAR), "traj": traj.numpy(), "losses": np.array(losses),
                "steps": np.array(steps), "tol": np.array(R2S_TOL), "max_iter": np.array(R2S_MAXIT)})
    return out


def golden_helix():
    d = W.paper_helix(steps=20)
    return run(d, [0], {1, 20})


def golden_star():
    d = W.star_robots(n_instances=1, steps=20)
    return run(d, list(range(6)), {1, 5, 20})


# discrete adjoint: rods of the 100-node adjoint workload's material and length, shortened to
# 20 nodes and 30 steps; case 0 starts from zero natural curvature (as the fitting problem
# does), case 1 from a seeded nonzero one
ADJ_RODS, ADJ_NODES, ADJ_STEPS = 2, 20, 30


def adjoint_case():
    d, target_kbar = W.adjoint_rods(n_rods=ADJ_RODS, n_nodes=ADJ_NODES, steps=ADJ_STEPS)
    return d, [target_kbar[r] for r in range(ADJ_RODS)]


def golden_adjoint():
    d, kstar = adjoint_case()
    _, _, target = AD.rollout(d, kstar)
    out = {"target_tips": target.numpy()}
    rng = np.random.Generator(np.random.PCG64(4))
    starts = [[np.zeros((ADJ_NODES - 2, 2)) for _ in range(ADJ_RODS)],
              [rng.normal(0.0, 1.0, size=(ADJ_NODES - 2, 2)) for _ in range(ADJ_RODS)]]
    for c, k0 in enumerate(starts):
        L, g, tips = AD.loss_and_grad(d, k0, target)
        out[f"kbar0_{c}"] = np.stack(k0)
        out[f"loss_{c}"] = np.array(L)
        out[f"grad_{c}"] = np.stack([gi.numpy() for gi in g])
        out[f"tips_{c}"] = tips.numpy()
    return out


# Real2Sim-style fit (Alg. 1 control flow, adjoint gradient) on the adjoint case, from zero
# natural curvature; step size 5e4 (the loss is in m^2, its gradient ~1e-5 per 1/m)
FIT_ALPHA, FIT_ITERS = 5e4, 4


def golden_fit():
    d, kstar = adjoint_case()
    _, _, target = AD.rollout(d, kstar)
    k0 = [np.zeros((ADJ_NODES - 2, 2)) for _ in range(ADJ_RODS)]
    ks, losses, alphas = AD.fit_natural_curvature(d, target.numpy(), k0, FIT_ALPHA, 1e-12, FIT_ITERS)
    out = {"target_tips": target.numpy(), "losses": np.array(losses), "alphas": np.array(alphas),
           "alpha": np.array(FIT_ALPHA), "iters": np.array(FIT_ITERS)}
    for i, k in enumerate(ks):
        out[f"kbar_{i}"] = np.stack([ki.numpy() for ki in k])
    return out


GOLDEN = {"cantilever": golden_cantilever, "batch": golden_batch, "helix": golden_helix, "star": golden_star,
          "adjoint": golden_adjoint, "cantilever_midpoint": golden_cantilever_midpoint,
          "star_midpoint": golden_star_midpoint, "fit": golden_fit, "batch100": golden_batch100,
          "star100": golden_star100, "adjoint_full": golden_adjoint_full, "real2sim": golden_real2sim,
          "coils": golden_coils}


if __name__ == "__main__":
    names = sys.argv[1:] or list(GOLDEN)
    for name in names:
        t0 = time.time()
        data = GOLDEN[name]()
        path = os.path.join(OUT, f"{name}.npz")
        np.savez_compressed(path, **data)
        print(f"{name}: wrote {path} in {time.time() - t0:.1f} s", flush=True)
