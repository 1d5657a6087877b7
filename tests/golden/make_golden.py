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
from oracle import der  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))

# rods of the 1024-rod batch compared one by one: the longest, the shortest and six seeded picks
BATCH_SAMPLE_SEED = 11


def batch_sample_ids(desc):
    ns = np.array([r["x0"].shape[0] for r in desc["rods"]])
    rng = np.random.Generator(np.random.PCG64(BATCH_SAMPLE_SEED))
    pick = [int(np.argmax(ns)), int(np.argmin(ns))] + [int(i) for i in rng.choice(len(ns), 6, replace=False)]
    return sorted(set(pick))


def run(desc, rod_ids, checkpoints, polish=1):
    """Step the system holding rod_ids and record rod states at the given step counts."""
    sys_, st = der.build(desc, rod_ids)
    out, iters = {}, []
    n = max(checkpoints)
    ls = desc.get("line_search", False)
    for k in range(1, n + 1):
        st, info = der.step(sys_, st, desc["dt"], desc["tol"], desc["max_iter"], polish=polish, line_search=ls)
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


def golden_helix():
    d = W.paper_helix(steps=20)
    return run(d, [0], {1, 20})


def golden_star():
    d = W.star_robots(n_instances=1, steps=20)
    return run(d, list(range(6)), {1, 5, 20})


GOLDEN = {"cantilever": golden_cantilever, "batch": golden_batch, "helix": golden_helix, "star": golden_star}


if __name__ == "__main__":
    names = sys.argv[1:] or list(GOLDEN)
    for name in names:
        t0 = time.time()
        data = GOLDEN[name]()
        path = os.path.join(OUT, f"{name}.npz")
        np.savez_compressed(path, **data)
        print(f"{name}: wrote {path} in {time.time() - t0:.1f} s", flush=True)
