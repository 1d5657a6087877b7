"""Benchmark: batched implicit DER steps on one MI355X, node-steps/s at a 1e-9 Newton residual.

Workload: 1024 independent clamped rods, N ~ U{20..400} nodes (seed 0), L ~ U(0.5, 2) m,
h ~ U(1e-3, 5e-3) m, E = 10^U(6, 8) Pa, natural curvature ~ N(0, 2^2) 1/m, gravity,
dt = 1e-3 s, FP64, all rods in one persistent launch.  A "step" is one backward-Euler time
step of the whole batch.  Prints one JSON line: the batch's rate and its FP64 roofline
(kernel time from HIP events on the launch's stream; HBM bytes from the committed counter
summary of the same kernel source, else null), the CPU oracle on a bounded sample, and the
warm start, star, midpoint, adjoint and per-rod figures.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --configs    # one line per benchmark configuration
    python bench.py --paper      # the paper's validation workloads against its wall times
    python bench.py --section self_contact   # one extra section alone (for profiling)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "node-steps/s, batched implicit DER at 1e-9 residual; plain vs warm-started"
# Algorithmic FP64 work of one Newton iteration per item, counted by the host program
# paper_2311_18126_amd/dm_flops over the step's own element math (csrc/dm_flops.cpp states the
# counting rules); the committed output is read here and checked against the program by the
# CPU tests.
FLOP_COUNT_FILE = os.path.join(ROOT, "profiles", "flop_count.json")
PEAK_FP64_VALU_TFLOPS = 78.6          # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
PEAK_BF16_MFMA_TFLOPS = 2500.0        # dense BF16 matrix-core peak, published
# 26-256-256-3 network, per row of a training step: forward 2 (26*256 + 256*256 + 256*3),
# input gradients of layers 3 and 2: 2 (256*3 + 256*256), weight gradients 2 (26*256 + 256*256 + 3*256)
INFER_FLOPS_PER_ROW = 2 * (26 * 256 + 256 * 256 + 256 * 3)
TRAIN_FLOPS_PER_ROW = 2 * INFER_FLOPS_PER_ROW + 2 * (256 * 3 + 256 * 256)
KERNEL_SOURCES = ["paper_2311_18126_amd/csrc/dm_kernels.hip", "paper_2311_18126_amd/csrc/dm_math.h",
                  "paper_2311_18126_amd/csrc/dm_layout.h", "paper_2311_18126_amd/csrc/dm_warm.h",
                  "paper_2311_18126_amd/csrc/dm_bf16.h", "paper_2311_18126_amd/csrc/dm_segment.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dm_step_kernel_rod_batch_traffic.json")


def rod_iteration_flops(n_nodes, count=None):
    """Counted FP64 operations of one Newton iteration of a clamped single rod of n nodes:
    stencils, stretch and twist inertia of the edges, node terms, their assembly into the band,
    the banded LU of the two arms with back substitution, the 10-DOF separator's dense LU and
    the arms' Schur blocks added into it, the update and the residual norm."""
    if count is None:
        with open(FLOP_COUNT_FILE) as f:
            count = json.load(f)
    n = np.asarray(n_nodes, dtype=np.float64)
    if np.any(n < 4):
        raise ValueError("the per-rod count assumes a 10-DOF separator and two arms (rods of 4 nodes or more)")
    dof = 4 * n - 1
    return ((n - 2) * (count["stencil"] + count["assembly_stencil"])
            + (n - 1) * (count["stretch"] + count["edge_inertia"] + count["assembly_edge"])
            + n * (count["node"] + count["assembly_node"])
            + (dof - 10) * (count["lu_row"] + count["backsub_row"]) + count["border_lu_10"] + 2 * count["schur_per_arm"]
            + dof * count["dof"])


def star_iteration_flops(limbs=6, limb_nodes=30, count=None):
    """Counted FP64 operations of one Newton iteration of a star of `limbs` rods of
    limb_nodes + 1 nodes joined at a hub: limb and hub stencils (every pair of hub edges),
    edges, nodes (contact and friction terms not counted: a lower bound), each limb's arm
    eliminated toward the 3 + 4 limbs border, the border's dense LU and the Schur blocks."""
    if count is None:
        with open(FLOP_COUNT_FILE) as f:
            count = json.load(f)
    assert limbs == 6, "the committed count holds the six-limb hub's border"
    n = limb_nodes + 1
    stencils = limbs * (n - 2) + limbs * (limbs - 1) // 2
    edges, nodes = limbs * (n - 1), limbs * (n - 1) + 1
    dof = limbs * (4 * n - 1) - 3 * (limbs - 1)
    eliminated = limbs * (4 * n - 1 - 7)
    return (stencils * (count["stencil"] + count["assembly_stencil"])
            + edges * (count["stretch"] + count["edge_inertia"] + count["assembly_edge"])
            + nodes * (count["node"] + count["assembly_node"])
            + eliminated * (count["lu_row"] + count["backsub_row"]) + count["border_lu_27"]
            + limbs * count["schur_per_arm"] + dof * count["dof"])


def kernel_hash():
    """Hash of the step kernel's sources and of the compiler flags they are built with."""
    from paper_2311_18126_amd import build as B
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    h.update(" ".join(f for f in B.FLAGS if not f.startswith(("-I", "/"))).encode())
    return h.hexdigest()[:16]


def measured_traffic(n_launch_steps):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None if the
    summary is missing or was taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t["bytes_per_step"] * n_launch_steps


def cpu_baseline(desc, budget_s=20.0, single_budget_s=8.0):
    """The CPU oracle, as is, on a bounded sample of the same workload: seeded rods of the
    batch, one step each, until the time budget is used (rank 0, one GPU only); then the same
    rods in the same order on one thread for a shorter budget."""
    import torch

    import workloads as W
    from oracle import der
    threads = min(os.cpu_count() or 1, 16)
    rng = np.random.Generator(np.random.PCG64(123))
    order = rng.permutation(len(desc["rods"]))

    def run(budget):
        nodes, t_used, rods = 0, 0.0, 0
        for r in order:
            sub = W.subset(desc, [int(r)])
            t0 = time.perf_counter()
            der.simulate(sub, steps=1)
            t_used += time.perf_counter() - t0
            nodes += sub["rods"][0]["x0"].shape[0]
            rods += 1
            if t_used > budget:
                break
        return nodes / t_used, rods, t_used
    torch.set_num_threads(threads)
    value, rods, t_used = run(budget_s)
    torch.set_num_threads(1)
    v1, rods1, t1 = run(single_budget_s)
    torch.set_num_threads(threads)
    return {"value": value, "unit": "node-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{rods} seeded rods of the 1024-rod batch, 1 step each, {t_used:.1f} s",
            "single_thread_value": v1,
            "single_thread_sample": f"the first {rods1} of those rods on 1 thread, {t1:.1f} s"}


def per_rod_baseline(dm, desc, steps, n=16):
    """The plain per-rod GPU step: seeded rods of the batch, each in its own simulation and
    launch (one workgroup at a time), same steps and residual."""
    rng = np.random.Generator(np.random.PCG64(321))
    ids = rng.choice(len(desc["rods"]), n, replace=False)
    import torch
    import workloads as W
    nodes, t_used = 0, 0.0
    for r in ids:
        sub = W.subset(desc, [int(r)])
        sim = dm.sim_from_description(sub, stream=torch.cuda.current_stream().cuda_stream)
        sim.step(sub["dt"], 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(sub["dt"], steps)
        torch.cuda.synchronize()
        t_used += time.perf_counter() - t0
        nodes += sub["rods"][0]["x0"].shape[0] * steps
        sim.close()
    return nodes / t_used


def timed_steps(sim, dt, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = sim.step(dt, steps)
    torch.cuda.synchronize()
    return st, time.perf_counter() - t0


def inference_rate(sim, dt, reps=10):
    """Matrix-core throughput of the network's guess for every node of the batch, run by
    dm_ws_predict with the step kernel's own device code (features, three layers, output).
    Each call is bracketed by events on the simulation's stream (torch's default stream); the
    shortest call is kept, and it still includes one launch latency."""
    import torch
    rows = sim.ws_rows
    buf = torch.empty((rows, 3), dtype=torch.float64, device="cuda")
    sim.ws_predict(dt, buf)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sim.ws_predict(dt, buf)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    flops = INFER_FLOPS_PER_ROW * rows
    return {"bound": "mfma", "achieved": flops / best / 1e12, "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s",
            "frac": flops / best / 1e12 / PEAK_BF16_MFMA_TFLOPS, "algorithmic_flops": float(flops),
            "rows": int(rows), "ms_per_call": best * 1e3}


def warm_start_section(dm, steps, log, train_steps=1000, skip=100):
    """Learned warm start at the stated size: a network trained, streamed, on 1000 steps of the
    1024-rod batch (seed 0) after its first 100 (the start-up transient, whose large targets
    would set the output scale): 1.0e6 rod-steps, 2.1e8 node rows, each chunk of 100 steps
    collected on the device, trained once and dropped; evaluated on 1024 fresh rods
    (N ~ U{50..400}, seed 3) over `steps` steps from rest against the plain step and the
    analytic predictors at the same residual."""
    import torch

    import workloads as W
    from paper_2311_18126_amd import warm_start as WS
    train = W.rod_batch(1024)
    sim = dm.sim_from_description(train)
    sim.step(train["dt"], skip)
    net = dm.Mlp(max_rows=65536)
    net.set_params(WS.init_params(0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch = 8192
    hist, n_rows = WS.train_streamed(net, sim, train["dt"], train_steps, chunk=100, batch=batch)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    rod_steps = len(train["rods"]) * train_steps
    sim.close()
    log(f"warm start: {n_rows} training rows ({rod_steps} rod-steps) streamed in {t_train:.1f} s, "
        f"loss {hist[0]:.3f} -> {hist[-1]:.3f}")
    ev = W.warm_start_eval(1024, steps=steps)
    nodes = float(sum(r["x0"].shape[0] for r in ev["rods"]))
    out = {"workload": "1024 fresh clamped rods, N~U{50..400} (seed 3), other parameters as the batch",
           "steps": steps, "training": f"1024-rod batch (seed 0), steps {skip + 1}..{skip + train_steps}, "
                                      "streamed in chunks of 100 steps",
           "training_rod_steps": rod_steps, "training_rows": int(n_rows),
           "train_and_collect_s": t_train, "training_loss_per_chunk": hist}
    # matrix-core throughput of training alone is not separated from the collection here
    out["training_mfma"] = {"bound": "mfma", "algorithmic_flops": float(TRAIN_FLOPS_PER_ROW * n_rows),
                            "achieved_including_collection": TRAIN_FLOPS_PER_ROW * n_rows / t_train / 1e12,
                            "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s"}
    for name, mode in (("plain", 0), ("explicit_predictor", 1), ("extrapolation", 3), ("third_order", 4),
                       ("network", 2)):
        sim = dm.sim_from_description(ev)
        sim.set_warm_start(net if mode == 2 else None, mode)
        st, wall = timed_steps(sim, ev["dt"], steps)
        assert (st["status"] == 0).all()
        out[f"{name}_value"] = nodes * steps / wall
        out[f"{name}_iters_per_step"] = float(st["iters"].sum() / st["iters"].size / steps)
        if mode == 2:
            out["network_fallbacks"] = int(st["fallbacks"].sum())
            out["inference_mfma"] = inference_rate(sim, ev["dt"])
        sim.close()
    net.close()
    return out


def star_section(dm, steps):
    """4096 six-limb stars on the floor with actuation (joined rods, arrowhead solve), from the
    plain Newton start and from the analytic warm starts (explicit predictor, second-order
    extrapolation), each from the same initial state; the warm-started end states are compared
    with the plain one."""
    import workloads as W
    d = W.star_robots(4096)
    out, x_plain = None, None
    for mode, name in ((0, None), (1, "explicit"), (3, "second_order")):
        sim = dm.sim_from_description(d)
        if mode:
            sim.set_warm_start(None, mode)
        sim.step(d["dt"], 1)
        st, wall = timed_steps(sim, d["dt"], steps)
        assert (st["status"] == 0).all()
        nodes = float(sim.num_nodes)
        x = sim.state()[0]
        res = {"value": nodes * steps / wall, "unit": "node-steps/s",
               "newton_iters_per_step": float(st["iters"].mean() / steps)}
        if mode == 0:
            x_plain = x
            out = {"workload": "4096 stars: 6 limbs x 30 nodes on a shared hub, floor contact and friction, "
                               "sinusoidal actuation (seed 1)", "steps": steps, **res, "block_size": sim.block_size,
                   "warm_started": {}}
        else:
            res["fallbacks"] = int(st["fallbacks"].sum())
            res["max_position_difference_vs_plain_m"] = float(np.abs(x - x_plain).max())
            out["warm_started"][name] = res
        sim.close()
    return out


def midpoint_section(dm, steps):
    """The 1024-rod batch stepped with the implicit-midpoint integrator (same rods, residual
    and launch as the headline figure), with adaptive halving (three levels): the undamped
    rule keeps the stiff modes ringing, and over a long run a step now and then needs halving."""
    import torch

    import workloads as W
    d = W.rod_batch(1024)
    sim = dm.sim_from_description(d)
    sim.set_integrator("midpoint")
    sim.set_adaptive(3)
    sim.step(d["dt"], 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = sim.step(d["dt"], steps, allow_failure=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    failed = int((st["status"] != 0).sum())
    nodes = float(sim.num_nodes)
    # a system that fails stops early, so the rate is reported only when none did
    out = {"workload": "1024-rod batch (seed 0) as above, implicit midpoint, adaptive halving", "steps": steps,
           "value": nodes * steps / wall if failed == 0 else None, "unit": "node-steps/s",
           "ms_per_step": 1e3 * wall / steps, "failed_systems": failed, "halved_steps": int(st["halvings"].sum()),
           "newton_iters_per_step": float(st["iters"].mean() / steps), "block_size": sim.block_size}
    sim.close()
    return out


def self_contact_section(dm, steps, n_rods=4096):
    """Coiled springs whose turns press on each other under gravity, stepped with each rod's
    edge-edge self-contact and friction inside the implicit step (pairs found at every Newton
    iterate, each rod's Newton matrix with its pairs' blocks), line search and adaptive halving
    (three levels), and the same batch without self-contact (band solve) for comparison."""
    import workloads as W
    d = W.coiled_springs(n_rods, steps=steps)
    out = {"workload": f"{n_rods} coiled springs: N ~ U{{40..80}}, h = 4 mm, pitch 8.1-8.4 mm, delta = 5e-4 m, "
                       f"mu = 0.3 (seed 13)", "steps": steps, "unit": "node-steps/s"}
    for key, on in (("with_self_contact", True), ("without", False)):
        dd = dict(d)
        if not on:
            dd.pop("self_contact")
        sim = dm.sim_from_description(dd)
        sim.set_adaptive(3)
        sim.step(d["dt"], 1)
        import torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = sim.step(d["dt"], steps, allow_failure=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        failed = int((st["status"] != 0).sum())
        # a system that fails stops early, so the rate is reported only when none did
        out[key] = {"value": float(sim.num_nodes) * steps / wall if failed == 0 else None,
                    "ms_per_step": 1e3 * wall / steps, "failed_systems": failed,
                    "newton_iters_per_step": float(st["iters"].mean() / steps),
                    "halved_steps": int(st["halvings"].sum()), "block_size": sim.block_size}
        sim.close()
    return out


def adjoint_section(dm):
    """Gradient of the tip-trajectory loss with respect to natural curvature: 256 rods x 100
    nodes x 200 steps, checkpoint every 20 (forward rollout + recompute + backward), timed after
    one untimed pass that captures the segment graphs."""
    import torch

    import workloads as W
    d, kstar = W.adjoint_rods()
    T = d["steps"]
    sim = dm.sim_from_description(d)
    start = sim.checkpoint_torch()
    sim.set_natural_curvature_all(kstar.reshape(-1))
    target = sim.rollout(d["dt"], T, ckpt_every=20)
    # one untimed forward + backward pass captures the segment graphs (a one-time setup cost)
    sim.restore(start)
    sim.set_natural_curvature_all(np.zeros(kstar.size))
    sim.adjoint(2.0 * (sim.rollout(d["dt"], T, ckpt_every=20) - target))
    sim.restore(start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tips = sim.rollout(d["dt"], T, ckpt_every=20)
    t1 = time.perf_counter()
    g = sim.adjoint(2.0 * (tips - target))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    nodes = 256 * 100.0
    return {"workload": "256 rods x 100 nodes x 200 steps, dt 1e-3, checkpoint every 20", "forward_s": t1 - t0,
            "backward_s": t2 - t1, "value": nodes * T / (t2 - t0), "unit": "node-steps/s (forward + adjoint)",
            "grad_norm": float(np.linalg.norm(g))}


def oracle_rate(make, threads, budget_s):
    """Node-steps/s of the CPU oracle, as is, on `threads` threads: calls make() -> (fn, nodes)
    repeatedly (each call one oracle unit of work over `nodes` node-steps) until the budget."""
    import torch
    torch.set_num_threads(threads)
    done, used = 0.0, 0.0
    while used < budget_s:
        fn, nodes = make()
        t0 = time.perf_counter()
        fn()
        used += time.perf_counter() - t0
        done += nodes
    return done / used


def paper_table(dm, log):
    """The paper's validation workloads (its Table II) under its own integrator, implicit
    midpoint, at its time steps and end times, each timed as one whole simulation in one
    launch, beside the paper's wall times on an 8-core desktop CPU.  Context only: other
    hardware, and the paper states no Newton tolerance (here 1e-9).  A step whose Newton solve
    fails is redone as two half steps (up to 8 levels); halvings are reported.  The same runs
    under backward Euler are reported beside them."""
    import torch

    import workloads as W
    pushes = np.linspace(-10.6, 10.5, 44)
    fr = W.paper_friction(push=float(pushes[0]), steps=300)
    fr["rods"] = [W.paper_friction(push=float(p), steps=300)["rods"][0] for p in pushes]
    cases = [
        ("a1 cantilever N=201, E=1e5 Pa, dt=0.5 s, T=100 s", W.paper_cantilever(E=1e5, dt=0.5, steps=200), 0.661),
        ("a2 cantilever N=201, E=1e7 Pa, dt=0.05 s, T=20 s", W.paper_cantilever(E=1e7, dt=0.05, steps=400), 1.24),
        ("b1 helix N=100, h=5 mm, E=1e7 Pa, dt=6e-3 s, T=10 s", W.paper_helix(E=1e7, h=5e-3, dt=6e-3, steps=1667), 7.30),
        ("b2 helix N=100, h=1 mm, E=1e9 Pa, dt=3e-3 s, T=2 s", W.paper_helix(E=1e9, h=1e-3, dt=3e-3, steps=667), 3.18),
        ("c axial friction N=26, 44 pushes in [-10.6, 10.5] N, dt=5e-3 s, T=1.5 s", fr, 1.59),
    ]
    def run(d, scheme):
        sim = dm.sim_from_description(d)
        sim.set_integrator(scheme)
        sim.set_adaptive(8)
        start = sim.checkpoint()
        sim.step(d["dt"], 2, allow_failure=True)
        sim.restore(start)
        steps = int(d["steps"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = sim.step(d["dt"], steps, allow_failure=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sim.close()
        return wall, float(st["iters"].sum() / st["iters"].size / steps), int(st["halvings"].sum()), \
            int((st["status"] != 0).sum())

    for name, d, paper_s in cases:
        steps = int(d["steps"])
        wall, iters, halv, failed = run(d, "midpoint")
        e_wall, e_iters, e_halv, e_failed = run(d, "euler")
        nodes = sum(r["x0"].shape[0] for r in d["rods"])
        row = {"workload": name, "integrator": "implicit midpoint", "systems": len(d["rods"]), "steps": steps,
               "wall_s": wall, "paper_wall_s": paper_s, "paper_over_this": paper_s / wall,
               "node_steps_per_s": nodes * steps / wall, "newton_iters_per_step": iters,
               "halvings": halv, "failed_systems": failed,
               "backward_euler": {"wall_s": e_wall, "newton_iters_per_step": e_iters, "halvings": e_halv,
                                  "failed_systems": e_failed}}
        log(f"paper: {name}: midpoint {wall:.3f} s, backward Euler {e_wall:.3f} s (paper {paper_s} s)")
        print(json.dumps(row), flush=True)


def config_table(dm, log):
    """One line per benchmark configuration: the plain per-system GPU step, the batched launch,
    the warm-started (second-order extrapolation) launch, the CPU oracle on one thread and on
    all cores (bounded samples), FP64 and HBM roofline fractions and Newton iterations per step.
    Each figure is node-steps/s at the 1e-9 residual."""
    import torch

    import workloads as W
    from oracle import adjoint as AD
    from oracle import der
    threads = min(os.cpu_count() or 1, 16)
    rows = []

    def gpu_run(desc, steps, warm=0, block=0):
        sim = dm.sim_from_description(desc, block_size=block)
        sim.set_warm_start(None, warm)
        sim.step(desc["dt"], 1)
        st, wall = timed_steps(sim, desc["dt"], steps)
        assert (st["status"] == 0).all()
        nodes = float(sim.num_nodes)
        kernel_s = sim.last_kernel_ms / 1e3
        iters = float(st["iters"].sum())
        sim.close()
        return nodes * steps / wall, iters / st["iters"].size / steps, kernel_s, nodes, iters

    def fp64_frac(flops, kernel_s):
        return flops / kernel_s / (PEAK_FP64_VALU_TFLOPS * 1e12)

    # single cantilever
    d = W.cantilever(steps=100)
    v, it, ks, nodes, iters = gpu_run(d, 100)
    vw, itw, _, _, _ = gpu_run(d, 100, warm=3)
    one = lambda: (lambda: der.simulate(d, steps=2), 2 * 51)
    rows.append({"config": "cantilever N=51, dt 1e-2, 100 steps", "plain_per_rod_gpu": v, "batched_gpu": None,
                 "warm_started_gpu": vw, "cpu_oracle_1_thread": oracle_rate(one, 1, 4.0),
                 "cpu_oracle_all_cores": oracle_rate(one, threads, 4.0), "cores": threads,
                 "fp64_roof_fraction": fp64_frac(float(rod_iteration_flops(51)) * iters, ks), "hbm_roof_fraction": None,
                 "newton_iters_plain": it, "newton_iters_warm": itw})
    log(f"configs: {rows[-1]}")
    # 1024-rod batch
    d = W.rod_batch(1024)
    n_r = np.array([r["x0"].shape[0] for r in d["rods"]], dtype=float)
    sim = dm.sim_from_description(d)
    sim.step(d["dt"], 1)
    st, wall = timed_steps(sim, d["dt"], 20)
    ks = sim.last_kernel_ms / 1e3
    sim.close()
    v = n_r.sum() * 20 / wall
    it = float(st["iters"].mean() / 20)
    vw, itw, _, _, _ = gpu_run(d, 20, warm=3)
    traffic = measured_traffic(20)
    rng = np.random.Generator(np.random.PCG64(123))
    order = iter(rng.permutation(len(d["rods"])))

    def one_rod():
        r = int(next(order))
        sub = W.subset(d, [r])
        return (lambda: der.simulate(sub, steps=1)), sub["rods"][0]["x0"].shape[0]
    c1 = oracle_rate(one_rod, 1, 6.0)
    call = oracle_rate(one_rod, threads, 6.0)
    rows.append({"config": "1024 rods N~U{20..400}, dt 1e-3", "plain_per_rod_gpu": per_rod_baseline(dm, d, 20),
                 "batched_gpu": v, "warm_started_gpu": vw, "cpu_oracle_1_thread": c1, "cpu_oracle_all_cores": call,
                 "cores": threads, "fp64_roof_fraction": fp64_frac(float((rod_iteration_flops(n_r) * st["iters"]).sum()), ks),
                 "hbm_roof_fraction": None if traffic is None else traffic / ks / 8e12,
                 "newton_iters_plain": it, "newton_iters_warm": itw})
    log(f"configs: {rows[-1]}")
    # six-limb stars
    d1 = W.star_robots(1, steps=10)
    v1, _, _, _, _ = gpu_run(d1, 10)
    d = W.star_robots(4096)
    v, it, ks, nodes, iters = gpu_run(d, 10)
    vw, itw, _, _, _ = gpu_run(d, 10, warm=3)
    star = lambda: (lambda: der.simulate(d1, steps=1), 6 * 30 + 1)
    rows.append({"config": "4096 six-limb stars, floor contact, actuation", "plain_per_rod_gpu": v1,
                 "batched_gpu": v, "warm_started_gpu": vw, "cpu_oracle_1_thread": oracle_rate(star, 1, 6.0),
                 "cpu_oracle_all_cores": oracle_rate(star, threads, 6.0), "cores": threads,
                 "fp64_roof_fraction": fp64_frac(star_iteration_flops() * iters, ks),
                 "hbm_roof_fraction": None, "newton_iters_plain": it, "newton_iters_warm": itw})
    log(f"configs: {rows[-1]}")
    # learned warm start (network) on fresh rods
    ws = warm_start_section(dm, 1000, log)
    rows.append({"config": "learned warm start, trained on 1e6 rod-steps of the 1024-rod batch, 1024 fresh rods "
                           "N~U{50..400}, 1000 steps", "plain_per_rod_gpu": None,
                 "batched_gpu": ws["plain_value"], "warm_started_gpu": ws["network_value"],
                 "warm_started_gpu_extrapolation": ws["extrapolation_value"],
                 "warm_started_gpu_third_order": ws["third_order_value"], "cpu_oracle_1_thread": None,
                 "cpu_oracle_all_cores": None, "cores": threads, "fp64_roof_fraction": None, "hbm_roof_fraction": None,
                 "newton_iters_plain": ws["plain_iters_per_step"], "newton_iters_warm": ws["network_iters_per_step"]})
    log(f"configs: {rows[-1]}")
    # adjoint
    adj = adjoint_section(dm)
    da, kstar = W.adjoint_rods(n_rods=1, n_nodes=100, steps=5)
    _, _, target = AD.rollout(da, [kstar[0]])
    k0 = [np.zeros((98, 2))]

    def adj_unit():
        return (lambda: AD.loss_and_grad(da, k0, target.numpy())), 100 * 5
    rows.append({"config": "adjoint 256 rods x 100 nodes x 200 steps (forward + backward)",
                 "plain_per_rod_gpu": None, "batched_gpu": adj["value"], "warm_started_gpu": None,
                 "cpu_oracle_1_thread": oracle_rate(adj_unit, 1, 8.0),
                 "cpu_oracle_all_cores": oracle_rate(adj_unit, threads, 8.0), "cores": threads,
                 "fp64_roof_fraction": None, "hbm_roof_fraction": None, "newton_iters_plain": None,
                 "newton_iters_warm": None})
    for r in rows:
        print(json.dumps(r), flush=True)


# per contact pair, the terms kernel's algorithmic traffic: reads the pair (2 int32), the four
# nodes' positions now and at the step start (4 x 2 x 24 B), their edge tables (2 x (2 int32 +
# radius)); writes the energy, gradient (12), Hessian (144) and friction forces (12) in float64
CONTACT_TERMS_BYTES_PER_PAIR = 8 + 192 + 2 * 16 + 8 * (1 + 12 + 144 + 12)


def contact_section(dm, reps=10):
    """Edge-edge contact of the entanglement gripper's scenes (4096 tangles of five 60-node
    fingers): detection (broad and narrow phase) and the pair terms (energy, gradient, Hessian,
    friction), each kernel timed by HIP events on the handle's stream."""
    import torch

    import workloads as W
    d = W.contact_tangle(4096)
    c = dm.Contact.from_rods(d["rods"], d["groups"], d["delta"], 1024,
                             stream=torch.cuda.current_stream().cuda_stream)
    x = torch.tensor(np.concatenate([r[0] for r in d["rods"]]), device="cuda")
    xp = torch.tensor(d["x_prev"], device="cuda")
    edges = sum(r[0].shape[0] - 1 for r in d["rods"])
    pairs, dst, counts, total = c.find(x)
    c.terms(x, pairs, counts, d["k_c"], x_prev=xp, dt=d["dt"], mu=d["mu"], nu=d["nu"], friction=True)
    tf, tt = [], []
    for _ in range(reps):
        c.find(x)
        tf.append(c.last_find_ms)
        c.terms(x, pairs, counts, d["k_c"], x_prev=xp, dt=d["dt"], mu=d["mu"], nu=d["nu"], friction=True)
        tt.append(c.last_terms_ms)
    mf, mt = float(np.mean(tf)), float(np.mean(tt))
    nbytes = CONTACT_TERMS_BYTES_PER_PAIR * total
    out = {"workload": "4096 tangles of the entanglement gripper: 5 fingers x 60 nodes, h = 5 mm, delta = 5e-4 m "
                       "(seed 7)", "edges": int(edges), "pairs": int(total),
           "detection_ms": mf, "detection_edges_per_s": edges / (mf * 1e-3),
           "terms_ms": mt, "terms_pairs_per_s": total / (mt * 1e-3),
           "terms_roofline": {"bound": "hbm", "achieved": nbytes / (mt * 1e-3) / 1e9, "peak": 8000.0,
                              "unit": "GB/s", "frac": nbytes / (mt * 1e-3) / 1e9 / 8000.0,
                              "bytes_per_pair": CONTACT_TERMS_BYTES_PER_PAIR}}
    c.close()
    return out


def real2sim_section(dm, n_robots=1024, n_configs=8, tol=1e-3, max_iter=200):
    """Alg. 1 (Real2Sim section) on a batch of two-limb manipulators with the paper's
    parameters: the target limb curvatures of each configuration are those the simulated
    robots show at seeded natural curvatures (a forward solve on the GPU), then every robot's
    natural curvatures are fitted to them from zero, configuration after configuration."""
    import torch

    import workloads as W
    d = W.two_limb_manipulator(n_robots=n_robots)
    kstar = W.limb_curvature_targets(n_configs=n_configs, n_robots=n_robots)
    sizes = [r["x0"].shape[0] - 2 for r in d["rods"]]

    def kbar_all(kv):
        return np.concatenate([np.stack([np.full(n, k), np.zeros(n)], 1).reshape(-1) for n, k in zip(sizes, kv)])
    stream = torch.cuda.current_stream().cuda_stream
    sim = dm.sim_from_description(d, line_search=True, stream=stream)
    targets = []
    for c in range(n_configs):
        sim.set_natural_curvature_all(kbar_all(kstar[c].reshape(-1)))
        sim.step(d["dt"], d["steps"])
        targets.append(sim.limb_curvatures())
    sim.close()
    targets = np.array(targets)
    sim = dm.sim_from_description(d, line_search=True, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    traj, steps, losses = sim.fit_limb_curvatures(d["dt"], d["steps"], targets, alpha0=0.1, tol=tol, max_iter=max_iter)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.close()
    return {"workload": f"{n_robots} two-limb manipulators (limbs of 76 mm, 12 nodes, radius 10 cm, silicone), "
                        f"{n_configs} target configurations from seeded natural curvatures",
            "tol": tol, "alpha0": 0.1, "wall_s": wall, "gradient_steps": int(steps.sum()),
            "configurations_per_s": n_robots * n_configs / wall,
            "converged_fraction": float((losses < tol).mean()),
            "max_kbar_error": float(np.abs(traj - kstar.reshape(n_configs, -1)).max())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-rod", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the batched step (for profiling)")
    ap.add_argument("--paper", action="store_true",
                    help="instead of the bench line, the paper's validation workloads under implicit midpoint")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--configs", action="store_true",
                    help="instead of the headline line, one line per benchmark configuration")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES bytes device to device once (calibrates the HBM byte counters)")
    ap.add_argument("--section", choices=["self_contact", "contact", "stars", "midpoint"], default=None,
                    help="only this extra section (for profiling), one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for --gpus {args.gpus}); independent rod batches "
              "would shard by rods across GPUs with no communication, and no multi-GPU launch is made.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2311_18126_amd as dm
    import workloads as W

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        n = args.copy_calibration // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 8 * n}), flush=True)
        return
    if args.configs:
        config_table(dm, log)
        return
    if args.paper:
        paper_table(dm, log)
        return
    if args.section:
        run = {"self_contact": lambda: self_contact_section(dm, 20, n_rods=256),
               "contact": lambda: contact_section(dm),
               "stars": lambda: star_section(dm, max(args.steps // 5, 5)),
               "midpoint": lambda: midpoint_section(dm, min(args.steps, 100))}[args.section]
        print(json.dumps({args.section: run()}), flush=True)
        return
    desc = W.rod_batch(1024)
    n_nodes = np.array([r["x0"].shape[0] for r in desc["rods"]])
    stream = torch.cuda.current_stream()
    sim = dm.sim_from_description(desc, stream=stream.cuda_stream, block_size=args.block)
    dt = desc["dt"]
    tuned = None
    if not args.no_autotune and args.block == 0:
        tuned = sim.autotune(dt, trial_steps=2)
        log(f"autotuned workgroup size {tuned}")
    if args.warmup > 0:
        sim.step(dt, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = sim.step(dt, args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_s = sim.last_kernel_ms / 1e3
    assert (stats["status"] == 0).all() and (stats["steps"] == args.steps).all(), np.unique(stats["status"])
    # systems are rods here, in order
    iters = stats["iters"].astype(np.float64)
    node_steps = float(n_nodes.sum()) * args.steps
    flops = float((rod_iteration_flops(n_nodes) * iters).sum())
    achieved = flops / kernel_s / 1e12
    traffic = measured_traffic(args.steps)
    out = {
        "metric": METRIC,
        "value": node_steps / wall,
        "unit": "node-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "1024 clamped rods, N~U{20..400} (seed 0), L~U(0.5,2) m, h~U(1,5) mm, "
                               "E=10^U(6,8) Pa, kbar~N(0,2^2)/m, gravity, dt=1e-3 s, Newton tol 1e-9",
                   "rods": int(len(n_nodes)), "nodes": int(n_nodes.sum()), "dt": dt,
                   "launch": "one persistent launch per call, one workgroup per rod",
                   "block_size": sim.block_size, "autotuned": tuned is not None},
        "newton_iters_per_step": float(iters.sum() / len(iters) / args.steps),
        "floor_steps": int(stats["floor_steps"].sum()),
        # largest residual among the steps accepted at their rounding floor, and that step's
        # computed floor (every floor-ended step has residual <= its floor by construction)
        "floor_residual_max": float(stats["floor_residual_max"].max()),
        "floor_estimate_at_max": float(stats["floor_estimate"][int(np.argmax(stats["floor_residual_max"]))]),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_VALU_TFLOPS, "traffic": traffic,
                     "kernel": "dm_step_kernel", "kernel_ms": 1e3 * kernel_s,
                     "algorithmic_flops": flops, "flops_from": "profiles/flop_count.json (dm_flops)",
                     "flops_per_node_iteration": flops / float((n_nodes * iters).sum())},
    }
    sim.close()
    if not args.no_extras:
        out["warm_start"] = warm_start_section(dm, 1000, log)
        out["stars"] = star_section(dm, max(args.steps // 5, 5))
        # over the whole 1000 steps some short stiff rods gain energy under the undamped rule
        # until Newton fails (22 of 1024 even with halving): the section times the first 100
        out["midpoint"] = midpoint_section(dm, min(args.steps, 100))
        out["adjoint"] = adjoint_section(dm)
        out["real2sim"] = real2sim_section(dm)
        out["contact"] = contact_section(dm)
        out["self_contact"] = self_contact_section(dm, 20, n_rods=256)
    if not args.no_per_rod:
        out["per_rod_plain_value"] = per_rod_baseline(dm, desc, min(args.steps, 20))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(desc)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
