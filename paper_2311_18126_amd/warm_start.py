"""Learned warm start: data from the solver's own trajectories, training and evaluation.

Every numerical step runs in libdmrod's kernels (features, targets, standardisation,
forward, backward, Adam); torch only provides device buffers and the shuffled row order.
"""
from __future__ import annotations

import numpy as np

from . import NET_IN, Mlp

N_IN, N_HID, N_OUT = NET_IN, 256, 3


def init_params(seed=0):
    """Seeded He-uniform weights and zero biases in the library's parameter layout
    (W1 [256][26], b1, W2 [256][256], b2, W3 [3][256], b3), float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for n_out, n_in in ((N_HID, N_IN), (N_HID, N_HID), (N_OUT, N_HID)):
        lim = np.sqrt(6.0 / n_in)
        parts.append(rng.uniform(-lim, lim, size=n_out * n_in))
        parts.append(np.zeros(n_out))
    return np.concatenate(parts).astype(np.float32)


def collect(sim, dt, steps, every=1):
    """Step `sim` for `steps` steps (plain Newton) and return device tensors (F, T) of the
    features at the start and the targets (the displacement beyond the third-order
    extrapolation) of every `every`-th step."""
    import torch
    rows = sim.ws_rows
    Fs, Ts = [], []
    for k in range(steps):
        take = k % every == 0
        if take:
            F = torch.empty((rows, N_IN), dtype=torch.float64, device="cuda")
            sim.ws_features(F)
        sim.step(dt, 1)
        if take:
            T = torch.empty((rows, N_OUT), dtype=torch.float64, device="cuda")
            sim.ws_targets(F, dt, T)
            Fs.append(F)
            Ts.append(T)
    return torch.cat(Fs), torch.cat(Ts)


def train(net: Mlp, F, T, epochs=2, batch=8192, lr=1e-3, seed=0, log=None):
    """Fit the standardisation on (F, T), then Adam over shuffled mini-batches (one library
    call per epoch; the shuffle is torch's seeded randperm).  Returns the mean loss of each
    epoch."""
    import torch
    net.fit_normalisation(F, T)
    g = torch.Generator(device=F.device)
    g.manual_seed(seed)
    n = F.shape[0]
    F, T = F.contiguous(), T.contiguous()
    hist = []
    for e in range(epochs):
        perm = torch.randperm(n, generator=g, device=F.device).to(torch.int32)
        hist.append(net.train_epoch(F, T, perm, batch, lr))
        if log:
            log(f"epoch {e}: loss {hist[-1]:.4e}")
    return hist


def train_streamed(net: Mlp, sim, dt, steps, chunk=100, batch=8192, lr=(1e-3, 3e-4), seed=0, log=None):
    """Train on the simulation's own trajectory as it is generated, without keeping it.  A
    calibration pass first steps through the whole horizon once, keeping the features and
    targets of the first step of every chunk, fits the standardisation on them (so the output
    scale covers the whole run, not its start) and restores the starting state.  Then `steps`
    steps (plain Newton) are taken again in chunks of `chunk`; the features and targets of every
    step of a chunk are collected on the device, trained once (one Adam epoch over its shuffled
    rows, the learning rate going linearly from lr[0] to lr[1] over the chunks) and dropped.
    The two steps after the restore are taken without training (see below).  Returns the mean
    loss per chunk and the number of rows trained on."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    hist, rows_seen = [], 0
    n_chunks = (steps + chunk - 1) // chunk
    start = sim.checkpoint_torch()
    Fs, Ts = [], []
    for c in range(n_chunks):
        m = min(chunk, steps - c * chunk)
        F, T = collect(sim, dt, m, every=m)
        Fs.append(F)
        Ts.append(T)
    net.fit_normalisation(torch.cat(Fs), torch.cat(Ts))
    del Fs, Ts
    sim.restore(start)
    # a restored state has no velocity history (a = j = 0): the first two steps' features are
    # not those of the trajectory, so they are stepped over
    sim.step(dt, 2)
    for c in range(n_chunks):
        m = min(chunk, steps - c * chunk) - (2 if c == 0 else 0)
        F, T = collect(sim, dt, m, every=1)
        n = F.shape[0]
        perm = torch.randperm(n, generator=g, device="cuda").to(torch.int32)
        rate = lr[0] + (lr[1] - lr[0]) * (c / max(n_chunks - 1, 1))
        hist.append(net.train_epoch(F, T, perm, min(batch, n), rate))
        rows_seen += (n // min(batch, n)) * min(batch, n)
        if log:
            log(f"chunk {c}: {n} rows, loss {hist[-1]:.4e}")
        del F, T, perm
    return hist, rows_seen


def save(net: Mlp, path):
    mean, std, scale = net.get_normalisation()
    np.savez(path, params=net.get_params(), mean=mean, std=std, scale=scale)


def load(path, max_rows, stream=None) -> Mlp:
    d = np.load(path)
    net = Mlp(max_rows, stream=stream)
    net.set_params(d["params"])
    net.set_normalisation(d["mean"], d["std"], d["scale"])
    return net
