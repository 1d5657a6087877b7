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


def save(net: Mlp, path):
    mean, std, scale = net.get_normalisation()
    np.savez(path, params=net.get_params(), mean=mean, std=std, scale=scale)


def load(path, max_rows, stream=None) -> Mlp:
    d = np.load(path)
    net = Mlp(max_rows, stream=stream)
    net.set_params(d["params"])
    net.set_normalisation(d["mean"], d["std"], d["scale"])
    return net
