"""Pins of the warm-start network oracle (oracle/mlp.py)."""
import numpy as np
import torch

from oracle import mlp


def test_bf16_rounding_matches_the_library_conversion():
    rng = np.random.Generator(np.random.PCG64(1))
    a = (rng.normal(size=20000) * 10.0 ** rng.integers(-30, 30, 20000)).astype(np.float32)
    a = np.concatenate([a, np.array([0.0, -0.0, 1.0, np.inf, -np.inf, 3.0e38, 1e-40, -1e-40], dtype=np.float32)])
    # exact ties: the low 16 bits are 0x8000, half-way between two bfloat16 values
    ties = ((rng.integers(0, 0x7F7F, 1000).astype(np.uint32) << 16) | 0x8000).astype(np.uint32).view(np.float32)
    a = np.concatenate([a, ties, -ties]).astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    got = mlp.bf16_round(a)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    assert np.isnan(mlp.bf16_round(np.array([np.nan], dtype=np.float32))[0])


def test_features_of_a_straight_rod():
    n = 5
    x = np.stack([np.linspace(0, 0.4, n), np.zeros(n), np.zeros(n)], 1)
    x[2, 2] = 0.01
    v = np.zeros((n, 3))
    v[:, 2] = np.arange(n)
    vp = np.zeros((n, 3))
    vp[:, 2] = 0.5 * np.arange(n)
    vp2 = np.zeros((n, 3))
    vp2[:, 2] = 0.25 * np.arange(n) ** 2
    kb = np.arange(2 * (n - 2), dtype=float).reshape(n - 2, 2)
    f = mlp.rod_features(x, v, vp, vp2, kb, 1e7, 2e-3, np.full(n - 1, 0.1))
    assert f[0, 2] == 0.0 and f[0, 5] == 1.0 and f[-1, 5] == 0.0 and f[-1, 2] == -1.0   # replicated ends
    assert f[2, 8] == 2 and f[2, 11] == 1.0                          # v and a = v - v_prev
    assert np.allclose(f[2, 12:15], [0.0, 0.0, -0.02]) and np.allclose(f[1, 12:15], [0.0, 0.0, 0.01])
    assert np.allclose(f[0, 12:15], [0.1, 0.0, 0.0])                 # x_1 - x_0 at the end
    assert np.allclose(f[:, 15], 7.0) and np.allclose(f[:, 16], 2e-3) and np.allclose(f[:, 17], 0.1)
    assert np.array_equal(f[0, 18:20], kb[0]) and np.array_equal(f[-1, 18:20], kb[-1])
    assert np.array_equal(f[2, 18:20], kb[1])
    # a_i = 0.5 i, a_prev_i = 0.5 i - 0.25 i^2: j_i = 0.25 i^2; the Laplacian of a is zero inside
    # (a is linear in i) and +-0.5 at the replicated ends
    assert np.allclose(f[:, 22], 0.25 * np.arange(n) ** 2) and np.allclose(f[:, 20:22], 0.0)
    assert np.allclose(f[1:-1, 25], 0.0) and f[0, 25] == 0.5 and f[-1, 25] == -0.5
    assert f.shape == (n, 26)


def test_backward_without_rounding_matches_automatic_differentiation():
    rng = np.random.Generator(np.random.PCG64(2))
    p = mlp.init_params(3)
    X = rng.normal(size=(64, mlp.N_IN)).astype(np.float32)
    T = rng.normal(size=(64, mlp.N_OUT)).astype(np.float32)
    L, _, g = mlp.loss_and_backward(p, X, T, rounding=False)
    Lr, gr = mlp.autograd_reference(p, X, T)
    assert abs(L - Lr) <= 1e-12 * abs(Lr)
    for k in gr:
        assert np.abs(g[k] - gr[k]).max() <= 1e-10 * np.abs(gr[k]).max(), k


def test_rounded_network_stays_within_the_bfloat16_error_bound():
    rng = np.random.Generator(np.random.PCG64(4))
    p = mlp.init_params(5)
    X = rng.normal(size=(256, mlp.N_IN)).astype(np.float32)
    T = rng.normal(size=(256, mlp.N_OUT)).astype(np.float32)
    y, _ = mlp.forward(p, X, rounding=True)
    y0, _ = mlp.forward(p, X, rounding=False)
    # five roundings to 8-bit significands on the way (input, two activations, three weights):
    # a relative perturbation of at most ~6 * 2^-8 per path
    assert np.linalg.norm(y - y0) <= 6 * 2.0 ** -8 * np.linalg.norm(y0)
    _, _, g = mlp.loss_and_backward(p, X, T, rounding=True)
    _, _, g0 = mlp.loss_and_backward(p, X, T, rounding=False)
    for k in g:
        assert np.linalg.norm(g[k] - g0[k]) <= 12 * 2.0 ** -8 * np.linalg.norm(g0[k]), k


def test_first_adam_step_has_its_closed_form():
    """With zero moments, the first bias-corrected step is -lr g / (|g| + eps)."""
    rng = np.random.Generator(np.random.PCG64(6))
    p = mlp.init_params(7)
    g = {k: rng.normal(size=a.shape) * 10.0 ** rng.integers(-6, 2, a.shape) for k, a in p.items()}
    p0 = {k: a.copy() for k, a in p.items()}
    mlp.adam_step(p, g, mlp.zeros_like(p), mlp.zeros_like(p), 1, lr=1e-3)
    for k in p:
        ref = (p0[k].astype(np.float64) - 1e-3 * g[k] / (np.abs(g[k]) + 1e-8)).astype(np.float32)
        assert np.array_equal(p[k], ref), k


def test_training_reduces_the_loss_on_a_smooth_target():
    rng = np.random.Generator(np.random.PCG64(8))
    p = mlp.init_params(9)
    X = rng.normal(size=(512, mlp.N_IN)).astype(np.float32)
    T = np.stack([np.sin(X[:, 0]), X[:, 1] * X[:, 2], np.tanh(X[:, 3])], 1).astype(np.float32)
    m, v = mlp.zeros_like(p), mlp.zeros_like(p)
    L0 = mlp.loss_and_backward(p, X, T)[0]
    for t in range(1, 61):
        L, _, g = mlp.loss_and_backward(p, X, T)
        mlp.adam_step(p, g, m, v, t)
    assert L < 0.5 * L0
