"""The allocation-free forward pass of the warm-start network (dm_mlp_forward_noalloc, for
callers that cannot allocate device memory) against the forward pass that uses the network's
own buffers (dm_mlp_forward): the same kernels, so the outputs must be equal bit for bit, on
two calls in a row (the second with fewer rows, so the static buffer still holds the first
call's rows beyond them), and a row count beyond the static buffer is refused."""
import os

import numpy as np
import pytest
import torch

NI = 26      # features per row of the warm-start network

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dm():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2311_18126_amd as m
    assert os.path.exists(m.LIB_PATH), "libdmrod.so is not built"
    return m


def features(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return torch.tensor(rng.normal(size=(n, NI)) * rng.uniform(0.1, 5.0, NI) + rng.normal(size=NI), device="cuda")


def test_noalloc_forward_equals_forward(dm):
    rng = np.random.Generator(np.random.PCG64(21))
    net = dm.Mlp(4096)
    lim = np.concatenate([np.full(256 * NI, np.sqrt(6 / NI)), np.zeros(256), np.full(256 * 256, np.sqrt(6 / 256)),
                          np.zeros(256), np.full(3 * 256, np.sqrt(6 / 256)), np.zeros(3)])
    params = (rng.uniform(-1.0, 1.0, lim.size) * lim).astype(np.float32)
    params[256 * NI:256 * (NI + 1)] = rng.normal(0, 0.1, 256).astype(np.float32)     # nonzero first-layer biases
    net.set_params(params)
    net.set_normalisation(rng.normal(size=NI), rng.uniform(0.5, 2.0, NI), np.array([1e-4, 3e-5, 2e-4]))
    for n, seed in ((dm.DM_MLP_NOALLOC_MAX_ROWS, 1), (300, 2), (1, 3)):
        print(f"case: noalloc forward, {n} rows", flush=True)
        F = features(n, seed)
        a = net.forward(F, torch.empty((n, 3), dtype=torch.float32, device="cuda"))
        b = net.forward_noalloc(F, torch.full((n, 3), float("nan"), dtype=torch.float32, device="cuda"))
        assert torch.isfinite(a).all()
        assert torch.equal(a, b), (n, float((a - b).abs().max()))
    with pytest.raises(dm.DmError) as e:
        n = dm.DM_MLP_NOALLOC_MAX_ROWS + 1
        net.forward_noalloc(features(n, 4), torch.empty((n, 3), dtype=torch.float32, device="cuda"))
    assert e.value.status == dm.DM_ERR_INVALID_ARG
    net.close()
