"""Device memory of a simulation through the allocator hook of dm_config (alloc / free_ /
alloc_ctx): the Python binding hands the library PyTorch's caching allocator, so PyTorch owns
the simulation's pages; with the hook off the library uses hipMalloc.  Both give the same
trajectory bit for bit."""
import os

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dm():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2311_18126_amd as m
    assert os.path.exists(m.LIB_PATH), "libdmrod.so is not built"
    return m


def test_simulation_buffers_come_from_torch(dm):
    d = W.rod_batch(64, seed=5, nmax=120)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    sim = dm.sim_from_description(d)                     # torch_memory=True (default)
    held = torch.cuda.memory_allocated() - base
    dofs = sum(4 * r["x0"].shape[0] - 1 for r in d["rods"])
    assert held >= 21 * 8 * dofs, (held, dofs)           # at least the band storage
    sim.step(d["dt"], 3)
    a = sim.state()
    sim.rollout(d["dt"], 4, 2)                           # checkpoint and tip buffers, grown on use
    assert torch.cuda.memory_allocated() - base > held   # come from torch too
    sim.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base         # every buffer went back at destroy
    ref = dm.sim_from_description(d, torch_memory=False)
    assert torch.cuda.memory_allocated() == base         # hipMalloc: torch sees nothing
    ref.step(d["dt"], 3)
    for u, w in zip(a, ref.state()):
        assert np.array_equal(u, w)
    ref.close()


def test_failed_allocation_is_reported(dm):
    """An allocator that refuses gives DM_ERR_OOM from dm_finalize, and nothing leaks."""
    import ctypes
    calls = {"alloc": 0, "free": 0}
    live = []

    def alloc(nbytes, ctx):
        calls["alloc"] += 1
        if calls["alloc"] > 5:
            return None
        p = torch.cuda.caching_allocator_alloc(int(nbytes))
        live.append(p)
        return p

    def free(ptr, ctx):
        calls["free"] += 1
        torch.cuda.caching_allocator_delete(ptr)
        live.remove(ptr)
    sim = dm.Sim(torch_memory=False)
    hooks = (dm.ALLOC_FN(alloc), dm.FREE_FN(free))
    L = dm.lib()
    cfg = dm.DmConfig()
    L.dm_config_default(ctypes.byref(cfg))
    cfg.alloc, cfg.free_ = hooks
    h = ctypes.c_void_p()
    assert L.dm_create(ctypes.byref(cfg), ctypes.byref(h)) == dm.DM_OK
    x = np.ascontiguousarray(W.straight_nodes(20, 0.5))
    rid = ctypes.c_int()
    assert L.dm_add_rod(h, 20, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1e-3, 1e7, 0.5, 1000.0,
                        ctypes.byref(rid)) == dm.DM_OK
    assert L.dm_finalize(h) == dm.DM_ERR_OOM
    assert calls["alloc"] == 6 and calls["free"] == 5 and not live
    L.dm_destroy(h)
    sim.close()
