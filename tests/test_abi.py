"""The C-ABI library loads and exports every function declared in include/dmrod.h
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmrod.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(dm_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def library():
    import paper_2311_18126_amd as dm
    if not os.path.exists(dm.LIB_PATH):
        from paper_2311_18126_amd import build
        build.build()
    return ctypes.CDLL(dm.LIB_PATH)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("dm_create", "dm_add_rod", "dm_add_joint", "dm_set_natural_curvature", "dm_finalize",
                 "dm_step", "dm_get_state", "dm_destroy", "dm_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(library):
    missing = [n for n in declared_functions() if not hasattr(library, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    import paper_2311_18126_amd as dm
    assert set(declared_functions()) <= set(dm._SIGS), set(declared_functions()) - set(dm._SIGS)


def test_config_struct_matches_header_defaults(library):
    import paper_2311_18126_amd as dm
    cfg = dm.DmConfig()
    dm.lib().dm_config_default(ctypes.byref(cfg))
    assert cfg.newton_tol == 1e-9 and cfg.max_iter == 50 and cfg.gravity[2] == -9.81
    assert cfg.block_size == 0 and cfg.floor_contact == 0 and cfg.floor_factor == 1.0
    assert not cfg.alloc and not cfg.free_ and not cfg.alloc_ctx


def test_missing_device_is_an_error_not_a_fallback(library):
    """Without a GPU, dm_create must fail with DM_ERR_HIP (the product never runs on the CPU)."""
    import torch

    import paper_2311_18126_amd as dm
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(dm.DmError) as e:
        dm.Sim()
    assert e.value.status == dm.DM_ERR_HIP


def test_fit_checks_array_sizes_before_the_library_call():
    """The binding refuses a target or start curvature of the wrong size (the C entry point
    reads the sizes it is told); no GPU is touched before the check."""
    import paper_2311_18126_amd as dm

    class Probe(dm.Sim):
        def __init__(self):     # no library call: only the size checks run
            pass
        num_rods = 2
        kbar_size = 12
    p = Probe()
    with pytest.raises(ValueError):
        p.fit_natural_curvature(1e-3, 4, np.zeros((4, 1, 3)))
    with pytest.raises(ValueError):
        p.fit_natural_curvature(1e-3, 4, np.zeros((4, 2, 3)), kbar0=np.zeros(5))
