"""Argument checks of the contact entry points, which run before any device work (no GPU
needed): each bad table is refused with DM_ERR_INVALID_ARG and a message."""
import ctypes
import os

import numpy as np
import pytest

import paper_2311_18126_amd as dm


def create(**kw):
    a = dict(n_nodes=4, edges=[(0, 1), (2, 3)], rod=[0, 1], arc0=[0.0, 0.0], ebar=[0.01, 0.01],
             radius=[5e-3, 5e-3], group_start=[0, 2], delta=5e-4, cap=16)
    a.update(kw)
    e = np.ascontiguousarray(a["edges"], dtype=np.int32).reshape(-1, 2)
    ne = e.shape[0]
    r = np.ascontiguousarray(a["rod"], dtype=np.int32)
    f = [np.ascontiguousarray(a[k], dtype=np.float64) for k in ("arc0", "ebar", "radius")]
    gs = np.ascontiguousarray(a["group_start"], dtype=np.int32)
    h = ctypes.c_void_p()
    IP, DP = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    st = dm.lib().dm_contact_create(0, None, a["n_nodes"], ne, e.ctypes.data_as(IP), r.ctypes.data_as(IP),
                                    *(v.ctypes.data_as(DP) for v in f), gs.size - 1, gs.ctypes.data_as(IP),
                                    a["delta"], a["cap"], ctypes.byref(h))
    return st, dm.lib().dm_contact_last_error().decode()


@pytest.mark.skipif(not os.path.exists(dm.LIB_PATH), reason="libdmrod.so is not built")
@pytest.mark.parametrize("kw,msg", [
    (dict(delta=0.0), "delta"),
    (dict(cap=0), "pair_capacity"),
    (dict(cap=4096), "pair_capacity"),
    (dict(group_start=[0, 1]), "group_start"),
    (dict(group_start=[0, 2, 1, 2]), "edges"),
    (dict(edges=[(0, 1), (2, 4)]), "node index"),
    (dict(edges=[(0, 1), (2, 2)]), "node index"),
    (dict(radius=[5e-3, 0.0]), "radius"),
    (dict(ebar=[0.01, float("nan")]), "radius, length"),
])
def test_bad_tables_are_refused(kw, msg):
    st, err = create(**kw)
    assert st == dm.DM_ERR_INVALID_ARG
    assert msg in err


@pytest.mark.skipif(not os.path.exists(dm.LIB_PATH), reason="libdmrod.so is not built")
def test_group_size_limit():
    n = 2049
    st, err = create(n_nodes=2 * n, edges=[(2 * i, 2 * i + 1) for i in range(n)], rod=list(range(n)),
                     arc0=[0.0] * n, ebar=[0.01] * n, radius=[5e-3] * n, group_start=[0, n])
    assert st == dm.DM_ERR_INVALID_ARG and "2049 edges" in err
