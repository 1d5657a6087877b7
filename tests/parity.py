"""Parity measures of GPU positions against the oracle's (shared by the GPU tests).

Absolute positions are O(1 m) while one step moves a node by 1e-5..1e-3 m, so a position
error relative to the positions alone says little about the step.  Every parity check also
measures the error against the displacement from the reference start shape x0 (the same start
for both sides, so the displacement error is the position error), as a 2-norm ratio and node by
node: the largest node error over the largest node displacement."""
import numpy as np


def measures(x, ref, x0):
    """(position-relative, displacement-relative, per-node) errors of x against ref."""
    x, ref, x0 = (np.asarray(a, dtype=np.float64).reshape(-1, 3) for a in (x, ref, x0))
    e = x - ref
    d = ref - x0
    pos = float(np.linalg.norm(e) / np.linalg.norm(ref))
    if not np.any(d):                      # nothing moved (a fully clamped rod): exact match
        return pos, (0.0 if not np.any(e) else np.inf), (0.0 if not np.any(e) else np.inf)
    disp = float(np.linalg.norm(e) / np.linalg.norm(d))
    node = float(np.linalg.norm(e, axis=1).max() / np.linalg.norm(d, axis=1).max())
    return pos, disp, node


def assert_parity(x, ref, x0, pos_tol, disp_tol, what=""):
    """Position error within pos_tol of the positions and within disp_tol of the displacement
    (2-norm and per node)."""
    pos, disp, node = measures(x, ref, x0)
    assert pos < pos_tol and disp < disp_tol and node < disp_tol, (what, pos, disp, node)
    return pos, disp, node
