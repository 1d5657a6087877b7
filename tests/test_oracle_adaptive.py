"""The oracle's adaptive time stepping (step_adaptive): a failed step is redone as two half
steps, recursively.  The halving rule is a reading (the paper names the option without a rule)
and composes steps pinned elsewhere, so these tests fix its bookkeeping: no failure leaves the
step untouched, a forced failure covers the interval exactly by smaller converged steps, and an
exhausted depth reports failure from the last converged substep."""
import numpy as np
import pytest

import workloads as W
from oracle import der


def test_without_failure_the_adaptive_step_is_the_plain_step():
    d = W.cantilever()
    sys_, st = der.build(d, [0])
    a, ok, iters, hv = der.step_adaptive(sys_, st.clone(), d["dt"], d["tol"], 50, max_halvings=3)
    b, info = der.step(sys_, st.clone(), d["dt"], d["tol"], 50)
    assert ok and hv == 0 and iters == info.iters
    assert np.array_equal(a.x.numpy(), b.x.numpy()) and a.time == b.time


def test_forced_failure_is_covered_by_converged_half_steps():
    """Newton limited to 3 iterations fails on the full cantilever step; the step is covered by
    halves (and quarters where needed), whose sizes sum to the step."""
    d = W.cantilever()
    sys_, st = der.build(d, [0])
    st, _ = der.step(sys_, st, d["dt"], d["tol"], 50)          # leave rest: later steps need 5 iterations
    _, info = der.step(sys_, st.clone(), d["dt"], d["tol"], 3)
    assert not info.converged
    a, ok, iters, hv = der.step_adaptive(sys_, st.clone(), d["dt"], d["tol"], 3, max_halvings=4)
    assert ok and hv >= 1
    assert a.time == pytest.approx(st.time + d["dt"], abs=1e-15)
    # the same interval by hand: halves, each split again if it fails
    def cover(s, h, depth):
        s1, info = der.step(sys_, s, h, d["tol"], 3)
        if info.converged:
            return s1, 0
        m, n1 = cover(s, 0.5 * h, depth + 1)
        e, n2 = cover(m, 0.5 * h, depth + 1)
        return e, 1 + n1 + n2
    b, nb = cover(st.clone(), d["dt"], 0)
    assert nb == hv
    assert np.array_equal(a.x.numpy(), b.x.numpy())


def test_exhausted_depth_fails_at_the_last_converged_substep():
    d = W.cantilever()
    sys_, st = der.build(d, [0])
    st, _ = der.step(sys_, st, d["dt"], d["tol"], 50)
    a, ok, _, hv = der.step_adaptive(sys_, st.clone(), d["dt"], d["tol"], 1, max_halvings=1)
    assert not ok and hv == 1
    assert st.time <= a.time < st.time + d["dt"]
