"""What a position guess can gain (oracle, CPU).

The warm start hands Newton a guess of the end-of-step positions and leaves the twists at the
step start.  On a rod of the warm-start evaluation set after 30 steps, the Newton iterations
from the step start, from the second- and third-order extrapolations, and from the exact
end-of-step positions themselves are counted at the step's 1e-9 residual: the exact positions
still leave 2 iterations, so no position guess (analytic or learned) can take a step below 2,
and the analytic extrapolation already reaches that count.  The residual is that of Eq. 16
(backward Euler) at the stated tolerance; the first Newton update has to bring the residual
below about 1e-4 N for one iteration to suffice, which the twist error of theta_n alone
exceeds."""
import torch

import workloads as W
from oracle import der


def test_exact_positions_still_take_two_newton_iterations():
    ev = W.warm_start_eval(64, steps=40)
    ns = [r["x0"].shape[0] for r in ev["rods"]]
    rid = min(range(len(ns)), key=lambda i: abs(ns[i] - 60))
    d = W.subset(ev, [rid])
    sys_, st = der.build(d)
    dt = d["dt"]
    hist = []
    for _ in range(30):
        hist.append(st.v.clone())
        st, info = der.step(sys_, st, dt)
        assert info.converged
    v, vp, vp2 = st.v, hist[-1], hist[-2]
    a, ap = v - vp, vp - vp2
    kap = der.natural_curvature(sys_, st.time + dt)
    q_star, info = der.newton_solve(sys_, st, dt, kap)
    xs, _ = der.unpack(sys_, q_star)
    iters = {}
    for name, xg in (("step start", st.x), ("second order", st.x + dt * (v + a)),
                     ("third order", st.x + dt * (v + 2 * a - ap)), ("exact positions", xs)):
        _, inf = der.newton_solve(sys_, st, dt, kap, q0=der.pack(xg, st.theta))
        assert inf.converged and not inf.at_floor
        iters[name] = inf.iters
    print(iters)
    assert iters["exact positions"] == 2
    assert iters["second order"] == iters["third order"] == 2
    assert iters["step start"] >= 2
    # the twists are what is left: exact positions and exact twists need no iteration
    _, inf = der.newton_solve(sys_, st, dt, kap, q0=q_star)
    assert inf.iters == 0
