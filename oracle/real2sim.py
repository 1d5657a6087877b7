"""Real2Sim fitting of natural curvature to target limb curvatures (oracle).

TEST INFRASTRUCTURE ONLY: used by tests/ to check the HIP path; never imported by the product
path.

The paper's Real2Sim section fits the natural curvatures of a joined two-limb soft manipulator
to curvatures measured on hardware (Alg. 1):

* the movement is quasi-static and each limb has about constant curvature; F(kbar) is the
  simulated configuration for natural curvatures kbar = (kbar_1, kbar_2), one per limb, and
  kappa_1, kappa_2 its limb curvatures from Eq. 5;
* the loss of one target configuration is lambda = |kappa*_1 - kappa_1| + |kappa*_2 - kappa_2|
  (Eq. 19);
* for every target configuration in turn: the step size alpha is reset to 0.1 and lambda_prev
  to infinity; loop: evaluate lambda at the current kbar, stop below the tolerance, halve
  alpha when lambda rose, keep lambda_prev, step kbar <- kbar - alpha grad lambda (Eq. 21);
  kbar carries over from one configuration to the next; the output is the trajectory of the
  fitted kbar, one entry per configuration.

Readings (the paper is silent on them):

* F(kbar) is reached by `n_settle` backward-Euler steps of a long time step `dt` (inertia
  negligible: a static solve) from the robot's current state, so that each evaluation continues
  from the previous one as a quasi-static sweep does; Newton runs with line search;
* a limb's curvature is the mean over its interior stencils of the first integrated curvature
  of Eq. 5 divided by the rest Voronoi length (1/m); kbar_j is the limb's natural curvature in
  1/m in the first material direction at every interior stencil (the second component zero);
* the gradient of Eq. 20 (forward differences) is replaced by the exact gradient of the static
  equilibrium: with R(q; kbar) = 0 the residual of the settled step (the settled state as its
  own step start), dq/dkbar = -J^-1 dR/dkbar, so grad lambda = -mu^T dR/dkbar with
  J^T mu = d lambda/dq;
* an iteration cap per configuration (the paper's loop has none).

Pinned by tests/test_oracle_real2sim.py: the gradient against central differences of re-settled
equilibria (the paper's own finite-difference route, made central), the stress-free case
without gravity (limb curvature equals the natural curvature, so the fit lands on the target),
and the recovery of known natural curvatures from the targets they produce.
"""
from __future__ import annotations

import math

import torch

from . import der


def kbar_rods(sys, kv):
    """Per-rod natural-curvature arrays (N-2, 2) in 1/m from one value per rod (first component)."""
    out = []
    for k, rn in enumerate(sys.rod_nodes):
        n = len(rn) - 2
        z = torch.zeros(n, dtype=der.DT)
        out.append(torch.stack([kv[k] * torch.ones(n, dtype=der.DT), z], 1))
    return out


def limb_curvatures(sys, x, theta, st):
    """Mean over each rod's interior stencils of kappa_1 (Eq. 5) over the rest Voronoi length,
    at positions x and twists theta with frames carried from the step start st (1/m)."""
    kap, _, _ = der.strains(sys, x, theta, st)
    out = []
    for k in range(len(sys.rod_nodes)):
        sel = sys.st_rod == k
        out.append((kap[sel, 0] / sys.Vbar[sel]).mean())
    return torch.stack(out)


def settle(sys, st, kv, dt, n_settle, tol=1e-9, max_iter=50, polish=1):
    """F(kbar): n_settle backward-Euler steps of dt with line search from the state st."""
    kb = kbar_rods(sys, kv)
    for _ in range(n_settle):
        st, info = der.step(sys, st, dt, tol, max_iter, kbar_rods=kb, polish=polish, line_search=True)
        if not info.converged:
            raise RuntimeError(f"real2sim settle: Newton did not converge ({info.history[-3:]})")
    return st


def curvature_gradient(sys, st, kv, weights, dt):
    """d (sum_j weights_j kappa_j) / d kbar at the settled state st (one value per rod), by the
    implicit-function theorem on the residual of a step of dt from st itself."""
    free = ~sys.fixed
    q = der.pack(st.x, st.theta)

    def R(qq, kk):
        kap = der.natural_curvature(sys, st.time + dt, kbar_rods(sys, kk))
        return der.residual(sys, qq, st, dt, kap)

    kv = torch.as_tensor(kv, dtype=der.DT)
    J = torch.func.jacfwd(R, argnums=0)(q, kv)[free][:, free]
    dR = torch.func.jacfwd(R, argnums=1)(q, kv)[free]
    w = torch.as_tensor(weights, dtype=der.DT)

    def objective(qq):
        x, th = der.unpack(sys, qq)
        return (w * limb_curvatures(sys, x, th, st)).sum()
    g = torch.func.grad(objective)(q)[free]
    mu = torch.linalg.solve(J.T, g)
    return -(mu @ dR)


def loss(target, kappa):
    """Eq. 19 summed over the limbs."""
    return float((torch.as_tensor(target, dtype=der.DT) - kappa).abs().sum())


def solve_natural_curvatures(desc, targets, dt=None, n_settle=None, alpha0=0.1, tol=1e-3, max_iter=200):
    """Alg. 1 for one robot (desc's rods are its limbs) over a sequence of target limb
    curvatures (S, n_rods).  Returns the fitted natural curvature after each configuration
    (S, n_rods), the loss of every evaluation in order, the number of gradient steps per
    configuration, and the final state."""
    dt = desc["dt"] if dt is None else dt
    n_settle = desc["steps"] if n_settle is None else n_settle
    sys, st = der.build(desc)
    n_rods = len(sys.rod_nodes)
    kv = torch.zeros(n_rods, dtype=der.DT)
    traj, losses, steps = [], [], []
    for tgt in targets:
        tgt = torch.as_tensor(tgt, dtype=der.DT)
        alpha, prev, it = alpha0, math.inf, 0
        while True:
            st = settle(sys, st, kv, dt, n_settle)
            kappa = limb_curvatures(sys, st.x, st.theta, st)
            lam = loss(tgt, kappa)
            losses.append(lam)
            if lam < tol or it >= max_iter:
                break
            if lam > prev:
                alpha *= 0.5
            prev = lam
            g = curvature_gradient(sys, st, kv, torch.sign(kappa - tgt), dt)
            kv = kv - alpha * g
            it += 1
        traj.append(kv.clone())
        steps.append(it)
    return torch.stack(traj), losses, steps, st


def curvatures_at(desc, kv_sequence, dt=None, n_settle=None):
    """The limb curvatures of the quasi-static configurations reached, in sequence, at the given
    natural curvatures (S, n_rods): the targets a fit to those natural curvatures would see."""
    dt = desc["dt"] if dt is None else dt
    n_settle = desc["steps"] if n_settle is None else n_settle
    sys, st = der.build(desc)
    out = []
    for kv in kv_sequence:
        st = settle(sys, st, torch.as_tensor(kv, dtype=der.DT), dt, n_settle)
        out.append(limb_curvatures(sys, st.x, st.theta, st))
    return torch.stack(out)
