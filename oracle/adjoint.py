"""Discrete adjoint of the backward-Euler DER trajectory (oracle).

TEST INFRASTRUCTURE ONLY: used by tests/ to check the HIP adjoint; never imported by
the product path.

The paper fits actuation inputs by gradient descent with finite-difference gradients
(Real2Sim section, Eq. 20).  Here the gradient of a trajectory loss with respect to the
per-stencil natural curvature is taken exactly, by the discrete adjoint of the step that
der.step implements:

* one step maps the state s_n = (x_n, v_n, theta_n, omega_n, t_n, d1_n) to s_{n+1} through
  the Newton root q of the residual R(q; s_n, kappa_bar) = 0 (Eq. 15) and the commit
  C(q; s_n) (velocity update after Eq. 16, frames carried to the new tangents by time-
  parallel transport);
* implicit-function theorem: for a cotangent qbar of q, lambda = J^-T qbar with J = dR/dq
  on the free DOFs, and every input p of R receives -lambda^T dR/dp;
* the reference-twist branch (beta_ref) is piecewise constant and carries no derivative;
  clamped DOFs never change, so their cotangents are dropped.

Loss used by the checks: L = sum over steps n = 1..T and rods of |x_tip,n - x*_tip,n|^2
with the tip the last node of each rod.

Parity of this module is pinned by brute-force central differences of the oracle's own
forward trajectory (tests/test_oracle_adjoint.py), which share no code with the adjoint
algebra here.
"""
from __future__ import annotations

import torch

from . import der


def _kbar_tensors(kbar):
    return [torch.as_tensor(k, dtype=der.DT) for k in kbar]


def rollout(desc, kbar, steps=None, tol=None, polish=2):
    """Forward trajectory with the given natural curvature per rod (list of (N-2, 2) arrays in
    1/m).  Returns (sys, states[0..T], tips (T, n_rods, 3))."""
    sys, st = der.build(desc)
    kb = _kbar_tensors(kbar)
    T = desc["steps"] if steps is None else steps
    tol = desc["tol"] if tol is None else tol
    states, tips = [st], []
    tip_ids = torch.tensor([int(r[-1]) for r in sys.rod_nodes])
    for _ in range(T):
        st, info = der.step(sys, st, desc["dt"], tol, desc["max_iter"], kbar_rods=kb, polish=polish)
        if not info.converged:
            raise RuntimeError("oracle rollout: Newton did not converge")
        states.append(st)
        tips.append(st.x[tip_ids])
    return sys, states, torch.stack(tips)


def tip_loss(tips, target_tips):
    """L = sum |tip - target|^2 and dL/dtips."""
    d = tips - target_tips
    return float((d * d).sum()), 2.0 * d


def _commit_fn(sys, dt):
    """s_{n+1} as a function of the Newton root q and the step-start state (der.commit)."""
    en = sys.edge_nodes

    def C(q, xn, thn, tref, d1ref):
        x, th = der.unpack(sys, q)
        e = x[en[:, 1]] - x[en[:, 0]]
        t = e / torch.linalg.norm(e, dim=1, keepdim=True)
        d1 = der.transport(tref, t, d1ref)
        return x, th, (x - xn) / dt, (th - thn) / dt, t, d1
    return C


def _residual_fn(sys, dt, beta_ref, time):
    """R(q; s_n, kappa_bar) of Eq. 15 with every state input an argument."""
    def R(q, xn, vn, thn, omn, tref, d1ref, kap):
        st = der.State(xn, thn, vn, omn, tref, d1ref, beta_ref, time)
        return der.residual(sys, q, st, dt, kap)
    return R


def adjoint(sys, states, kbar, dt, dL_dtips):
    """Gradient of a loss of the tip trajectory with respect to each rod's natural curvature.

    states: s_0..s_T from rollout; dL_dtips: (T, n_rods, 3), the loss gradient with respect
    to the tip positions after steps 1..T.  Returns a list of (N-2, 2) tensors (per rod, in
    the units of kbar, 1/m)."""
    kb = _kbar_tensors(kbar)
    T = len(states) - 1
    free = ~sys.fixed
    tip_ids = torch.tensor([int(r[-1]) for r in sys.rod_nodes])
    nn, ne = sys.n_nodes, sys.n_edges
    z3n = torch.zeros(nn, 3, dtype=der.DT)
    z3e = torch.zeros(ne, 3, dtype=der.DT)
    ze = torch.zeros(ne, dtype=der.DT)
    ax, av, ath, aom, atref, ad1 = z3n.clone(), z3n.clone(), ze.clone(), ze.clone(), z3e.clone(), z3e.clone()
    gkap = torch.zeros(sys.st_nodes.shape[0], 2, dtype=der.DT)
    C = _commit_fn(sys, dt)
    for n in reversed(range(T)):
        ax = ax.clone()
        ax[tip_ids] += torch.as_tensor(dL_dtips[n], dtype=der.DT)
        s0, s1 = states[n], states[n + 1]
        q = der.pack(s1.x, s1.theta)
        kap = der.natural_curvature(sys, s0.time + dt, kb)
        # commit: cotangents of s_{n+1} -> cotangent of q and direct ones of s_n
        _, vjp_c = torch.func.vjp(C, q, s0.x, s0.theta, s0.t_ref, s0.d1_ref)
        qbar, xb_c, thb_c, trb_c, d1b_c = vjp_c((ax, ath, av, aom, atref, ad1))
        # implicit-function theorem through R(q; s_n, kappa_bar) = 0
        Rf = _residual_fn(sys, dt, s0.beta_ref, s0.time)
        J = torch.func.jacfwd(Rf, argnums=0)(q, s0.x, s0.v, s0.theta, s0.omega, s0.t_ref, s0.d1_ref, kap)
        lam = torch.zeros_like(q)
        lam[free] = torch.linalg.solve(J[free][:, free].T, qbar[free])
        _, vjp_r = torch.func.vjp(lambda *a: Rf(q, *a), s0.x, s0.v, s0.theta, s0.omega, s0.t_ref, s0.d1_ref, kap)
        xr, vr, thr, omr, trr, d1r, kr = vjp_r(lam)
        ax, av, ath, aom = xb_c - xr, -vr, thb_c - thr, -omr
        atref, ad1 = trb_c - trr, d1b_c - d1r
        gkap = gkap - kr
    out = []
    for k, rn in enumerate(sys.rod_nodes):
        sel = torch.nonzero(sys.st_rod == k).flatten()
        idx = sys.st_index[sel] - 1
        g = torch.zeros(len(rn) - 2, 2, dtype=der.DT)
        g[idx] = gkap[sel] * sys.Vbar[sel][:, None]
        out.append(g)
    return out


def loss_and_grad(desc, kbar, target_tips, steps=None, polish=2):
    """Convenience: forward rollout, tip loss against target tips, and its adjoint gradient."""
    sys, states, tips = rollout(desc, kbar, steps, polish=polish)
    L, dL = tip_loss(tips, torch.as_tensor(target_tips, dtype=der.DT))
    return L, adjoint(sys, states, kbar, desc["dt"], dL), tips


def fit_natural_curvature(desc, target_tips, kbar0, alpha0, tol, max_iter, polish=2):
    """Gradient descent on the natural curvature in the control flow of the paper's Real2Sim
    algorithm (Alg. 1): evaluate the loss of the current kbar; stop below tol; halve the step
    size when the loss rose since the previous iterate; step kbar <- kbar - alpha grad
    (Eq. 21), the gradient here being the discrete adjoint of the tip loss instead of the
    forward differences of Eq. 20.  At most max_iter gradient steps.  Returns the kbar after
    every step (first entry kbar0), the loss of every evaluated iterate and the step size of
    every step."""
    kbar = [torch.as_tensor(k, dtype=der.DT).clone() for k in kbar0]
    alpha, prev = alpha0, float("inf")
    ks, losses, alphas = [[k.clone() for k in kbar]], [], []
    for _ in range(max_iter + 1):
        L, g, _ = loss_and_grad(desc, kbar, target_tips, polish=polish)
        losses.append(L)
        if L < tol or len(losses) == max_iter + 1:
            break
        if L > prev:
            alpha *= 0.5
        prev = L
        kbar = [k - alpha * gi for k, gi in zip(kbar, g)]
        ks.append([k.clone() for k in kbar])
        alphas.append(alpha)
    return ks, losses, alphas
