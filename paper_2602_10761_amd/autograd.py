"""Gradients of the charging objectives through the particle step (torch.autograd).

J(theta) per ensemble = (mean particle charge after n steps, charge received by
the walls per unit time), theta = (k_c, dU, e) per ensemble: the condenser
charge-transfer coefficient, contact potential difference and restitution
coefficient.  Backward runs the library's reverse-mode step (tf_adjoint_step)
with the discrete events of the run held fixed, over checkpointed segments:
forward stores the particle state every `segment` steps; backward restores
each segment's checkpoint, re-runs it with recording and reverses it.

The simulation's statistics also count the recomputed steps; the particle
state after backward equals the state after forward.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .runtime import FIX_WALL, KEYS, TriboSim


def objectives(sim: TriboSim, wall0, n_steps: int):
    out = np.zeros((sim.n_ens, 2))
    for e in range(sim.n_ens):
        q = sim.state(e)["q"]
        st = sim.stats(e)
        w = (int(st["wallq"].sum()) - wall0[e]) * 2.0 ** -FIX_WALL
        out[e, 0] = float(q.mean()) if q.numel() else 0.0
        out[e, 1] = w / (n_steps * sim.ens[e].params["dt"])
    return out


class TriboRun(torch.autograd.Function):
    """TriboRun.apply(theta[n_ens, 3], sim, n_steps, segment) -> J[n_ens, 2]."""

    @staticmethod
    def forward(ctx, theta, sim: TriboSim, n_steps: int, segment: int):
        if segment < 1 or segment > sim.traj_steps:
            raise ValueError("segment must be in [1, traj_steps of the simulation]")
        th = theta.detach().to("cpu", torch.float64).numpy().reshape(sim.n_ens, 3)
        sim.set_params(th)
        wall0 = [int(sim.stats(e)["wallq"].sum()) for e in range(sim.n_ens)]
        ckpts, lens = [], []
        done = 0
        while done < n_steps:
            k = min(segment, n_steps - done)
            ckpts.append([{k2: v.clone() for k2, v in sim.state(e).items()} for e in range(sim.n_ens)])
            lens.append(k)
            sim.step(k)
            done += k
        J = objectives(sim, wall0, n_steps)
        ctx.sim = sim
        ctx.theta = th.copy()       # backward re-runs the segments at this theta
        ctx.ckpts = ckpts
        ctx.lens = lens
        ctx.final = [sim.state(e) for e in range(sim.n_ens)]
        ctx.n_steps = n_steps
        return torch.as_tensor(J, dtype=theta.dtype if theta.is_floating_point() else torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        sim: TriboSim = ctx.sim
        g = gJ.detach().to("cpu", torch.float64).numpy().reshape(sim.n_ens, 2)
        dev = sim.dev
        lam = []
        w_wall = np.zeros((sim.n_ens, 2))
        for e in range(sim.n_ens):
            n = sim.ens[e].n
            L = {k: torch.zeros(n, dtype=torch.float64, device=dev) for k in KEYS}
            if n:
                L["q"].fill_(g[e, 0] / n)
            lam.append(L)
            w_wall[e, :] = g[e, 1] / (ctx.n_steps * sim.ens[e].params["dt"])
        # the segments are re-run at the theta of this forward (another apply or
        # set_params on the same simulation may have changed it since); the
        # simulation's parameters are restored afterwards
        theta_before = sim.theta.copy()
        sim.set_params(ctx.theta)
        dth = torch.zeros((sim.n_ens, 3), dtype=torch.float64, device=dev)
        for ck, k in zip(reversed(ctx.ckpts), reversed(ctx.lens)):
            for e in range(sim.n_ens):
                sim.set_state(e, ck[e])
            sim.step(k, record=True)
            sim.adjoint(lam, w_wall, dtheta=dth)
        for e in range(sim.n_ens):
            sim.set_state(e, ctx.final[e])
        sim.set_params(theta_before)
        return dth.cpu(), None, None, None


def charging_gradient(sim: TriboSim, theta: np.ndarray, n_steps: int, segment: int = 50):
    """(J, dJ/dtheta) with dJ[e] = [dJ1/dtheta, dJ2/dtheta] ([n_ens, 2, 3])."""
    th = torch.tensor(np.asarray(theta, dtype=np.float64).reshape(sim.n_ens, 3), requires_grad=True)
    J = TriboRun.apply(th, sim, n_steps, segment)
    grads = np.zeros((sim.n_ens, 2, 3))
    for m in range(2):
        # one objective per backward pass (each pass recomputes the segments)
        sel = torch.zeros_like(J)
        sel[:, m] = 1.0
        (g,) = torch.autograd.grad(J, th, grad_outputs=sel, retain_graph=(m == 0))
        grads[:, m, :] = g.numpy()
    return J.detach().numpy(), grads
