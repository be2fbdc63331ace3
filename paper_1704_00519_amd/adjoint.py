"""Gradients through the time steps of the library.

The nested shock-bubble (a planar shock in ambient gas hitting a bubble with
an outer shell and an inner core) is parameterised by the shell density, the
core density and the shock Mach number.  The functional is the x-position of
the bubble's volume centroid at the final step,

    J = sum_i (alpha^shell_i + alpha^core_i) x_i / sum_i (alpha^shell_i + alpha^core_i).

Every time step and every reverse (adjoint) step runs in the library
(``mm_step`` with a tape, ``mm_adjoint_step``).  Only the map from the three
parameters to the initial primitive fields and the inflow state (the normal
shock relations) and from those to Q^0 = alpha^0 U(W) is differentiated here,
with torch on the host.  The step sizes are a fixed schedule (those of a
reference run), replayed by the library; the gradient is that of J at fixed
step sizes.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib

GAMMA_AMBIENT = 1.4


def rankine_hugoniot(mach, gamma=GAMMA_AMBIENT, rho0=1.0, p0=1.0):
    """Post-shock (rho, u, p) behind a right-moving normal shock of Mach
    ``mach`` entering gas at rest (rho0, p0); ideal gas, closed form.  Works
    on torch tensors (differentiable) and floats."""
    c0 = (gamma * p0 / rho0) ** 0.5
    m2 = mach * mach
    p1 = p0 * (2.0 * gamma * m2 - (gamma - 1.0)) / (gamma + 1.0)
    rho1 = rho0 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    s = mach * c0
    u1 = s - s * rho0 / rho1
    return rho1, u1, p1


def bubble_fields(params, X, post):
    """Primitive fields [3][4][ny][nx] and inflow state (4) of the nested
    bubble for params = (rho_shell, rho_core, mach) (torch, float64)."""
    rho_o, rho_i, mach = params[0], params[1], params[2]
    rho1, u1, p1 = rankine_hugoniot(mach)
    one = torch.ones_like(X)
    zero = torch.zeros_like(X)
    post = torch.as_tensor(post)
    amb = torch.stack([torch.where(post, rho1 * one, one), torch.where(post, u1 * one, zero),
                       zero, torch.where(post, p1 * one, one)])
    shell = torch.stack([rho_o * one, zero, zero, one])
    core = torch.stack([rho_i * one, zero, zero, one])
    W = torch.stack([amb, shell, core])
    inflow = torch.stack([rho1, u1, torch.zeros_like(rho1), p1])
    return W, inflow


def conserved(W, gammas, pinfs):
    """alpha-free conserved state U(W) per material, [M][4][ny][nx]."""
    out = []
    for m in range(W.shape[0]):
        r, u, v, p = W[m, 0], W[m, 1], W[m, 2], W[m, 3]
        g, pi = gammas[m], pinfs[m]
        E = (p + g * pi) / (g - 1.0) + 0.5 * r * (u * u + v * v)
        out.append(torch.stack([r, r * u, r * v, E]))
    return torch.stack(out)


def centroid(alpha, x):
    """J and dJ/dalpha for alpha [3][ny][nx] (numpy), x the cell centres."""
    a = alpha[1] + alpha[2]
    S = a.sum()
    J = float((a * x).sum() / S)
    g = np.zeros_like(alpha)
    g[1] = (x - J) / S
    g[2] = (x - J) / S
    return J, g


class NestedBubble:
    """The nested shock-bubble on a given grid; ``workload`` is the dict of
    ``workloads.shock_bubble`` (its level set, indicator and configuration
    are used; its primitive fields are rebuilt from the parameters)."""

    def __init__(self, workload, x_shock=0.5):
        self.w = workload
        cfg = workload["cfg"]
        nx, ny = cfg["nx"], cfg["ny"]
        dx = (cfg["x1"] - cfg["x0"]) / nx
        x = cfg["x0"] + (np.arange(nx) + 0.5) * dx
        self.x = np.broadcast_to(x, (ny, nx)).copy()
        self.X = torch.tensor(self.x, dtype=torch.float64)
        self.post = self.x < x_shock

    def fields(self, params):
        return bubble_fields(params, self.X, self.post)

    def solver(self, params, stream=None):
        W, inflow = self.fields(torch.as_tensor(params, dtype=torch.float64))
        cfg = dict(self.w["cfg"])
        cfg["inflow_W"] = [float(v) for v in inflow]
        cfg["reinit"] = 0  # the adjoint is built without the redistancing
        s = _lib.Solver(cfg, stream=stream)
        s.init(self.w["phi"], self.w["chi"], W.numpy())
        return s

    def run(self, params, steps, record=0, dts=None, stream=None):
        """Forward run; returns (J, solver, alpha^0).  With dts, step n uses
        the fixed size dts[n] (the library replays the schedule)."""
        s = self.solver(params, stream)
        alpha0 = s.get()["alpha"]
        if dts is not None:
            if len(dts) < steps:
                raise ValueError("the schedule is shorter than the run")
            s.set_dt_schedule(np.asarray(dts[:steps], np.float64))
        s.step(steps, record=record)
        J, _ = centroid(s.get()["alpha"], self.x)
        return J, s, alpha0

    def pullback(self, params, alpha0, lamQ0, lam_inflow):
        """dJ/dparams from the adjoint of Q^0 and of the inflow state."""
        cfg = self.w["cfg"]
        with torch.enable_grad():  # also inside an autograd backward
            p = torch.as_tensor(params, dtype=torch.float64).detach().clone().requires_grad_(True)
            W, inflow = self.fields(p)
            U = conserved(W, cfg["gamma"], cfg["pinf"])
            a = torch.tensor(alpha0, dtype=torch.float64)
            Q0 = torch.where(a[:, None] > 0.0, a[:, None] * U, torch.zeros_like(U))
            L = (torch.tensor(lamQ0) * Q0).sum() + (torch.tensor(lam_inflow) * inflow).sum()
            (g,) = torch.autograd.grad(L, p)
        return g.numpy()


def nominal_schedule(problem, params, steps, stream=None):
    """Step sizes of the CFL run at ``params`` (the schedule a gradient
    study holds fixed)."""
    _, s, _ = problem.run(params, steps, record=1, stream=stream)
    dts = s.tape()[2]
    s.close()
    return dts


class CentroidGradient(torch.autograd.Function):
    """J(params) of a NestedBubble after ``steps`` steps of the fixed step
    sizes ``dts`` (a schedule, e.g. ``nominal_schedule`` at a reference
    point), with the gradient from the library's reverse steps (a checkpoint
    every K steps).  The step sizes are inputs held fixed, not functions of
    params, so forward and backward are derivatives of the same function:
    J(params) = centroid after the scheduled steps."""

    @staticmethod
    def forward(ctx, params, problem, steps, K, dts):
        J, s, alpha0 = problem.run(params.detach().numpy(), steps, record=K, dts=dts)
        ctx.problem, ctx.steps, ctx.solver, ctx.alpha0 = problem, steps, s, alpha0
        ctx.save_for_backward(params)
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        (params,) = ctx.saved_tensors
        g = reverse_gradient(ctx.problem, ctx.solver, ctx.alpha0, ctx.steps,
                             params.detach().numpy())
        return gJ * torch.tensor(g), None, None, None, None


def reverse_gradient(problem, solver, alpha0, steps, params):
    """Walk the recorded steps backwards from dJ/dalpha at the end."""
    _, lam_alpha = centroid(solver.get()["alpha"], problem.x)
    if steps == 1:
        lamQ0, _ = solver.adjoint_step(lamAlpha=lam_alpha)
    else:
        solver.adjoint_step(lamAlpha=lam_alpha, out=False)
        for _ in range(steps - 2):
            solver.adjoint_step(out=False)
        lamQ0, _ = solver.adjoint_step()
    lam_inflow = solver.adjoint_inflow()
    return problem.pullback(params, alpha0, lamQ0, lam_inflow)
