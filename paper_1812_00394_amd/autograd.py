"""torch.autograd wrapper of the discrete adjoint.

    problem = Problem(mesh, params, rho=..., u=..., k=..., omega=..., n_steps=400, ckpt_every=20,
                      wall_mask=1)
    p = torch.tensor([theta, sigma_k1, sigma_w1, beta_star, a1], dtype=torch.float64, requires_grad=True)
    J = FVLBMObjective.apply(p, problem)        # (F_x, F_y, J_R) of the final state
    (J @ w).backward()                           # p.grad = d(w . J)/dp from the adjoint run

The forward runs the recorded steps on the GPU (fvlbm_record) and evaluates the surface
functionals; backward seeds the adjoint with the incoming gradient and returns dJ/dp for the inflow
angle and the four SST constants (fvlbm_adjoint_step).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import fvlbm as F

PARAM_NAMES = ("theta", "sigma_k1", "sigma_w1", "beta_star", "a1")


@dataclass
class Problem:
    mesh: F.Mesh
    params: dict
    rho: np.ndarray
    u: np.ndarray
    k: np.ndarray | None = None
    omega: np.ndarray | None = None
    n_steps: int = 400
    ckpt_every: int = 20
    wall_mask: int = 1
    precision: str = "fp64"
    f0: np.ndarray | None = None          # optional non-equilibrium initial f [9][n]
    last_state: object = field(default=None, repr=False)

    def with_params(self, p):
        d = dict(self.params)
        for name, v in zip(PARAM_NAMES, p):
            d[name] = float(v)
        return d


class FVLBMObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, problem: Problem):
        pv = params.detach().cpu().numpy().astype(np.float64)
        st = F.State(problem.mesh, problem.with_params(pv), precision=problem.precision, rho=problem.rho,
                     u=problem.u, k=problem.k, omega=problem.omega)
        if problem.f0 is not None:
            st.set_state(problem.f0, problem.k, problem.omega)
        st.record(problem.n_steps, problem.ckpt_every)
        Fv, jr = st.forces(problem.wall_mask)
        ctx.state = st
        ctx.mask = problem.wall_mask
        ctx.dtype = params.dtype
        problem.last_state = st
        return torch.tensor([Fv[0], Fv[1], jr], dtype=params.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        seed = grad_out.detach().cpu().numpy().astype(np.float64)
        dp = ctx.state.adjoint(ctx.mask, seed)
        return torch.tensor(dp, dtype=ctx.dtype), None


class LiftDragObjective(torch.autograd.Function):
    """(C_l, C_d) of the final recorded state as a function of the five parameters; backward runs
    fvlbm_adjoint_lift_drag (the reverse run plus the explicit turn of the lift and drag directions
    with theta).  problem.lift_drag_ref = (u_ref, chord)."""

    @staticmethod
    def forward(ctx, params, problem: Problem, u_ref: float, chord: float = 1.0):
        pv = params.detach().cpu().numpy().astype(np.float64)
        st = F.State(problem.mesh, problem.with_params(pv), precision=problem.precision, rho=problem.rho,
                     u=problem.u, k=problem.k, omega=problem.omega)
        if problem.f0 is not None:
            st.set_state(problem.f0, problem.k, problem.omega)
        st.record(problem.n_steps, problem.ckpt_every)
        cl, cd = st.lift_drag(problem.wall_mask, u_ref, chord)
        ctx.state, ctx.mask, ctx.ref, ctx.dtype = st, problem.wall_mask, (u_ref, chord), params.dtype
        problem.last_state = st
        return torch.tensor([cl, cd], dtype=params.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        seed = grad_out.detach().cpu().numpy().astype(np.float64)
        dp, _ = ctx.state.adjoint_lift_drag(ctx.mask, ctx.ref[0], ctx.ref[1], seed)
        return torch.tensor(dp, dtype=ctx.dtype), None, None, None
