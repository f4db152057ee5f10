"""Differentiable rollouts over the library's hand-written adjoint.

torch.autograd.Function wrappers whose forward passes call dg2p_prim_to_cons
and dg2p_rk_step and whose backward passes call dg2p_prim_to_cons_vjp and
dg2p_rk_step_vjp.  ``Rollout`` advances n SSP-RK3 steps with a frozen time
step, keeps the state every ``checkpoint_every`` steps, and in the backward
pass recomputes one segment at a time from its checkpoint before reversing
its steps (memory: one segment of states instead of the whole trajectory).
The surface-tension coefficient is a differentiable input.

The interface-shape loss of the adjoint workload and the seeded perturbed
target run are built here as well.
"""

import numpy as np
import torch

from . import dg2p, workloads


def _params_with_sigma(base, sigma):
    return dg2p.make_params({**base, "sigma": float(sigma)})


class PrimToCons(torch.autograd.Function):
    """Conserved state from primitive fields (layout of dg2p_prim_to_cons)."""

    @staticmethod
    def forward(ctx, prim, mesh, params):
        ctx.mesh, ctx.params = mesh, params
        ctx.save_for_backward(prim)
        return dg2p.prim_to_cons(mesh, params, prim.detach().contiguous())

    @staticmethod
    def backward(ctx, U_bar):
        (prim,) = ctx.saved_tensors
        return dg2p.prim_to_cons_vjp(ctx.mesh, ctx.params, prim.contiguous(), U_bar.contiguous()), None, None


class Rollout(torch.autograd.Function):
    """U_T = Phi^n(U_0; sigma) with Phi one SSP-RK3 step of frozen step dt."""

    @staticmethod
    def forward(ctx, U0, sigma, mesh, base_params, n_steps, dt, checkpoint_every):
        P = _params_with_sigma(base_params, sigma.item())
        U = U0.detach().contiguous().clone()
        ckpts = []
        for s in range(n_steps):
            if s % checkpoint_every == 0:
                ckpts.append(U.clone())
            dg2p.rk_step(mesh, P, U, dt)
        ctx.mesh, ctx.P, ctx.n, ctx.every = mesh, P, n_steps, checkpoint_every
        ctx.dt = dt
        ctx.ckpts = ckpts
        return U

    @staticmethod
    def backward(ctx, U_bar):
        mesh, P, n, every, dt = ctx.mesh, ctx.P, ctx.n, ctx.every, ctx.dt
        Ub = U_bar.contiguous().clone()
        sb = torch.zeros(1, dtype=torch.float64, device=Ub.device)
        spare = torch.empty_like(Ub)
        for seg in reversed(range(len(ctx.ckpts))):
            s0 = seg * every
            s1 = min(s0 + every, n)
            states = [ctx.ckpts[seg]]
            U = ctx.ckpts[seg].clone()
            for _ in range(s0, s1 - 1):
                dg2p.rk_step(mesh, P, U, dt)
                states.append(U.clone())
            for s in reversed(range(s0, s1)):
                dg2p.rk_step_vjp(mesh, P, states[s - s0], dt, Ub, param_bar=sb, out=spare)
                Ub, spare = spare, Ub
        ctx.ckpts = None
        return Ub, sb.reshape(()), None, None, None, None, None


def alpha_misfit(U, alpha_target, W, d):
    """L = 1/2 sum_nodes W_j (alpha_j - alpha_target_j)^2 (W: element node weights)."""
    r = U[3 + d] - alpha_target
    return 0.5 * (r * r * W).sum()


class AdjointProblem:
    """The adjoint workload: droplet with viscosity and surface tension,
    gradient of the alpha misfit at the final time with respect to the nodal
    initial velocity and the surface-tension coefficient.

    Controls: u0 (d, E, nn) and sigma.  The target is the same run from
    u0 + 1e-2 * (smooth seeded field) and 1.2 sigma.  dt is frozen from the
    unperturbed initial state.
    """

    def __init__(self, n_elem=None, n_steps=None, checkpoint_every=None, cfl=0.1, bc=None):
        cfg = workloads.config("adjoint2d", n_elem=n_elem)
        if bc is not None:   # boundary kinds per axis, e.g. [("no_slip", "no_slip"), ("slip_wall", "slip_wall")]
            cfg["bc"] = [tuple(b) for b in bc]
        self.cfg = cfg
        self.d = cfg["dim"]
        self.n_steps = cfg["steps"] if n_steps is None else n_steps
        self.every = cfg["checkpoint_every"] if checkpoint_every is None else checkpoint_every
        self.base = dict(cfg["params"])
        self.P = dg2p.make_params(self.base)
        self.mesh = dg2p.mesh_from_config(cfg, self.P)
        X = self.mesh.node_coords()
        pf = workloads.primitive_fields(cfg, X)
        self.prim0 = dg2p.prim_tensor(pf, self.d)
        self.u0 = self.prim0[4:4 + self.d].clone()
        self.sigma0 = float(self.base["sigma"])
        W = torch.from_numpy(self.mesh.node_weights()).cuda()
        self.W = W.expand(self.mesh.E, self.mesh.nn)
        U0 = dg2p.prim_to_cons(self.mesh, self.P, self.prim0)
        self.dt = dg2p.max_dt(self.mesh, self.P, U0, cfl=cfl)
        pert = torch.from_numpy(workloads.adjoint_target_perturbation(X)).cuda()
        with torch.no_grad():
            UT = self.final_state(self.u0 + 1e-2 * pert, 1.2 * self.sigma0)
        self.alpha_target = UT[3 + self.d].clone()

    def prim(self, u0):
        return torch.cat([self.prim0[:4], u0, self.prim0[4 + self.d:]], dim=0)

    def final_state(self, u0, sigma):
        sig = torch.as_tensor(sigma, dtype=torch.float64, device="cuda")
        U0 = PrimToCons.apply(self.prim(u0).contiguous(), self.mesh, self.P)
        return Rollout.apply(U0, sig, self.mesh, self.base, self.n_steps, self.dt, self.every)

    def loss(self, u0, sigma):
        return alpha_misfit(self.final_state(u0, sigma), self.alpha_target, self.W, self.d)

    def gradient(self, u0=None, sigma=None):
        """(L, dL/du0, dL/dsigma) by the hand-written adjoint."""
        u0 = (self.u0 if u0 is None else u0).clone().requires_grad_(True)
        sig = torch.tensor(self.sigma0 if sigma is None else sigma, dtype=torch.float64, device="cuda",
                           requires_grad=True)
        L = self.loss(u0, sig)
        gu, gs = torch.autograd.grad(L, (u0, sig))
        return float(L), gu, float(gs)

    def fd_directions(self, k):
        """Seeded direction k with unit W-norm: (du0, dsigma)."""
        du, ds = workloads.fd_direction(tuple(self.u0.shape), k)
        du = torch.from_numpy(du).cuda()
        ds = ds * self.sigma0
        nrm = float(torch.sqrt((du * du * self.W).sum() + ds * ds))
        return du / nrm, ds / nrm
