"""Adjoint workload on the GPU: gradients of the final-time alpha misfit with
respect to the nodal initial velocity and the surface tension, by the
hand-written reverse pass with checkpointed recomputation, checked against
central finite differences (16 seeded unit directions) and against the
oracle's autograd adjoint of its own rollout."""

import math

import numpy as np
import pytest
import torch

import oracle
from paper_2306_05002_amd import workloads

pytestmark = pytest.mark.gpu


def _adj():
    from paper_2306_05002_amd import adjoint
    return adjoint


def fd_agreement(prob, n_dir=16, h=1e-6):
    L0, gu, gs = prob.gradient()
    worst = 0.0
    rows = []
    for k in range(n_dir):
        du, ds = prob.fd_directions(k)
        with torch.no_grad():
            Lp = float(prob.loss(prob.u0 + h * du, prob.sigma0 + h * ds))
            Lm = float(prob.loss(prob.u0 - h * du, prob.sigma0 - h * ds))
        fd = (Lp - Lm) / (2 * h)
        ad = float((gu * du).sum()) + gs * ds
        rel = abs(fd - ad) / max(abs(fd), abs(ad), 1e-300)
        rows.append((k, fd, ad, rel))
        worst = max(worst, rel)
    return L0, worst, rows


def test_adjoint_fd_reduced():
    prob = _adj().AdjointProblem(n_elem=(16, 16), n_steps=24, checkpoint_every=5)
    L0, worst, rows = fd_agreement(prob)
    for r in rows:
        print("dir %2d fd % .12e adj % .12e rel %.2e" % r)
    assert L0 > 0.0
    assert worst < 1e-6, worst


def test_adjoint_fd_walls():
    """The same gradient with extrapolation in x and slip walls in y (the
    ghosts' reverse), against central differences.  (The workload's
    translating droplet driven into walls on both axes loses positivity
    within ten steps; the residual VJP of the other kinds is tested against
    the oracle in test_gpu_parity.py.)"""
    prob = _adj().AdjointProblem(n_elem=(12, 12), n_steps=16, checkpoint_every=5,
                                 bc=[("extrapolate", "extrapolate"), ("slip_wall", "slip_wall")])
    L0, worst, rows = fd_agreement(prob, n_dir=8)
    for r in rows:
        print("dir %2d fd % .12e adj % .12e rel %.2e" % r)
    assert L0 > 0.0
    assert worst < 1e-6, worst


def test_adjoint_matches_oracle_autograd():
    """Same problem on both sides, each with its own forward, target run and
    frozen dt; the oracle differentiates its rollout with torch.autograd."""
    ne, steps = (8, 8), 10
    adj = _adj()
    prob = adj.AdjointProblem(n_elem=ne, n_steps=steps, checkpoint_every=3)
    L_g, gu_g, gs_g = prob.gradient()

    cfg = workloads.config("adjoint2d", n_elem=ne)
    prm = oracle.Params(**cfg["params"])
    om = oracle.OracleMesh(2, 3, ne, cfg["lo"], cfg["hi"], cfg["bc"])
    X = om.node_coords().numpy()
    pf = workloads.primitive_fields(cfg, X)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)
    u0 = T(pf["u"])
    sig0 = prm.sigma

    def final(u, s):
        import dataclasses
        p = dataclasses.replace(prm, sigma=s)
        U = oracle.prim_to_cons(T(pf["alpha"]), T(pf["psi"]), T(pf["rho1"]), T(pf["rho2"]), u, T(pf["P"]), p)
        for _ in range(steps):
            U = oracle.rk_step(U, dt, om, p)
        return U

    U00 = oracle.prim_to_cons(T(pf["alpha"]), T(pf["psi"]), T(pf["rho1"]), T(pf["rho2"]), u0, T(pf["P"]), prm)
    dt = oracle.max_dt(U00, om, prm)
    pert = T(workloads.adjoint_target_perturbation(X))
    with torch.no_grad():
        a_t = final(u0 + 1e-2 * pert, 1.2 * sig0)[5]
    W = om.node_weights()
    u = u0.clone().requires_grad_(True)
    s = torch.tensor(sig0, dtype=torch.float64, requires_grad=True)
    L = 0.5 * (((final(u, s)[5] - a_t) ** 2) * W).sum()
    gu_o, gs_o = torch.autograd.grad(L, (u, s))
    print("L", L_g, float(L), "sigma grad", gs_g, float(gs_o))
    assert abs(L_g - float(L)) <= 1e-10 * float(L)
    err_u = float((gu_g.cpu() - gu_o).abs().max() / gu_o.abs().max())
    print("u0 gradient normwise error", err_u)
    # thin interface: the CSF delta function is differentiated through
    # grad alpha / |grad alpha| where grad alpha comes from cancellation
    assert err_u <= 1e-7
    assert abs(gs_g - float(gs_o)) <= 1e-7 * abs(float(gs_o))


@pytest.mark.timeout(300)
def test_adjoint_fd_full_size():
    """The adjoint workload at its full size: 128 x 128, 400 steps,
    checkpoints every 20 steps; 16 seeded directions, h = 1e-6."""
    prob = _adj().AdjointProblem()
    L0, worst, rows = fd_agreement(prob)
    for r in rows:
        print("dir %2d fd % .12e adj % .12e rel %.2e" % r)
    assert worst < 1e-6, worst
