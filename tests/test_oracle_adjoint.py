"""Pins of the oracle's adjoint (CPU): dot-product identity against central
finite differences of the oracle residual and of one SSP-RK3 step, and the
surface-tension cotangent against the exact linear dependence on sigma."""

import pytest
import torch

import oracle
from helpers import oracle_setup

torch.set_default_dtype(torch.float64)


@pytest.mark.parametrize("name,ne", [("drop1d", (9,)), ("adjoint2d", (4, 3))])
def test_rhs_vjp_dot_product_vs_fd(name, ne):
    """<J v, w> (central difference, h = 1e-6) = <v, J^T w> (autograd)."""
    cfg, om, prm, U0 = oracle_setup(name, n_elem=ne)
    g = torch.Generator().manual_seed(5)
    v = torch.randn(U0.shape, generator=g) * U0.abs().amax(dim=(1, 2), keepdim=True) * 1e-3
    w = torch.randn(U0.shape, generator=g)
    h = 1e-6
    Jv = (oracle.rhs(U0 + h * v, om, prm) - oracle.rhs(U0 - h * v, om, prm)) / (2 * h)
    Ub, _ = oracle.adjoint.rhs_vjp(U0, w, om, prm)
    lhs, rhs_ = float((Jv * w).sum()), float((v * Ub).sum())
    assert abs(lhs - rhs_) <= 1e-6 * max(abs(lhs), abs(rhs_))


def test_sigma_cotangent_is_exact_derivative():
    """R is affine in sigma: <w, R(sigma2) - R(sigma1)> / (sigma2 - sigma1) = sigma_bar."""
    cfg, om, prm, U0 = oracle_setup("adjoint2d", n_elem=(4, 4))
    w = torch.randn(U0.shape, generator=torch.Generator().manual_seed(2))
    import dataclasses
    R1 = oracle.rhs(U0, om, dataclasses.replace(prm, sigma=0.0))
    R2 = oracle.rhs(U0, om, dataclasses.replace(prm, sigma=1.0))
    want = float((w * (R2 - R1)).sum())
    _, sb = oracle.adjoint.rhs_vjp(U0, w, om, prm)
    assert abs(sb - want) <= 1e-10 * abs(want)


def test_rk_step_vjp_dot_product():
    cfg, om, prm, U0 = oracle_setup("adjoint2d", n_elem=(3, 3))
    dt = oracle.max_dt(U0, om, prm)
    g = torch.Generator().manual_seed(7)
    v = torch.randn(U0.shape, generator=g) * U0.abs().amax(dim=(1, 2), keepdim=True) * 1e-3
    w = torch.randn(U0.shape, generator=g)
    h = 1e-6
    Jv = (oracle.rk_step(U0 + h * v, dt, om, prm) - oracle.rk_step(U0 - h * v, dt, om, prm)) / (2 * h)
    Ub, _ = oracle.adjoint.rk_step_vjp(U0, dt, w, om, prm)
    lhs, rhs_ = float((Jv * w).sum()), float((v * Ub).sum())
    assert abs(lhs - rhs_) <= 1e-6 * max(abs(lhs), abs(rhs_))
