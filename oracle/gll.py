"""Gauss-Lobatto-Legendre tables (test infrastructure only).

The paper discretises each element with Lagrange polynomials of degree p
(Section "Discontinuous Galerkin discretisation", the local expansion of the
solution and the function space V).  We use the nodal GLL collocation
reading: interpolation and quadrature at the p+1 GLL points.

Nodes: -1, +1 and the roots of P_p'(x) (P_p = Legendre polynomial).
Weights: w_j = 2 / (p (p+1) P_p(x_j)^2).
Derivative matrix: D[a, b] = l_b'(x_a) (l_b = Lagrange basis polynomial),
built from barycentric weights.
"""

import math

import torch


def _legendre(p, x):
    """P_p(x) and P_p'(x) by the three-term recurrence (Bonnet)."""
    p0, p1 = 1.0, x
    if p == 0:
        return 1.0, 0.0
    for k in range(2, p + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    # derivative from (1 - x^2) P_p' = p (P_{p-1} - x P_p)
    dp = p * (p0 - x * p1) / (1.0 - x * x) if abs(x) < 1.0 else (
        0.5 * p * (p + 1) * (1.0 if x > 0 else (-1.0) ** (p + 1)))
    return p1, dp


def gll_nodes_weights(p):
    """GLL nodes (ascending) and weights for degree p >= 1, as float64 tensors."""
    if p < 1:
        raise ValueError("p must be >= 1")
    n = p + 1
    xs = []
    for j in range(n):
        if j == 0:
            xs.append(-1.0)
            continue
        if j == p:
            xs.append(1.0)
            continue
        # interior roots of P_p': Newton from the Chebyshev-Gauss-Lobatto guess
        x = -math.cos(math.pi * j / p)
        for _ in range(100):
            # g(x) = P_p'(x); g'(x) from the Legendre ODE:
            # (1-x^2) P'' = 2x P' - p(p+1) P
            P, dP = _legendre(p, x)
            d2P = (2.0 * x * dP - p * (p + 1) * P) / (1.0 - x * x)
            dx = dP / d2P
            x -= dx
            if abs(dx) < 1e-17:
                break
        xs.append(x)
    w = []
    for x in xs:
        P, _ = _legendre(p, x)
        w.append(2.0 / (p * (p + 1) * P * P))
    return (torch.tensor(xs, dtype=torch.float64),
            torch.tensor(w, dtype=torch.float64))


def derivative_matrix(x):
    """D[a, b] = l_b'(x_a) for the Lagrange basis on nodes x (barycentric form)."""
    n = x.numel()
    xv = [float(v) for v in x]
    lam = []
    for j in range(n):
        prod = 1.0
        for k in range(n):
            if k != j:
                prod *= (xv[j] - xv[k])
        lam.append(1.0 / prod)
    D = torch.zeros(n, n, dtype=torch.float64)
    for a in range(n):
        s = 0.0
        for b in range(n):
            if a != b:
                D[a, b] = (lam[b] / lam[a]) / (xv[a] - xv[b])
                s += float(D[a, b])
        D[a, a] = -s  # rows annihilate constants
    return D
