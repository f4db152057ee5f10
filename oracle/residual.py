"""The semi-discrete DG operator dU/dt = R(U) (test infrastructure only).

Paper passages followed (Tonicello & Ihme, arXiv 2306.05002):
  * the model (system of Section "Five equation model"): phase-field
    transport with the Allen-Cahn flux a_1, level-set transport, the two
    partial densities with R_l = rho_l^(0) a_l, momentum with f (x) u, tau,
    CSF and gravity, energy with f k, sum_l rho_l H_l a_l, tau.u, CSF and
    gravity work;
  * the interface flux a_1 = Gamma (eps grad phi - phi (1-phi) n) with the
    normal taken from the level set, n = grad psi / |grad psi|;
  * the local DG weak form (Section "Discontinuous Galerkin
    discretisation", the weak form after integration by parts with the
    element mass matrix); under GLL collocation the summation-by-parts
    identity makes it equal to the strong form used below (pinned by a test);
  * transport of phi and psi as a volume source plus the hat/tilde face
    fluxes of the quasi-conservative form, with the half jump
    [[phi]] = (phi+ - phi-)/2 and the average {{phi}};
  * Lax-Friedrichs fluxes for partial densities, momentum and energy, and
    symmetric interior penalty fluxes for every term built from a_l (the
    statement closing the per-equation weak forms).

Readings where the paper is silent (all also listed in the design notes):
  * "-" is the element's own (interior) trace, "+" the neighbour's; the
    characteristic speed c of the hat flux is the same face speed
    lambda = max(|u.m| + c_mix) over both sides that the Lax-Friedrichs flux
    uses;
  * every a_l-built flux is s_q * a_1 with a scalar s_q per equation
    (a_2 = -a_1): s = (rho1_0, -rho2_0, (rho1_0-rho2_0) u, (rho1_0-rho2_0) k
    + rho1 H1 - rho2 H2, 1, 0) for (q1, q2, rho u, rho E, alpha, psi);
  * SIPG: numerical normal flux {{a}}.m - eta (alpha_i - alpha_e) with
    eta = c_ip Gamma eps (p+1)^2 / h, face coefficient s_bar = {{s_q}}, plus
    the symmetric term  +{{s_bar Gamma eps grad v}}.[[alpha]] ;
  * viscous stresses: incomplete interior penalty (average + penalty,
    no symmetric term), eta_v = c_ip {{mu}} (p+1)^2 / h;
  * n = g / sqrt(g.g + delta^2), delta_Gamma = sqrt(|grad alpha|^2 +
    delta^2) - delta, delta = grad_reg;
  * boundary ghosts: slip wall mirrors the state and gradients in the
    normal direction; Dirichlet prescribes (q1, q2, rho u, rho E, alpha) and
    keeps the interior psi and gradients; extrapolation copies the interior;
    no-slip wall negates the whole momentum, mirrors the scalar gradients and
    keeps the velocity gradient; the Riemann-invariant boundary (zero
    velocity and pressure P_b outside, Section "Rayleigh-Taylor
    instability") builds its ghost state from the two characteristic
    invariants (_riemann_ghost) and keeps the interior gradients.

Every element evaluates all of its own faces (the neighbour's element-local
gradients are recomputed from the neighbour's nodal data), so any subset of
elements can be evaluated on its own: that is what lets the tests check
full-size grids on sampled elements.
"""

import torch

from .physics import primitives


def _dk(f, k, mesh):
    """Broken derivative along axis k: (1/J_k) sum_b D[a, b] f(..b..)."""
    dim = f.dim() - 1 - k
    g = torch.movedim(f, dim, -1) @ mesh.D.T
    return torch.movedim(g, -1, dim) / mesh.J[k]


def _grad(f, mesh):
    return torch.stack([_dk(f, k, mesh) for k in range(mesh.d)])


def _raw(X, mesh, prm):
    """Nodal state plus the element-local gradients every flux needs."""
    d = mesh.d
    raw = dict(Q=X, gA=_grad(X[3 + d], mesh), gP=_grad(X[4 + d], mesh))
    if prm.viscous:
        rho = X[0] + X[1]
        u = torch.stack([X[2 + j] / rho for j in range(d)])
        raw["gU"] = torch.stack([_grad(u[j], mesh) for j in range(d)])  # [j][k] = d_k u_j
    return raw


def _pointwise(raw, d, prm):
    """Node-local quantities from a (trace of a) raw state."""
    Q = raw["Q"]
    pr = primitives(Q, d, prm)
    u, P, kin = pr["u"], pr["P"], pr["kin"]
    alpha = Q[3 + d]
    gA, gP = raw["gA"], raw["gP"]
    delta = prm.grad_reg
    nrm = torch.sqrt((gP * gP).sum(0) + delta * delta)
    nhat = gP / nrm
    a = prm.Gamma * (prm.eps * gA - (alpha * (1.0 - alpha)) * nhat)
    r1, r2 = prm.rho0
    s = [torch.full_like(alpha, r1), torch.full_like(alpha, -r2)]
    s += [(r1 - r2) * u[j] for j in range(d)]
    s += [(r1 - r2) * kin + pr["rH1"] - pr["rH2"]]
    s = torch.stack(s)                                     # (d+3, ...)
    # convective fluxes Fc[q][k]
    Fc = [torch.stack([Q[0] * u[k] for k in range(d)]),
          torch.stack([Q[1] * u[k] for k in range(d)])]
    for j in range(d):
        Fc.append(torch.stack([Q[2 + j] * u[k] + (P if j == k else 0.0 * P)
                               for k in range(d)]))
    Fc.append(torch.stack([(Q[2 + d] + P) * u[k] for k in range(d)]))
    Fc = torch.stack(Fc)                                   # (d+3, d, ...)
    out = dict(pr=pr, nhat=nhat, a=a, s=s, Fc=Fc)
    if prm.viscous:
        gU = raw["gU"]
        mu = prm.mu[0] * alpha + prm.mu[1] * (1.0 - alpha)
        div = sum(gU[j][j] for j in range(d))
        tau = torch.stack([torch.stack([
            mu * (gU[j][k] + gU[k][j] - (2.0 / 3.0) * (div if j == k else 0.0 * div))
            for k in range(d)]) for j in range(d)])        # tau[j][k]
        V = [torch.zeros_like(Fc[0]), torch.zeros_like(Fc[0])]
        V += [tau[j] for j in range(d)]
        V.append(torch.stack([sum(tau[j][k] * u[j] for j in range(d))
                              for k in range(d)]))
        out["mu"] = mu
        out["V"] = torch.stack(V)                          # (d+3, d, ...)
    return out


def _trace(t, k, idx):
    """Values on the face node layer idx along axis k (node axes are last,
    x fastest)."""
    return t.select(t.dim() - 1 - k, idx)


def _trace_raw(raw, k, idx):
    return {key: _trace(v, k, idx) for key, v in raw.items()}


def _riemann_ghost(Q, k, side, d, P_b, prm):
    """Far-field ghost state of a Riemann-invariant boundary with zero velocity
    and pressure P_b outside (Section "Rayleigh-Taylor instability": top
    boundary).  With n the outward normal and the mixture treated as a
    stiffened gas at the interior composition (gamma - 1 = 1/xi), the outgoing
    invariant J+ = u.n + 2 xi c comes from the interior and the incoming one
    J- = -2 xi c_far from the far field (u = 0, P = P_b, interior density);
    the boundary state has u.n = (J+ + J-)/2 and c = (J+ - J-)/(4 xi), the
    pressure that gives this c at the interior density, and interior partial
    densities, tangential velocity, alpha and psi."""
    pr = primitives(Q, d, prm)
    rho, xi, pi = pr["rho"], pr["xi"], pr["pi"]
    sm = 1.0 if side == 1 else -1.0
    un = sm * pr["u"][k]
    c_far = torch.sqrt(((1.0 + xi) * P_b + pi) / (xi * rho))
    j_out = un + 2.0 * xi * pr["c"]
    j_in = -2.0 * xi * c_far
    un_b = 0.5 * (j_out + j_in)
    c_b = (j_out - j_in) / (4.0 * xi)
    P_g = (xi * rho * c_b * c_b - pi) / (1.0 + xi)
    u_g = pr["u"].clone()
    u_g[k] = u_g[k] + sm * (un_b - un)
    G = Q.clone()
    for j in range(d):
        G[2 + j] = rho * u_g[j]
    G[2 + d] = xi * P_g + pi + 0.5 * rho * (u_g * u_g).sum(0)
    return G


def _ghost(rawI, kind, k, side, d, bc_vals, prm):
    """Ghost trace for a non-periodic boundary face, built from the interior trace."""
    if kind == "extrapolate":
        return dict(rawI)
    if kind in ("slip_wall", "no_slip"):
        # mirror image: scalar gradients have their normal component negated.
        # Slip wall: the normal momentum flips and the velocity gradient is
        # mirrored too (no tangential stress); no-slip wall: the whole momentum
        # flips (zero velocity on the wall) and the velocity gradient is kept
        # (the wall takes the interior shear stress).
        Q = rawI["Q"].clone()
        if kind == "slip_wall":
            Q[2 + k] = -Q[2 + k]
        else:
            for j in range(d):
                Q[2 + j] = -Q[2 + j]
        sgn = torch.ones(d, dtype=torch.float64)
        sgn[k] = -1.0
        shp = (d,) + (1,) * (rawI["gA"].dim() - 1)
        g = dict(Q=Q, gA=rawI["gA"] * sgn.view(shp), gP=rawI["gP"] * sgn.view(shp))
        if "gU" in rawI:
            if kind == "slip_wall":
                shp2 = (d, d) + (1,) * (rawI["gU"].dim() - 2)
                g["gU"] = rawI["gU"] * (sgn[:, None] * sgn[None, :]).view(shp2)
            else:
                g["gU"] = rawI["gU"]
        return g
    if kind == "riemann":
        g = dict(rawI)
        g["Q"] = _riemann_ghost(rawI["Q"], k, side, d, float(bc_vals[0]), prm)
        return g
    if kind == "dirichlet":
        Q = rawI["Q"].clone()
        vals = torch.as_tensor(bc_vals, dtype=torch.float64)
        for f in range(4 + d):                 # q1, q2, rho u, rho E, alpha
            Q[f] = torch.zeros_like(Q[f]) + vals[f]
        g = dict(rawI)
        g["Q"] = Q
        return g
    raise ValueError(kind)


def _where_raw(mask, A, B):
    """Per-element select between two raw traces (mask has shape (B,))."""
    out = {}
    for key in A:
        t = A[key]
        lead = {"Q": 1, "gA": 1, "gP": 1, "gU": 2}[key]
        m = mask.view((1,) * lead + (-1,) + (1,) * (t.dim() - lead - 1))
        out[key] = torch.where(m, A[key], B[key])
    return out


def _place(face_val, k, vec):
    """Spread a face-layer tensor along axis k with weights vec (length n)."""
    n = vec.numel()
    v = vec.view((n,) + (1,) * k)
    return face_val.unsqueeze(face_val.dim() - k) * v


def _face_contrib(mesh, prm, k, side, I, E, rawI, rawE):
    """Contributions of one face of every batch element to its own nodes."""
    d, n, p = mesh.d, mesh.n, mesh.p
    sm = -1.0 if side == 0 else 1.0                       # m = sm * e_k
    QI, QE = rawI["Q"], rawE["Q"]
    uI, uE = I["pr"]["u"], E["pr"]["u"]
    umI, umE = sm * uI[k], sm * uE[k]
    lam = torch.maximum(torch.abs(umI) + I["pr"]["c"], torch.abs(umE) + E["pr"]["c"])
    h = mesh.h[k]
    eta = prm.c_ip * prm.Gamma * prm.eps * (p + 1) ** 2 / h
    amI, amE = sm * I["a"][k], sm * E["a"][k]
    alI, alE = QI[3 + d], QE[3 + d]
    ahat = 0.5 * (amI + amE) - eta * (alI - alE)
    L = 1.0 / (float(mesh.w[0]) * mesh.J[k])
    ncons = d + 3
    contrib = []
    for q in range(ncons):
        FmI, FmE = sm * I["Fc"][q][k], sm * E["Fc"][q][k]
        Fhat = 0.5 * (FmI + FmE) - 0.5 * lam * (QE[q] - QI[q])
        sbar = 0.5 * (I["s"][q] + E["s"][q])
        t = (FmI - Fhat) + (sbar * ahat - I["s"][q] * amI)
        if prm.viscous and q >= 2:
            VmI, VmE = sm * I["V"][q][k], sm * E["V"][q][k]
            mubar = 0.5 * (I["mu"] + E["mu"])
            etav = prm.c_ip * mubar * (p + 1) ** 2 / h
            if q < 2 + d:
                j = q - 2
                pen = etav * (uI[j] - uE[j])
            else:
                pen = etav * sum((uI[j] - uE[j]) * (0.5 * (uI[j] + uE[j]))
                                 for j in range(d))
            Vhat = 0.5 * (VmI + VmE) - pen
            t = t + (Vhat - VmI)
        contrib.append(L * t)
    KA = 0.5 * (lam - umI) * (alE - alI)
    contrib.append(L * (KA + (ahat - amI)))
    psI, psE = QI[4 + d], QE[4 + d]
    contrib.append(L * (0.5 * (lam - umI) * (psE - psI)))
    contrib = torch.stack(contrib)                        # (F, B, face...)
    idx = 0 if side == 0 else n - 1
    onehot = torch.zeros(n, dtype=torch.float64)
    onehot[idx] = 1.0
    R = _place(contrib, k, onehot)
    # SIPG symmetric term along the normal lines through the face nodes
    jump = alI - alE
    wts = torch.stack([mesh.D[idx, a] / (2.0 * mesh.w[a] * mesh.J[k] ** 2)
                       for a in range(n)])
    sym = []
    for q in range(ncons):
        sbar = 0.5 * (I["s"][q] + E["s"][q])
        sym.append(sm * sbar * prm.Gamma * prm.eps * jump)
    sym.append(sm * prm.Gamma * prm.eps * jump)
    sym.append(torch.zeros_like(jump))
    R = R + _place(torch.stack(sym), k, wts)
    return R


def _rhs_batch(U, mesh, prm, el):
    d, n, F = mesh.d, mesh.n, mesh.nf
    shp = (F, el.numel()) + (n,) * d
    X = U[:, el].reshape(shp)
    raw = _raw(X, mesh, prm)
    own = _pointwise(raw, d, prm)
    u = own["pr"]["u"]
    a = own["a"]
    # volume terms (strong form)
    R = []
    for q in range(d + 3):
        flux = -own["Fc"][q] + own["s"][q] * a
        if prm.viscous:
            flux = flux + own["V"][q]
        R.append(sum(_dk(flux[k], k, mesh) for k in range(d)))
    R.append(-(u * raw["gA"]).sum(0) + sum(_dk(a[k], k, mesh) for k in range(d)))
    R.append(-(u * raw["gP"]).sum(0))
    R = torch.stack(R)
    # sources: gravity and continuum surface force
    rho = own["pr"]["rho"]
    nhat = own["nhat"]
    if torch.is_tensor(prm.sigma) or prm.sigma != 0.0:
        kappa = -sum(_dk(nhat[k], k, mesh) for k in range(d))
        delta = prm.grad_reg
        dG = torch.sqrt((raw["gA"] * raw["gA"]).sum(0) + delta * delta) - delta
        csf = prm.sigma * kappa * dG
    else:
        csf = None
    src = [torch.zeros_like(rho), torch.zeros_like(rho)]
    eng = torch.zeros_like(rho)
    for j in range(d):
        sj = rho * prm.g[j]
        ej = rho * prm.g[j] * u[j]
        if csf is not None:
            sj = sj + csf * nhat[j]
            ej = ej + csf * u[j] * nhat[j]
        src.append(sj)
        eng = eng + ej
    src += [eng, torch.zeros_like(rho), torch.zeros_like(rho)]
    R = R + torch.stack(src)
    # faces
    for k in range(d):
        for side in (0, 1):
            nb, bnd = mesh.neighbour(el, k, side)
            idxI = 0 if side == 0 else n - 1
            idxE = n - 1 if side == 0 else 0
            rawI = _trace_raw(raw, k, idxI)
            Y = U[:, nb].reshape(shp)
            rawE = _trace_raw(_raw(Y, mesh, prm), k, idxE)
            kind = mesh.bc[k][side]
            if kind != "periodic" and bool(bnd.any()):
                ghost = _ghost(rawI, kind, k, side, d, mesh.bc_state.get((k, side)), prm)
                rawE = _where_raw(bnd, ghost, rawE)
            I = _pointwise(rawI, d, prm)
            E = _pointwise(rawE, d, prm)
            R = R + _face_contrib(mesh, prm, k, side, I, E, rawI, rawE)
    return R.reshape(F, el.numel(), n ** d)


def rhs(U, mesh, prm, elems=None, chunk=8192):
    """R(U) of the semi-discrete scheme, U and R in layout [field, element, node].

    ``elems`` (LongTensor) restricts the evaluation to those elements; the
    result then has shape (F, len(elems), nn).
    """
    if elems is None:
        elems = torch.arange(mesh.E)
    elems = torch.as_tensor(elems, dtype=torch.long)
    parts = [_rhs_batch(U, mesh, prm, elems[s:s + chunk])
             for s in range(0, elems.numel(), chunk)]
    return torch.cat(parts, dim=1)
