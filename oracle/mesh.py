"""Structured Cartesian element grid for the oracle (test infrastructure only).

The paper partitions the domain into non-overlapping elements with outward
unit normals on their boundaries (Section "Discontinuous Galerkin
discretisation", the partition of Omega and the surface integral of the
local weak form).  Here the elements are the cells of an axis-aligned box
split into N_x (x N_y (x N_z)) equal cells; each element carries (p+1)^d GLL
nodes, and the map from the reference cube is affine with Jacobian
J_k = h_k / 2 per axis.

Flat layouts (the same ones the library documents in its public header):
  element index  e = e_x + N_x (e_y + N_y e_z)
  node index     j = a_x + n (a_y + n a_z),  n = p + 1
  state          U[f, e, j]
"""

import torch

from .gll import gll_nodes_weights, derivative_matrix

BC_KINDS = ("periodic", "slip_wall", "dirichlet", "extrapolate", "no_slip", "riemann")


class OracleMesh:
    def __init__(self, dim, order, n_elem, lo, hi, bc=None, bc_state=None):
        if dim not in (1, 2, 3):
            raise ValueError("dim must be 1, 2 or 3")
        self.d = dim
        self.p = order
        self.n = order + 1
        self.N = tuple(int(v) for v in n_elem[:dim])
        self.lo = tuple(float(v) for v in lo[:dim])
        self.hi = tuple(float(v) for v in hi[:dim])
        if bc is None:
            bc = [("periodic", "periodic")] * dim
        self.bc = [tuple(bc[k]) for k in range(dim)]
        for k in range(dim):
            for s in range(2):
                if self.bc[k][s] not in BC_KINDS:
                    raise ValueError(f"unknown bc {self.bc[k][s]}")
            if (self.bc[k][0] == "periodic") != (self.bc[k][1] == "periodic"):
                raise ValueError("periodic must be set on both sides of an axis")
        self.bc_state = {} if bc_state is None else dict(bc_state)
        self.h = tuple((self.hi[k] - self.lo[k]) / self.N[k] for k in range(dim))
        self.J = tuple(0.5 * self.h[k] for k in range(dim))
        self.xi, self.w = gll_nodes_weights(order)
        self.D = derivative_matrix(self.xi)
        self.E = 1
        for v in self.N:
            self.E *= v
        self.nn = self.n ** dim
        self.nf = dim + 5

    # ---- element indexing -------------------------------------------------
    def elem_multi(self, e):
        """(e_x, e_y, e_z) components of flat element indices (LongTensor)."""
        out = []
        r = e.clone()
        for k in range(self.d):
            out.append(r % self.N[k])
            r = torch.div(r, self.N[k], rounding_mode="floor")
        return out

    def elem_flat(self, comps):
        e = torch.zeros_like(comps[0])
        stride = 1
        for k in range(self.d):
            e = e + comps[k] * stride
            stride *= self.N[k]
        return e

    def neighbour(self, e, k, side):
        """Neighbour across face (axis k, side 0 = low / 1 = high).

        Returns (neighbour flat index, boundary mask).  Across a periodic
        boundary the index wraps; across any other boundary the mask is True
        and the returned index is the element itself (a placeholder: the
        caller replaces that side by a ghost state).
        """
        comps = self.elem_multi(e)
        step = -1 if side == 0 else 1
        c = comps[k] + step
        if self.bc[k][side] == "periodic":
            bnd = torch.zeros_like(c, dtype=torch.bool)
            c = c % self.N[k]
        else:
            bnd = (c < 0) | (c >= self.N[k])
            c = torch.where(bnd, comps[k], c)
        comps = list(comps)
        comps[k] = c
        return self.elem_flat(comps), bnd

    # ---- geometry ---------------------------------------------------------
    def node_coords(self):
        """Physical node coordinates, float64 tensor of shape (d, E, nn)."""
        e = torch.arange(self.E)
        comps = self.elem_multi(e)
        j = torch.arange(self.nn)
        out = torch.empty(self.d, self.E, self.nn, dtype=torch.float64)
        for k in range(self.d):
            a_k = torch.div(j, self.n ** k, rounding_mode="floor") % self.n
            ref = self.xi[a_k]                                   # (nn,)
            out[k] = (self.lo[k] + self.h[k] * comps[k].to(torch.float64)[:, None]
                      + self.J[k] * (ref[None, :] + 1.0))
        return out

    def node_weights(self):
        """Diagonal mass matrix W_j = prod_k w_{a_k} J_k, shape (nn,)."""
        j = torch.arange(self.nn)
        W = torch.ones(self.nn, dtype=torch.float64)
        for k in range(self.d):
            a_k = torch.div(j, self.n ** k, rounding_mode="floor") % self.n
            W = W * self.w[a_k] * self.J[k]
        return W

    def node_shape(self):
        return (self.n,) * self.d
