"""FP64 CPU oracle for the two-phase DG residual (TEST INFRASTRUCTURE ONLY).

This package is the independent, slow, obviously-correct reference against
which the HIP path is checked.  It is test infrastructure: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import or run it.  The product path (``paper_2306_05002_amd``) never imports
it, and it never imports the product path.  The two share no code; they share
only the seeded primitive-field generators of
``paper_2306_05002_amd.workloads`` (which hold none of the method's
arithmetic), and the oracle itself does not even import those.

Everything is written with plain PyTorch CPU float64 tensor operations
(vectorised over elements) so that ``torch.autograd`` gives the oracle its own
discrete adjoint.  Each function cites the part of Tonicello & Ihme,
"A high-order diffused-interface approach for two-phase compressible flow
simulations using a Discontinuous Galerkin framework" (arXiv 2306.05002) it
follows.

Modules
  gll       Gauss-Lobatto-Legendre nodes, weights and the derivative matrix
  mesh      structured Cartesian element grid, neighbours, node coordinates
  physics   stiffened-gas closure, primitives, initial-condition map
  residual  the semi-discrete DG operator dU/dt = R(U)
  stepper   time-step rule, SSP-RK3 and monitors
  adjoint   loss, checkpointed rollout and autograd gradients
  kinematic the phase field and level set under a prescribed velocity (RK4,
            L1 and mass errors), the level-set re-initialisation, and the
            velocity of a nodal stream function

Pinning status (what fixes each function other than itself) is listed in the
tests under ``tests/test_oracle_*.py``.  The readings of the paper's silent
points (penalty constant, symmetric SIPG term, viscous numerical flux,
mixture sound speed, boundary ghosts, time-step rule) are parity unpinned at
the level of "is this what the authors ran": no implementation or hot-path
number of theirs exists to compare with.
"""

from .gll import gll_nodes_weights, derivative_matrix
from .mesh import OracleMesh
from .physics import Params, primitives, prim_to_cons
from .residual import rhs
from .stepper import max_rate, max_dt, rk_step, monitors
from . import adjoint

__all__ = [
    "gll_nodes_weights", "derivative_matrix", "OracleMesh", "Params",
    "primitives", "prim_to_cons", "rhs", "max_rate", "max_dt", "rk_step",
    "monitors", "adjoint",
]
