"""Inexact Braess-Sarazin relaxation.

Oracle (test infrastructure only).  Follows the paper's "Braess-Sarazin
relaxation scheme" subsection (the block factorisation with L replaced by
t D, equations bseq1 and bseq2, and the Braess-Sarazin algorithm): with D
the diagonal of the velocity block L and the approximate Schur complement
S = -(1/t) B D^{-1} B^T, one relaxation step on the residual (r_u, r_p)
of the current iterate

  1. approximately solves  S dp = r_p - (1/t) B D^{-1} r_u  by weighted
     Jacobi sweeps on S, starting from dp = 0;
  2. computes  du = (1/t) D^{-1} (r_u - B^T dp);
  3. updates  p += omega_bs dp,  u += omega_bs du.

The matrices are the blocks of the assembled, Dirichlet-eliminated
operator (identity rows on Dirichlet velocity DoFs, whose B^T rows and B
columns are zero), so Dirichlet DoFs receive (omega_bs / t) r_u there.

Readings (the paper reports parameters found by experiment only for the
other schemes): t, omega_bs, the Jacobi weight and the number of Jacobi
sweeps are arguments.  The defaults t = 1, omega_bs = 1, weight 1, two
sweeps are the best of a small FGMRES study with this V-cycle (64 x 64, 5
levels: 6 iterations with V(2,2), 13 with V(1,1)); one sweep with weight 1
does not converge, one with weight 0.8 needs 8 and 18.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from stokes_inputs import grid_sizes


class BraessSarazinSmoother:
    def __init__(self, A: sp.csr_matrix, N: int, t: float = 1.0, omega_bs: float = 1.0,
                 jacobi_weight: float = 1.0, jacobi_sweeps: int = 2):
        g = grid_sizes(N)
        nv = g.off_p
        A = sp.csr_matrix(A)
        self.A = A
        self.nv = nv
        self.L = A[:nv, :nv].tocsr()
        self.BT = A[:nv, nv:].tocsr()
        self.B = A[nv:, :nv].tocsr()
        self.t = float(t)
        self.omega_bs = float(omega_bs)
        self.jacobi_weight = float(jacobi_weight)
        self.jacobi_sweeps = int(jacobi_sweeps)
        self.Dinv = 1.0 / self.L.diagonal()
        # S = -(1/t) B D^{-1} B^T and its diagonal
        self.S = (-(1.0 / self.t) * (self.B @ sp.diags(self.Dinv) @ self.BT)).tocsr()
        self.Sdiag = self.S.diagonal()

    def schur_rhs(self, r: np.ndarray) -> np.ndarray:
        """r_p - (1/t) B D^{-1} r_u (right-hand side of equation bseq1)."""
        ru, rp = r[:self.nv], r[self.nv:]
        return rp - (1.0 / self.t) * (self.B @ (self.Dinv * ru))

    def schur_jacobi(self, rhs: np.ndarray) -> np.ndarray:
        """Weighted Jacobi sweeps on S dp = rhs from dp = 0."""
        dp = np.zeros_like(rhs)
        for _ in range(self.jacobi_sweeps):
            dp = dp + self.jacobi_weight * (rhs - self.S @ dp) / self.Sdiag
        return dp

    def correction(self, r: np.ndarray) -> np.ndarray:
        """The unweighted update (du, dp) for the residual r."""
        dp = self.schur_jacobi(self.schur_rhs(r))
        du = (1.0 / self.t) * self.Dinv * (r[:self.nv] - self.BT @ dp)
        return np.concatenate([du, dp])

    def sweep(self, x: np.ndarray, b: np.ndarray) -> np.ndarray:
        r = b - self.A @ x
        return x + self.omega_bs * self.correction(r)
