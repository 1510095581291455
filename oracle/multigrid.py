"""Monolithic geometric multigrid V-cycle.

Oracle (test infrastructure only).  Follows the paper's Algorithm 1 (level
0 coarsest): relax, compute the residual, restrict it with P^T, recurse (or
solve exactly on level 0), correct with P, relax again; every level starts
from a zero initial guess.

Readings: the coarse operators are rediscretised on each level (equal to
the Galerkin product P^T A P for constant viscosity, which a test checks);
a per-element viscosity (array of N^2 values, index ey*N + ex) is coarsened
by the arithmetic mean of the four children, and its Vanka patches are then
all distinct ("simple" Vanka: one stored inverse per patch);
with coarse_operator="galerkin" the coarse operators are instead the
products A_{l-1} = P^T A_l P formed from the finest level down (identity
rows on the coarse Dirichlet DoFs, whose columns of P are zero), the
alternative for a per-element viscosity;
the relaxation is the additive Vanka sweep (or, with relaxation="bs", the
inexact Braess-Sarazin step of braess_sarazin.py), nu_pre sweeps before and
nu_post after the coarse correction; the level-0 solve is exact, with the
constant-pressure null space handled by bordering the matrix with
c = (0, 1_p): [[A_0, c], [c^T, 0]] [e; lambda] = [r; 0], solved by dense
LU (a library primitive).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from stokes_inputs import grid_sizes
from stokes_inputs import velocity_dirichlet_mask
from .fem import stokes_system
from .transfer import prolongation
from .braess_sarazin import BraessSarazinSmoother
from .vanka import VankaSmoother


class Level:
    def __init__(self, N: int, nu, omega: float, shared, relax: bool, relaxation: str = "vanka",
                 bs=None, A=None, progress=None):
        self.N = N
        if A is None:
            self.A, _, self.dmask, _ = stokes_system(N, nu)
        else:
            self.A, self.dmask = A, velocity_dirichlet_mask(N)
        if progress is not None:
            progress(f"{N}x{N} operator assembled")
        self.n = self.A.shape[0]
        if not relax:
            self.smoother = None
        elif relaxation == "bs":
            self.smoother = BraessSarazinSmoother(self.A, N, **(bs or {}))
        else:
            if np.ndim(nu) > 0:
                shared = False  # per-element viscosity: every patch differs
            self.smoother = VankaSmoother(self.A, N, self.dmask, omega, shared)


class Hierarchy:
    """Levels l = 0 (coarsest) .. L-1 (finest) with N_l = N / 2^(L-1-l)."""

    def __init__(self, N: int, levels: int, nu: float = 1.0, omega: float = 0.5,
                 nu_pre: int = 2, nu_post: int = 2, shared=None, relaxation: str = "vanka",
                 bs=None, coarse_operator: str = "rediscretise", progress=None):
        if levels < 2:
            raise ValueError("need at least two levels")
        if N % (1 << (levels - 1)):
            raise ValueError("N must be divisible by 2^(levels-1)")
        self.L = levels
        self.nu_pre, self.nu_post = nu_pre, nu_post
        nus = [nu]
        if np.ndim(nu) > 0:
            for l in range(levels - 1):
                Nl = N >> l
                v = np.asarray(nus[-1], dtype=np.float64).reshape(Nl, Nl)
                nus.append(0.25 * (v[0::2, 0::2] + v[0::2, 1::2] + v[1::2, 0::2] + v[1::2, 1::2]).ravel())
        else:
            nus = [nu] * levels
        self.nu_levels = nus[::-1]  # index l = level (0 coarsest)
        if coarse_operator not in ("rediscretise", "galerkin"):
            raise ValueError("coarse_operator must be 'rediscretise' or 'galerkin'")
        self.P = [None] + [prolongation(N >> (levels - l)) for l in range(1, levels)]
        ops = [None] * levels
        if coarse_operator == "galerkin":
            ops[-1], _, _, _ = stokes_system(N, nus[0])
            for l in range(levels - 1, 0, -1):
                Nc = N >> (levels - l)
                Ac = (self.P[l].T @ ops[l] @ self.P[l]).tocsr()
                Ac = (Ac + sp.diags(velocity_dirichlet_mask(Nc).astype(np.float64))).tocsr()
                Ac.eliminate_zeros()
                Ac.sort_indices()
                ops[l - 1] = Ac
        self.levels = []
        for l in range(levels):
            Nl = N >> (levels - 1 - l)
            self.levels.append(Level(Nl, self.nu_levels[l], omega, shared, relax=(l > 0),
                                     relaxation=relaxation, bs=bs, A=ops[l], progress=progress))
            if progress is not None:  # (a report only: long setups of large meshes)
                progress(f"level {l} ({Nl}x{Nl}) built")
        # bordered coarse matrix
        A0 = self.levels[0].A.toarray()
        g0 = grid_sizes(self.levels[0].N)
        n0 = A0.shape[0]
        c = np.zeros(n0)
        c[g0.off_p:] = 1.0
        Ab = np.zeros((n0 + 1, n0 + 1))
        Ab[:n0, :n0] = A0
        Ab[:n0, n0] = c
        Ab[n0, :n0] = c
        self.coarse_bordered = Ab
        self.coarse_lu = sla.lu_factor(Ab)

    def coarse_solve(self, r0: np.ndarray) -> np.ndarray:
        rhs = np.concatenate([r0, [0.0]])
        return sla.lu_solve(self.coarse_lu, rhs)[:-1]

    def mg(self, l: int, b: np.ndarray) -> np.ndarray:
        """MG(l, b) of Algorithm 1 with a zero initial guess."""
        lev = self.levels[l]
        x = np.zeros(lev.n)
        for _ in range(self.nu_pre):
            x = lev.smoother.sweep(x, b)
        r = b - lev.A @ x
        bc = self.P[l].T @ r
        if l - 1 == 0:
            e = self.coarse_solve(bc)
        else:
            e = self.mg(l - 1, bc)
        x = x + self.P[l] @ e
        for _ in range(self.nu_post):
            x = lev.smoother.sweep(x, b)
        return x

    def vcycle(self, r: np.ndarray) -> np.ndarray:
        """Preconditioner application z = M r on the finest level."""
        return self.mg(self.L - 1, r)

    @property
    def A(self):
        return self.levels[-1].A

    def patch_updates_per_cycle(self) -> int:
        """Patch solves in one V(nu_pre, nu_post) cycle (relaxed levels)."""
        return sum((self.nu_pre + self.nu_post) * (lev.N + 1) ** 2
                   for lev in self.levels[1:])
