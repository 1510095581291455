"""Restarted flexible GMRES with right preconditioning.

Oracle (test infrastructure only).  The paper uses its own FGMRES with the
multigrid V-cycle as a (non-symmetric, possibly varying) preconditioner and
gives no further detail; this follows Saad's flexible GMRES (1993):
Arnoldi by modified Gram-Schmidt on A z_j with z_j = M(v_j), Givens
rotations on the Hessenberg matrix, x = x0 + Z_m y_m.

Readings (the paper is silent): Euclidean norm over all DoFs; convergence
when the rotated residual estimate |g_{j+1}| <= rtol * ||b - A x_0||; after
each restart and at the end the true residual is recomputed and iteration
continues while it exceeds the tolerance; an exact breakdown
(h_{j+1,j} == 0) ends the cycle with the exact solution of the subspace.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class FgmresResult:
    x: np.ndarray
    iterations: int
    restarts: int
    converged: bool
    beta0: float
    true_rel_res: float
    est_history: list = field(default_factory=list)


def fgmres(A, b, x0, precond, rtol=1e-8, restart=30, max_iters=500,
           fixed_iters=None) -> FgmresResult:
    """Solve A x = b.  ``A`` supports ``@``; ``precond(v)`` returns z.

    With ``fixed_iters`` the solver runs exactly that many Arnoldi steps
    (restarting every ``restart``) regardless of the tolerance, which is
    how solutions are compared at equal iteration counts."""
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - A @ x
    beta0 = float(np.linalg.norm(r))
    hist = [1.0]
    if beta0 == 0.0:
        return FgmresResult(x, 0, 0, True, 0.0, 0.0, hist)
    target = rtol * beta0
    total = 0
    restarts = 0
    limit = fixed_iters if fixed_iters is not None else max_iters
    while True:
        beta = float(np.linalg.norm(r))
        m = restart
        V = np.zeros((m + 1, len(b)))
        Z = np.zeros((m, len(b)))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = precond(V[j])
            w = A @ Z[j]
            for i in range(j + 1):  # modified Gram-Schmidt
                H[i, j] = float(w @ V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            for i in range(j):  # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            denom = float(np.hypot(H[j, j], H[j + 1, j]))
            cs[j] = H[j, j] / denom
            sn[j] = H[j + 1, j] / denom
            breakdown = H[j + 1, j] == 0.0
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            H[j, j] = denom
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / beta0)
            if fixed_iters is None and abs(g[j + 1]) <= target:
                break
            if breakdown or total >= limit:
                break
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k]) if k else np.zeros(0)
        x = x + Z[:k].T @ y
        r = b - A @ x
        rn = float(np.linalg.norm(r))
        if fixed_iters is not None:
            if total >= fixed_iters:
                return FgmresResult(x, total, restarts, rn <= target, beta0, rn / beta0, hist)
        elif rn <= target:
            return FgmresResult(x, total, restarts, True, beta0, rn / beta0, hist)
        if total >= limit:
            return FgmresResult(x, total, restarts, False, beta0, rn / beta0, hist)
        restarts += 1
