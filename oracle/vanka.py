"""Additive Vanka relaxation.

Oracle (test infrastructure only).  Follows the paper's "Vanka relaxation
scheme" subsection (equation vksystem and Algorithm 3): one patch per
pressure (Q1) node, holding that pressure DoF and both velocity components
at every Q2 node of the (up to four) elements touching the node; the patch
matrix A_i = V_i A V_i^T is extracted from the assembled, Dirichlet-
eliminated global matrix and inverted once (the inverses do not change
between iterations); one sweep solves every patch against the same residual
and adds the weighted corrections, x += sum_i V_i^T W_i A_i^{-1} V_i r.

Readings (the paper gives no weight values): W_i = omega * diag(1/m_j),
with m_j the number of patches containing DoF j, and weight 0 on Dirichlet
DoFs.  Boundary nodes have patches too (the paper's Table 1 patch counts
include them), of 31 DoFs on edges and 19 at corners.

Patch-local numbering (51 slots, absent slots -1): u_x at the 5x5 Q2 nodes
(2I-2+a, 2J-2+b) in slot b*5+a, u_y in slot 25+b*5+a, the pressure in
slot 50.  Patch index k = J*(N+1) + I.

The "tuned" variant of the paper shares one inverse among all patches with
identical matrices: on a uniform mesh the matrix depends only on the
distance class of I and of J (0, 1, interior, N-1, N), 25 classes in all.
``patch_inverses(..., shared=True)`` extracts one representative per class
from the assembled matrix; ``shared=False`` extracts every patch.  A test
checks that the two agree.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from stokes_inputs import grid_sizes

PATCH_SLOTS = 51


def patch_dofs(N: int) -> np.ndarray:
    """Global DoF indices of every patch, shape ((N+1)^2, 51), -1 = absent."""
    g = grid_sizes(N)
    s2 = g.q2_side
    nodes = np.arange(N + 1)
    II, JJ = np.meshgrid(nodes, nodes, indexing="xy")
    II, JJ = II.ravel(), JJ.ravel()
    idx = -np.ones(((N + 1) ** 2, PATCH_SLOTS), dtype=np.int64)
    for b in range(5):
        for a in range(5):
            qi = 2 * II - 2 + a
            qj = 2 * JJ - 2 + b
            ok = (qi >= 0) & (qi < s2) & (qj >= 0) & (qj < s2)
            node = qj * s2 + qi
            idx[:, b * 5 + a] = np.where(ok, g.off_ux + node, -1)
            idx[:, 25 + b * 5 + a] = np.where(ok, g.off_uy + node, -1)
    idx[:, 50] = g.off_p + JJ * (N + 1) + II
    return idx


def distance_class(i: np.ndarray, N: int) -> np.ndarray:
    """0: on the low boundary, 1: one element in, 2: interior, 3: one element
    from the high boundary, 4: on the high boundary."""
    i = np.asarray(i)
    c = np.full(i.shape, 2, dtype=np.int64)
    c[i == 1] = 1
    c[i == N - 1] = 3
    c[i == 0] = 0
    c[i == N] = 4
    return c


def patch_classes(N: int) -> np.ndarray:
    nodes = np.arange(N + 1)
    II, JJ = np.meshgrid(nodes, nodes, indexing="xy")
    return (distance_class(JJ.ravel(), N) * 5 + distance_class(II.ravel(), N))


def extract_patch_matrix(A: sp.csr_matrix, dofs: np.ndarray) -> np.ndarray:
    """Dense V_i A V_i^T for the present DoFs of one patch."""
    S = dofs[dofs >= 0]
    return A[S][:, S].toarray()


def patch_inverses(A: sp.csr_matrix, N: int, shared: bool):
    """Inverse of every patch matrix, zero-padded to the 51 slots.

    Returns (inv, classes): with shared=False inv has shape (P, 51, 51);
    with shared=True shape (25, 51, 51), one per class, and ``classes``
    maps patch -> class."""
    idx = patch_dofs(N)
    cls = patch_classes(N)

    def padded_inverse(dofs):
        present = dofs >= 0
        Ak = extract_patch_matrix(A, dofs)
        Ainv = np.linalg.inv(Ak)
        out = np.zeros((PATCH_SLOTS, PATCH_SLOTS))
        pos = np.nonzero(present)[0]
        out[np.ix_(pos, pos)] = Ainv
        return out

    if not shared:
        inv = np.stack([padded_inverse(idx[k]) for k in range(idx.shape[0])])
        return inv, cls
    inv = np.zeros((25, PATCH_SLOTS, PATCH_SLOTS))
    for c in range(25):
        members = np.nonzero(cls == c)[0]
        if members.size:
            inv[c] = padded_inverse(idx[members[0]])
    return inv, cls


def local_patch_matrix(N: int, I: int, J: int, nu: float = 1.0):
    """V_i A V_i^T for the patch at Q1 node (I, J) of an N x N mesh without
    assembling the global matrix: the entries between patch DoFs summed over
    the element matrices of every element that touches the patch, then the
    Dirichlet DoFs eliminated (identity rows and columns).  Returns the dense
    matrix on the present slots and the patch's global DoF indices."""
    from .fem import element_matrices
    g = grid_sizes(N)
    s2, s1 = g.q2_side, g.q1_side
    E = element_matrices(1.0 / N)
    dofs = patch_dofs_one(N, I, J)
    present = np.nonzero(dofs >= 0)[0]
    S = dofs[present]
    pos = {int(d): k for k, d in enumerate(S)}
    A = np.zeros((len(S), len(S)))
    for ey in range(max(0, J - 2), min(N, J + 2)):
        for ex in range(max(0, I - 2), min(N, I + 2)):
            q2 = [(2 * ey + bb) * s2 + 2 * ex + aa for bb in range(3) for aa in range(3)]
            q1 = [(ey + d) * s1 + ex + c for d in range(2) for c in range(2)]
            for f, Bk in ((0, E["Bx"]), (1, E["By"])):
                off = g.off_ux if f == 0 else g.off_uy
                for a_ in range(9):
                    ia = pos.get(off + q2[a_])
                    if ia is None:
                        continue
                    for b_ in range(9):
                        ib = pos.get(off + q2[b_])
                        if ib is not None:
                            A[ia, ib] += nu * E["L"][a_, b_]
                    for k in range(4):
                        ip = pos.get(g.off_p + q1[k])
                        if ip is not None:
                            A[ip, ia] += Bk[k, a_]
                            A[ia, ip] += Bk[k, a_]
    for k, d in enumerate(S):
        if d < g.off_p:
            node = d % g.n_q2
            qi, qj = node % s2, node // s2
            if qi == 0 or qj == 0 or qi == s2 - 1 or qj == s2 - 1:
                A[k, :] = 0.0
                A[:, k] = 0.0
                A[k, k] = 1.0
    return A, S


def patch_dofs_one(N: int, I: int, J: int) -> np.ndarray:
    """The 51-slot DoF list of the patch at Q1 node (I, J), -1 = absent."""
    g = grid_sizes(N)
    s2 = g.q2_side
    idx = -np.ones(PATCH_SLOTS, dtype=np.int64)
    for b in range(5):
        for a in range(5):
            qi, qj = 2 * I - 2 + a, 2 * J - 2 + b
            if 0 <= qi < s2 and 0 <= qj < s2:
                idx[b * 5 + a] = g.off_ux + qj * s2 + qi
                idx[25 + b * 5 + a] = g.off_uy + qj * s2 + qi
    idx[50] = g.off_p + J * (N + 1) + I
    return idx


def sampled_sweep_update(N: int, x: np.ndarray, b: np.ndarray, dofs, omega: float = 0.5,
                         nu: float = 1.0) -> np.ndarray:
    """The change one additive sweep makes at the given DoFs, computed one DoF
    at a time: sum over the patches i containing DoF j of
    (omega/m_j) (A_i^{-1} V_i r)_j, with r from residual_rows and A_i from
    local_patch_matrix (for meshes too large to assemble).  Dirichlet DoFs do
    not change."""
    from .fem import residual_rows
    g = grid_sizes(N)
    s2 = g.q2_side
    inv_cache = {}
    out = np.zeros(len(dofs))
    for n_, d in enumerate(dofs):
        d = int(d)
        if d < g.off_p:
            node = d % g.n_q2
            qi, qj = node % s2, node // s2
            if qi == 0 or qj == 0 or qi == s2 - 1 or qj == s2 - 1:
                continue
            Is = [I for I in range((qi - 1) // 2, qi // 2 + 2) if abs(2 * I - qi) <= 2 and 0 <= I <= N]
            Js = [J for J in range((qj - 1) // 2, qj // 2 + 2) if abs(2 * J - qj) <= 2 and 0 <= J <= N]
            patches = [(I, J) for J in Js for I in Is]
        else:
            node = d - g.off_p
            patches = [(node % (N + 1), node // (N + 1))]
        total = 0.0
        for I, J in patches:
            key = (int(distance_class(np.array(I), N)), int(distance_class(np.array(J), N)))
            if key not in inv_cache:
                Ak, _ = local_patch_matrix(N, I, J, nu)
                inv_cache[key] = np.linalg.inv(Ak)
            S = patch_dofs_one(N, I, J)
            S = S[S >= 0]
            r = residual_rows(N, x, b, S, nu)
            pos = int(np.nonzero(S == d)[0][0])
            total += inv_cache[key][pos] @ r
        out[n_] = omega / len(patches) * total
    return out


def multiplicities(N: int) -> np.ndarray:
    """m_j = number of patches containing DoF j, counted by brute force."""
    idx = patch_dofs(N)
    g = grid_sizes(N)
    flat = idx[idx >= 0]
    return np.bincount(flat, minlength=g.n).astype(np.float64)


def vanka_weights(N: int, dmask: np.ndarray, omega: float) -> np.ndarray:
    """Per-DoF weight omega/m_j, zero on the Dirichlet set."""
    m = multiplicities(N)
    w = omega / m
    w[dmask] = 0.0
    return w


class VankaSmoother:
    """Precomputed data of one level's additive Vanka sweep."""

    def __init__(self, A: sp.csr_matrix, N: int, dmask: np.ndarray,
                 omega: float = 0.5, shared: bool | None = None):
        if shared is None:
            shared = N > 32
        self.A = A
        self.N = N
        self.omega = omega
        self.idx = patch_dofs(N)
        self.inv, self.cls = patch_inverses(A, N, shared)
        self.shared = shared
        self.w = vanka_weights(N, dmask, omega)
        self.n = A.shape[0]

    def patch_corrections(self, r: np.ndarray) -> np.ndarray:
        """delta_i = A_i^{-1} V_i r for every patch, shape (P, 51)."""
        R = np.where(self.idx >= 0, r[np.maximum(self.idx, 0)], 0.0)
        if not self.shared:
            return np.einsum("pij,pj->pi", self.inv, R)
        D = np.empty_like(R)
        for c in range(25):
            sel = self.cls == c
            if np.any(sel):
                D[sel] = R[sel] @ self.inv[c].T
        return D

    def apply_to_residual(self, r: np.ndarray) -> np.ndarray:
        """sum_i V_i^T W_i A_i^{-1} V_i r."""
        D = self.patch_corrections(r)
        ok = self.idx >= 0
        flat = self.idx[ok]
        contrib = (D * self.w[np.maximum(self.idx, 0)])[ok]
        return np.bincount(flat, weights=contrib, minlength=self.n)

    def sweep(self, x: np.ndarray, b: np.ndarray) -> np.ndarray:
        """One additive sweep: r = b - A x; x + sum_i V_i^T W_i A_i^{-1} V_i r."""
        r = b - self.A @ x
        return x + self.apply_to_residual(r)
