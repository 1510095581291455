"""Grid transfers between nested uniform meshes.

Oracle (test infrastructure only).  Follows the paper's multigrid section:
one interpolation operator P from the coarse Q2/Q1 spaces to their fine
analogues (the finite-element interpolation, since the spaces are nested)
and its transpose as restriction, as used by the V-cycle algorithm
(Algorithm 1).

P is built from its definition: the fine nodal value is the coarse
finite-element function evaluated at the fine node.  The 1D matrices are
obtained by evaluating the coarse 1D Lagrange basis at the fine node
coordinates; the 2D operators are their tensor products (the bases are
tensor products).  Reading for the Dirichlet set (the paper is silent):
rows of fine Dirichlet DoFs and columns of coarse Dirichlet DoFs are
zeroed, so restricted residuals vanish on coarse Dirichlet DoFs and
corrections never touch fine boundary values.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from stokes_inputs import grid_sizes, velocity_dirichlet_mask
from .fem import lagrange_1d, Q2_NODES_1D, Q1_NODES_1D


def interpolation_1d(nc: int, degree: int) -> np.ndarray:
    """Dense 1D interpolation from the coarse mesh with nc elements to the
    fine mesh with 2 nc elements, for continuous Lagrange elements of the
    given degree (1 or 2).  Shape (degree*2*nc + 1, degree*nc + 1)."""
    nodes = Q2_NODES_1D if degree == 2 else Q1_NODES_1D
    nf = 2 * nc
    n_fine = degree * nf + 1
    n_coarse = degree * nc + 1
    Hc = 1.0 / nc
    xf = np.arange(n_fine) / (degree * nf)
    P = np.zeros((n_fine, n_coarse))
    for i, x in enumerate(xf):
        e = min(int(np.floor(x / Hc)), nc - 1)
        t = (x - e * Hc) / Hc
        V, _ = lagrange_1d(nodes, np.array([t]))
        for a in range(degree + 1):
            P[i, degree * e + a] += V[a, 0]
    P[np.abs(P) < 1e-15] = 0.0
    return P


def prolongation(nc: int) -> sp.csr_matrix:
    """P_{l-1}: coarse full vector (nc elements per side) -> fine full vector
    (2 nc per side), block diagonal over (u_x, u_y, p), with the Dirichlet
    rows/columns zeroed as described in the module docstring."""
    P2 = sp.csr_matrix(interpolation_1d(nc, 2))
    P1 = sp.csr_matrix(interpolation_1d(nc, 1))
    Q2 = sp.kron(P2, P2, format="csr")  # index j*side + i -> kron(P_y, P_x)
    Q1 = sp.kron(P1, P1, format="csr")
    P = sp.block_diag([Q2, Q2, Q1], format="csr")
    fmask = velocity_dirichlet_mask(2 * nc)
    cmask = velocity_dirichlet_mask(nc)
    P = sp.diags((~fmask).astype(float)) @ P @ sp.diags((~cmask).astype(float))
    P = P.tocsr()
    P.eliminate_zeros()
    assert P.shape == (grid_sizes(2 * nc).n, grid_sizes(nc).n)
    return P


def prolong_rows(nc: int, ec: np.ndarray, rows) -> np.ndarray:
    """(P ec)[rows] computed row by row from the 1D interpolation matrices
    (the tensor-product definition of P), for meshes too large to assemble
    P.  Same Dirichlet reading as ``prolongation``."""
    return _tensor_rows(nc, ec, rows, transpose=False)


def restrict_rows(nc: int, rf: np.ndarray, rows) -> np.ndarray:
    """(P^T rf)[rows] for coarse rows, computed one coarse DoF at a time."""
    return _tensor_rows(nc, rf, rows, transpose=True)


def _tensor_rows(nc, v, rows, transpose):
    gf, gc = grid_sizes(2 * nc), grid_sizes(nc)
    fmask = velocity_dirichlet_mask(2 * nc)
    cmask = velocity_dirichlet_mask(nc)
    P1d = {2: interpolation_1d(nc, 2), 1: interpolation_1d(nc, 1)}
    out = np.empty(len(rows))
    for n_, row in enumerate(rows):
        row = int(row)
        g_out, g_in = (gc, gf) if transpose else (gf, gc)
        m_out, m_in = (cmask, fmask) if transpose else (fmask, cmask)
        if m_out[row]:
            out[n_] = 0.0
            continue
        if row < g_out.off_p:
            deg, f = 2, row // g_out.n_q2
            node = row % g_out.n_q2
            side_out, side_in = g_out.q2_side, g_in.q2_side
            off_in = g_in.off_ux if f == 0 else g_in.off_uy
        else:
            deg, node = 1, row - g_out.off_p
            side_out, side_in = g_out.q1_side, g_in.q1_side
            off_in = g_in.off_p
        i, j = node % side_out, node // side_out
        M = P1d[deg].T if transpose else P1d[deg]
        ci = np.nonzero(M[i])[0]
        cj = np.nonzero(M[j])[0]
        acc = 0.0
        for jj in cj:
            for ii in ci:
                k = off_in + jj * side_in + ii
                if not m_in[k]:
                    acc += M[j, jj] * M[i, ii] * v[k]
        out[n_] = acc
    return out
