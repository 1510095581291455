"""Q2-Q1 Taylor-Hood finite elements on a uniform N x N mesh of [0,1]^2.

Oracle (test infrastructure only).  Follows the paper's "Problem setup" and
"Discretization" sections: the Stokes weak form with a(u,v) = nu int grad u :
grad v, the velocity space of continuous biquadratics, the pressure space of
continuous bilinears, and the saddle-point matrix [[L, B^T], [B, 0]] of the
equation labelled stokesmatrix, with L_ij = a(psi_j, psi_i) and
B_kj = b(psi_j, phi_k).

Readings (listed with the others in the design notes):
  * b(v, q) = -int q div v, so that the discrete pressure approximates +p of
    the strong form -nu lap u + grad p = f (the printed sign of b would give
    -p);
  * Dirichlet data on both velocity components on every edge;
  * the pressure is defined up to a constant; comparisons use zero
    mass-weighted mean.

Everything is computed from the definitions: 1D Lagrange bases evaluated at
3-point Gauss-Legendre nodes (exact for the polynomial degrees involved),
element integrals by tensor quadrature, global matrices by COO summation.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from stokes_inputs import grid_sizes, q2_boundary_mask, velocity_dirichlet_mask

# ----------------------------------------------------------------------------
# 1D building blocks on the reference interval [0, 1]
# ----------------------------------------------------------------------------

Q2_NODES_1D = np.array([0.0, 0.5, 1.0])
Q1_NODES_1D = np.array([0.0, 1.0])


def gauss_legendre_01(npts: int):
    """Gauss-Legendre points and weights mapped to [0, 1]."""
    t, w = np.polynomial.legendre.leggauss(npts)
    return 0.5 * (t + 1.0), 0.5 * w


def lagrange_1d(nodes: np.ndarray, t: np.ndarray):
    """Values and derivatives of the Lagrange basis on ``nodes`` at points t.

    Returns (V, D) of shape (len(nodes), len(t)), V[a, q] = l_a(t_q)."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    n = len(nodes)
    V = np.ones((n, t.size))
    D = np.zeros((n, t.size))
    for a in range(n):
        for m in range(n):
            if m == a:
                continue
            V[a] *= (t - nodes[m]) / (nodes[a] - nodes[m])
        # derivative: sum over dropped factor
        for k in range(n):
            if k == a:
                continue
            term = np.full(t.size, 1.0 / (nodes[a] - nodes[k]))
            for m in range(n):
                if m == a or m == k:
                    continue
                term *= (t - nodes[m]) / (nodes[a] - nodes[m])
            D[a] += term
    return V, D


# ----------------------------------------------------------------------------
# Element integrals
# ----------------------------------------------------------------------------

def q2_basis_2d(s, t, h):
    """Biquadratic basis on the element [0,h]^2 at reference points (s, t).

    Local index b*3 + a for the node at (a h/2, b h/2).  Returns values and
    physical x/y derivatives, each of shape (9, npts)."""
    Vs, Ds = lagrange_1d(Q2_NODES_1D, s)
    Vt, Dt = lagrange_1d(Q2_NODES_1D, t)
    val = np.empty((9, len(s)))
    dx = np.empty((9, len(s)))
    dy = np.empty((9, len(s)))
    for b in range(3):
        for a in range(3):
            k = b * 3 + a
            val[k] = Vs[a] * Vt[b]
            dx[k] = Ds[a] * Vt[b] / h
            dy[k] = Vs[a] * Dt[b] / h
    return val, dx, dy


def q1_basis_2d(s, t):
    """Bilinear basis, local index d*2 + c for the node at (c h, d h)."""
    Vs, _ = lagrange_1d(Q1_NODES_1D, s)
    Vt, _ = lagrange_1d(Q1_NODES_1D, t)
    val = np.empty((4, len(s)))
    for d in range(2):
        for c in range(2):
            val[d * 2 + c] = Vs[c] * Vt[d]
    return val


def _element_quadrature(npts: int, h: float):
    g, w = gauss_legendre_01(npts)
    S, T = np.meshgrid(g, g, indexing="xy")
    W = np.outer(w, w) * h * h  # W[j, i] for point (g_i, g_j)
    return S.ravel(), T.ravel(), W.ravel()


def element_matrices(h: float):
    """Element matrices on one square element of side h.

    Returns dict with
      'L'  (9x9): int grad psi_i . grad psi_j      (multiply by nu)
      'Bx' (4x9): -int phi_k d psi_j / dx
      'By' (4x9): -int phi_k d psi_j / dy
      'M'  (9x9): int psi_i psi_j
      'Mp' (4x4): int phi_k phi_l
      'wp' (4,) : int phi_k
    """
    s, t, w = _element_quadrature(3, h)
    val, dx, dy = q2_basis_2d(s, t, h)
    pv = q1_basis_2d(s, t)
    L = (dx * w) @ dx.T + (dy * w) @ dy.T
    L = 0.5 * (L + L.T)  # symmetric by definition; remove quadrature rounding
    Bx = -(pv * w) @ dx.T
    By = -(pv * w) @ dy.T
    M = (val * w) @ val.T
    M = 0.5 * (M + M.T)
    Mp = (pv * w) @ pv.T
    wp = pv @ w
    return {"L": L, "Bx": Bx, "By": By, "M": M, "Mp": Mp, "wp": wp}


# ----------------------------------------------------------------------------
# Element-to-global maps and assembly
# ----------------------------------------------------------------------------

def element_dof_maps(N: int):
    """Global Q2 and Q1 node indices of every element (ex, ey), element index
    ey*N + ex.  Returns (q2 (ne, 9), q1 (ne, 4))."""
    s2, s1 = 2 * N + 1, N + 1
    e = np.arange(N)
    EX, EY = np.meshgrid(e, e, indexing="xy")
    EX, EY = EX.ravel(), EY.ravel()
    q2 = np.empty((N * N, 9), dtype=np.int64)
    for b in range(3):
        for a in range(3):
            q2[:, b * 3 + a] = (2 * EY + b) * s2 + 2 * EX + a
    q1 = np.empty((N * N, 4), dtype=np.int64)
    for d in range(2):
        for c in range(2):
            q1[:, d * 2 + c] = (EY + d) * s1 + EX + c
    return q2, q1



def assemble_coo(rows, cols, vals, n: int) -> sp.csr_matrix:
    """Sum duplicate (row, col) contributions in the order they are given
    (stable sort, then sequential reduction), so that equal element
    contributions produce bitwise equal global entries (exact symmetry and
    translation invariance)."""
    rows = np.ravel(rows)
    cols = np.ravel(cols)
    vals = np.ravel(vals)
    order = np.lexsort((cols, rows))  # stable
    r, c, v = rows[order], cols[order], vals[order]
    if r.size == 0:
        return sp.csr_matrix((n, n))
    start = np.ones(r.size, dtype=bool)
    start[1:] = (r[1:] != r[:-1]) | (c[1:] != c[:-1])
    pos = np.nonzero(start)[0]
    sums = np.add.reduceat(v, pos)
    A = sp.csr_matrix((sums, (r[pos], c[pos])), shape=(n, n))
    A.sort_indices()
    return A


def assemble_stokes(N: int, nu=1.0) -> sp.csr_matrix:
    """Unconstrained saddle-point matrix [[L,0,Bx^T],[0,L,By^T],[Bx,By,0]].

    ``nu`` is a scalar or a per-element array (index ey*N + ex)."""
    g = grid_sizes(N)
    h = 1.0 / N
    E = element_matrices(h)
    q2, q1 = element_dof_maps(N)
    ne = N * N
    nu_e = np.broadcast_to(np.asarray(nu, dtype=np.float64), (ne,))
    ux = q2 + g.off_ux
    uy = q2 + g.off_uy
    pp = q1 + g.off_p
    blocks = []
    Lv = nu_e[:, None, None] * E["L"][None]
    for u in (ux, uy):
        blocks.append((np.broadcast_to(u[:, :, None], (ne, 9, 9)),
                       np.broadcast_to(u[:, None, :], (ne, 9, 9)), Lv))
    for u, Bk in ((ux, E["Bx"]), (uy, E["By"])):
        Bv = np.broadcast_to(Bk[None], (ne, 4, 9))
        r = np.broadcast_to(pp[:, :, None], (ne, 4, 9))
        c = np.broadcast_to(u[:, None, :], (ne, 4, 9))
        blocks.append((r, c, Bv))
        blocks.append((c, r, Bv))  # transpose block B^T
    rows = np.concatenate([np.ravel(b[0]) for b in blocks])
    cols = np.concatenate([np.ravel(b[1]) for b in blocks])
    vals = np.concatenate([np.ravel(b[2]) for b in blocks])
    return assemble_coo(rows, cols, vals, g.n)


def assemble_q2_mass(N: int) -> sp.csr_matrix:
    """Scalar Q2 mass matrix on the (2N+1)^2 nodes."""
    h = 1.0 / N
    E = element_matrices(h)
    q2, _ = element_dof_maps(N)
    ne = N * N
    r = np.broadcast_to(q2[:, :, None], (ne, 9, 9))
    c = np.broadcast_to(q2[:, None, :], (ne, 9, 9))
    v = np.broadcast_to(E["M"][None], (ne, 9, 9))
    return assemble_coo(r, c, v, (2 * N + 1) ** 2)


def pressure_weights(N: int) -> np.ndarray:
    """int phi_k over the domain for every Q1 node k (the row sums of the
    pressure mass matrix), assembled element by element."""
    E = element_matrices(1.0 / N)
    _, q1 = element_dof_maps(N)
    w = np.zeros((N + 1) ** 2)
    np.add.at(w, q1.ravel(), np.broadcast_to(E["wp"][None], q1.shape).ravel())
    return w


# ----------------------------------------------------------------------------
# Dirichlet elimination and right-hand sides
# ----------------------------------------------------------------------------

def apply_dirichlet(A_full: sp.csr_matrix, b_full: np.ndarray, g_full: np.ndarray,
                    dmask: np.ndarray):
    """Symmetric elimination of the Dirichlet set D (mask ``dmask``):
    b_F -= A_FD g_D, rows and columns of D zeroed, A_DD = I, b_D = g_D."""
    n = A_full.shape[0]
    gD = np.where(dmask, g_full, 0.0)
    b = b_full - A_full @ gD
    b[dmask] = g_full[dmask]
    keep = sp.diags((~dmask).astype(np.float64))
    A = (keep @ A_full @ keep).tocsr()
    A = A + sp.diags(dmask.astype(np.float64))
    A = A.tocsr()
    A.eliminate_zeros()
    A.sort_indices()
    assert A.shape == (n, n)
    return A, b


def rhs_from_nodal_force(N: int, f_nodal: np.ndarray) -> np.ndarray:
    """Velocity load b_u = M_Q2 f_h for f_h the Q2 interpolant of the nodal
    force (shape (2, (2N+1)^2)); pressure load 0.  Full vector layout."""
    g = grid_sizes(N)
    M = assemble_q2_mass(N)
    b = np.zeros(g.n)
    b[g.off_ux:g.off_ux + g.n_q2] = M @ f_nodal[0]
    b[g.off_uy:g.off_uy + g.n_q2] = M @ f_nodal[1]
    return b


def rhs_from_function(N: int, f, nu: float = 1.0, npts: int = 3) -> np.ndarray:
    """Velocity load b_u,i = int f . psi_i by npts x npts Gauss quadrature per
    element; ``f(x, y, nu)`` returns the two force components."""
    g = grid_sizes(N)
    h = 1.0 / N
    s, t, w = _element_quadrature(npts, h)
    val, _, _ = q2_basis_2d(s, t, h)
    q2, _ = element_dof_maps(N)
    e = np.arange(N)
    EX, EY = np.meshgrid(e, e, indexing="xy")
    X = (EX.ravel()[:, None] + s[None, :]) * h
    Y = (EY.ravel()[:, None] + t[None, :]) * h
    f1, f2 = f(X, Y, nu)
    b = np.zeros(g.n)
    for comp, fc in ((0, f1), (1, f2)):
        loc = (fc * w[None, :]) @ val.T  # (ne, 9)
        off = g.off_ux if comp == 0 else g.off_uy
        np.add.at(b, (q2 + off).ravel(), loc.ravel())
    return b


def lift_vector(N: int, g_nodal: np.ndarray) -> np.ndarray:
    """Full vector equal to the Dirichlet data on D and zero elsewhere."""
    gs = grid_sizes(N)
    x = np.zeros(gs.n)
    bm = q2_boundary_mask(N)
    x[gs.off_ux:gs.off_ux + gs.n_q2][bm] = g_nodal[0][bm]
    x[gs.off_uy:gs.off_uy + gs.n_q2][bm] = g_nodal[1][bm]
    return x


def stokes_system(N: int, nu=1.0, f_nodal=None, g_nodal=None, b_load=None):
    """Constrained system (A, b, dmask, x_lift) for nodal force ``f_nodal``
    (or a precomputed velocity load ``b_load``) and Dirichlet data
    ``g_nodal`` (both shape (2, (2N+1)^2); None means zero)."""
    gs = grid_sizes(N)
    A_full = assemble_stokes(N, nu)
    if b_load is None:
        b_load = (rhs_from_nodal_force(N, f_nodal) if f_nodal is not None
                  else np.zeros(gs.n))
    if g_nodal is None:
        g_nodal = np.zeros((2, gs.n_q2))
    dmask = velocity_dirichlet_mask(N)
    xl = lift_vector(N, g_nodal)
    A, b = apply_dirichlet(A_full, b_load, xl, dmask)
    return A, b, dmask, xl


# ----------------------------------------------------------------------------
# Rows of the constrained operator one by one (for sampled checks on meshes
# too large to assemble)
# ----------------------------------------------------------------------------

def residual_rows(N: int, x: np.ndarray, b: np.ndarray, rows, nu: float = 1.0) -> np.ndarray:
    """(b - A x)[rows] for the Dirichlet-eliminated operator, each row summed
    over the element matrices of the elements that contain its DoF (the
    definition of assembly); Dirichlet columns are dropped and Dirichlet rows
    are identity rows."""
    g = grid_sizes(N)
    h = 1.0 / N
    E = element_matrices(h)
    s2, s1 = g.q2_side, g.q1_side
    out = np.empty(len(rows))

    def q2_free(qi, qj):
        return 0 < qi < s2 - 1 and 0 < qj < s2 - 1

    for n_, row in enumerate(rows):
        row = int(row)
        acc = 0.0
        if row < g.off_p:
            f = row // g.n_q2
            node = row % g.n_q2
            qi, qj = node % s2, node // s2
            if not q2_free(qi, qj):
                out[n_] = b[row] - x[row]
                continue
            off = g.off_ux if f == 0 else g.off_uy
            Bk = E["Bx"] if f == 0 else E["By"]
            for ey in range((qj - 1) // 2, qj // 2 + 1):
                for ex in range((qi - 1) // 2, qi // 2 + 1):
                    if not (0 <= ex < N and 0 <= ey < N):
                        continue
                    li = (qj - 2 * ey) * 3 + (qi - 2 * ex)
                    for bb in range(3):
                        for aa in range(3):
                            cj, ci = 2 * ey + bb, 2 * ex + aa
                            if q2_free(ci, cj):
                                acc += nu * E["L"][li, bb * 3 + aa] * x[off + cj * s2 + ci]
                    for d in range(2):
                        for c in range(2):
                            acc += Bk[d * 2 + c, li] * x[g.off_p + (ey + d) * s1 + ex + c]
        else:
            node = row - g.off_p
            I, J = node % s1, node // s1
            for ey in (J - 1, J):
                for ex in (I - 1, I):
                    if not (0 <= ex < N and 0 <= ey < N):
                        continue
                    lk = (J - ey) * 2 + (I - ex)
                    for bb in range(3):
                        for aa in range(3):
                            cj, ci = 2 * ey + bb, 2 * ex + aa
                            if q2_free(ci, cj):
                                q = cj * s2 + ci
                                acc += E["Bx"][lk, bb * 3 + aa] * x[g.off_ux + q]
                                acc += E["By"][lk, bb * 3 + aa] * x[g.off_uy + q]
        out[n_] = b[row] - acc
    return out


# ----------------------------------------------------------------------------
# Null space and errors
# ----------------------------------------------------------------------------

def pressure_mean(N: int, x: np.ndarray) -> float:
    """Mass-weighted mean of the discrete pressure: int p_h / |Omega|."""
    gs = grid_sizes(N)
    w = pressure_weights(N)
    return float(w @ x[gs.off_p:]) / float(w.sum())


def normalise_pressure(N: int, x: np.ndarray) -> np.ndarray:
    gs = grid_sizes(N)
    y = np.array(x, dtype=np.float64, copy=True)
    y[gs.off_p:] -= pressure_mean(N, y)
    return y


def discretisation_errors(N: int, x: np.ndarray, name: str, npts: int = 5):
    """L2 and H1-seminorm velocity errors and L2 pressure error against the
    manufactured solution ``name`` by npts x npts Gauss quadrature per
    element; both pressures are reduced to zero mean first."""
    from stokes_inputs import MANUFACTURED
    sol = MANUFACTURED[name]
    gs = grid_sizes(N)
    h = 1.0 / N
    s, t, w = _element_quadrature(npts, h)
    val, dx, dy = q2_basis_2d(s, t, h)
    pv = q1_basis_2d(s, t)
    q2, q1 = element_dof_maps(N)
    e = np.arange(N)
    EX, EY = np.meshgrid(e, e, indexing="xy")
    X = (EX.ravel()[:, None] + s[None, :]) * h
    Y = (EY.ravel()[:, None] + t[None, :]) * h
    xn = normalise_pressure(N, x)
    ux = xn[gs.off_ux:gs.off_ux + gs.n_q2][q2]
    uy = xn[gs.off_uy:gs.off_uy + gs.n_q2][q2]
    pp = xn[gs.off_p:][q1]
    u1, u2 = sol.u(X, Y)
    g11, g12, g21, g22 = sol.grad_u(X, Y)
    pe = sol.p(X, Y)
    # exact pressure mean by the same quadrature
    pe_mean = float((pe * w[None, :]).sum())
    e_u = (ux @ val - u1) ** 2 + (uy @ val - u2) ** 2
    e_g = ((ux @ dx - g11) ** 2 + (ux @ dy - g12) ** 2
           + (uy @ dx - g21) ** 2 + (uy @ dy - g22) ** 2)
    e_p = (pp @ pv - (pe - pe_mean)) ** 2
    return (float(np.sqrt((e_u * w).sum())), float(np.sqrt((e_g * w).sum())),
            float(np.sqrt((e_p * w).sum())))
