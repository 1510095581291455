"""Field-by-field comparison of vectors in the [u_x | u_y | p] layout.

After a Vanka sweep, a V-cycle or a solve the pressure block can be about
1/h^2 larger than the velocity blocks (at N = 40 a sweep leaves |p| ~ 2e4
against |u| ~ 8), so one relative error over the whole vector would test the
velocity only to ~1e-9 when the bound reads 1e-12.  These helpers measure
each field against its own magnitude and report the worst field.
"""

from __future__ import annotations

import math

import numpy as np


def mesh_of(n: int) -> int:
    """N such that 2 (2N+1)^2 + (N+1)^2 == n (a level vector's length)."""
    # 9 N^2 + 10 N + 3 = n
    N = int(round((-10 + math.sqrt(100 - 36 * (3 - n))) / 18))
    for M in (N - 1, N, N + 1):
        if M >= 1 and 2 * (2 * M + 1) ** 2 + (M + 1) ** 2 == n:
            return M
    raise ValueError(f"{n} is not the length of a Q2-Q1 level vector")


def field_slices(n: int):
    N = mesh_of(n)
    nq2 = (2 * N + 1) ** 2
    return (slice(0, nq2), slice(nq2, 2 * nq2), slice(2 * nq2, n))


def rel(a, b) -> float:
    """Worst over the fields of max|a_f - b_f| / max|b_f| (0 for a field
    that is zero in both)."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    assert a.shape == b.shape, (a.shape, b.shape)
    worst = 0.0
    for sl in field_slices(b.size):
        d = np.abs(a[sl] - b[sl]).max()
        if d == 0.0:
            continue
        worst = max(worst, d / max(np.abs(b[sl]).max(), 1e-300))
    return worst


def rel2(a, b) -> float:
    """Worst over the fields of ||a_f - b_f||_2 / ||b_f||_2."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    assert a.shape == b.shape, (a.shape, b.shape)
    worst = 0.0
    for sl in field_slices(b.size):
        d = np.linalg.norm(a[sl] - b[sl])
        if d == 0.0:
            continue
        worst = max(worst, d / max(np.linalg.norm(b[sl]), 1e-300))
    return worst
