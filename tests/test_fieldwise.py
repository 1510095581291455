"""CPU checks of the per-field comparison used by the GPU parity tests."""

import numpy as np

from fieldwise import field_slices, mesh_of, rel, rel2
from stokes_inputs import grid_sizes


def test_mesh_of_every_level_size():
    for N in (1, 2, 4, 8, 16, 40, 1024, 4096):
        assert mesh_of(grid_sizes(N).n) == N
    for bad in (0, 5, grid_sizes(16).n + 1):
        try:
            mesh_of(bad)
        except ValueError:
            continue
        raise AssertionError(bad)


def test_velocity_error_is_not_hidden_by_a_large_pressure():
    """A sweep-like vector: pressure 1e4 times the velocity.  A velocity-only
    error of 1e-10 relative to the velocity would read ~1e-14 under one max
    over all fields; per field it reads 1e-10."""
    N = 40
    g = grid_sizes(N)
    rng = np.random.default_rng(0)
    b = rng.uniform(-1, 1, g.n)
    b[g.off_p:] *= 2e4
    a = b.copy()
    a[g.off_ux + 7] += 1e-10 * np.abs(b[:g.off_uy]).max()
    whole = np.abs(a - b).max() / np.abs(b).max()
    assert whole < 1e-13
    assert abs(rel(a, b) - 1e-10) < 1e-12
    sl = field_slices(g.n)
    assert rel2(a, b) > 1e-12 and rel2(a, b) == np.linalg.norm((a - b)[sl[0]]) / np.linalg.norm(b[sl[0]])
    assert rel(b, b) == 0.0 and rel2(b, b) == 0.0
