"""Pins of the soft steric forces (oracle/forces.py)."""
import numpy as np

from oracle import forces
from tests.conftest import golden_rows


def test_paper_wall_energy_example():
    (u0, b, expect), = golden_rows("steric_wall_energy.txt")
    assert abs(float(forces.potential(0.0, 1.0, float(u0), float(b))) - float(expect)) < 1e-12


def test_continuity_and_force_is_minus_gradient():
    for d in (1.0, 2.0):
        for u0, b in ((1.0, 0.1), (4.0, 0.3)):
            e = 1e-12
            assert abs(forces.potential(d - e, d, u0, b) - forces.potential(d + e, d, u0, b)) < 1e-9
            assert abs(forces.force_magnitude(d - e, d, u0, b) - forces.force_magnitude(d + e, d, u0, b)) < 1e-9
            for r in (0.3 * d, 0.9 * d, d + 0.05, d + 0.4):
                h = 1e-6
                fd = -(forces.potential(r + h, d, u0, b) - forces.potential(r - h, d, u0, b)) / (2 * h)
                assert abs(fd - forces.force_magnitude(r, d, u0, b)) < 1e-6 * max(1.0, u0 / b)


def test_pair_forces_balance_and_point_apart():
    rng = np.random.default_rng(4)
    pos = np.column_stack([rng.uniform(0, 4, 12), rng.uniform(0, 4, 12), rng.uniform(1.0, 2.0, 12)])
    f = forces.forces(pos, 1.0, 1.0, 0.1, f_grav_z=0.0)
    wall = forces.force_magnitude(pos[:, 2], 1.0, 1.0, 0.1)
    internal = f.copy()
    internal[:, 2] -= wall
    assert np.abs(internal.sum(0)).max() < 1e-10 * np.abs(internal).max()
    two = forces.forces(np.array([[0.0, 0.0, 5.0], [1.9, 0.0, 5.0]]), 1.0, 1.0, 0.1, 0.0)
    assert two[0, 0] < 0 and two[1, 0] > 0 and abs(two[0, 0] - (-10.0)) < 1e-12
    rows = forces.forces(pos, 1.0, 1.0, 0.1, -1.0, rows=np.array([3, 7]))
    full = forces.forces(pos, 1.0, 1.0, 0.1, -1.0)
    assert np.allclose(rows, full[[3, 7]], rtol=0, atol=1e-15)
