"""Input recipes: the seeded generators shared by the oracle tests, the GPU tests and the bench."""
import numpy as np
from scipy.spatial import cKDTree

from paper_1612_00474_amd import workloads as wl


def test_sheet_recipe():
    pos = wl.sheet(3000, seed=2)
    side = wl.side_for_area_fraction(3000, wl.PHI)
    assert pos.shape == (3000, 3)
    assert np.all((pos[:, :2] >= 0) & (pos[:, :2] < side))
    assert np.all((pos[:, 2] >= 1.1) & (pos[:, 2] <= 2.5))
    assert np.array_equal(pos, wl.sheet(3000, seed=2))


def test_sedimented_sheet_recipe():
    # area fraction 0.25, exponential height profile of mean ~1.6a above 1.1a, no overlaps
    n = 4000
    pos = wl.sedimented_sheet(n, seed=3)
    side = wl.side_for_area_fraction(n, 0.25)
    assert np.all((pos[:, :2] >= 0) & (pos[:, :2] < side))
    assert pos[:, 2].min() >= 1.1
    assert 1.55 <= pos[:, 2].mean() <= 1.75
    d, _ = cKDTree(pos).query(pos, k=2)
    assert d[:, 1].min() >= 2.0
    assert np.array_equal(pos, wl.sedimented_sheet(n, seed=3))
    assert not np.array_equal(pos, wl.sedimented_sheet(n, seed=4))
