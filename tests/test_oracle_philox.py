"""Pins of the counter-based generator (oracle/philox.py)."""
import numpy as np
import scipy.stats

from oracle import philox
from tests.conftest import golden_rows


def test_known_answer_vector():
    for row in golden_rows("philox4x64_10_kat.txt"):
        ctr = [int(v) for v in row[:4]]
        key = [int(v) for v in row[4:6]]
        out = philox.philox4x64(np.array([ctr], dtype=np.uint64), np.array(key, dtype=np.uint64))[0]
        assert [int(v) for v in out] == [int(v, 16) for v in row[6:10]]


def test_matches_numpy_philox():
    rng = np.random.default_rng(0)
    for _ in range(20):
        key = rng.integers(0, 2 ** 63, size=2, dtype=np.uint64)
        ctr = rng.integers(0, 2 ** 63, size=4, dtype=np.uint64)
        ctr[0] = ctr[0] % np.uint64(2 ** 40) + np.uint64(1)
        # numpy's generator advances its counter by one before producing a block
        bg = np.random.Philox(key=key, counter=ctr - np.array([1, 0, 0, 0], dtype=np.uint64))
        ref = bg.random_raw(4 * 5).reshape(5, 4)
        ctrs = np.tile(ctr, (5, 1))
        ctrs[:, 0] += np.arange(5, dtype=np.uint64)
        got = philox.philox4x64(ctrs, key)
        assert np.array_equal(got, ref)


def test_normals_distribution_and_layout():
    x = philox.normals(200003, seed=12345, stream=0, step=7)
    assert x.shape == (200003,)
    assert scipy.stats.kstest(x, "norm").pvalue > 1e-3
    y = philox.normals(200003, seed=12345, stream=1, step=7)
    assert abs(np.corrcoef(x, y)[0, 1]) < 0.01
    # prefix property: a shorter draw is a prefix of a longer one
    assert np.array_equal(philox.normals(10, 5, 0, 3), philox.normals(1000, 5, 0, 3)[:10])
    u = philox.uniforms(np.array([0, 2 ** 64 - 1], dtype=np.uint64))
    assert 0.0 < u[0] < 1e-15 and 1.0 - 1e-15 < u[1] < 1.0
