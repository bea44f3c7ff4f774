"""Pins of the random finite difference and the divergence of M (oracle/stochastic.py)."""
import math

import numpy as np
import pytest

from oracle import mobility, stochastic

A = 1.0


@pytest.mark.parametrize("z", [1.2, 1.7, 3.5])
def test_single_sphere_divergence_above_a(z):
    h = z / A
    expect = (9 / (8 * h ** 2) - 3 / (2 * h ** 4) + 5 / (8 * h ** 6)) / (6 * math.pi * A ** 2)
    d = stochastic.divergence(np.array([[0.2, -0.4, z]]), A, 1.0)
    assert abs(d[0, 2] - expect) <= 1e-14 * abs(expect)
    assert d[0, 0] == 0.0 and d[0, 1] == 0.0


@pytest.mark.parametrize("z", [0.3, 0.8])
def test_single_sphere_divergence_below_a(z):
    # M_zz = H0(z/a)^2 mu_perp(1)/(6 pi eta a), mu_perp(1) = 1/4
    expect = (2 * z / A ** 2) * 0.25 / (6 * math.pi * A)
    d = stochastic.divergence(np.array([[0.0, 0.0, z]]), A, 1.0)
    assert abs(d[0, 2] - expect) <= 1e-14 * expect


def _config():
    # overlapping pairs, a sphere below z = a, none within 1e-3 of a kink (z = 0, z = a)
    return np.array([[0.0, 0.0, 1.3], [1.5, 0.4, 1.9], [0.8, -1.1, 0.6],
                     [3.5, 1.0, 2.4], [2.6, -0.5, 1.05]])


def test_central_differences_over_all_directions_match_divergence():
    pos = _config()
    n = len(pos)
    delta = 1e-5
    acc = np.zeros(3 * n)
    for k in range(3 * n):
        e = np.zeros(3 * n)
        e[k] = 1.0
        up = mobility.dense_matvec(pos + 0.5 * delta * e.reshape(n, 3), e.reshape(n, 3), None, A)
        um = mobility.dense_matvec(pos - 0.5 * delta * e.reshape(n, 3), e.reshape(n, 3), None, A)
        acc += ((up - um) / delta).ravel()
    d = stochastic.divergence(pos, A, 1.0).ravel()
    assert np.abs(acc - d).max() <= 1e-7 * np.abs(d).max()


def test_rfd_mean_matches_divergence():
    pos = _config()[:3]
    rng = np.random.default_rng(9)
    K = 1200
    samples = np.array([stochastic.rfd(pos, rng.standard_normal(pos.shape), 1e-4, A).ravel()
                        for _ in range(K)])
    mean = samples.mean(0)
    se = samples.std(0) / math.sqrt(K)
    d = stochastic.divergence(pos, A, 1.0).ravel()
    assert np.all(np.abs(mean - d) <= 4.5 * se + 1e-12)


def test_one_sided_rfd_mean_matches_divergence():
    # one-sided difference: unbiased up to O(delta) (Sec. II.A)
    pos = _config()[:3]
    rng = np.random.default_rng(10)
    K = 1200
    samples = np.array([stochastic.rfd_one_sided(pos, rng.standard_normal(pos.shape), 1e-4,
                                                 A).ravel() for _ in range(K)])
    mean = samples.mean(0)
    se = samples.std(0) / math.sqrt(K)
    d = stochastic.divergence(pos, A, 1.0).ravel()
    assert np.all(np.abs(mean - d) <= 4.5 * se + 1e-3 * np.abs(d).max())


def test_one_sided_and_centred_rfd_agree_to_first_order_in_delta():
    # (kT/delta)[M(q+delta w)w - M(q)w] - centred = (delta/2) w.grad(M w) + O(delta^2): halving
    # delta halves the gap
    pos = _config()[:5]
    wt = np.random.default_rng(4).standard_normal(pos.shape)
    gap = [np.linalg.norm(stochastic.rfd_one_sided(pos, wt, d, A) - stochastic.rfd(pos, wt, d, A))
           for d in (2e-3, 1e-3)]
    assert gap[1] == pytest.approx(gap[0] / 2, rel=0.02)


def test_rfd_scales_with_kT():
    pos = _config()
    wt = np.random.default_rng(1).standard_normal(pos.shape)
    d1 = stochastic.rfd(pos, wt, 1e-4, A, 1.0, 1.0)
    d2 = stochastic.rfd(pos, wt, 1e-4, A, 1.0, 2.5)
    assert np.allclose(d2, 2.5 * d1, rtol=1e-14, atol=0)


def test_free_space_rfd_mean_vanishes():
    # the unbounded RPY tensor is divergence-free (both branches), so the drift has mean zero
    pos = _config()[:3]
    rng = np.random.default_rng(12)
    K = 800
    samples = np.array([stochastic.rfd(pos, rng.standard_normal(pos.shape), 1e-4, A,
                                       wall=False).ravel() for _ in range(K)])
    se = samples.std(0) / math.sqrt(K)
    assert np.all(np.abs(samples.mean(0)) <= 4.5 * se + 1e-12)
