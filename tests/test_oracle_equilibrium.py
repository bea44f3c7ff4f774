"""Pins of the equilibrium height density (oracle/equilibrium.py) used by the GPU
equilibrium check (App. B: equilibrium distribution of heights; Sec. II.A: the drift makes
exp(-U/kT) invariant)."""
import numpy as np
import pytest

from oracle import equilibrium as eq
from oracle import forces
from tests.conftest import golden_rows

KW = dict(a=1.0, u0=4.0, b=0.1, f_grav_z=-2.0, kT=1.0)


def test_density_is_normalised_and_positive():
    h = eq.grid(6.0, 2001)
    p = eq.boltzmann_density(h, **KW)
    assert np.all(p >= 0.0)
    assert np.trapezoid(p, h) == pytest.approx(1.0, rel=1e-12)
    c = eq.cdf(h, p)
    assert c[0] == 0.0 and c[-1] == pytest.approx(1.0) and np.all(np.diff(c) >= 0.0)


def test_log_density_slope_is_the_total_force():
    # kT d ln P / dh = -dU/dh must be the z force the dynamics feels: wall (d = a) plus
    # gravity, evaluated independently by oracle.forces on a lone sphere
    h = eq.grid(6.0, 60001)
    p = eq.boltzmann_density(h, **KW)
    for z in (1.05, 1.2, 1.5, 2.0, 3.0, 0.7):
        k = int(round(z / (h[1] - h[0])))
        slope = (np.log(p[k + 1]) - np.log(p[k - 1])) / (h[k + 1] - h[k - 1])
        f = forces.forces(np.array([[0.3, -0.2, h[k]]]), KW["a"], KW["u0"], KW["b"],
                          KW["f_grav_z"])[0, 2]
        assert slope * KW["kT"] == pytest.approx(f, rel=1e-6, abs=1e-6), z


def test_mzz_follows_the_wall_self_mobility_series_far_from_the_wall():
    # M_zz (6 pi eta a) = 1 - 9/8 eps + 1/2 eps^3 + O(eps^4), eps = a/h (golden fixture)
    coef = {int(o): int(n) / int(d) for dn, o, n, d in golden_rows("wall_self_mobility_series.txt")
            if dn == "perp"}
    eta = 0.7
    for hgt in (20.0, 40.0):
        eps = 1.0 / hgt
        series = sum(c * eps ** o for o, c in coef.items())
        m = eq.mzz(np.array([hgt]), 1.0, eta)[0] * 6.0 * np.pi * eta
        assert abs(m - series) <= 2.0 * eps ** 4


def test_the_check_separates_a_missing_drift():
    # the density left invariant without the drift differs visibly from P(h)
    h = eq.grid(6.0, 601)
    p = eq.boltzmann_density(h, **KW)
    q = eq.no_drift_density(h, eta=1.0 / (6.0 * np.pi), **KW)
    assert np.abs(eq.cdf(h, p) - eq.cdf(h, q)).max() > 0.08


def test_ks_distance_of_exact_samples_is_small():
    h = eq.grid(6.0, 6001)
    c = eq.cdf(h, eq.boltzmann_density(h, **KW))
    u = np.random.default_rng(0).uniform(size=40000)
    x = np.interp(u, c, h)                       # inverse-CDF samples
    assert eq.ks_distance(x, h, c) < 0.01
    assert eq.ks_distance(x + 0.1, h, c) > 0.05  # a shifted sample is caught
