"""Equilibrium height distribution of one sphere above the wall.

Test infrastructure only (see ``oracle/__init__``).

The integrators of Sec. II.A (eqs. EM, AB with the random finite difference for the drift
kT div M) are built to leave the Gibbs-Boltzmann distribution exp(-U/kT) invariant; App. B
checks the equilibrium distribution of heights.  For one sphere with the wall part of the soft
potential (Sec. III, eq. soft_potential: d = a, r = h) and gravity f_g along z, the height is
distributed as

    P(h) = exp(-(U_wall(h) - f_g h)/kT) / Z.

Without the drift term the same dynamics (Ito, height-dependent mobility M_zz(h)) would instead
leave P(h) M_zz(h)^-1 / Z' invariant: the zero-flux condition of its Fokker-Planck equation,
M F p = kT d(M p)/dh, gives M p ~ exp(-U/kT).  The tests use this second density to show that
the check can tell a missing drift from a correct one.

Both densities are tabulated on a uniform grid of heights and normalised with the trapezoidal
rule; CDFs are cumulative trapezoidal sums.

Pinned by (tests/test_oracle_equilibrium.py): kT d ln P/dh equals the total z force of
``oracle.forces`` on a lone sphere; P integrates to one; M_zz matches the wall self-mobility
series of the golden fixture far from the wall.
"""
from __future__ import annotations

import numpy as np

from . import forces, mobility


def height_potential(h, a=1.0, u0=1.0, b=0.1, f_grav_z=-1.0):
    """U_wall(h) - f_g h (soft wall of eq. soft_potential with d = a, plus gravity)."""
    h = np.asarray(h, dtype=np.float64)
    return forces.potential(h, a, u0, b) - f_grav_z * h


def grid(h_max=4.0, n=4001):
    return np.linspace(0.0, h_max, n)


def _normalise(h, p):
    return p / np.trapezoid(p, h)


def boltzmann_density(h, a=1.0, u0=1.0, b=0.1, f_grav_z=-1.0, kT=1.0):
    """P(h) on the grid ``h`` (normalised over it)."""
    e = height_potential(h, a, u0, b, f_grav_z) / kT
    return _normalise(h, np.exp(-(e - e.min())))


def mzz(h, a=1.0, eta=1.0):
    """M_zz of a lone sphere at height h (regularised mobility, App. A)."""
    out = np.empty(len(h))
    for k, z in enumerate(h):
        M, _ = mobility.dense(np.array([[0.0, 0.0, z]]), a, eta)
        out[k] = M[2, 2]
    return out


def no_drift_density(h, a=1.0, u0=1.0, b=0.1, f_grav_z=-1.0, kT=1.0, eta=1.0):
    """The invariant density of the same dynamics without kT div M (h > 0 only)."""
    p = boltzmann_density(h, a, u0, b, f_grav_z, kT)
    m = mzz(h, a, eta)
    q = np.where(m > 0.0, p / np.where(m > 0.0, m, 1.0), 0.0)
    return _normalise(h, q)


def cdf(h, p):
    """Cumulative trapezoidal integral of the density p on the grid h."""
    c = np.concatenate([[0.0], np.cumsum(0.5 * (p[1:] + p[:-1]) * np.diff(h))])
    return c / c[-1]


def ks_distance(samples, h, c):
    """sup |F_empirical - F| for samples against the tabulated CDF c on grid h."""
    x = np.sort(np.asarray(samples, dtype=np.float64))
    n = x.size
    f = np.interp(x, h, c)
    hi = np.arange(1, n + 1) / n - f
    lo = f - np.arange(0, n) / n
    return float(max(hi.max(), lo.max()))
