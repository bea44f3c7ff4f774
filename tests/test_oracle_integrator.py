"""Pins of the time integrators (oracle/integrator.py): deterministic orders of accuracy."""
import math

import numpy as np
import pytest
import scipy.integrate

from oracle import forces, integrator, mobility

A = 1.0
PHYS = dict(f_grav_z=-1.0, torque=(0.0, 1.0, 0.0), u0=1.0, b=0.1)


def _velocity(q):
    pos = q.reshape(-1, 3)
    F = forces.forces(pos, A, PHYS["u0"], PHYS["b"], PHYS["f_grav_z"])
    T = np.tile(np.array(PHYS["torque"]), (len(pos), 1))
    return mobility.dense_matvec(pos, F, T, A).ravel()


@pytest.fixture(scope="module")
def reference():
    q0 = np.array([[0.0, 0.0, 1.6], [2.5, 0.3, 2.0]])
    t_end = 0.8
    sol = scipy.integrate.solve_ivp(lambda t, q: _velocity(q), (0.0, t_end), q0.ravel(),
                                    method="DOP853", rtol=1e-12, atol=1e-13)
    return q0, t_end, sol.y[:, -1].reshape(-1, 3)


def _run(q0, t_end, nsteps, scheme):
    dt = t_end / nsteps
    q = q0.copy()
    u_prev = None
    zero = np.zeros_like(q0)
    for _ in range(nsteps):
        q, u_prev, *_ = integrator.step(q, u_prev, zero, zero, dt=dt, delta=1e-4, lanczos_tol=1e-8,
                                        scheme=scheme, kT=0.0, a=A, **PHYS)
    return q


@pytest.mark.parametrize("scheme,order", [("sab", 2.0), ("em", 1.0)])
def test_deterministic_order(reference, scheme, order):
    q0, t_end, qref = reference
    errs = [np.abs(_run(q0, t_end, n, scheme) - qref).max() for n in (8, 16, 32)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - order) < 0.25), (errs, rates)


# ---- stochastic terms at kT > 0 (eqs. EM and AB): one sphere above the wall, no force ------

def _mu(h):
    """Wall self-mobilities of one sphere, parallel and perpendicular (Faxen; Lorentz/Brenner
    to O((a/h)^5)), written out from the textbook series, not from the oracle."""
    mu_par = 1 - 9 / (16 * h) + 1 / (8 * h ** 3) - 1 / (16 * h ** 5)
    mu_perp = 1 - 9 / (8 * h) + 1 / (2 * h ** 3) - 1 / (8 * h ** 5)
    return mu_par, mu_perp


def _dmu_perp_dh(h):
    return 9 / (8 * h ** 2) - 3 / (2 * h ** 4) + 5 / (8 * h ** 6)


LONE = dict(f_grav_z=0.0, torque=(0.0, 0.0, 0.0), u0=0.0, b=0.1)


@pytest.mark.parametrize("scheme", ["sab", "em"])
@pytest.mark.parametrize("kT,dt,a,eta", [(1.0, 0.01, 1.0, 1.0), (2.5, 0.004, 0.8, 1.3)])
def test_noise_term_of_a_lone_sphere(scheme, kT, dt, a, eta):
    z = 1.9 * a
    q = np.array([[0.4, -0.2, z]])
    W = np.array([[0.7, -1.3, 0.45]])
    u_prev = np.zeros((1, 3)) if scheme == "sab" else None
    new, u, *_ = integrator.step(q, u_prev, W, np.zeros((1, 3)), dt=dt, delta=1e-4,
                                 lanczos_tol=1e-12, scheme=scheme, kT=kT, a=a, eta=eta, **LONE)
    mu_par, mu_perp = _mu(z / a)
    expect = (np.sqrt(2 * kT * dt) * np.sqrt(np.array([mu_par, mu_par, mu_perp]))
              * W[0] / np.sqrt(6 * math.pi * eta * a))
    assert np.abs(u).max() == 0.0
    assert np.abs((new - q)[0] - expect).max() <= 1e-13 * np.abs(expect).max()


@pytest.mark.parametrize("scheme", ["sab", "em"])
@pytest.mark.parametrize("kT,dt,a,eta", [(1.0, 0.01, 1.0, 1.0), (2.5, 0.004, 0.8, 1.3)])
def test_drift_term_of_a_lone_sphere(scheme, kT, dt, a, eta):
    z = 1.6 * a
    q = np.array([[0.4, -0.2, z]])
    u_prev = np.zeros((1, 3)) if scheme == "sab" else None
    zhat = np.array([[0.0, 0.0, 1.0]])
    new, *_ = integrator.step(q, u_prev, np.zeros((1, 3)), zhat, dt=dt, delta=1e-4,
                              lanczos_tol=1e-12, scheme=scheme, kT=kT, a=a, eta=eta, **LONE)
    # d/dz [mu_perp(z/a) / (6 pi eta a)] = mu_perp'(h) / (6 pi eta a^2)
    expect = dt * kT * _dmu_perp_dh(z / a) / (6 * math.pi * eta * a * a)
    disp = (new - q)[0]
    assert disp[0] == 0.0 and disp[1] == 0.0
    # centred difference: O(delta^2) truncation, O(eps/delta) rounding
    assert abs(disp[2] - expect) <= 1e-8 * abs(expect)


def test_stochastic_terms_add():
    q = np.array([[0.1, 0.3, 1.4]])
    W = np.array([[0.2, 0.9, -0.6]])
    zhat = np.array([[0.0, 0.0, 1.0]])
    kw = dict(dt=0.01, delta=1e-4, lanczos_tol=1e-12, kT=1.7, **LONE)
    both = integrator.step(q, None, W, zhat, **kw)[0] - q
    noise = integrator.step(q, None, W, np.zeros((1, 3)), **kw)[0] - q
    drift = integrator.step(q, None, np.zeros((1, 3)), zhat, **kw)[0] - q
    assert np.abs(both - (noise + drift)).max() <= 1e-15
