"""Pins of the time integrators (oracle/integrator.py): deterministic orders of accuracy."""
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
