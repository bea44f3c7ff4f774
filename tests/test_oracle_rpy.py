"""Pins of the unbounded RPY tensors (oracle/rpy.py)."""
import numpy as np
import pytest
import sympy as sp

from oracle import rpy
from tests.quadrature import double_average, oseen

A = 1.0


def _dirs():
    return [np.array([0.6, 0.8, 0.0]), np.array([0.3, -0.4, np.sqrt(0.75)])]


@pytest.mark.parametrize("dist", [2.5, 4.0])
def test_far_tt_is_surface_average_of_oseen(dist):
    for d in _dirs():
        qj = dist * d
        ref = double_average(oseen, np.zeros(3), qj, A, 32)
        got = rpy.free_tt((np.zeros(3) - qj)[:, None], A)[:, :, 0]
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("dist", [0.7, 1.3, 1.8])
def test_overlap_tt_is_surface_average_of_oseen(dist):
    # singular integrand on the intersection circle: product rule error ~1e-3 at nt = 32,
    # Richardson step with nt = 16 brings it to ~1e-4
    d = _dirs()[1]
    qj = dist * d
    q32 = double_average(oseen, np.zeros(3), qj, A, 32)
    q16 = double_average(oseen, np.zeros(3), qj, A, 16)
    ref = q32 + (q32 - q16) / 7.0
    got = rpy.free_tt((np.zeros(3) - qj)[:, None], A)[:, :, 0]
    assert np.abs(got - ref).max() <= 1e-3 * np.abs(ref).max()


@pytest.mark.parametrize("dist", [0.7, 1.5, 3.0])
def test_tr_is_surface_average_of_torque_traction(dist):
    d = _dirs()[1]
    qj = dist * d
    q32 = double_average(oseen, np.zeros(3), qj, A, 32, torque=True)
    q16 = double_average(oseen, np.zeros(3), qj, A, 16, torque=True)
    ref = q32 + (q32 - q16) / 7.0
    got = rpy.free_tr((np.zeros(3) - qj)[:, None], A)[:, :, 0]
    assert np.abs(got - ref).max() <= 1e-3 * np.abs(ref).max()


def test_far_form_is_faxen_on_oseen():
    r = sp.symbols("r1:4", real=True)
    a = sp.Symbol("a", positive=True)
    rv = sp.Matrix(r)
    rn = sp.sqrt(rv.dot(rv))
    S = sp.eye(3) / rn + rv * rv.T / rn ** 3
    fax = S.applyfunc(lambda e: e + a ** 2 / 3 * sum(sp.diff(e, v, 2) for v in r))
    far = rpy.symbolic_free_tt("far")
    far = far.subs(sp.Symbol("a", positive=True), a)
    pt = {r[0]: sp.Rational(5, 3), r[1]: sp.Rational(-7, 4), r[2]: sp.Rational(2, 5), a: sp.Rational(3, 4)}
    assert all(sp.simplify((fax[i] - far[i]).subs(pt)) == 0 for i in range(9))


def test_continuity_at_contact_and_self_value():
    for d in _dirs():
        lo = rpy.free_tt(((2 * A - 1e-12) * d)[:, None], A)[:, :, 0]
        hi = rpy.free_tt(((2 * A + 1e-12) * d)[:, None], A)[:, :, 0]
        assert np.abs(lo - hi).max() < 1e-10
        lo = rpy.free_tr(((2 * A - 1e-12) * d)[:, None], A)[:, :, 0]
        hi = rpy.free_tr(((2 * A + 1e-12) * d)[:, None], A)[:, :, 0]
        assert np.abs(lo - hi).max() < 1e-10
    # r = 0: Stokes drag 1/(6 pi eta a) (times 8 pi eta) and no rotation coupling
    z = np.zeros((3, 1))
    assert np.allclose(rpy.free_tt(z, A)[:, :, 0], 4.0 / (3.0 * A) * np.eye(3), rtol=0, atol=1e-15)
    assert np.all(rpy.free_tr(z, A) == 0.0)


def test_rotlet_direction():
    # a torque about +z at the origin turns the fluid counter-clockwise: +y velocity at +x
    r = np.array([[5.0], [0.0], [0.0]])
    u = rpy.free_tr(r, A)[:, :, 0] @ np.array([0.0, 0.0, 1.0])
    assert u[1] > 0 and abs(u[0]) < 1e-15 and abs(u[2]) < 1e-15


@pytest.mark.parametrize("dist", [0.9, 3.0])
def test_divergence_free(dist):
    rng = np.random.default_rng(3)
    y0 = dist * _dirs()[1]
    dy = rpy.free_tt_dy((np.zeros(3) - y0)[:, None], A)[:, :, 0]
    assert np.abs(dy.sum(axis=1)).max() < 1e-13
    # and the symbolic derivative agrees with central differences
    h = 1e-5
    for b in range(3):
        e = np.zeros(3)
        e[b] = h
        fp = rpy.free_tt((np.zeros(3) - (y0 + e))[:, None], A)[:, b, 0]
        fm = rpy.free_tt((np.zeros(3) - (y0 - e))[:, None], A)[:, b, 0]
        assert np.allclose((fp - fm) / (2 * h), dy[:, b], atol=1e-8)
