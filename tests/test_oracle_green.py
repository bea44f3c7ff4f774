"""Pins of Blake's image tensor (oracle/green.py): no slip, Stokes equations, reciprocity."""
import sympy as sp
import pytest

from oracle import green

X = sp.symbols("x1:4", real=True)
Y = sp.symbols("y1:4", real=True)
PT = {X[0]: sp.Rational(3, 7), X[1]: sp.Rational(-2, 5), X[2]: sp.Rational(9, 5),
      Y[0]: sp.Rational(1, 3), Y[1]: sp.Rational(5, 4), Y[2]: sp.Rational(7, 3)}


@pytest.fixture(scope="module")
def G():
    return green.blake_total(X, Y)


@pytest.fixture(scope="module")
def Gimg():
    return green.blake_image(X, Y)


def test_no_slip_on_wall(G):
    for pt in ({X[0]: sp.Rational(3, 7), X[1]: sp.Rational(-2, 5), X[2]: 0,
                Y[0]: sp.Rational(1, 3), Y[1]: sp.Rational(5, 4), Y[2]: sp.Rational(7, 3)},
               {X[0]: 5, X[1]: 1, X[2]: 0, Y[0]: -2, Y[1]: 3, Y[2]: sp.Rational(1, 9)}):
        vals = G.subs(pt)
        assert all(sp.simplify(v) == 0 for v in vals)


def test_incompressible(G):
    for j in range(3):
        div = sum(sp.diff(G[i, j], X[i]) for i in range(3))
        assert sp.simplify(div.subs(PT)) == 0


def test_stokes_momentum(Gimg):
    # lap u = grad p for some p  <=>  curl(lap u) = 0 for every column of the regular part
    for j in range(3):
        L = [sum(sp.diff(Gimg[i, j], v, 2) for v in X) for i in range(3)]
        curl = [sp.diff(L[2], X[1]) - sp.diff(L[1], X[2]),
                sp.diff(L[0], X[2]) - sp.diff(L[2], X[0]),
                sp.diff(L[1], X[0]) - sp.diff(L[0], X[1])]
        assert all(sp.simplify(c.subs(PT)) == 0 for c in curl)


def test_reciprocity(Gimg):
    swap = {X[0]: Y[0], X[1]: Y[1], X[2]: Y[2], Y[0]: X[0], Y[1]: X[1], Y[2]: X[2]}
    for i in range(3):
        for j in range(3):
            d = Gimg[i, j] - Gimg[j, i].xreplace(swap)
            assert sp.simplify(d.subs(PT)) == 0


def test_image_part_decays_and_is_opposite_oseen_far_from_wall(Gimg):
    # far above the wall the image part is small compared with the Oseen part
    pt = {X[0]: 0, X[1]: 0, X[2]: 1000, Y[0]: 1, Y[1]: 0, Y[2]: 1000}
    val = float(sp.Abs(Gimg[0, 0].subs(pt)))
    assert val < 1e-3
