"""Stokes Green's function above a no-slip plane wall (symbolic, sympy).

Test infrastructure only (see ``oracle/__init__``).

Sec. II.B of the paper uses Blake's method-of-images solution for a point force
in the half space z > 0 bounded by a no-slip wall at z = 0.  For a point force
at y = (y1, y2, h) the velocity at x is u_i(x) = G_ij(x, y) F_j with

    8 pi eta G = S(r) + G_img,     r = x - y,
    S(r)_ij    = delta_ij / |r| + r_i r_j / |r|^3          (Oseen tensor)

and, writing R = x - (y1, y2, -h) for the separation from the image point and
D = diag(1, 1, -1),

    G_img_ij = - S(R)_ij
               + 2 h D_jj d/dR_j [ h R_i / |R|^3 - S(R)_i3 ]      (no sum over j).

The first term is an image Stokeslet of opposite sign; the bracket holds the
image Stokes doublet (S(R)_i3 column) and the source doublet (h R_i/|R|^3).

Pinned by (tests/test_oracle_green.py): the total G vanishes on z = 0
(no slip); each column is divergence free in x and the curl of its Laplacian
vanishes (Stokes equations with a pressure); reciprocity
G_ij(x, y) = G_ji(y, x); the image part is regular in the fluid.  A tensor with
the Oseen singularity, satisfying the Stokes equations, vanishing on the wall
and decaying at infinity is unique, so these checks fix G.
"""
from __future__ import annotations

import sympy as sp


def oseen(rvec: sp.Matrix) -> sp.Matrix:
    """8 pi eta times the Oseen tensor for separation ``rvec``."""
    rn = sp.sqrt(rvec.dot(rvec))
    return sp.eye(3) / rn + rvec * rvec.T / rn ** 3


def image_vector(x, y) -> sp.Matrix:
    """R = x - y_img, with y_img = (y1, y2, -y3) the mirror image of y in z = 0."""
    return sp.Matrix([x[0] - y[0], x[1] - y[1], x[2] + y[2]])


def blake_image(x, y) -> sp.Matrix:
    """8 pi eta times the image part of Blake's tensor; entry [i, j] = velocity i from force j.

    ``x`` (field point) and ``y`` (source point) are sequences of three sympy symbols.
    The derivative d/dR_j is taken as d/dx_j, since R depends on x only through x - y_img.
    """
    h = y[2]
    R = image_vector(x, y)
    Rn = sp.sqrt(R.dot(R))
    S = oseen(R)
    D = (1, 1, -1)
    G = sp.zeros(3, 3)
    for i in range(3):
        bracket = h * R[i] / Rn ** 3 - S[i, 2]
        for j in range(3):
            G[i, j] = -S[i, j] + 2 * h * D[j] * sp.diff(bracket, x[j])
    return G


def blake_total(x, y) -> sp.Matrix:
    """8 pi eta times Blake's full tensor (Oseen part plus image part)."""
    r = sp.Matrix([x[0] - y[0], x[1] - y[1], x[2] - y[2]])
    return oseen(r) + blake_image(x, y)
