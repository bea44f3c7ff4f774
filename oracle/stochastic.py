"""Stochastic drift: centred random finite difference and the divergence it estimates.

Test infrastructure only (see ``oracle/__init__``).

Sec. II.A of the paper, last term of eq. EM / eq. AB: with W~ a vector of
i.i.d. standard normals, the centred random finite difference

    D = (kT / delta) [ M(q + delta/2 W~) W~ - M(q - delta/2 W~) W~ ]

equals kT (div_q . M)(q) in expectation up to O(delta^2).  Only the
translation-translation mobility M enters (eq. BD); M_C does not.

``divergence`` evaluates (div . M)_{i alpha} = sum_j sum_beta dM_{i alpha, j beta}/dq_{j beta}
exactly: M_ij = H(z_i) H(z_j) M~(q~_i, q~_j) (App. A, eq. effMob), so the chain rule
brings in H'(z) = 1/a on 0 < z < a and kills the z derivative of M~ where the
height is clamped (z < a).  For j = i the block depends on q_i through both
arguments; its total z derivative is used.

Pinned by (tests/test_oracle_stochastic.py): for one sphere above a the
divergence is z-hat times d/dz of the perpendicular self-mobility
(1/(6 pi eta a^2))(9/(8h^2) - 3/(2h^4) + 5/(8h^6)), h = z/a, and for 0 < z < a it
is z-hat (2z/a^2)(1/4)/(6 pi eta a); the deterministic central difference
summed over all 3N unit directions matches ``divergence`` to O(delta^2); the
sample mean of the RFD (centred and one-sided) over many W~ matches it within its standard
error.
"""
from __future__ import annotations

import math

import numpy as np

from . import faxen, mobility, rpy


def rfd(pos, w_tilde, delta, a=1.0, eta=1.0, kT=1.0, rows=None, workers=1, wall=True,
        box=None):
    """Centred random finite difference (kT/delta)[M(q+)W~ - M(q-)W~], shape (n, 3)."""
    pos = np.asarray(pos, dtype=np.float64)
    wt = np.asarray(w_tilde, dtype=np.float64).reshape(pos.shape)
    qp = pos + 0.5 * delta * wt
    qm = pos - 0.5 * delta * wt
    up = mobility.matvec(qp, wt, None, a, eta, rows=rows, workers=workers, wall=wall, box=box)
    um = mobility.matvec(qm, wt, None, a, eta, rows=rows, workers=workers, wall=wall, box=box)
    return (kT / delta) * (up - um)


def rfd_one_sided(pos, w_tilde, delta, a=1.0, eta=1.0, kT=1.0, rows=None, workers=1,
                  wall=True, box=None):
    """One-sided random finite difference (kT/delta)[M(q + delta W~)W~ - M(q)W~], shape (n, 3).

    Sec. II.A allows a one-sided difference in place of the centred one; it equals
    kT (div . M) in expectation up to O(delta)."""
    pos = np.asarray(pos, dtype=np.float64)
    wt = np.asarray(w_tilde, dtype=np.float64).reshape(pos.shape)
    up = mobility.matvec(pos + delta * wt, wt, None, a, eta, rows=rows, workers=workers,
                         wall=wall, box=box)
    u0 = mobility.matvec(pos, wt, None, a, eta, rows=rows, workers=workers, wall=wall, box=box)
    return (kT / delta) * (up - u0)


def divergence(pos, a=1.0, eta=1.0):
    """Exact (div_q . M)(q), shape (n, 3) (App. A regularisation included)."""
    pos = np.asarray(pos, dtype=np.float64)
    qt, H = mobility.regularize(pos, a)
    z = pos[:, 2]
    dH = np.where((z > 0.0) & (z < a), 1.0 / a, 0.0)
    above = (z > a).astype(np.float64)
    n = len(pos)
    s = 1.0 / (8.0 * math.pi * eta)
    out = np.zeros((n, 3))
    for i in range(n):
        js = np.concatenate([np.arange(i), np.arange(i + 1, n)])
        if js.size:
            qi = np.repeat(qt[i][:, None], js.size, axis=1)
            qj = qt[js].T
            r = qi - qj
            R = (rpy.free_tt(r, a) + faxen.wall_tt(qi, qj, a)) * s
            dR = (rpy.free_tt_dy(r, a) + faxen.wall_tt_dy(qi, qj, a)) * s
            per_j = H[js] * (dR[:, 0] + dR[:, 1] + above[js] * dR[:, 2]) + dH[js] * R[:, 2]
            out[i] += H[i] * per_j.sum(axis=1)
        # self block: H_i^2 S(z~_i), S = Stokes drag + wall self part
        S2 = (faxen.wall_tt_self(qt[i, 2], a)[:, 2] + np.array([0.0, 0.0, 4.0 / (3.0 * a)])) * s
        dS2 = faxen.wall_tt_self_dz(qt[i, 2], a)[:, 2] * s
        out[i] += 2.0 * H[i] * dH[i] * S2 + H[i] ** 2 * above[i] * dS2
    return out
