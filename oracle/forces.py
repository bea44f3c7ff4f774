"""Soft steric forces and gravity.

Test infrastructure only (see ``oracle/__init__``).

Sec. III, eq. soft_potential of the paper:

    U(r) = U0 + U0 (d - r)/b     for r < d,
    U(r) = U0 exp(-(r - d)/b)    for r >= d,

with d = 2a and r the centre distance for sphere pairs, and d = a and r the
height z for the sphere-wall interaction.  The force is -grad U: magnitude
f(r) = -U'(r) = U0/b for r < d and (U0/b) exp(-(r - d)/b) for r >= d, directed
along (q_i - q_j)/|q_i - q_j| for pairs and along +z for the wall.  Gravity adds
a constant force f_g z-hat (f_g < 0 pulls towards the wall).  No cutoff.
Coincident centres (r = 0) exert no force (the direction is undefined).

Pinned by (tests/test_oracle_forces.py): U and f are continuous at r = d;
f = -dU/dr by finite differences; the force on a pair is equal and opposite;
the paper's worked value (1 + a/b) U0 = 44 kT for U0 = 4 kT, b = 0.1a is the
wall energy at z = 0.
"""
from __future__ import annotations

import numpy as np


def potential(r, d, u0, b):
    r = np.asarray(r, dtype=np.float64)
    return np.where(r < d, u0 + u0 * (d - r) / b, u0 * np.exp(-(r - d) / b))


def force_magnitude(r, d, u0, b):
    """f(r) = -U'(r)."""
    r = np.asarray(r, dtype=np.float64)
    return np.where(r < d, u0 / b, (u0 / b) * np.exp(-(r - d) / b))


def forces(pos, a=1.0, u0=1.0, b=0.1, f_grav_z=-1.0, rows=None, wall=True, box=None):
    """Total force on each sphere (or on ``rows``), shape (n, 3) / (len(rows), 3).
    ``wall=False``: no wall repulsion (free space).  ``box=(L_x, L_y)``: pair separations
    by the minimum image convention (App. B)."""
    pos = np.asarray(pos, dtype=np.float64)
    n = len(pos)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    out = np.zeros((len(rows), 3))
    for k, i in enumerate(rows):
        r = pos[i] - pos
        if box is not None:
            for c, length in enumerate(box):
                r[:, c] -= length * np.round(r[:, c] / length)
        rn = np.sqrt(np.sum(r * r, axis=1))
        ok = (np.arange(n) != i) & (rn > 0.0)
        f = force_magnitude(rn[ok], 2.0 * a, u0, b)
        out[k] = np.sum((f / rn[ok])[:, None] * r[ok], axis=0)
    z = pos[rows, 2]
    if wall:
        out[:, 2] += force_magnitude(z, a, u0, b)
    out[:, 2] += f_grav_z
    return out
