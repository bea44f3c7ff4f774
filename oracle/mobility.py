"""Regularised Rotne-Prager-Blake mobility: dense assembly and matrix-free products.

Test infrastructure only (see ``oracle/__init__``).

Definitions (paper, Sec. II.B, Sec. III and App. A):

* Pair mobility for spheres clear of the wall: unbounded RPY part (``rpy``,
  eq. mobilityOverlap, both branches) plus the Faxen-applied image part
  (``faxen``, eq. mobilityDifferential), Sec. II.B.  The self block (j = i) is
  the same integral with j = i: Stokes drag I/(6 pi eta a) plus the image part
  at x = y.
* Translation-rotation block M_C, eq. mobilityDifferentialTR, the same way.
* Wall overlap regularisation, App. A eq. effMob:  M = B M~ B with
  B_ii = H0(z_i/a) I, H0(x) = clamp(x, 0, 1), and M~ evaluated at the clamped
  heights max(z, a).  The paper states B only for M; the same B is applied to
  M_C here, so that the whole 6N grand mobility stays B (.) B and a sphere on the
  wall stops moving whatever force or torque acts (App. A, first requirement).

Velocity of the spheres: U = M F + M_C T (the deterministic drift of eq. BD with
the active term of Sec. III).

Free space (``wall=False``, the contrast drawn in Sec. II.C): the unbounded RPY
blocks alone, unclamped heights and H = 1.

Pseudo-periodic boundary conditions (``box=(L_x, L_y)``, App. B): each pair block is the
sum over the source's minimum image and its images in the eight neighbour cells, so M
depends on the positions modulo the box only.

Pinned by (tests/test_oracle_mobility.py): symmetry and positive definiteness of
dense M (eigvalsh), zero rows for spheres at or below the wall, the textbook wall
self-mobility series, the 1/r^3 decay of the screened pair interaction for
r >> h (Sec. II.C), quadrature of the integral definition.  The box option: invariance
under whole-box moves and common shifts, O(L^-3) decay of the image terms, and equality
with the unbounded mobility of the system copied into the 3 x 3 cells around the unit
cell, each source's nine copies summed (App. B's image set).
"""
from __future__ import annotations

import concurrent.futures as cf
import math
import multiprocessing as mp

import numpy as np

from . import faxen, rpy


def regularize(pos, a, wall=True):
    """Clamped positions q~ = (x, y, max(z, a)) and weights H0(z/a) (App. A, eq. effMob).

    Free space (``wall=False``): no clamping, H = 1."""
    pos = np.asarray(pos, dtype=np.float64)
    qt = pos.copy()
    if not wall:
        return qt, np.ones(len(pos))
    qt[:, 2] = np.maximum(pos[:, 2], a)
    H = np.clip(pos[:, 2] / a, 0.0, 1.0)
    return qt, H


def image_offsets(box):
    """Horizontal offsets (k_x L_x, k_y L_y, 0) of the unit cell and its eight neighbours."""
    lx, ly = box
    return [np.array([kx * lx, ky * ly, 0.0]) for kx in (-1, 0, 1) for ky in (-1, 0, 1)]


def minimum_image(qi, qj, box):
    """Sources moved by whole box lengths so that x_i - x_j and y_i - y_j lie in
    [-L/2, L/2] (the minimum image convention of App. B).  Arrays (3, n)."""
    qj = np.array(qj, dtype=np.float64, copy=True)
    for c, length in enumerate(box):
        qj[c] += length * np.round((qi[c] - qj[c]) / length)
    return qj


def pair_blocks(qi, qj, a, eta, wall=True, box=None):
    """Translation and translation-rotation blocks M~_ij, M~C_ij of clamped positions.

    ``qi``, ``qj``: arrays (3, n) of targets and sources (already clamped).
    Returns (tt, tr), each (3, 3, n), in mobility units.  ``wall=False``: the unbounded
    RPY blocks alone (free space).  ``box=(L_x, L_y)``: pseudo-periodic boundary conditions
    of App. B, the sum over the source's minimum image and its eight neighbour-cell images.
    """
    qi = np.asarray(qi, dtype=np.float64)
    qj = np.asarray(qj, dtype=np.float64)
    if box is not None:
        qw = minimum_image(qi, qj, box)
        tt, tr = 0.0, 0.0
        for off in image_offsets(box):
            t1, t2 = pair_blocks(qi, qw + off[:, None], a, eta, wall)
            tt, tr = tt + t1, tr + t2
        return tt, tr
    r = qi - qj
    tt = rpy.free_tt(r, a)
    tr = rpy.free_tr(r, a)
    if wall:
        tt = tt + faxen.wall_tt(qi, qj, a)
        tr = tr + faxen.wall_tr(qi, qj, a)
    s = 1.0 / (8.0 * math.pi * eta)
    return tt * s, tr * s


_PAIR_CHUNK = 1 << 17


def dense(pos, a=1.0, eta=1.0, wall=True, box=None):
    """Dense (3N, 3N) matrices M and M_C (FP64).  Practical for N up to ~2000."""
    qt, H = regularize(pos, a, wall)
    n = len(qt)
    M = np.zeros((n, 3, n, 3))
    MC = np.zeros((n, 3, n, 3))
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    I = I.ravel()
    J = J.ravel()
    for s in range(0, I.size, _PAIR_CHUNK):
        ii = I[s:s + _PAIR_CHUNK]
        jj = J[s:s + _PAIR_CHUNK]
        tt, tr = pair_blocks(qt[ii].T, qt[jj].T, a, eta, wall, box)
        w = H[ii] * H[jj]
        M[ii, :, jj, :] = (tt * w).transpose(2, 0, 1)
        MC[ii, :, jj, :] = (tr * w).transpose(2, 0, 1)
    return M.reshape(3 * n, 3 * n), MC.reshape(3 * n, 3 * n)


def _rows_product(args):
    rows, qt, H, force, torque, a, eta, wall, box = args
    n = len(qt)
    out = np.zeros((len(rows), 3))
    step = max(1, _PAIR_CHUNK // n)
    for s in range(0, len(rows), step):
        blk = rows[s:s + step]
        ii = np.repeat(blk, n)
        jj = np.tile(np.arange(n), len(blk))
        tt, tr = pair_blocks(qt[ii].T, qt[jj].T, a, eta, wall, box)
        acc = np.zeros((3, len(ii)))
        if force is not None:
            acc += np.einsum("abk,kb->ak", tt, force[jj])
        if torque is not None:
            acc += np.einsum("abk,kb->ak", tr, torque[jj])
        acc *= H[jj]
        out[s:s + len(blk)] = H[blk][:, None] * acc.reshape(3, len(blk), n).sum(axis=2).T
    return out


def matvec(pos, force=None, torque=None, a=1.0, eta=1.0, rows=None, workers=1, wall=True,
           box=None):
    """U = M F + M_C T by direct summation over all sources (matrix-free).

    ``rows``: optional indices of the target spheres to evaluate (row sampling);
    the result then has shape (len(rows), 3).  ``workers`` > 1 splits the targets
    over a pool of forked processes.
    """
    qt, H = regularize(pos, a, wall)
    n = len(qt)
    force = None if force is None else np.asarray(force, dtype=np.float64)
    torque = None if torque is None else np.asarray(torque, dtype=np.float64)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    if rows.size == 0:
        return np.zeros((0, 3))
    if workers <= 1:
        return _rows_product((rows, qt, H, force, torque, a, eta, wall, box))
    # compile the lambdified tensors before forking so the children inherit them
    pair_blocks(qt[:1].T, qt[:1].T, a, eta, wall)
    parts = np.array_split(rows, min(workers * 4, rows.size))
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
        res = list(ex.map(_rows_product, [(p, qt, H, force, torque, a, eta, wall, box)
                                          for p in parts]))
    return np.vstack(res)


def dense_matvec(pos, force=None, torque=None, a=1.0, eta=1.0, wall=True, box=None):
    """U = M F + M_C T through the dense matrices (small N)."""
    M, MC = dense(pos, a, eta, wall, box)
    n = len(pos)
    u = np.zeros(3 * n)
    if force is not None:
        u += M @ np.asarray(force, dtype=np.float64).ravel()
    if torque is not None:
        u += MC @ np.asarray(torque, dtype=np.float64).ravel()
    return u.reshape(n, 3)
