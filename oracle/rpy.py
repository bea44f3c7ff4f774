"""Unbounded Rotne-Prager-Yamakawa tensors for equal spheres of radius a.

Test infrastructure only (see ``oracle/__init__``).

These are the free-space parts of the pair mobility (Sec. II.B and Sec. III of
the paper): for non-overlapping spheres they are the Faxen form
(eq. mobilityDifferential) applied to the Oseen tensor; for overlapping spheres
(|r| < 2a) they are the double surface average of eq. mobilityOverlap, the
unbounded RPY forms to which the paper adds the wall corrections.  All values
carry the factor 8 pi eta.  r = q_i - q_j (target minus source), rhat = r/|r|.

Translation-translation (velocity of i per force on j):
    |r| >= 2a:  (1/|r|) [ (1 + 2a^2/(3 r^2)) I + (1 - 2a^2/r^2) rhat rhat ]
    |r| <  2a:  (4/(3a)) [ (1 - 9|r|/(32a)) I + (3|r|/(32a)) rhat rhat ]
Translation-rotation (velocity of i per torque T on j, U = c T x r):
    |r| >= 2a:  c = 1/|r|^3
    |r| <  2a:  c = (1 - 3|r|/(8a)) / (2 a^3)

At r = 0 the translation block is the Stokes self-mobility 4/(3a) I
(= I/(6 pi eta a) after dividing by 8 pi eta) and the rotation block vanishes.

Pinned by (tests/test_oracle_rpy.py): both branches equal brute-force
quadratures of the double surface average of the Oseen tensor (and of the
torque traction 3/(8 pi a^3) T x n for the rotation block) over the two sphere
surfaces; for |r| >= 2a the form equals (1 + a^2/3 lap) of the Oseen tensor
symbolically; the branches meet continuously at |r| = 2a; both are divergence
free.
"""
from __future__ import annotations

import functools

import numpy as np
import sympy as sp


def _geometry(r):
    r = np.asarray(r, dtype=np.float64)
    rn = np.sqrt(np.sum(r * r, axis=0))
    safe = np.where(rn > 0.0, rn, 1.0)
    rhat = np.where(rn > 0.0, r / safe, 0.0)
    return rn, rhat


def free_tt(r, a):
    """8 pi eta times the unbounded RPY translation tensor; r of shape (3, n) -> (3, 3, n)."""
    rn, rhat = _geometry(r)
    rr = rhat[:, None, :] * rhat[None, :, :]
    eye = np.eye(3)[:, :, None]
    far = rn >= 2.0 * a
    rs = np.where(far, rn, 1.0)
    c_i = np.where(far, (1.0 + 2.0 * a * a / (3.0 * rs * rs)) / rs,
                   4.0 / (3.0 * a) * (1.0 - 9.0 * rn / (32.0 * a)))
    c_rr = np.where(far, (1.0 - 2.0 * a * a / (rs * rs)) / rs,
                    4.0 / (3.0 * a) * (3.0 * rn / (32.0 * a)))
    return c_i[None, None, :] * eye + c_rr[None, None, :] * rr


def free_tr(r, a):
    """8 pi eta times the unbounded RPY translation-rotation tensor.

    Entry [alpha, beta]: velocity component alpha of sphere i per torque component
    beta on sphere j, i.e. U = c (T x r).
    """
    r = np.asarray(r, dtype=np.float64)
    rn, _ = _geometry(r)
    far = rn >= 2.0 * a
    rs = np.where(far, rn, 1.0)
    c = np.where(far, 1.0 / rs ** 3, (1.0 - 3.0 * rn / (8.0 * a)) / (2.0 * a ** 3))
    out = np.zeros((3, 3) + rn.shape)
    # (T x r)_alpha = eps_{alpha beta gamma} T_beta r_gamma
    for al in range(3):
        for be in range(3):
            for ga in range(3):
                e = _eps(al, be, ga)
                if e:
                    out[al, be] += e * c * r[ga]
    return out


def _eps(i, j, k):
    return int(sp.LeviCivita(i, j, k))


# ---- symbolic versions, used for derivatives (divergence of M) -----------------------

_R = sp.symbols("r1:4", real=True)
_A = sp.Symbol("a", positive=True)


def symbolic_free_tt(branch: str) -> sp.Matrix:
    """The same tensor as ``free_tt`` for one branch ("far" or "near"), in sympy."""
    r = sp.Matrix(_R)
    rn = sp.sqrt(r.dot(r))
    rr = r * r.T / rn ** 2
    if branch == "far":
        return (1 + 2 * _A ** 2 / (3 * rn ** 2)) / rn * sp.eye(3) + (1 - 2 * _A ** 2 / rn ** 2) / rn * rr
    return sp.Rational(4, 3) / _A * ((1 - 9 * rn / (32 * _A)) * sp.eye(3) + 3 * rn / (32 * _A) * rr)


@functools.lru_cache(maxsize=None)
def _dy_fn(branch: str):
    # d/dy_beta of T[alpha, beta](x - y) = - d/dr_beta T[alpha, beta](r)
    T = symbolic_free_tt(branch)
    entries = [-sp.diff(T[al, be], _R[be]) for al in range(3) for be in range(3)]
    return sp.lambdify((_R, _A), entries, modules="numpy", cse=True)


def free_tt_dy(r, a):
    """[alpha, beta] = d/dy_beta of 8 pi eta free_tt[alpha, beta](x - y), no sum; r = x - y."""
    r = np.asarray(r, dtype=np.float64)
    rn = np.sqrt(np.sum(r * r, axis=0))
    out = np.zeros((3, 3) + rn.shape)
    for branch, mask in (("far", rn >= 2.0 * a), ("near", (rn < 2.0 * a) & (rn > 0.0))):
        if not np.any(mask):
            continue
        vals = _dy_fn(branch)(tuple(r[:, mask]), a)
        for k, v in enumerate(vals):
            out[k // 3, k % 3, mask] = v
    return out
