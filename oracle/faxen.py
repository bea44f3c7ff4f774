"""Faxen operators applied to the wall image tensor (symbolic derivation, numeric evaluation).

Test infrastructure only (see ``oracle/__init__``).

Definitions followed (Sec. II.B and Sec. III of the paper):

* Translation-translation, eq. mobilityDifferential: the pair mobility is
  (I + a^2/6 lap_x)(I + a^2/6 lap_y) G(x, y) at x = q_i, y = q_j.  The wall
  correction is this operator applied to the image part of Blake's tensor
  (``green.blake_image``).  It is used for overlapping spheres as well: the
  overlap correction does not depend on the boundary (Sec. II.B), so only the
  unbounded part switches form (``rpy``).

* Translation-rotation, eq. mobilityDifferentialTR: (I + a^2/6 lap_x)(1/2 curl_y) G.
  The velocity of sphere i from a torque T on sphere j is

      U_alpha = 1/2 eps_{beta k l} d/dy_k [(1 + a^2/6 lap_x) G_{alpha l}] T_beta,

  the convention under which the same operator applied to the Oseen tensor gives
  the rotlet T x r / (8 pi eta |r|^3), r = x - y (checked in tests).

All tensors carry the factor 8 pi eta (divide by it to get mobilities).

The derivation (sympy differentiation of the closed-form image tensor) takes tens
of seconds, so the resulting expressions are pickled under ``oracle/.cache`` keyed
by a hash of the source files that define them; the cache holds only this
module's own derived expressions.

Pinned by (tests/test_oracle_mobility.py): the self limit x = y reproduces the
textbook wall series of Faxen (parallel) and Lorentz (perpendicular) through
O((a/h)^3) and the rolling coupling 3/32 (a/h)^4; the pair tensors equal
sphere-surface quadratures of the image tensor (the integral form,
eq. mobilityOverlap) for spheres clear of the wall and of each other; the
assembled matrix is symmetric positive definite.
"""
from __future__ import annotations

import functools
import hashlib
import os
import pickle

import numpy as np
import sympy as sp

from . import green

_HERE = os.path.dirname(os.path.abspath(__file__))

X = sp.symbols("x1:4", real=True)   # field point (target sphere centre)
Y = sp.symbols("y1:4", real=True)   # source point (source sphere centre)
A = sp.Symbol("a", positive=True)   # sphere radius
Z = sp.Symbol("z", positive=True)   # height used for the self block


def _lap(expr, v):
    return sum(sp.diff(expr, s, 2) for s in v)


def _derive():
    """Build every symbolic expression the oracle evaluates (8 pi eta units)."""
    Gimg = green.blake_image(X, Y)
    faxen_x = lambda e: e + A ** 2 / 6 * _lap(e, X)
    faxen_y = lambda e: e + A ** 2 / 6 * _lap(e, Y)

    # Translation-translation wall correction.
    Wtt = Gimg.applyfunc(lambda g: faxen_x(faxen_y(g)))

    # Translation-rotation wall correction.
    Gx = Gimg.applyfunc(faxen_x)
    Wtr = sp.zeros(3, 3)
    for al in range(3):
        for be in range(3):
            s = 0
            for k in range(3):
                for l in range(3):
                    e = sp.LeviCivita(be, k, l)
                    if e != 0:
                        s += sp.Rational(1, 2) * e * sp.diff(Gx[al, l], Y[k])
            Wtr[al, be] = s

    # d/dy_beta of Wtt[alpha, beta] (no sum), for the divergence of M.
    dWtt = sp.zeros(3, 3)
    for al in range(3):
        for be in range(3):
            dWtt[al, be] = sp.diff(Wtt[al, be], Y[be])

    # Self block: Wtt at x = y = (0, 0, z) and its total z derivative.
    at_self = {X[0]: 0, X[1]: 0, Y[0]: 0, Y[1]: 0, X[2]: Z, Y[2]: Z}
    Wself = Wtt.subs(at_self)
    Wself_dz = Wself.applyfunc(lambda e: sp.diff(e, Z))
    Wtr_self = Wtr.subs(at_self)
    return dict(Wtt=list(Wtt), Wtr=list(Wtr), dWtt=list(dWtt),
                Wself=list(Wself), Wself_dz=list(Wself_dz), Wtr_self=list(Wtr_self))


def _source_key() -> str:
    h = hashlib.sha256()
    for name in ("green.py", "faxen.py"):
        with open(os.path.join(_HERE, name), "rb") as f:
            h.update(f.read())
    h.update(sp.__version__.encode())
    return h.hexdigest()[:20]


@functools.lru_cache(maxsize=1)
def expressions():
    """The derived sympy expressions (from the on-disk cache when it matches the sources)."""
    cache_dir = os.environ.get("RPB_ORACLE_CACHE", os.path.join(_HERE, ".cache"))
    path = os.path.join(cache_dir, f"faxen-{_source_key()}.pkl")
    try:
        with open(path, "rb") as f:
            return pickle.load(f)
    except (OSError, EOFError, pickle.UnpicklingError):
        pass
    exprs = _derive()
    try:
        os.makedirs(cache_dir, exist_ok=True)
        tmp = f"{path}.{os.getpid()}.tmp"
        with open(tmp, "wb") as f:
            pickle.dump(exprs, f)
        os.replace(tmp, path)
    except OSError:
        pass
    return exprs


def _tensor_fn(entries, args):
    f = sp.lambdify(args, entries, modules="numpy", cse=True)

    def fn(*vals):
        out = f(*vals)
        shape = np.broadcast(*[np.asarray(v) for v in out]).shape
        return np.stack([np.broadcast_to(np.asarray(v, dtype=np.float64), shape)
                         for v in out]).reshape((3, 3) + shape)
    return fn


@functools.lru_cache(maxsize=None)
def _compiled(name: str):
    e = expressions()[name]
    if name in ("Wself", "Wself_dz", "Wtr_self"):
        return _tensor_fn(e, (Z, A))
    return _tensor_fn(e, (X, Y, A))


def wall_tt(x, y, a):
    """8 pi eta W_tt(x, y): arrays x, y of shape (3, n) -> (3, 3, n)."""
    return _compiled("Wtt")(tuple(x), tuple(y), a)


def wall_tr(x, y, a):
    """8 pi eta W_tr(x, y): [alpha, beta] = velocity alpha of x from torque beta at y."""
    return _compiled("Wtr")(tuple(x), tuple(y), a)


def wall_tt_dy(x, y, a):
    """[alpha, beta] = d/dy_beta of 8 pi eta W_tt[alpha, beta](x, y) (no sum)."""
    return _compiled("dWtt")(tuple(x), tuple(y), a)


def wall_tt_self(z, a):
    """8 pi eta W_tt(q, q) for q = (., ., z): shape (3, 3) + shape(z)."""
    return _compiled("Wself")(z, a)


def wall_tt_self_dz(z, a):
    """Total z derivative of ``wall_tt_self``."""
    return _compiled("Wself_dz")(z, a)


def wall_tr_self(z, a):
    """8 pi eta W_tr(q, q) for q = (., ., z)."""
    return _compiled("Wtr_self")(z, a)
