"""One Brownian dynamics time step: Euler-Maruyama or stochastic Adams-Bashforth.

Test infrastructure only (see ``oracle/__init__``).

Sec. II.A of the paper.  With u^n = M^n F^n + M_C^n T (deterministic velocity
including the active torque term of Sec. III), g^n ~ M^{n 1/2} W^n (Lanczos,
Sec. II.C) and D^n the centred RFD with W~^n:

    EM  (eq. EM):  q^{n+1} = q^n + dt u^n + sqrt(2 kT dt) g^n + dt D^n
    SAB (eq. AB):  q^{n+1} = q^n + dt (3/2 u^n - 1/2 u^{n-1}) + sqrt(2 kT dt) g^n + dt D^n

The first SAB step has no u^{-1}; it takes u^{-1} = u^0, i.e. an EM step
(reading: the paper does not say how the multistep scheme is started).
u^n is returned so the caller can keep it for the next step.

Pinned by (tests/test_oracle_integrator.py): with kT = 0 SAB is the
two-step Adams-Bashforth method (second-order convergence on a deterministic
two-sphere trajectory against a tight ODE solve) and EM is forward Euler
(first order).  At kT > 0, for one sphere above the wall with no force: the noise
term alone equals sqrt(2 kT dt) (6 pi eta a)^{-1/2} diag(sqrt mu_par, sqrt mu_par,
sqrt mu_perp) W (the textbook wall self-mobilities), and the drift term alone,
with W~ = z-hat, equals dt kT d/dz of the perpendicular self-mobility; both schemes
give the same stochastic terms, and they add.
"""
from __future__ import annotations

import math

import numpy as np

from . import forces as forces_mod
from . import lanczos, mobility, stochastic


def step(pos, u_prev, w, w_tilde, *, dt, delta, lanczos_tol, lanczos_max_iter=64,
         scheme="sab", f_grav_z=-1.0, torque=(0.0, 1.0, 0.0), u0=1.0, b=0.1,
         a=1.0, eta=1.0, kT=1.0, dense=None, rfd="centred", wall=True,
         lanczos_precond=False, box=None):
    """Advance ``pos`` by one step.  Returns (new_pos, u_now, lanczos_iterations, eps, status).

    ``u_prev``: previous deterministic velocity or None (first step).  ``rfd``: "centred"
    or "one_sided" random finite difference for the drift.  ``wall=False``: free space.
    ``lanczos_precond``: block-diagonal preconditioned Lanczos for the noise.
    ``box=(L_x, L_y)``: pseudo-periodic boundary conditions (App. B).  ``w``,
    ``w_tilde``: (n, 3) normal variates.  ``dense``: use dense matrices (default
    for n <= 1500).
    """
    pos = np.asarray(pos, dtype=np.float64)
    n = len(pos)
    if dense is None:
        dense = n <= 1500
    F = forces_mod.forces(pos, a, u0, b, f_grav_z, wall=wall, box=box)
    T = np.tile(np.asarray(torque, dtype=np.float64), (n, 1))
    if dense:
        M, MC = mobility.dense(pos, a, eta, wall, box)
        u = (M @ F.ravel() + MC @ T.ravel()).reshape(n, 3)
        apply_m = lambda v: M @ v
    else:
        u = mobility.matvec(pos, F, T, a, eta, wall=wall, box=box)
        apply_m = lambda v: mobility.matvec(pos, v.reshape(n, 3), None, a, eta,
                                            wall=wall, box=box).ravel()
    if lanczos_precond:
        scale = lanczos.block_diagonal_scale(pos, a, eta, wall)
        g, iters, eps, status = lanczos.lanczos_sqrt_precond(apply_m, scale, np.asarray(w).ravel(),
                                                             lanczos_tol, lanczos_max_iter)
    else:
        g, iters, eps, status = lanczos.lanczos_sqrt(apply_m, np.asarray(w).ravel(),
                                                     lanczos_tol, lanczos_max_iter)
    rfd_fn = stochastic.rfd if rfd == "centred" else stochastic.rfd_one_sided
    drift = rfd_fn(pos, w_tilde, delta, a, eta, kT, wall=wall, box=box)
    if scheme == "em" or u_prev is None:
        det = u
    else:
        det = 1.5 * u - 0.5 * np.asarray(u_prev)
    new = pos + dt * det + math.sqrt(2.0 * kT * dt) * g.reshape(n, 3) + dt * drift
    return new, u, iters, eps, status

