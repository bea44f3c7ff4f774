"""Krylov (Lanczos) approximation of M^{1/2} W and the dense symmetric square root.

Test infrastructure only (see ``oracle/__init__``).

Sec. II.C of the paper: m Lanczos iterations build the Krylov space
K_m(M, W) = span{W, M W, ..., M^{m-1} W}; the noise is approximated in it as
g_m = ||W|| V_m T_m^{1/2} e_1 (Ando et al.), with V_m the orthonormal Lanczos
basis and T_m the tridiagonal projection of M.  The iteration stops when the
relative change eps_m = ||g_m - g_{m-1}|| / ||g_{m-1}|| falls below the
tolerance.  Readings where the paper is silent: the basis is fully
re-orthogonalised against all previous vectors at every step (m is small);
eps_m needs two iterates, so m >= 2 unless the Krylov space is invariant
(beta_m = 0, where g_m is exact); the square root of T_m comes from its
eigendecomposition T_m = Q Lambda Q^T.

Pinned by (tests/test_oracle_lanczos.py): against the dense symmetric square
root (``sqrtm_dense``) of the assembled mobility at tight tolerance; at m = 3N
iterations the result is the exact M^{1/2} W; for one sphere the result equals
the closed-form diagonal square root; the sample covariance of g over many W
approaches M (fluctuation-dissipation, eq. BD).  The preconditioned variant at
m = 3N equals L B^{1/2} W with (L B^{1/2})(L B^{1/2})^T = M, and its scale reproduces the
wall self-mobility series.
``tridiag_sqrt_e1`` matches the closed-form root of a 2 x 2 matrix, the diagonal case and
scipy's Schur-based ``sqrtm`` of the dense T.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def lanczos_sqrt(apply_m, w, tol, max_iter=64, breakdown_rel=1e-14, notspd_rel=1e-12):
    """Return (g, iterations, eps, status) with g ~ M^{1/2} w.

    ``apply_m``: callable v -> M v on flat FP64 vectors.  ``status`` is "ok"
    (eps < tol), "breakdown" (invariant Krylov space, g exact), "noconv"
    (max_iter reached; g is the last iterate) or "notspd" (a Ritz value below
    -notspd_rel * largest).
    """
    w = np.asarray(w, dtype=np.float64).ravel()
    wn = np.linalg.norm(w)
    if wn == 0.0:
        return np.zeros_like(w), 0, 0.0, "ok"
    V = [w / wn]
    alphas, betas = [], []
    g_prev = None
    eps = np.inf
    for m in range(1, max_iter + 1):
        v = V[-1]
        u = apply_m(v)
        alpha = float(v @ u)
        u = u - alpha * v
        if m > 1:
            u = u - betas[-1] * V[-2]
        Vm = np.array(V)
        u = u - Vm.T @ (Vm @ u)          # full re-orthogonalisation
        beta = float(np.linalg.norm(u))
        alphas.append(alpha)

        lam, Q = scipy.linalg.eigh_tridiagonal(np.array(alphas), np.array(betas))
        if lam.min() < -notspd_rel * max(lam.max(), 0.0):
            return Vm.T @ (wn * Q @ (np.sqrt(np.maximum(lam, 0.0)) * Q[0])), m, eps, "notspd"
        y = wn * Q @ (np.sqrt(np.maximum(lam, 0.0)) * Q[0])
        g = Vm.T @ y
        if g_prev is not None:
            eps = float(np.linalg.norm(g - g_prev) / np.linalg.norm(g_prev))
            if eps < tol:
                return g, m, eps, "ok"
        if beta <= breakdown_rel * max(abs(x) for x in alphas):
            return g, m, (eps if g_prev is not None else 0.0), "breakdown"
        betas.append(beta)
        V.append(u / beta)
        g_prev = g
    return g, max_iter, eps, "noconv"


def tridiag_sqrt_e1(alpha, beta, wnorm=1.0):
    """|w| T^{1/2} e_1 for the symmetric tridiagonal T with diagonal ``alpha`` and
    off-diagonal ``beta`` (len(alpha) - 1 entries): the small dense step of Sec. II.C that
    turns the Lanczos coefficients into the coordinates of g_m in the Krylov basis.  From the
    eigendecomposition T = Q Lambda Q^T, negative eigenvalues clamped at zero as in
    ``lanczos_sqrt``."""
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    lam, Q = scipy.linalg.eigh_tridiagonal(alpha, beta)
    return wnorm * Q @ (np.sqrt(np.maximum(lam, 0.0)) * Q[0])


def sqrtm_dense(M):
    """Symmetric square root Q Lambda^{1/2} Q^T of a symmetric PSD matrix."""
    lam, Q = np.linalg.eigh(np.asarray(M, dtype=np.float64))
    return (Q * np.sqrt(np.maximum(lam, 0.0))) @ Q.T


def block_diagonal_scale(pos, a=1.0, eta=1.0, wall=True):
    """L with L^2 = the diagonal of the self blocks M_ii, flat (3N,).

    With the wall each self block is diagonal, diag(mu_par, mu_par, mu_perp) times H_i^2
    (App. A); a sphere at or below the wall (H = 0) keeps L = 1, so its zero rows of M stay
    zero rows of B.  The blocks are read off the dense oracle matrix of each lone sphere.
    """
    from . import mobility
    pos = np.asarray(pos, dtype=np.float64)
    out = np.ones(3 * len(pos))
    for i, q in enumerate(pos):
        M, _ = mobility.dense(q[None, :], a, eta, wall)
        d = np.diag(M)
        out[3 * i:3 * i + 3] = np.where(d > 0.0, np.sqrt(np.where(d > 0.0, d, 1.0)), 1.0)
    return out


def lanczos_sqrt_precond(apply_m, scale, w, tol, max_iter=64):
    """Square-root preconditioned Lanczos (the preconditioning Sec. II.C tried): with
    P = L L^T block diagonal (here diagonal, L = diag(scale)), run Lanczos on
    B = L^-1 M L^-T and return g = L B^{1/2} w, whose covariance over w is L B L^T = M.
    The stopping test is applied to the B-space iterates.  Returns (g, m, eps, status)."""
    scale = np.asarray(scale, dtype=np.float64)
    y, m, eps, status = lanczos_sqrt(lambda v: apply_m(v / scale) / scale, w, tol, max_iter)
    return scale * y, m, eps, status
