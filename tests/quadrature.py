"""Product Gauss rule on a sphere surface and double surface averages (test helper).

Used to check the pair mobilities against their integral definition (paper,
eq. mobilityOverlap): the velocity of sphere i is the average over its surface
S_i of the flow made by a force density spread over S_j.  A force F on sphere j
is the uniform density F/(4 pi a^2); a torque T is the density
3/(8 pi a^3) T x n (its moment about the centre is T).
"""
import numpy as np


def sphere_rule(nt, nph, rot=0.0):
    """Unit normals (3, nt*nph) and weights summing to 4 pi."""
    mu, wmu = np.polynomial.legendre.leggauss(nt)
    ph = (np.arange(nph) + 0.5) * 2.0 * np.pi / nph + rot
    M, P = np.meshgrid(mu, ph, indexing="ij")
    s = np.sqrt(1.0 - M * M)
    n = np.stack([s * np.cos(P), s * np.sin(P), M], axis=0).reshape(3, -1)
    w = (wmu[:, None] * np.ones(nph)[None, :] * 2.0 * np.pi / nph).ravel()
    return n, w


def double_average(kernel, qi, qj, a, nt, torque=False):
    """(1/4pi a^2) int_{S_i} int_{S_j} kernel(x, y) density(y) dS_y dS_x as a 3x3 matrix.

    ``kernel(x, y)`` returns (3, 3, k) for points x, y of shape (3, k).  With
    ``torque`` the matrix maps a torque T to the velocity (density 3/(8 pi a^3) T x n);
    otherwise it maps a force F (density F/(4 pi a^2)).
    """
    ni, wi = sphere_rule(nt, 2 * nt, 0.1)
    nj, wj = sphere_rule(nt, 2 * nt, 0.37)
    qi = np.asarray(qi, dtype=np.float64)
    qj = np.asarray(qj, dtype=np.float64)
    y = qj[:, None] + a * nj
    out = np.zeros((3, 3))
    if torque:
        # (T x n)_l = eps_{l b c} T_b n_c  ->  matrix E[l, b] per point
        E = np.zeros((3, 3, nj.shape[1]))
        E[0, 1], E[0, 2] = nj[2], -nj[1]
        E[1, 0], E[1, 2] = -nj[2], nj[0]
        E[2, 0], E[2, 1] = nj[1], -nj[0]
    for k in range(ni.shape[1]):
        x = np.repeat((qi + a * ni[:, k])[:, None], y.shape[1], axis=1)
        K = kernel(x, y)
        if torque:
            K = np.einsum("alk,lbk->abk", K, E) * (3.0 / (8.0 * np.pi * a ** 3)) * a * a
            out += wi[k] * (K * wj).sum(-1)
        else:
            out += wi[k] * (K * wj).sum(-1) / (4.0 * np.pi)
    return out / (4.0 * np.pi)


def oseen(x, y):
    """8 pi eta times the Oseen tensor between point arrays x, y (3, k)."""
    r = x - y
    rn = np.sqrt((r * r).sum(0))
    return np.eye(3)[:, :, None] / rn + r[:, None, :] * r[None, :, :] / rn ** 3
