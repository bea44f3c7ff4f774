"""Seeded synthetic workloads: sheets of spheres above a no-slip wall at z = 0.

This module only draws random inputs (positions, force/torque vectors, noise
vectors, system sizes) and holds none of the mobility arithmetic, so both the
HIP path and the CPU oracle can use it.

The shapes follow the paper's workloads: a quasi-two-dimensional suspension
sedimented over a wall at projected area fraction phi (Sec. II.C, Fig. 1 uses
phi = 0.25; Sec. III uses sheets of N = 2^15 rollers), heights of the order of
the gravitational height h_g (Sec. III), in reduced units a = eta = kT = 1.
The paper's own initial states come from Monte Carlo sampling of the
Gibbs-Boltzmann distribution, which is not reproduced here: uniform
x, y over a square and uniform heights stand in for it.

Substreams of ``numpy.random.SeedSequence(seed).spawn(5)``:
0 positions, 1 forces/torques, 2 Lanczos noise W, 3 RFD noise W~, 4 sizes.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

STREAM_POS, STREAM_FT, STREAM_W, STREAM_WT, STREAM_SIZES = range(5)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic configuration (reduced units: a = eta = kT = 1)."""

    name: str
    n: int                      # spheres per system
    side: float                 # square side L of the x-y box
    z_lo: float                 # heights are uniform in [z_lo, z_hi]
    z_hi: float
    reject_below: float = 0.0   # RSA: minimum 3-D centre distance (0 = none)
    precision: str = "fp64"     # "fp64" or "mixed"
    steps: int = 1
    dt: float = 0.01
    delta: float = 1e-4         # RFD length
    lanczos_tol: float = 1e-3
    f_grav_z: float = -1.0      # gravity force on every sphere (z component)
    torque: tuple = (0.0, 1.0, 0.0)
    steric_u0: float = 1.0      # soft potential strength U0 (Sec. III, eq. soft_potential)
    steric_b: float = 0.1       # soft potential range b
    nsys: int = 1               # > 1: batched independent suspensions
    n_lo: int = 0               # batched sizes uniform in [n_lo, n_hi]
    n_hi: int = 0
    a: float = 1.0
    eta: float = 1.0
    kT: float = 1.0


def side_for_area_fraction(n: int, phi: float, a: float = 1.0) -> float:
    """Square side L with projected area fraction n*pi*a^2/L^2 = phi."""
    return math.sqrt(n * math.pi * a * a / phi)


PHI = 0.4

WORKLOADS = {
    # Small FP64 case: one matvec and one Lanczos solve, dense check possible.
    "sheet256_rsa": Workload("sheet256_rsa", 256, 32.0, 1.1, 3.0, reject_below=2.05,
                             lanczos_tol=1e-6),
    # FP64 time stepping: 100 stochastic Adams-Bashforth steps.
    "sheet16k_fp64": Workload("sheet16k_fp64", 16384, side_for_area_fraction(16384, PHI),
                              1.1, 2.5, steps=100),
    # Mixed precision at N = 65,536 (the headline size).
    "sheet64k_mixed": Workload("sheet64k_mixed", 65536, side_for_area_fraction(65536, PHI),
                               1.1, 2.5, precision="mixed", steps=10),
    # 64 independent suspensions of uneven size, float64 and mixed precision.
    "batch64_uneven": Workload("batch64_uneven", 0, 0.0, 1.1, 2.5, nsys=64,
                               n_lo=1024, n_hi=8192),
    "batch64_uneven_mixed": Workload("batch64_uneven_mixed", 0, 0.0, 1.1, 2.5, nsys=64,
                                     n_lo=1024, n_hi=8192, precision="mixed"),
    # Large sheet.
    "sheet256k_mixed": Workload("sheet256k_mixed", 262144, side_for_area_fraction(262144, PHI),
                                1.1, 2.0, precision="mixed", steps=20, dt=0.005),
}


def substreams(seed: int, k: int = 5):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


def sample_positions(n: int, side: float, z_lo: float, z_hi: float,
                     reject_below: float = 0.0, rng=None, seed: int = 0) -> np.ndarray:
    """(n, 3) float64 positions: x, y uniform in [0, side), z uniform in [z_lo, z_hi].

    With ``reject_below > 0`` candidates are placed one by one and rejected when
    closer than ``reject_below`` (3-D centre distance) to an accepted sphere
    (random sequential addition).
    """
    if rng is None:
        rng = substreams(seed)[STREAM_POS]
    if reject_below <= 0.0:
        xy = rng.uniform(0.0, side, size=(n, 2))
        z = rng.uniform(z_lo, z_hi, size=(n, 1))
        return np.ascontiguousarray(np.hstack([xy, z]))
    out = np.empty((n, 3))
    k = 0
    tries = 0
    while k < n:
        tries += 1
        if tries > 10_000_000:
            raise RuntimeError("random sequential addition did not place all spheres")
        c = np.array([rng.uniform(0.0, side), rng.uniform(0.0, side), rng.uniform(z_lo, z_hi)])
        if k and np.min(np.sum((out[:k] - c) ** 2, axis=1)) < reject_below ** 2:
            continue
        out[k] = c
        k += 1
    return out


def normal_vectors(n: int, rng, count: int = 1):
    """``count`` arrays of shape (n, 3) of i.i.d. N(0, 1) float64 values."""
    vs = [np.ascontiguousarray(rng.standard_normal((n, 3))) for _ in range(count)]
    return vs if count > 1 else vs[0]


def make_inputs(w: Workload, seed: int = 0):
    """Positions, forces, torques, W and W~ for a single-system workload."""
    s = substreams(seed)
    pos = sample_positions(w.n, w.side, w.z_lo, w.z_hi, w.reject_below, rng=s[STREAM_POS])
    force, torque = normal_vectors(w.n, s[STREAM_FT], 2)
    wv = normal_vectors(w.n, s[STREAM_W])
    wt = normal_vectors(w.n, s[STREAM_WT])
    return dict(pos=pos, force=force, torque=torque, w=wv, w_tilde=wt)


def batch_sizes(w: Workload, seed: int = 0) -> np.ndarray:
    """System sizes of a batched workload, uniform integers in [n_lo, n_hi]."""
    rng = substreams(seed)[STREAM_SIZES]
    return rng.integers(w.n_lo, w.n_hi + 1, size=w.nsys).astype(np.int64)


def make_batch(w: Workload, seed: int = 0):
    """Concatenated positions of ``w.nsys`` systems and their offsets (prefix sums)."""
    sizes = batch_sizes(w, seed)
    s = substreams(seed)
    rng = s[STREAM_POS]
    pos = [sample_positions(int(n), side_for_area_fraction(int(n), PHI), w.z_lo, w.z_hi, rng=rng)
           for n in sizes]
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    return np.ascontiguousarray(np.vstack(pos)), offs


def sheet(n: int, z_lo: float = 1.1, z_hi: float = 2.5, phi: float = PHI, seed: int = 0):
    """A uniform sheet of ``n`` spheres at area fraction ``phi`` (positions only)."""
    s = substreams(seed)
    return sample_positions(n, side_for_area_fraction(n, phi), z_lo, z_hi, rng=s[STREAM_POS])


def sedimented_sheet(n: int, phi: float = 0.25, h_mean: float = 1.6, h_min: float = 1.1,
                     seed: int = 0, a: float = 1.0) -> np.ndarray:
    """A sedimented-looking sheet: x, y at projected area fraction ``phi``, heights
    h_min + Exp(h_mean - h_min) (mean ``h_mean``, the exponential profile of a gravitational
    height over the wall), no two centres closer than 2a (random sequential addition on a
    cell grid).  Stands in for the equilibrium states of the Lanczos convergence study
    (phi = 0.25, characteristic height 1.6a)."""
    rng = substreams(seed)[STREAM_POS]
    side = side_for_area_fraction(n, phi, a)
    d2 = (2.0 * a) ** 2
    cell = 2.0 * a
    nc = max(1, int(side // cell))
    grid = {}
    out = np.empty((n, 3))
    k = tries = 0
    while k < n:
        tries += 1
        if tries > 200 * n + 1000:
            raise RuntimeError("random sequential addition did not place all spheres")
        x, y = rng.uniform(0.0, side, 2)
        z = h_min + rng.exponential(h_mean - h_min)
        cx, cy = int(x / side * nc) % nc, int(y / side * nc) % nc
        ok = True
        for ix in (cx - 1, cx, cx + 1):
            for iy in (cy - 1, cy, cy + 1):
                for j in grid.get((ix % nc, iy % nc), ()):
                    q = out[j]
                    if (q[0] - x) ** 2 + (q[1] - y) ** 2 + (q[2] - z) ** 2 < d2:
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        out[k] = (x, y, z)
        grid.setdefault((cx, cy), []).append(k)
        k += 1
    return out
