"""Pins of the wall-corrected mobility (oracle/faxen.py, oracle/mobility.py)."""
import functools
import math
from fractions import Fraction

import numpy as np
import pytest
import sympy as sp

from oracle import faxen, green, mobility
from paper_1612_00474_amd import workloads as wl
from tests.conftest import golden_rows
from tests.quadrature import double_average

A = 1.0


@functools.lru_cache(maxsize=1)
def _gimg_numeric():
    X = sp.symbols("x1:4", real=True)
    Y = sp.symbols("y1:4", real=True)
    f = sp.lambdify((X, Y), list(green.blake_image(X, Y)), modules="numpy", cse=True)

    def k(x, y):
        vals = f(tuple(x), tuple(y))
        return np.stack([np.broadcast_to(np.asarray(v, dtype=float), x.shape[1:]) for v in vals]).reshape(
            (3, 3) + x.shape[1:])
    return k


PAIRS = [  # (q_i, q_j): clear of the wall; the third pair overlaps (|r| < 2a)
    (np.array([0.0, 0.0, 1.5]), np.array([2.3, -1.1, 2.2])),
    (np.array([0.4, 0.2, 3.0]), np.array([-5.0, 1.0, 1.2])),
    (np.array([0.0, 0.0, 1.7]), np.array([0.9, 0.5, 2.4])),
]


@pytest.mark.parametrize("k", range(len(PAIRS)))
def test_wall_tt_equals_double_surface_average_of_image(k):
    qi, qj = PAIRS[k]
    ref = double_average(_gimg_numeric(), qi, qj, A, 24)
    got = faxen.wall_tt(qi[:, None], qj[:, None], A)[:, :, 0]
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("k", range(len(PAIRS)))
def test_wall_tr_equals_double_surface_average_of_image(k):
    qi, qj = PAIRS[k]
    ref = double_average(_gimg_numeric(), qi, qj, A, 24, torque=True)
    got = faxen.wall_tr(qi[:, None], qj[:, None], A)[:, :, 0]
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


def test_self_mobility_matches_wall_series():
    # mu(h) in units of 1/(6 pi eta a); compare Taylor coefficients in eps = a/h through eps^3
    rows = golden_rows("wall_self_mobility_series.txt")
    eps = sp.Symbol("eps", positive=True)
    z = sp.Symbol("z", positive=True)
    a = sp.Symbol("a", positive=True)
    W = faxen.expressions()["Wself"]
    for direction, idx in (("par", 0), ("perp", 8)):
        mu = 1 + sp.Rational(3, 4) * a * W[idx]          # (6 pi eta a)/(8 pi eta) = 3a/4
        mu = sp.simplify(mu.subs(z, a / eps))
        ser = sp.series(mu, eps, 0, 4).removeO()
        for d, order, num, den in rows:
            if d == direction:
                assert sp.Rational(int(num), int(den)) == ser.coeff(eps, int(order))


def test_rolling_coupling_matches_far_field_result():
    (num, den, power), = golden_rows("rolling_coupling.txt")
    C = Fraction(int(num), int(den))
    for h in (1.0, 1.7, 4.0):
        Wtr = faxen.wall_tr_self(np.array(h), A)
        Ux = Wtr[0, 1] / (8 * math.pi)          # velocity x per torque y (eta = 1)
        expect = float(C) * (A / h) ** int(power) / (6 * math.pi * A ** 2)
        assert abs(Ux - expect) <= 1e-14 * expect
        assert abs(Wtr[1, 0] / (8 * math.pi) + expect) <= 1e-14 * expect
        assert np.abs(Wtr[2]).max() == 0.0 and abs(Wtr[0, 0]) < 1e-18


def test_pair_tends_to_self_block():
    q = np.array([0.3, -0.2, 1.6])
    self_tt = faxen.wall_tt_self(np.array(q[2]), A)
    for e in (1e-4, 1e-6):
        qj = q + e * np.array([0.6, 0.0, 0.8])
        w = faxen.wall_tt(q[:, None], qj[:, None], A)[:, :, 0]
        assert np.abs(w - self_tt).max() < 50 * e


@pytest.fixture(scope="module")
def c1_dense():
    inp = wl.make_inputs(wl.WORKLOADS["sheet256_rsa"], 0)
    return inp, mobility.dense(inp["pos"], A, 1.0)


def test_dense_symmetric_positive_definite(c1_dense):
    _, (M, _) = c1_dense
    assert np.linalg.norm(M - M.T) / np.linalg.norm(M) <= 1e-14
    assert np.linalg.eigvalsh(M).min() > 0.0


def test_spd_with_overlaps_and_wall_overlaps():
    rng = np.random.default_rng(7)
    pos = np.column_stack([rng.uniform(0, 6, 60), rng.uniform(0, 6, 60), rng.uniform(0.2, 2.5, 60)])
    pos[5, 2] = 0.0      # centre on the wall
    pos[6, 2] = -0.3     # below the wall
    pos[8, 2] = 1.5
    pos[7] = pos[8] + np.array([0.0, 0.0, 1e-3])   # nearly coincident
    pos[9, :2] = pos[10, :2]
    pos[9, 2], pos[10, 2] = 0.4, 0.7              # coincident after clamping to z = a
    M, MC = mobility.dense(pos, A, 1.0)
    assert np.linalg.norm(M - M.T) / np.linalg.norm(M) <= 1e-14
    lam = np.linalg.eigvalsh(M)
    assert lam.min() > -1e-14 * lam.max()
    for i in (5, 6):  # rows and columns vanish exactly on/below the wall (App. A)
        assert np.all(M[3 * i:3 * i + 3] == 0.0) and np.all(M[:, 3 * i:3 * i + 3] == 0.0)
        assert np.all(MC[3 * i:3 * i + 3] == 0.0) and np.all(MC[:, 3 * i:3 * i + 3] == 0.0)
    # without exactly coincident (clamped) centres the nonzero part is positive definite
    keep = np.ones(len(pos), bool)
    keep[[5, 6, 9]] = False
    Mk, _ = mobility.dense(pos[keep], A, 1.0)
    lam = np.linalg.eigvalsh(Mk)
    assert lam.min() > 1e-8 * lam.max()


def test_wall_screening_decays_as_inverse_cube():
    # Sec. II.C: pair interaction above a wall decays like 1/r^3 for r >> h
    h = 1.5
    rs = np.array([50.0, 100.0, 200.0, 400.0])
    qi = np.tile(np.array([0.0, 0.0, h])[:, None], (1, rs.size))
    qj = np.vstack([rs, np.zeros_like(rs), np.full_like(rs, h)])
    tt, _ = mobility.pair_blocks(qi, qj, A, 1.0)
    # the slowest component (parallel, along the separation) sets the decay; the
    # transverse and normal components decay faster (1/r^5)
    norm = np.sqrt((tt ** 2).sum(axis=(0, 1)))
    assert abs(np.polyfit(np.log(rs), np.log(norm), 1)[0] + 3.0) < 0.02
    assert abs(np.polyfit(np.log(rs), np.log(np.abs(tt[1, 1])), 1)[0] + 5.0) < 0.02
    # without the wall part the decay is 1/r
    from oracle import rpy
    free = rpy.free_tt(qi - qj, A)[0, 0]
    assert abs(np.polyfit(np.log(rs), np.log(free), 1)[0] + 1.0) < 0.01


def test_matrix_free_equals_dense(c1_dense):
    inp, (M, MC) = c1_dense
    u_dense = (M @ inp["force"].ravel() + MC @ inp["torque"].ravel()).reshape(-1, 3)
    u = mobility.matvec(inp["pos"], inp["force"], inp["torque"], A, 1.0)
    assert np.abs(u - u_dense).max() <= 1e-15 * np.abs(u_dense).max() * 10
    rows = np.array([0, 17, 255])
    ur = mobility.matvec(inp["pos"], inp["force"], inp["torque"], A, 1.0, rows=rows, workers=2)
    assert np.abs(ur - u_dense[rows]).max() <= 1e-14 * np.abs(u_dense).max()


# ---- free space (wall = False): the unbounded RPY tensors alone ---------------------------

def _free_config():
    # overlapping pairs and spheres at and below z = 0: no wall, so nothing is clamped
    return np.array([[0.0, 0.0, 1.3], [1.5, 0.4, 1.9], [0.8, -1.1, 0.6], [3.5, 1.0, -2.4],
                     [2.6, -0.5, 0.0], [0.2, 0.3, 1.0]])


def test_free_space_self_block_is_stokes_drag():
    for z in (-3.0, 0.0, 0.4, 2.0):
        M, _ = mobility.dense(np.array([[0.1, 0.2, z]]), 1.3, 0.7, wall=False)
        assert np.allclose(M, np.eye(3) / (6 * math.pi * 0.7 * 1.3), rtol=1e-14, atol=0)


def test_free_space_is_translation_invariant_and_spd():
    pos = _free_config()
    M0, C0 = mobility.dense(pos, wall=False)
    M1, C1 = mobility.dense(pos + np.array([3.0, -7.0, 11.0]), wall=False)
    assert np.allclose(M0, M1, rtol=1e-13, atol=1e-16)
    assert np.allclose(C0, C1, rtol=1e-13, atol=1e-16)
    assert np.allclose(M0, M0.T, rtol=0, atol=1e-15)
    assert np.linalg.eigvalsh(M0).min() > 0.0
    # the wall breaks the invariance
    W0, _ = mobility.dense(pos + np.array([0.0, 0.0, 5.0]))
    W1, _ = mobility.dense(pos + np.array([0.0, 0.0, 9.0]))
    assert np.abs(W0 - W1).max() > 1e-3


def test_wall_mobility_tends_to_free_space_far_from_the_wall():
    # the image part of the self term decays like a/h (-9/16 a/h parallel, -9/8 a/h normal)
    pos = _free_config() + np.array([0.0, 0.0, 3.0])
    free, _ = mobility.dense(pos, wall=False)
    for lift in (1e3, 1e4):
        wall, _ = mobility.dense(pos + np.array([0.0, 0.0, lift]))
        gap = np.abs(wall - free).max() / np.abs(free).max()
        assert gap < 2.0 / lift


def test_free_space_matrix_free_product_matches_dense():
    pos = _free_config()
    rng = np.random.default_rng(3)
    F, T = rng.standard_normal(pos.shape), rng.standard_normal(pos.shape)
    M, MC = mobility.dense(pos, wall=False)
    ref = (M @ F.ravel() + MC @ T.ravel()).reshape(-1, 3)
    assert np.allclose(mobility.matvec(pos, F, T, wall=False), ref, rtol=1e-13, atol=1e-16)


# ---- pseudo-periodic boundary conditions (App. B): minimum image + 8 neighbour cells ------

BOX = (9.0, 7.5)


def _box_config():
    rng = np.random.default_rng(17)
    pos = np.column_stack([rng.uniform(0, BOX[0], 7), rng.uniform(0, BOX[1], 7),
                           rng.uniform(1.05, 2.5, 7)])
    pos[1, :2] = pos[0, :2] + [1.2, 0.9]       # an overlapping pair
    pos[2, 2] = 0.8                            # a sphere below z = a
    return pos


def test_periodic_mobility_depends_on_positions_modulo_the_box():
    pos = _box_config()
    M, MC = mobility.dense(pos, box=BOX)
    moved = pos.copy()
    moved[:, 0] += 3.3                         # common shift
    moved[:, 1] -= 1.1
    moved[3, 0] += 2 * BOX[0]                  # whole-box jumps of single spheres
    moved[5, 1] -= BOX[1]
    M2, MC2 = mobility.dense(moved, box=BOX)
    assert np.allclose(M2, M, rtol=1e-12, atol=1e-15)
    assert np.allclose(MC2, MC, rtol=1e-12, atol=1e-15)
    assert np.allclose(M, M.T, rtol=0, atol=1e-15)


def test_periodic_images_decay_like_the_screened_interaction():
    # the eight neighbour cells add O(L^-3) (wall-screened far field, Sec. II.C): doubling the
    # box divides the difference from the unbounded sheet by about 8
    pos = _box_config()[:4] - np.array([4.5, 3.75, 0.0])
    pos[:, :2] *= 0.4
    free, _ = mobility.dense(pos)
    gaps = []
    for L in (40.0, 80.0):
        M, _ = mobility.dense(pos, box=(L, L))
        gaps.append(np.abs(M - free).max())
    assert 6.0 < gaps[0] / gaps[1] < 10.5


def test_periodic_forces_use_the_minimum_image():
    from oracle import forces
    pair = np.array([[0.3, 2.0, 1.5], [BOX[0] - 0.6, 2.4, 1.7]])
    near = pair.copy()
    near[1, 0] -= BOX[0]                       # the same pair, unwrapped
    fp = forces.forces(pair, 1.0, 1.0, 0.1, -1.0, box=BOX)
    fn = forces.forces(near, 1.0, 1.0, 0.1, -1.0)
    assert np.allclose(fp, fn, rtol=1e-14, atol=1e-14)
    assert np.abs(fp[:, 0]).max() > 1.0        # they do repel


def test_periodic_image_set_is_the_nine_cell_replica():
    # App. B: a pair's hydrodynamic block is the sum over the source's minimum image and its
    # images in the eight neighbour cells (a sphere also feels its own eight images).  Built
    # here without the box option: copy every sphere into the 3 x 3 cells around the unit cell,
    # assemble the unbounded (wall) mobility of the 9N spheres, and sum each original target's
    # column blocks over the nine copies of each source.  The spheres sit in a corner of side
    # below L/2, so every pair's minimum image is the pair itself.
    box = (12.0, 10.0)
    rng = np.random.default_rng(23)
    n = 5
    pos = np.column_stack([rng.uniform(0, 5.0, n), rng.uniform(0, 4.5, n),
                           rng.uniform(1.05, 2.5, n)])
    pos[1, :2] = pos[0, :2] + [1.1, 0.7]       # an overlapping pair
    pos[2, 2] = 0.7                            # a sphere below z = a
    M, MC = mobility.dense(pos, box=box)
    cells = [(kx, ky) for kx in (-1, 0, 1) for ky in (-1, 0, 1)]
    reps = np.concatenate([pos + np.array([kx * box[0], ky * box[1], 0.0]) for kx, ky in cells])
    Mr, MCr = mobility.dense(reps)
    home = cells.index((0, 0))
    for big, small in ((Mr, M), (MCr, MC)):
        ref = big.reshape(9, n, 3, 9, n, 3)[home].sum(axis=2).reshape(3 * n, 3 * n)
        assert np.abs(small - ref).max() <= 1e-14 * np.abs(ref).max()
