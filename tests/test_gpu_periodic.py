"""Pseudo-periodic boundary conditions (App. B: forces by the minimum image convention,
hydrodynamics over the unit cell and its eight neighbour cells): GPU parity against the
oracle's box option, through the C ABI."""
import numpy as np
import pytest

from oracle import forces, integrator, mobility
from tests.gpu_util import max_element, close, dev, host, rel2, require_gpu

pytestmark = pytest.mark.gpu

BOX = (40.0, 30.0)
FP64_TOL, MIXED_TOL = 1e-12, 1e-5


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_1612_00474_amd import Context
    c = Context(0, box=BOX)
    yield c
    c.close()


def _boxed(n, seed):
    rng = np.random.default_rng(seed)
    pos = np.column_stack([rng.uniform(0, BOX[0], n), rng.uniform(0, BOX[1], n),
                           rng.uniform(1.05, 2.5, n)])
    pos[0] = [0.4, 15.0, 1.3]                  # a pair across the x edge
    pos[1] = [BOX[0] - 0.7, 15.6, 1.5]
    pos[2] = [10.0, -0.3, 1.2]                 # a pair across the y edge, one outside the box
    pos[3] = [10.5, BOX[1] + 0.5, 1.4]
    pos[4, 0] += 2 * BOX[0]                    # far outside: only its image matters
    pos[5, 2] = 0.7                            # below z = a
    return pos


@pytest.mark.parametrize("sym", [1, 0])
@pytest.mark.parametrize("n", [6, 257])
def test_periodic_product_matches_oracle(ctx, n, sym):
    pos = _boxed(n, 60 + n)
    rng = np.random.default_rng(n)
    F, T = rng.standard_normal(pos.shape), rng.standard_normal(pos.shape)
    for torque in (None, T):
        ref = mobility.dense_matvec(pos, F, torque, box=BOX)
        for precision, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL)):
            ctx.set_tuning(precision, symmetric=sym)
            u = host(ctx.matvec(dev(pos), dev(F), None if torque is None else dev(torque),
                                precision))
            assert close(u, ref, tol), (n, sym, precision, torque is None)


def test_periodic_forces_match_oracle(ctx):
    pos = _boxed(300, 9)
    ref = forces.forces(pos, 1.0, 1.0, 0.1, -1.0, box=BOX)
    f = host(ctx.forces(dev(pos), -1.0, 1.0, 0.1))
    assert close(f, ref, 1e-12)


def test_periodic_step_matches_oracle(ctx):
    from paper_1612_00474_amd import StepState
    pos = _boxed(80, 10)
    rng = np.random.default_rng(10)
    W, Wt = rng.standard_normal(pos.shape), rng.standard_normal(pos.shape)
    state = StepState(dev(pos))
    it, eps, st = ctx.sab_step(state, dt=0.01, delta=1e-4, lanczos_tol=1e-300,
                               lanczos_max_iter=6, w=dev(W), w_tilde=dev(Wt), steric_u0=1.0,
                               steric_b=0.1)
    new, u, m, _, _ = integrator.step(pos, None, W, Wt, dt=0.01, delta=1e-4,
                                      lanczos_tol=1e-300, lanczos_max_iter=6, u0=1.0, b=0.1,
                                      box=BOX)
    assert it == m == 6
    assert close(host(state.pos) - pos, new - pos, 1e-10)
    assert close(host(state.u_prev), u, 1e-12)


def test_periodic_rejections(ctx):
    from paper_1612_00474_amd import Context, RpbError
    pos = dev(_boxed(20, 11))
    F = dev(np.ones((20, 3)))
    with pytest.raises(RpbError):
        ctx.matvec_batched(pos, [0, 10, 20], F, None, "fp64")
    small = Context(0, box=(10.0, 30.0))      # 10 < 2 (2a + 40 b) = 12
    with pytest.raises(RpbError):
        small.forces(pos, -1.0, 1.0, 0.1)
    small.close()
    bad = Context(0, box=(10.0, 0.0))
    with pytest.raises(RpbError):
        bad.matvec(pos, F, None)
    bad.close()


def test_periodic_forces_small_box(ctx):
    # a box with fewer than three cells of the steric cutoff per side takes the all-pairs path
    from paper_1612_00474_amd import Context
    small_box = (14.0, 13.0)
    c = Context(0, box=small_box)
    try:
        rng = np.random.default_rng(31)
        pos = np.column_stack([rng.uniform(-3.0, 17.0, 40), rng.uniform(-2.0, 15.0, 40),
                               rng.uniform(1.05, 2.5, 40)])
        ref = forces.forces(pos, 1.0, 1.0, 0.1, -1.0, box=small_box)
        f = host(c.forces(dev(pos), -1.0, 1.0, 0.1))
        assert close(f, ref, 1e-12)
    finally:
        c.close()


def test_periodic_product_several_tiles():
    # 1,100 spheres: several 256- or 512-sphere tiles and a ragged last one, so the symmetric
    # kernel's off-diagonal tile pairs (one image loop serving both directions) are exercised
    require_gpu()
    from paper_1612_00474_amd import Context
    box = (90.0, 70.0)
    rng = np.random.default_rng(21)
    n = 1100
    pos = np.column_stack([rng.uniform(0, box[0], n), rng.uniform(0, box[1], n),
                           rng.uniform(1.05, 2.5, n)])
    pos[0] = [0.3, 35.0, 1.3]                  # pairs across both edges
    pos[n - 1] = [box[0] - 0.6, 35.4, 1.6]
    pos[1] = [20.0, 0.2, 1.2]
    pos[n - 2] = [20.5, box[1] - 0.4, 1.4]
    pos[2, 0] -= 3 * box[0]                    # far outside the box
    pos[3, 2] = 0.6                            # below z = a
    F, T = rng.standard_normal(pos.shape), rng.standard_normal(pos.shape)
    rows = np.concatenate([np.arange(6), rng.choice(n, 40, replace=False), [n - 2, n - 1]])
    c = Context(0, box=box)
    try:
        for torque in (None, T):
            ref = mobility.matvec(pos, F, torque, rows=rows, box=box)
            for precision, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL)):
                for tpt, sym in ((1, 1), (2, 1), (1, 0), (2, 0)):
                    c.set_tuning(precision, tpt=tpt, symmetric=sym)
                    u = host(c.matvec(dev(pos), dev(F), None if torque is None else dev(torque),
                                      precision))[rows]
                    err = rel2(u, ref)
                    assert err <= tol and max_element(u, ref) <= 10 * tol, (tpt, sym, precision, torque is None, err)
    finally:
        c.close()


def test_periodic_full_size_row_sampled():
    # the 65,536-sphere sheet in a box of its own side, force-only products as the benchmark
    # times them (launch shape from the tuner), against the oracle on sampled rows
    require_gpu()
    from paper_1612_00474_amd import Context
    from paper_1612_00474_amd import workloads as wl
    w = wl.WORKLOADS["sheet64k_mixed"]
    inp = wl.make_inputs(w, 0)
    box = (w.side, w.side)
    rows = np.random.default_rng(17).choice(w.n, 3, replace=False)
    rows[0] = w.n - 1
    ref = mobility.matvec(inp["pos"], inp["force"], None, rows=rows, box=box)
    c = Context(0, box=box)
    try:
        P, F = dev(inp["pos"]), dev(inp["force"])
        for precision, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL)):
            c.autotune(P, None, precision)
            err = rel2(host(c.matvec(P, F, None, precision))[rows], ref)
            print(f"periodic sheet64k {precision}: rel2 = {err:.3e} over {len(rows)} rows")
            assert err <= tol and max_element(host(c.matvec(P, F, None, precision))[rows], ref) <= 10 * tol
    finally:
        c.close()
