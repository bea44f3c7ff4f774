"""Sphere radius and viscosity other than 1: the kernels work in units of a (the packed
lengths divided by a, the torques by a, each result by 8 pi eta a), so every path is checked
against the oracle at a = 0.8, eta = 1.3 (through the C ABI)."""
import math

import numpy as np
import pytest

from oracle import forces, integrator, mobility
from paper_1612_00474_amd import workloads as wl
from tests.gpu_util import close, dev, host, rel2, require_gpu

pytestmark = pytest.mark.gpu

A, ETA = 0.8, 1.3
FP64_TOL, MIXED_TOL = 1e-12, 1e-5


def _sheet(n, seed, wall=True):
    rng = np.random.default_rng(seed)
    side = A * max(2.0, math.sqrt(n * math.pi / 0.4))
    z = rng.uniform(0.7 * A, 2.6 * A, n) if wall else rng.uniform(-3.0, 3.0, n)
    return np.column_stack([rng.uniform(0, side, n), rng.uniform(0, side, n), z])


@pytest.mark.parametrize("wall", [True, False])
@pytest.mark.parametrize("n", [300, 700])
def test_products_at_other_radius(n, wall):
    require_gpu()
    from paper_1612_00474_amd import Context
    c = Context(0, a=A, eta=ETA, wall=wall)
    try:
        pos = _sheet(n, 70 + n, wall)
        rng = np.random.default_rng(n)
        F, T = rng.standard_normal(pos.shape), rng.standard_normal(pos.shape)
        ref = mobility.dense_matvec(pos, F, T, a=A, eta=ETA, wall=wall)
        for precision, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL)):
            for sym in (1, 0):
                c.set_tuning(precision, symmetric=sym)
                u = host(c.matvec(dev(pos), dev(F), dev(T), precision))
                assert close(u, ref, tol), (precision, sym)
            FF = np.stack([F, T])
            um = host(c.matvec_multi(dev(pos), dev(FF), precision))
            for v in range(2):
                refv = mobility.dense_matvec(pos, FF[v], None, a=A, eta=ETA, wall=wall)
                assert close(um[v], refv, tol)
    finally:
        c.close()


def test_periodic_product_at_other_radius():
    require_gpu()
    from paper_1612_00474_amd import Context
    box = (30.0, 24.0)
    c = Context(0, a=A, eta=ETA, box=box)
    try:
        rng = np.random.default_rng(5)
        pos = np.column_stack([rng.uniform(-2, 32, 200), rng.uniform(-2, 26, 200),
                               rng.uniform(0.9, 2.0, 200)])
        F, T = rng.standard_normal(pos.shape), rng.standard_normal(pos.shape)
        ref = mobility.dense_matvec(pos, F, T, a=A, eta=ETA, box=box)
        for precision, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL)):
            assert close(host(c.matvec(dev(pos), dev(F), dev(T), precision)), ref, tol)
        fref = forces.forces(pos, A, 1.0, 0.1, -1.0, box=box)
        assert close(host(c.forces(dev(pos), -1.0, 1.0, 0.1)), fref, 1e-12)
    finally:
        c.close()


def test_step_at_other_radius():
    # the step's two-vector launch (M F + M_C T with the rollers' torque, and M W), the
    # Lanczos solve, the RFD and the forces at a = 0.8
    require_gpu()
    from paper_1612_00474_amd import Context, StepState
    c = Context(0, a=A, eta=ETA, kT=1.0)
    try:
        n = 600
        w = wl.Workload("r", n, A * wl.side_for_area_fraction(n, 0.4), 1.1 * A, 2.5 * A)
        pos = wl.make_inputs(w, 3)["pos"]
        rng = np.random.default_rng(4)
        W, Wt = rng.standard_normal(pos.shape), rng.standard_normal(pos.shape)
        state = StepState(dev(pos))
        kw = dict(dt=0.01, delta=1e-4, lanczos_tol=1e-300, lanczos_max_iter=8)
        it, eps, st = c.sab_step(state, w=dev(W), w_tilde=dev(Wt), steric_u0=1.0, steric_b=0.1,
                                 f_grav_z=-1.0, torque=(0.0, 1.0, 0.0), **kw)
        new, u, m, _, _ = integrator.step(pos, None, W, Wt, u0=1.0, b=0.1, f_grav_z=-1.0,
                                          torque=(0.0, 1.0, 0.0), a=A, eta=ETA, **kw)
        assert it == m == 8
        assert close(host(state.u_prev), u, 1e-12)
        assert close(host(state.pos) - pos, new - pos, 1e-10)
    finally:
        c.close()
