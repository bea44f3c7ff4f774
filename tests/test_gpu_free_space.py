"""Free-space mode (wall = 0: the unbounded RPY tensors of Sec. II.B alone, the contrast drawn
in Sec. II.C): GPU parity against the oracle's free-space option, through the C ABI."""
import math

import numpy as np
import pytest

from oracle import integrator, lanczos, mobility
from tests.gpu_util import close, dev, host, rel2, require_gpu

pytestmark = pytest.mark.gpu

FP64_TOL, MIXED_TOL = 1e-12, 1e-5


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_1612_00474_amd import Context
    c = Context(0, wall=False)
    yield c
    c.close()


def _cloud(n, seed):
    # a 3-D cloud straddling z = 0 (no wall), with overlapping pairs
    rng = np.random.default_rng(seed)
    side = (n * 4.19 / 0.2) ** (1.0 / 3.0)
    return rng.uniform(-0.5 * side, 0.5 * side, size=(n, 3))


@pytest.mark.parametrize("sym", [1, 0])
@pytest.mark.parametrize("n", [1, 7, 300, 1100])
def test_free_space_product_matches_oracle(ctx, n, sym):
    pos = _cloud(n, 40 + n)
    rng = np.random.default_rng(n)
    F, T = rng.standard_normal(pos.shape), rng.standard_normal(pos.shape)
    for torque in (None, T):
        ref = mobility.dense_matvec(pos, F, torque, wall=False)
        for precision, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL)):
            ctx.set_tuning(precision, symmetric=sym)
            u = host(ctx.matvec(dev(pos), dev(F), None if torque is None else dev(torque),
                                precision))
            assert close(u, ref, tol), (n, sym, precision, torque is None)


def test_free_space_differs_from_the_wall_product(ctx):
    from paper_1612_00474_amd import Context
    pos = _cloud(200, 3) + np.array([0.0, 0.0, 20.0])
    F = np.random.default_rng(3).standard_normal(pos.shape)
    w = Context(0)
    uw = host(w.matvec(dev(pos), dev(F), None, "fp64"))
    w.close()
    uf = host(ctx.matvec(dev(pos), dev(F), None, "fp64"))
    assert close(uf, mobility.dense_matvec(pos, F, None, wall=False), FP64_TOL)
    assert close(uw, mobility.dense_matvec(pos, F, None), FP64_TOL)
    assert rel2(uf, uw) > 1e-3


def test_free_space_lanczos_matches_dense_root(ctx):
    pos = _cloud(150, 5)
    W = np.random.default_rng(5).standard_normal(pos.shape)
    M, _ = mobility.dense(pos, wall=False)
    exact = lanczos.sqrtm_dense(M) @ W.ravel()
    g, it, eps, st = ctx.lanczos(dev(pos), dev(W), 1e-8)
    assert close(host(g).ravel(), exact, 1e-6)


def test_free_space_step_matches_oracle(ctx):
    from paper_1612_00474_amd import StepState
    pos = _cloud(120, 6)
    rng = np.random.default_rng(6)
    W, Wt = rng.standard_normal(pos.shape), rng.standard_normal(pos.shape)
    state = StepState(dev(pos))
    it, eps, st = ctx.sab_step(state, dt=0.01, delta=1e-4, lanczos_tol=1e-300,
                               lanczos_max_iter=6, w=dev(W), w_tilde=dev(Wt), steric_u0=1.0,
                               steric_b=0.1)
    new, u, m, _, _ = integrator.step(pos, None, W, Wt, dt=0.01, delta=1e-4,
                                      lanczos_tol=1e-300, lanczos_max_iter=6, u0=1.0, b=0.1,
                                      wall=False)
    assert it == m == 6
    assert close(host(state.pos) - pos, new - pos, 1e-10)
    assert close(host(state.u_prev), u, 1e-12)


def test_free_space_batched_product(ctx):
    sizes = [300, 1, 90]
    parts = [_cloud(n, 70 + n) for n in sizes]
    pos = np.vstack(parts)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    F = np.random.default_rng(7).standard_normal(pos.shape)
    for precision, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL)):
        u = host(ctx.matvec_batched(dev(pos), offs, dev(F), None, precision))
        for s in range(len(sizes)):
            a, b = offs[s], offs[s + 1]
            ref = mobility.dense_matvec(pos[a:b], F[a:b], None, wall=False)
            assert close(u[a:b], ref, tol), (s, precision)
