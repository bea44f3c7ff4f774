"""Products whose triangle of tile pairs is walked in several chunks: a context created with the
partial-sum limit forced down to 64 KiB (RPB_CHUNK_KIB) splits even small systems into many
launches, each followed by its reduction into the result.  Checked against the oracle
(Sec. II.B) and against the one-chunk products of a default context, for the single-vector
symmetric kernel at 1, 2 and 4 targets per lane (with the source parts of small systems), the
multi-vector kernel, and a time step whose first products share one launch."""
import os

import numpy as np
import pytest

from oracle import mobility
from paper_1612_00474_amd import workloads as wl
from tests.gpu_util import close, dev, host, max_element, rel2, require_gpu

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}
ORDER_TOL = {"fp64": 1e-13, "mixed": 2e-6}   # same arithmetic, another summation order


def _context(chunk_kib=None):
    from paper_1612_00474_amd import Context
    if chunk_kib is None:
        return Context(0)
    os.environ["RPB_CHUNK_KIB"] = str(chunk_kib)
    try:
        return Context(0)
    finally:
        del os.environ["RPB_CHUNK_KIB"]


@pytest.fixture(scope="module")
def ctxs():
    require_gpu()
    small, whole = _context(64), _context()
    yield small, whole
    small.close()
    whole.close()


def _config(n, seed):
    rng = np.random.default_rng(seed)
    side = np.sqrt(n * np.pi / 0.4)
    pos = np.column_stack([rng.uniform(0, side, n), rng.uniform(0, side, n),
                           rng.uniform(0.8, 2.6, n)])
    return pos, rng.standard_normal((n, 3)), rng.standard_normal((n, 3))


@pytest.mark.parametrize("n", [700, 1100, 2100])
@pytest.mark.parametrize("tpt", [1, 2, 4])
def test_chunked_symmetric_product(ctxs, n, tpt):
    small, whole = ctxs
    pos, F, T = _config(n, 10 + n + tpt)
    ref = mobility.dense_matvec(pos, F, T)
    P, Fd, Td = dev(pos), dev(F), dev(T)
    for precision in ("fp64", "mixed"):
        for c in ctxs:
            c.set_tuning(precision, tpt=tpt, symmetric=1)
        u = host(small.matvec(P, Fd, Td, precision))
        u1 = host(whole.matvec(P, Fd, Td, precision))
        print(f"n={n} tpt={tpt} {precision}: chunked vs oracle {rel2(u, ref):.2e} "
              f"({max_element(u, ref):.2e}), vs one chunk {rel2(u, u1):.2e}")
        assert close(u, ref, TOL[precision]), (n, tpt, precision)
        assert close(u, u1, ORDER_TOL[precision]), (n, tpt, precision)
        assert np.array_equal(u, host(small.matvec(P, Fd, Td, precision)))   # reproducible


@pytest.mark.parametrize("n", [300, 700])
def test_chunked_multi_vector_product(ctxs, n):
    small, whole = ctxs
    pos, _, _ = _config(n, 50 + n)
    FF = np.random.default_rng(n).standard_normal((5, n, 3))
    M, _ = mobility.dense(pos)
    ref = np.stack([(M @ f.ravel()).reshape(n, 3) for f in FF])
    for precision in ("fp64", "mixed"):
        u = host(small.matvec_multi(dev(pos), dev(FF), precision))
        u1 = host(whole.matvec_multi(dev(pos), dev(FF), precision))
        for v in range(len(FF)):
            assert close(u[v], ref[v], TOL[precision]), (n, precision, v)
        assert close(u, u1, ORDER_TOL[precision]), (n, precision)


@pytest.mark.parametrize("precision,tol_u,tol_x", [("fp64", 1e-12, 1e-10), ("mixed", 1e-5, 1e-5)])
def test_chunked_step_products(ctxs, precision, tol_u, tol_x):
    # M F + M_C T and the first Lanczos product M W in one launch, walked in chunks
    from oracle import integrator
    from paper_1612_00474_amd import StepState
    small, _ = ctxs
    pos = wl.sheet(700, phi=0.4, seed=4)
    rng = np.random.default_rng(12)
    W, Wt = rng.standard_normal(pos.shape), rng.standard_normal(pos.shape)
    kw = dict(f_grav_z=-1.0, torque=(0.0, 1.0, 0.0))
    state = StepState(dev(pos))
    it, eps, st = small.sab_step(state, dt=0.01, delta=1e-4, lanczos_tol=1e-300,
                                 lanczos_max_iter=6, precision=precision, rfd_precision="fp64",
                                 w=dev(W), w_tilde=dev(Wt), steric_u0=1.0, steric_b=0.1, **kw)
    new, u, m, _, _ = integrator.step(pos, None, W, Wt, dt=0.01, delta=1e-4, lanczos_tol=1e-300,
                                      lanczos_max_iter=6, **kw)
    assert it == m == 6
    assert close(host(state.u_prev), u, tol_u)
    assert close(host(state.pos) - pos, new - pos, tol_x)
