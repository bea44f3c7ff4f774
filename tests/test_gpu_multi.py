"""GPU parity of the multi-vector product and the multi-vector Lanczos solve against the FP64
oracle (through the C ABI): U_v = M F_v for several vectors of one configuration, and one
Lanczos process per vector."""
import math

import numpy as np
import pytest

from oracle import lanczos, mobility
from paper_1612_00474_amd import workloads as wl
from tests.gpu_util import max_element, close, dev, host, rel2, require_gpu

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12     # relative 2-norm, float64 path
MIXED_TOL = 1e-5     # relative 2-norm, float32 pair terms


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_1612_00474_amd import Context
    c = Context(0)
    yield c
    c.close()


def suspension(n, seed, wall=True):
    rng = np.random.default_rng(seed)
    side = max(2.0, math.sqrt(n * math.pi / 0.4))
    z = rng.uniform(0.8, 2.6, n) if wall else rng.uniform(-3.0, 3.0, n)
    return np.column_stack([rng.uniform(0, side, n), rng.uniform(0, side, n), z])


@pytest.mark.parametrize("wall", [True, False])
@pytest.mark.parametrize("n,nvec", [(1, 1), (2, 3), (65, 4), (256, 5), (300, 2), (700, 9)])
def test_multi_matches_oracle_per_vector(ctx, n, nvec, wall):
    # several tiles with a ragged last one, partial 64-source blocks, vector counts that leave
    # zero-padded slots in the last launch
    from paper_1612_00474_amd import Context
    c = ctx if wall else Context(0, wall=False)
    pos = suspension(n, 10 + n, wall)
    F = np.random.default_rng(20 + n).standard_normal((nvec, n, 3))
    M, _ = mobility.dense(pos, wall=wall)
    ref = np.stack([(M @ F[v].ravel()).reshape(n, 3) for v in range(nvec)])
    P, Fd = dev(pos), dev(F)
    for precision, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL)):
        u = host(c.matvec_multi(P, Fd, precision))
        for v in range(nvec):
            assert close(u[v], ref[v], tol), (precision, n, v)
        # agrees with the single-vector product to rounding
        one = np.stack([host(c.matvec(P, dev(F[v]), None, precision)) for v in range(nvec)])
        assert close(u, one, (1e-13 if precision == "fp64" else 2e-6))
        assert np.array_equal(u, host(c.matvec_multi(P, Fd, precision)))   # reproducible
    if not wall:
        c.close()


def test_multi_overlaps_and_self_pairs(ctx):
    # overlapping and coincident (clamped) spheres take the complete pair form, the self pair
    # r = 0 included, inside the diagonal tiles and across tiles
    from tests.gpu_util import awkward_config
    pos = np.concatenate([awkward_config(200, 5), awkward_config(100, 6) + [0.5, 0.5, 0.0]])
    n = len(pos)
    F = np.random.default_rng(3).standard_normal((3, n, 3))
    M, _ = mobility.dense(pos)
    u = host(ctx.matvec_multi(dev(pos), dev(F), "fp64"))
    for v in range(3):
        assert close(u[v], (M @ F[v].ravel()).reshape(n, 3), FP64_TOL)


def test_multi_full_size_row_sampled(ctx):
    # N = 65,536 sheet, four vectors in one launch: sampled rows against the oracle
    w = wl.WORKLOADS["sheet64k_mixed"]
    inp = wl.make_inputs(w, 0)
    rng = np.random.default_rng(31)
    F = rng.standard_normal((4, w.n, 3))
    rows = rng.choice(w.n, 12, replace=False)
    rows[0] = w.n - 1
    P, Fd = dev(inp["pos"]), dev(F)
    for precision, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL)):
        u = host(ctx.matvec_multi(P, Fd, precision))
        for v in range(4):
            ref = mobility.matvec(inp["pos"], F[v], None, rows=rows)
            err = rel2(u[v][rows], ref)
            print(f"multi N=65536 {precision} vector {v}: rel2 = {err:.3e} over 12 rows")
            assert err <= tol and max_element(u[v][rows], ref) <= 10 * tol


def test_multi_error_paths(ctx):
    import torch
    from paper_1612_00474_amd import Context
    from paper_1612_00474_amd._lib import RPB_EINVAL, RPB_ENONFINITE, RpbError
    pos = suspension(40, 1)
    P, F = dev(pos), dev(np.ones((2, 40, 3)))
    with pytest.raises(RpbError) as e:
        ctx.matvec_multi(P, F, out=F)
    assert e.value.status == RPB_EINVAL
    bad = P.clone()
    bad[3, 2] = float("inf")
    with pytest.raises(RpbError) as e:
        ctx.matvec_multi(bad, F)
    assert e.value.status == RPB_ENONFINITE
    with pytest.raises(RpbError) as e:
        ctx.lanczos_multi(P, F, 1e-6, max_iter=0)
    assert e.value.status == RPB_EINVAL
    boxed = Context(0, box=(20.0, 20.0))
    try:
        with pytest.raises(RpbError) as e:
            boxed.matvec_multi(P, F)
        assert e.value.status == RPB_EINVAL
        with pytest.raises(RpbError) as e:
            boxed.lanczos_multi(P, F, 1e-6)
        assert e.value.status == RPB_EINVAL
    finally:
        boxed.close()
    none = torch.empty((0, 40, 3), dtype=torch.float64, device="cuda")
    assert ctx.matvec_multi(P, none).shape == (0, 40, 3)
    empty = torch.empty((0, 3), dtype=torch.float64, device="cuda")
    assert ctx.matvec_multi(empty, torch.empty((2, 0, 3), dtype=torch.float64,
                                               device="cuda")).shape == (2, 0, 3)


@pytest.fixture(scope="module")
def c1():
    inp = wl.make_inputs(wl.WORKLOADS["sheet256_rsa"], 0)
    M, _ = mobility.dense(inp["pos"])
    return inp, M


@pytest.mark.parametrize("m", [1, 3, 8])
def test_lanczos_multi_fixed_iterations(ctx, c1, m):
    inp, M = c1
    n = len(inp["pos"])
    W = np.random.default_rng(41).standard_normal((6, n, 3))
    g, it, eps, st = ctx.lanczos_multi(dev(inp["pos"]), dev(W), 1e-300, max_iter=m,
                                       allow_noconv=True)
    g = host(g)
    for v in range(6):
        ref, mref, _, _ = lanczos.lanczos_sqrt(lambda x: M @ x, W[v].ravel(), 1e-300, max_iter=m)
        assert it[v] == m == mref
        assert close(g[v].ravel(), ref, 1e-12)


def test_lanczos_multi_tolerance_per_vector(ctx, c1):
    # each process stops on its own test: iteration counts and eps as the oracle's, results
    # within the tolerance of the dense root; a scaled copy of a vector converges alike
    inp, M = c1
    n = len(inp["pos"])
    W = np.random.default_rng(42).standard_normal((5, n, 3))
    W[4] = 3.0 * W[0]
    W[3] = 0.0
    W[3, 7] = [1.0, 0.0, 0.0]          # one sphere only: few iterations
    root = lanczos.sqrtm_dense(M)
    P = dev(inp["pos"])
    for precision in ("fp64", "mixed"):
        g, it, eps, st = ctx.lanczos_multi(P, dev(W), 1e-6, precision=precision)
        g = host(g)
        for v in range(5):
            _, mref, eps_ref, _ = lanczos.lanczos_sqrt(lambda x: M @ x, W[v].ravel(), 1e-6)
            err = rel2(g[v].ravel(), root @ W[v].ravel())
            print(f"lanczos multi {precision} v{v}: m = {it[v]} (oracle {mref}), err {err:.2e}")
            assert err <= 1e-5 and max_element(g[v].ravel(), root @ W[v].ravel()) <= 10 * 1e-5
            if precision == "fp64":
                assert it[v] == mref and abs(eps[v] - eps_ref) <= 1e-9 * max(eps_ref, 1e-30)
        # each vector's result as the single-vector solve
        if precision == "fp64":
            assert it[4] == it[0]
            for v in range(5):
                one, m1, _, _ = ctx.lanczos(P, dev(W[v]), 1e-6)
                assert m1 == it[v]
                assert close(g[v], host(one), 1e-12)
