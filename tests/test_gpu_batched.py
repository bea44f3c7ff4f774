"""GPU parity of the batched (persistent-launch) products, Lanczos, step and hipGraph step."""
import numpy as np
import pytest

from oracle import integrator, lanczos, mobility
from paper_1612_00474_amd import workloads as wl
from tests.gpu_util import close, dev, host, rel2, require_gpu

pytestmark = pytest.mark.gpu

SIZES = [300, 1, 0, 7, 700, 256, 1100]     # includes an empty system and ragged tiles


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_1612_00474_amd import Context
    c = Context(0)
    yield c
    c.close()


def _batch(sizes=SIZES, seed=0):
    rng = np.random.default_rng(seed)
    parts = [wl.sample_positions(n, wl.side_for_area_fraction(max(n, 1), 0.4), 1.1, 2.5, rng=rng)
             if n else np.zeros((0, 3)) for n in sizes]
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    pos = np.vstack(parts)
    return pos, offs, rng


@pytest.mark.parametrize("sym,btpt", [(1, 1), (1, 2), (0, 1), (0, 2)])
@pytest.mark.parametrize("torque", [False, True])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_batched_product_matches_oracle_per_system(ctx, precision, tol, torque, sym, btpt):
    # symmetric (system, tile pair) items and ordered (system, target tile, source chunk) items
    from paper_1612_00474_amd import Context
    c = Context(0)
    c.set_tuning(precision, batch_symmetric=sym, batch_tpt=btpt, batch_chunk=256, batch_wgs=64)
    pos, offs, rng = _batch()
    F = rng.standard_normal(pos.shape)
    T = rng.standard_normal(pos.shape) if torque else None
    u = host(c.matvec_batched(dev(pos), offs, dev(F), dev(T) if torque else None, precision))
    for s in range(len(SIZES)):
        a, b = offs[s], offs[s + 1]
        if a == b:
            continue
        ref = mobility.dense_matvec(pos[a:b], F[a:b], None if T is None else T[a:b])
        assert close(u[a:b], ref, tol), (s, precision)
    c.close()


def test_batched_equals_single_calls(ctx):
    pos, offs, rng = _batch(seed=1)
    F = rng.standard_normal(pos.shape)
    P, Fd = dev(pos), dev(F)
    for precision in ("fp64", "mixed"):
        ub = host(ctx.matvec_batched(P, offs, Fd, None, precision))
        for s in range(len(SIZES)):
            a, b = offs[s], offs[s + 1]
            if a == b:
                continue
            us = host(ctx.matvec(dev(pos[a:b]), dev(F[a:b]), None, precision))
            assert close(ub[a:b], us, (1e-14 if precision == "fp64" else 1e-6))


def test_batched_lanczos_fixed_m(ctx):
    pos, offs, rng = _batch([40, 130, 7], seed=2)
    W = rng.standard_normal(pos.shape)
    g, it, eps, st = ctx.lanczos_batched(dev(pos), offs, dev(W), 1e-300, max_iter=6, allow_noconv=True)
    g = host(g)
    for s in range(3):
        a, b = offs[s], offs[s + 1]
        M, _ = mobility.dense(pos[a:b])
        ref, m, _, _ = lanczos.lanczos_sqrt(lambda v: M @ v, W[a:b].ravel(), 1e-300, max_iter=6)
        assert it[s] == m
        assert close(g[a:b].ravel(), ref, 1e-12)


def test_batched_lanczos_tolerance_per_system(ctx):
    pos, offs, rng = _batch([60, 200, 1, 90], seed=3)
    W = rng.standard_normal(pos.shape)
    g, it, eps, st = ctx.lanczos_batched(dev(pos), offs, dev(W), 1e-6)
    g = host(g)
    for s in range(4):
        a, b = offs[s], offs[s + 1]
        M, _ = mobility.dense(pos[a:b])
        _, m, _, _ = lanczos.lanczos_sqrt(lambda v: M @ v, W[a:b].ravel(), 1e-6)
        exact = lanczos.sqrtm_dense(M) @ W[a:b].ravel()
        assert it[s] == m, (s, it, m)
        assert close(g[a:b].ravel(), exact, 1e-5)


def test_batched_step_matches_oracle(ctx):
    pos, offs, rng = _batch([50, 120, 33], seed=4)
    W, Wt = rng.standard_normal(pos.shape), rng.standard_normal(pos.shape)
    P = dev(pos)
    U = dev(np.zeros_like(pos))
    it, eps, st = ctx.sab_step_batched(P, U, offs, 0, False, dt=0.01, delta=1e-4, lanczos_tol=1e-300,
                                       lanczos_max_iter=6, w=dev(W), w_tilde=dev(Wt),
                                       steric_u0=1.0, steric_b=0.1)
    got = host(P)
    for s in range(3):
        a, b = offs[s], offs[s + 1]
        new, u, m, _, _ = integrator.step(pos[a:b], None, W[a:b], Wt[a:b], dt=0.01, delta=1e-4,
                                          lanczos_tol=1e-300, lanczos_max_iter=6, u0=1.0, b=0.1)
        assert it[s] == m == 6
        assert close(got[a:b] - pos[a:b], new - pos[a:b], 1e-10)
        assert close(host(U)[a:b], u, 1e-12)


@pytest.mark.parametrize("precision,tol_u,tol_x", [("fp64", 1e-12, 1e-10), ("mixed", 1e-5, 1e-5)])
def test_batched_step_over_several_tiles(ctx, precision, tol_u, tol_x):
    # systems of several 256-sphere tiles (ragged), an empty and a one-sphere system: the joint
    # persistent launch of M F + M_C T (rollers' torque) and the first Lanczos product M W
    sizes = [300, 0, 700, 1, 257]
    pos, offs, rng = _batch(sizes, seed=6)
    W, Wt = rng.standard_normal(pos.shape), rng.standard_normal(pos.shape)
    P, U = dev(pos), dev(np.zeros_like(pos))
    phys = dict(f_grav_z=-1.0, torque=(0.0, 1.0, 0.0))
    it, eps, st = ctx.sab_step_batched(P, U, offs, 0, False, dt=0.01, delta=1e-4,
                                       lanczos_tol=1e-300, lanczos_max_iter=6, w=dev(W),
                                       w_tilde=dev(Wt), steric_u0=1.0, steric_b=0.1,
                                       precision=precision, rfd_precision="fp64", **phys)
    got, gu = host(P), host(U)
    for s in range(len(sizes)):
        a, b = offs[s], offs[s + 1]
        if a == b:
            continue
        new, u, m, _, _ = integrator.step(pos[a:b], None, W[a:b], Wt[a:b], dt=0.01, delta=1e-4,
                                          lanczos_tol=1e-300, lanczos_max_iter=6, u0=1.0, b=0.1,
                                          **phys)
        # float32 products cannot show the exact breakdown (beta ~ 1e-14 max|alpha|) of the
        # one-sphere system, whose Krylov space is exhausted after its 3 dimensions
        assert it[s] == m if precision == "fp64" else it[s] <= 6
        assert close(gu[a:b], u, tol_u), (s, precision)
        assert close(got[a:b] - pos[a:b], new - pos[a:b], tol_x), (s, precision)


def test_graph_replays_match_eager_steps(ctx):
    import torch
    pos, offs, rng = _batch([200, 900, 31, 450], seed=5)
    kw = dict(dt=0.01, delta=1e-4, lanczos_tol=1e-4, lanczos_max_iter=12, seed=7,
              steric_u0=1.0, steric_b=0.1, precision="mixed")
    Pg, Ug = dev(pos), dev(np.zeros_like(pos))
    Pe, Ue = dev(pos), dev(np.zeros_like(pos))
    graph = ctx.step_graph(Pg, Ug, offs, 0, False, **kw)
    assert np.array_equal(host(Pg), pos)           # creation does not advance the state
    other = dev(rng.standard_normal((500, 3)))
    for k in range(4):
        graph.launch()
        torch.cuda.synchronize()
        # eager work of the program between the replays
        ctx.matvec(other, other, None, "fp64")
        torch.cuda.synchronize()
        ite, epse, _ = ctx.sab_step_batched(Pe, Ue, offs, k, k > 0, **kw)
        step, itg, epsg, _ = graph.status()
        assert step == k + 1
        assert np.array_equal(itg, ite)
        assert np.array_equal(host(Pg), host(Pe)), k
        assert np.array_equal(host(Ug), host(Ue)), k
    graph.close()


def test_uneven_batch_rows_sampled(ctx):
    # the 64-suspension workload: check a few rows of a few systems against the oracle
    w = wl.WORKLOADS["batch64_uneven"]
    pos, offs = wl.make_batch(w, 0)
    rng = np.random.default_rng(6)
    F = rng.standard_normal(pos.shape)
    u = host(ctx.matvec_batched(dev(pos), offs, dev(F), None, "mixed"))
    for s in (0, 17, 63):
        a, b = offs[s], offs[s + 1]
        rows = rng.choice(b - a, 8, replace=False)
        ref = mobility.matvec(pos[a:b], F[a:b], None, rows=rows)
        assert close(u[a:b][rows], ref, 1e-5)


def test_autotune_picks_a_candidate_and_keeps_parity(ctx):
    from paper_1612_00474_amd import Context
    c = Context(0)
    pos = wl.sheet(3000, seed=8)
    rng = np.random.default_rng(8)
    F = rng.standard_normal(pos.shape)
    P, Fd = dev(pos), dev(F)
    shape, ms = c.autotune(P, None, "mixed", reps=1)
    assert shape["tpt"] in (1, 2) and shape["target_wgs"] in (2048, 4096, 8192, 16384) and ms > 0
    shape2, ms2 = c.autotune(P, None, "mixed", reps=1)      # cached: no timing
    assert shape2 == shape and ms2 == -1.0
    ref = mobility.matvec(pos, F, None, rows=np.arange(0, 3000, 50))
    assert close(host(c.matvec(P, Fd, None, "mixed"))[::50], ref, 1e-5)
    pos_b, offs, _ = _batch(seed=9)
    shape_b, _ = c.autotune(dev(pos_b), offs, "fp64", reps=1)
    assert shape_b["batch_chunk"] in (512, 1024, 2048) and shape_b["batch_wgs"] in (1024, 2048, 4096)
    Fb = rng.standard_normal(pos_b.shape)
    u = host(c.matvec_batched(dev(pos_b), offs, dev(Fb), None, "fp64"))
    a, b = offs[4], offs[5]
    assert close(u[a:b], mobility.dense_matvec(pos_b[a:b], Fb[a:b], None), 1e-12)
    c.close()
