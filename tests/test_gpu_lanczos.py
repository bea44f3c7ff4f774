"""GPU parity of lanczos_sqrt_apply against the FP64 oracle (through the C ABI)."""
import math

import numpy as np
import pytest

from oracle import lanczos, mobility
from paper_1612_00474_amd import workloads as wl
from tests.gpu_util import max_element, close, dev, host, rel2, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_1612_00474_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c1():
    inp = wl.make_inputs(wl.WORKLOADS["sheet256_rsa"], 0)
    M, _ = mobility.dense(inp["pos"])
    return inp, M


def _close(got, ref, tol, what=""):
    """Relative 2-norm within tol and every element within 10 tol of the largest."""
    err = rel2(got, ref)
    emax = float(np.abs(np.asarray(got) - ref).max() / np.abs(ref).max())
    print(f"{what}: rel2 {err:.2e}, max element {emax:.2e}")
    assert err <= tol and emax <= 10 * tol, what


@pytest.mark.parametrize("m", [1, 2, 5, 9, 24, 48, 64])
def test_fixed_iterations_fp64(ctx, c1, m):
    # up to the largest Krylov space the device eigensolve takes (64)
    inp, M = c1
    w = inp["w"]
    ref, mref, _, _ = lanczos.lanczos_sqrt(lambda v: M @ v, w.ravel(), 1e-300, max_iter=m)
    g, it, eps, st = ctx.lanczos(dev(inp["pos"]), dev(w), 1e-300, max_iter=m, allow_noconv=True)
    assert it == m == mref
    _close(host(g).ravel(), ref, 1e-12, f"sheet256 m={m}")


@pytest.fixture(scope="module")
def multi_tile():
    # 1,100 spheres: three tiles of the symmetric kernel (the last one ragged), so every
    # product of the solve runs the off-diagonal tile pairs and the lane rotation
    pos = wl.sheet(1100, phi=0.4, seed=11)
    M, _ = mobility.dense(pos)
    w = np.random.default_rng(12).standard_normal((1100, 3))
    return pos, M, w


@pytest.mark.parametrize("m", [5, 16, 40])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_fixed_iterations_several_tiles(ctx, multi_tile, m, precision, tol):
    pos, M, w = multi_tile
    ref, mref, _, _ = lanczos.lanczos_sqrt(lambda v: M @ v, w.ravel(), 1e-300, max_iter=m)
    g, it, eps, st = ctx.lanczos(dev(pos), dev(w), 1e-300, max_iter=m, precision=precision,
                                 allow_noconv=True)
    assert it == m == mref
    _close(host(g).ravel(), ref, tol, f"n=1100 {precision} m={m}")


def test_spheres_below_the_wall_exhaust_the_krylov_space(ctx):
    # spheres at or below the wall have zero rows and columns (App. A), so M has the eigenvalue
    # 0 and the Krylov space of w is the live subspace plus one direction: the solve ends in a
    # breakdown (invariant space, exact result) once those 3 x 8 + 1 directions are spanned
    # (one iteration later when the last beta is rounding noise just above the threshold)
    rng = np.random.default_rng(31)
    live = np.column_stack([rng.uniform(0, 9, 8), rng.uniform(0, 9, 8), rng.uniform(1.1, 2.5, 8)])
    dead = np.column_stack([rng.uniform(0, 9, 4), rng.uniform(0, 9, 4), rng.uniform(-1.0, 0.0, 4)])
    pos = np.vstack([live, dead])
    M, _ = mobility.dense(pos)
    w = rng.standard_normal((12, 3))
    ref, mref, _, status = lanczos.lanczos_sqrt(lambda v: M @ v, w.ravel(), 1e-300, 64)
    assert status == "breakdown" and mref <= 26
    exact = lanczos.sqrtm_dense(M) @ w.ravel()
    assert close(ref, exact, 1e-7)
    g, it, eps, st = ctx.lanczos(dev(pos), dev(w), 1e-300, 64)
    assert st == 0 and 25 <= it <= 26
    _close(host(g).ravel(), exact, 1e-7, "below-wall breakdown")
    # at a fixed m before the space is exhausted: a Ritz value converges to the eigenvalue 0
    # at rounding level eps lambda_max within a few iterations, and the square root is not
    # Lipschitz at 0, so it contributes ~(eps lambda_max)^{1/2} ~ 1e-8 |g| on either side with
    # its own rounding: the two agree to ~sqrt(u), not to u, in this degenerate case
    ref20 = lanczos.lanczos_sqrt(lambda v: M @ v, w.ravel(), 1e-300, 20)[0]
    g20 = ctx.lanczos(dev(pos), dev(w), 1e-300, 20, allow_noconv=True)[0]
    _close(host(g20).ravel(), ref20, 1e-7, "below-wall m=20")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-7), ("mixed", 1e-5)])
def test_two_identical_clusters_far_apart(ctx, precision, tol):
    # two copies of one cluster 5,000 radii apart: the coupling is screened to ~1e-12, so M has
    # nearly double eigenvalues and T_m nearly degenerate Ritz pairs in the eigensolve
    rng = np.random.default_rng(41)
    a = np.column_stack([rng.uniform(0, 8, 10), rng.uniform(0, 8, 10), rng.uniform(1.1, 2.5, 10)])
    pos = np.vstack([a, a + np.array([5000.0, 0.0, 0.0])])
    M, _ = mobility.dense(pos)
    w = rng.standard_normal((20, 3))
    exact = lanczos.sqrtm_dense(M) @ w.ravel()
    g, it, eps, st = ctx.lanczos(dev(pos), dev(w), 1e-9, 64, precision=precision)
    print(f"clusters {precision}: m = {it}, eps = {eps:.2e}, status {st}")
    _close(host(g).ravel(), exact, tol, f"clusters {precision}")


def test_tolerance_run_matches_dense_root(ctx, c1):
    inp, M = c1
    w = inp["w"].ravel()
    _, mref, eps_ref, _ = lanczos.lanczos_sqrt(lambda v: M @ v, w, 1e-6)
    exact = lanczos.sqrtm_dense(M) @ w
    for precision in ("fp64", "mixed"):
        g, it, eps, st = ctx.lanczos(dev(inp["pos"]), dev(inp["w"]), 1e-6, precision=precision)
        err = rel2(host(g).ravel(), exact)
        print(f"lanczos {precision}: m = {it} (oracle {mref}), eps = {eps:.2e}, err vs dense root {err:.2e}")
        assert err <= 1e-5 and max_element(host(g).ravel(), exact) <= 10 * 1e-5
        if precision == "fp64":
            assert it == mref and abs(eps - eps_ref) <= 1e-9 * eps_ref


def test_single_sphere_is_exact(ctx):
    pos = np.array([[0.1, 0.2, 1.8]])
    w = np.array([[0.7, -1.2, 0.4]])
    h = 1.8
    mu_par = 1 - 9 / (16 * h) + 1 / (8 * h ** 3) - 1 / (16 * h ** 5)
    mu_perp = 1 - 9 / (8 * h) + 1 / (2 * h ** 3) - 1 / (8 * h ** 5)
    ref = np.sqrt(np.array([mu_par, mu_par, mu_perp]) / (6 * math.pi)) * w[0]
    g, it, eps, st = ctx.lanczos(dev(pos), dev(w), 1e-10)
    assert it <= 2
    assert np.abs(host(g)[0] - ref).max() <= 1e-14 * np.abs(ref).max()


def test_no_convergence_status(ctx, c1):
    from paper_1612_00474_amd._lib import RPB_ENOCONV, RpbError
    inp, _ = c1
    with pytest.raises(RpbError) as e:
        ctx.lanczos(dev(inp["pos"]), dev(inp["w"]), 1e-12, max_iter=3)
    assert e.value.status == RPB_ENOCONV
    g, it, eps, st = ctx.lanczos(dev(inp["pos"]), dev(inp["w"]), 1e-12, max_iter=3, allow_noconv=True)
    assert st == RPB_ENOCONV and it == 3 and eps > 1e-12


def test_full_size_properties(ctx):
    # N = 16,384 (time-stepping sheet): the wall screens the interactions, so the tolerance
    # 1e-3 is met in a few iterations (Sec. II.C); |g|^2 = w^T M w for the symmetric root.
    inp = wl.make_inputs(wl.WORKLOADS["sheet16k_fp64"], 0)
    P, W = dev(inp["pos"]), dev(inp["w"])
    g, it, eps, st = ctx.lanczos(P, W, 1e-3)
    Mw = host(ctx.matvec(P, W, None, "fp64"))
    g = host(g)
    wMw = float(np.sum(inp["w"] * Mw))
    print(f"sheet16k: m = {it}, eps = {eps:.2e}, |g|^2 / w.Mw - 1 = {float(np.sum(g * g)) / wMw - 1:.2e}")
    assert it <= 12 and eps < 1e-3
    assert abs(float(np.sum(g * g)) / wMw - 1.0) <= 1e-3
    # mixed and float64 agree at a fixed number of iterations
    g64 = host(ctx.lanczos(P, W, 1e-300, max_iter=6, allow_noconv=True)[0])
    g32 = host(ctx.lanczos(P, W, 1e-300, max_iter=6, precision="mixed", allow_noconv=True)[0])
    assert close(g32, g64, 1e-5)


@pytest.mark.parametrize("m", [1, 3, 7])
def test_preconditioned_fixed_iterations_fp64(ctx, c1, m):
    # square-root preconditioning: Lanczos on B = L^-1 M L^-1, result L B^{1/2} w
    inp, M = c1
    pos = inp["pos"].copy()
    pos[5, 2] = 0.7                      # one sphere below z = a (H < 1 scales its L)
    Mp, _ = mobility.dense(pos)
    L = lanczos.block_diagonal_scale(pos)
    w = inp["w"]
    ref, mref, _, _ = lanczos.lanczos_sqrt_precond(lambda v: Mp @ v, L, w.ravel(), 1e-300, m)
    g, it, eps, st = ctx.lanczos(dev(pos), dev(w), 1e-300, max_iter=m, allow_noconv=True,
                                 precond=True)
    assert it == m == mref
    assert close(host(g).ravel(), ref, 1e-12)


def test_preconditioned_tolerance_run_is_a_root_of_m(ctx, c1):
    inp, M = c1
    L = lanczos.block_diagonal_scale(inp["pos"])
    S = L[:, None] * lanczos.sqrtm_dense(M / np.outer(L, L))      # S S^T = M
    w = inp["w"].ravel()
    for precision, tol in (("fp64", 1e-5), ("mixed", 1e-4)):
        g, it, eps, st = ctx.lanczos(dev(inp["pos"]), dev(inp["w"]), 1e-6, precision=precision,
                                     precond=True)
        assert close(host(g).ravel(), S @ w, tol), precision


@pytest.mark.parametrize("precond", [False, True])
def test_stop_read_one_iteration_late_changes_nothing(ctx, c1, precond):
    # The solve enqueues one iteration past its stop before the host reads the stop flag; that
    # iteration must leave the result alone and must not count as a pair-kernel launch.  A run
    # capped at the same m never enqueues past its last iteration, so the two agree bitwise.
    import torch
    inp, _ = c1
    P, W = dev(inp["pos"]), dev(inp["w"])
    for precision in ("fp64", "mixed"):
        torch.cuda.synchronize()
        ctx.timing(True)
        ctx.timing_read()
        g, it, eps, st = ctx.lanczos(P, W, 1e-6, precision=precision, precond=precond)
        _, launches, _ = ctx.timing_read()
        ctx.timing(False)
        assert 2 <= it < 64
        assert launches == it, (precision, it, launches)
        capped, it2, eps2, _ = ctx.lanczos(P, W, 1e-6, max_iter=it, precision=precision,
                                           precond=precond)
        assert it2 == it and eps2 == eps
        assert torch.equal(g, capped), precision
        # back to back: the previous solve's last status copy cannot leak into this one
        again, it3, eps3, _ = ctx.lanczos(P, W, 1e-6, precision=precision, precond=precond)
        assert it3 == it and eps3 == eps and torch.equal(g, again)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-4)])
def test_not_spd_is_reported(precision, tol):
    # a crowded pseudo-periodic configuration whose truncated image sum is indefinite (App. B):
    # RPB_ENOTSPD at the oracle's iteration, with the last iterate (built from the non-negative
    # part of the Ritz spectrum) in the output
    require_gpu()
    from paper_1612_00474_amd import Context
    from paper_1612_00474_amd._lib import RPB_ENOTSPD
    from tests.test_oracle_lanczos import _not_spd_fixture
    box, m_ref, pos, w = _not_spd_fixture()
    M, _ = mobility.dense(pos, box=box)
    g_ref, mo, _, status = lanczos.lanczos_sqrt(lambda v: M @ v, w, 1e-300, 64)
    assert status == "notspd" and mo == m_ref
    c = Context(0, box=box)
    try:
        g, m, eps, st = c.lanczos(dev(pos), dev(w.reshape(-1, 3)), 1e-300, 64, precision,
                                  allow_noconv=True, allow_notspd=True)
        err = rel2(host(g).ravel(), g_ref)
        print(f"not SPD {precision}: status {st}, m = {m} (oracle {mo}), rel2 {err:.2e}")
        assert st == RPB_ENOTSPD and m == mo
        assert err <= tol and max_element(host(g).ravel(), g_ref) <= 10 * tol
        assert "negative Ritz value" in c.last_error()
    finally:
        c.close()


def test_small_and_large_solves_alternate(ctx, c1, multi_tile):
    # A 256-sphere solve runs its eigensolve on the context's second stream and a 1,100-sphere
    # solve runs it in line; alternating the two on one context reproduces each bitwise (the
    # status ring's slots and the streams' ordering carry nothing from one solve to the next).
    import torch
    inp, _ = c1
    pos_l, _, w_l = multi_tile
    cases = [(dev(inp["pos"]), dev(inp["w"])), (dev(pos_l), dev(w_l))]
    first = [ctx.lanczos(P, W, 1e-5, allow_noconv=True) for P, W in cases]
    for _ in range(3):
        for (P, W), (g0, it0, eps0, _) in zip(cases, first):
            g, it, eps, _ = ctx.lanczos(P, W, 1e-5, allow_noconv=True)
            assert it == it0 and eps == eps0 and torch.equal(g, g0)
