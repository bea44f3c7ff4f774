"""GPU parity of sab_step (one stochastic Adams-Bashforth / Euler-Maruyama step) against the oracle."""
import numpy as np
import pytest

from oracle import integrator, philox
from paper_1612_00474_amd import workloads as wl
from tests.gpu_util import max_element, close, dev, host, rel2, require_gpu

pytestmark = pytest.mark.gpu

PHYS = dict(f_grav_z=-1.0, torque=(0.0, 1.0, 0.0))
M_FIXED = 8   # fixed Lanczos iteration count so that both sides take the same Krylov space


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_1612_00474_amd import Context
    c = Context(0)
    yield c
    c.close()


def _setup(n=200, seed=0):
    w = wl.Workload("step", n, wl.side_for_area_fraction(n, 0.4), 1.1, 2.5)
    return wl.make_inputs(w, seed)


def _oracle_step(pos, u_prev, W, Wt, scheme, rfd="centred"):
    return integrator.step(pos, u_prev, W, Wt, dt=0.01, delta=1e-4, lanczos_tol=1e-300,
                           lanczos_max_iter=M_FIXED, scheme=scheme, u0=1.0, b=0.1, rfd=rfd,
                           **PHYS)


@pytest.mark.parametrize("scheme,rfd", [("sab", "centred"), ("em", "centred"),
                                        ("sab", "one_sided"), ("em", "one_sided")])
def test_two_steps_match_oracle(ctx, scheme, rfd):
    from paper_1612_00474_amd import StepState
    inp = _setup()
    rng = np.random.default_rng(3)
    state = StepState(dev(inp["pos"]))
    pos = inp["pos"].copy()
    u_prev = None
    for k in range(2):
        W, Wt = rng.standard_normal(pos.shape), rng.standard_normal(pos.shape)
        it, eps, st = ctx.sab_step(state, dt=0.01, delta=1e-4, lanczos_tol=1e-300,
                                   lanczos_max_iter=M_FIXED, scheme=scheme, w=dev(W), w_tilde=dev(Wt),
                                   steric_u0=1.0, steric_b=0.1, rfd_scheme=rfd, **PHYS)
        new, u, mref, _, _ = _oracle_step(pos, u_prev, W, Wt, scheme, rfd)
        got = host(state.pos)
        err = rel2(got - pos, new - pos)
        print(f"{scheme}/{rfd} step {k}: displacement rel2 = {err:.3e}")
        assert it == mref == M_FIXED
        assert err <= 1e-10 and max_element(got - pos, new - pos) <= 10 * 1e-10
        assert close(host(state.u_prev), u, 1e-12)
        # continue both trajectories from the device state (one-step parity)
        pos = got.copy()
        u_prev = host(state.u_prev).copy()
    assert state.step == 2 and state.have_prev


def test_preconditioned_step_matches_oracle(ctx):
    from paper_1612_00474_amd import StepState
    inp = _setup()
    rng = np.random.default_rng(8)
    W, Wt = rng.standard_normal(inp["pos"].shape), rng.standard_normal(inp["pos"].shape)
    state = StepState(dev(inp["pos"]))
    it, eps, st = ctx.sab_step(state, dt=0.01, delta=1e-4, lanczos_tol=1e-300,
                               lanczos_max_iter=M_FIXED, w=dev(W), w_tilde=dev(Wt), steric_u0=1.0,
                               steric_b=0.1, lanczos_precond=True, **PHYS)
    new, u, m, _, _ = integrator.step(inp["pos"], None, W, Wt, dt=0.01, delta=1e-4,
                                      lanczos_tol=1e-300, lanczos_max_iter=M_FIXED, u0=1.0, b=0.1,
                                      lanczos_precond=True, **PHYS)
    assert it == m == M_FIXED
    assert close(host(state.pos) - inp["pos"], new - inp["pos"], 1e-10)


def test_device_noise_matches_oracle_generator(ctx):
    from paper_1612_00474_amd import StepState
    inp = _setup(n=120, seed=1)
    state = StepState(dev(inp["pos"]))
    state.step = 41
    ctx.sab_step(state, dt=0.01, delta=1e-4, lanczos_tol=1e-300, lanczos_max_iter=M_FIXED, seed=99,
                 steric_u0=1.0, steric_b=0.1, **PHYS)
    n = len(inp["pos"])
    W = philox.normals(3 * n, 99, 0, 41).reshape(n, 3)
    Wt = philox.normals(3 * n, 99, 1, 41).reshape(n, 3)
    new, *_ = _oracle_step(inp["pos"], None, W, Wt, "sab")
    assert close(host(state.pos) - inp["pos"], new - inp["pos"], 1e-10)


def test_mixed_precision_step(ctx):
    from paper_1612_00474_amd import StepState
    inp = _setup(n=256, seed=2)
    rng = np.random.default_rng(8)
    W, Wt = rng.standard_normal(inp["pos"].shape), rng.standard_normal(inp["pos"].shape)
    state = StepState(dev(inp["pos"]))
    ctx.sab_step(state, dt=0.01, delta=1e-4, lanczos_tol=1e-300, lanczos_max_iter=M_FIXED,
                 precision="mixed", rfd_precision="fp64", w=dev(W), w_tilde=dev(Wt),
                 steric_u0=1.0, steric_b=0.1, **PHYS)
    new, *_ = _oracle_step(inp["pos"], None, W, Wt, "sab")
    err = rel2(host(state.pos) - inp["pos"], new - inp["pos"])
    print(f"mixed step: displacement rel2 = {err:.3e}")
    assert err <= 1e-5 and max_element(host(state.pos) - inp["pos"], new - inp["pos"]) <= 10 * 1e-5


@pytest.mark.parametrize("precision,rfd_precision,rfd,tol_u,tol_x", [
    ("fp64", "fp64", "centred", 1e-12, 1e-10),
    ("mixed", "fp64", "centred", 1e-5, 1e-5),
    ("fp64", "fp64", "one_sided", 1e-12, 1e-10),
    ("mixed", "mixed", "one_sided", 1e-5, 2e-3)])
def test_step_products_over_several_tiles(ctx, precision, rfd_precision, rfd, tol_u, tol_x):
    # N = 700: three tiles of the launch that evaluates M F + M_C T (with the rollers' torque)
    # together with the first Lanczos product M W and, for the one-sided RFD in the step's own
    # precision, M W~ at q; ragged last tile included.  Mixed RFD: float32 products differenced
    # over delta = 1e-4 (a-priori ~1e-3 relative in the drift, a small part of the displacement)
    from paper_1612_00474_amd import StepState
    inp = _setup(n=700, seed=4)
    rng = np.random.default_rng(12)
    W, Wt = rng.standard_normal(inp["pos"].shape), rng.standard_normal(inp["pos"].shape)
    state = StepState(dev(inp["pos"]))
    it, eps, st = ctx.sab_step(state, dt=0.01, delta=1e-4, lanczos_tol=1e-300,
                               lanczos_max_iter=M_FIXED, precision=precision,
                               rfd_precision=rfd_precision, rfd_scheme=rfd, w=dev(W),
                               w_tilde=dev(Wt), steric_u0=1.0, steric_b=0.1, **PHYS)
    new, u, mref, _, _ = _oracle_step(inp["pos"], None, W, Wt, "sab", rfd)
    err_u = rel2(host(state.u_prev), u)
    err_x = rel2(host(state.pos) - inp["pos"], new - inp["pos"])
    print(f"{precision}/{rfd_precision} {rfd} step N=700: u rel2 = {err_u:.3e}, "
          f"displacement rel2 = {err_x:.3e}")
    assert it == mref == M_FIXED
    assert err_u <= tol_u and max_element(host(state.u_prev), u) <= 10 * tol_u
    assert err_x <= tol_x and max_element(host(state.pos) - inp["pos"], new - inp["pos"]) <= 10 * tol_x


@pytest.mark.parametrize("box", [None, "periodic"])
@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -float("inf")])
def test_non_finite_position_leaves_state_alone(box, bad):
    # the step reads its position check back only after the forces (cell list) and the first
    # product are enqueued; a NaN or Inf must still end in RPB_ENONFINITE with the state as it
    # was, and the next good step must run normally
    import torch
    from paper_1612_00474_amd import Context, StepState
    from paper_1612_00474_amd._lib import RPB_ENONFINITE, RpbError
    require_gpu()
    inp = _setup(n=300, seed=4)
    side = wl.side_for_area_fraction(300, 0.4)
    c = Context(0, box=(side, side)) if box else Context(0)
    try:
        kw = dict(dt=0.01, delta=1e-4, lanczos_tol=1e-4, **PHYS)
        for precision in ("fp64", "mixed"):
            state = StepState(dev(inp["pos"]))
            c.sab_step(state, precision=precision, **kw)
            good_pos, good_u = state.pos.clone(), state.u_prev.clone()
            for row, comp in ((0, 2), (150, 0), (299, 1)):
                state.pos[row, comp] = bad
                before = state.pos.clone()
                with pytest.raises(RpbError) as e:
                    c.sab_step(state, precision=precision, **kw)
                assert e.value.status == RPB_ENONFINITE
                assert np.array_equal(host(state.pos), host(before), equal_nan=True)
                assert torch.equal(state.u_prev, good_u)
                assert state.step == 1 and state.have_prev
                state.pos.copy_(good_pos)
            it, _, _ = c.sab_step(state, precision=precision, **kw)
            assert it >= 2 and state.step == 2
            assert torch.isfinite(state.pos).all() and torch.isfinite(state.u_prev).all()
    finally:
        c.close()
