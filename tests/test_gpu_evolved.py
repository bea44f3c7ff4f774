"""One-step parity at states a trajectory actually reaches: the 16,384-sphere float64 sheet
(area fraction 0.4, gravity -1, torque (0, 1, 0), soft repulsion U0 = 1, b = 0.1) advanced by
stochastic Adams-Bashforth steps (Sec. II.A eq. AB) with device noise at dt = 0.01.  After 50
and after 99 steps the GPU state is handed to the oracle, which evaluates at that state

  - the forces (Sec. III eq. soft_potential plus gravity), all spheres;
  - the deterministic velocity u^n = M F + M_C T (Sec. II.B, Sec. III) on 64 rows, against the
    u^n the next GPU step stores;
  - the centred RFD drift (Sec. II.A) with a seeded W~ on 64 rows, against rfd_drift.

Trajectories are stochastic and tolerance-based Lanczos may stop at another iteration on the
two sides, so whole trajectories are never compared, only these one-step quantities.
"""
import numpy as np
import pytest

from oracle import forces, mobility, stochastic
from paper_1612_00474_amd import workloads as wl
from tests.gpu_util import dev, host, max_element, rel2, require_gpu

pytestmark = pytest.mark.gpu

W = wl.WORKLOADS["sheet16k_fp64"]
SNAPSHOTS = (50, 99)
NROWS = 64


@pytest.fixture(scope="module")
def trajectory():
    """{k: (q^k, u^k)}: the state after k steps and the u^k stored by step k + 1."""
    require_gpu()
    from paper_1612_00474_amd import Context, StepState
    c = Context(0)
    inp = wl.make_inputs(W, 0)
    state = StepState(dev(inp["pos"]))
    kw = dict(dt=W.dt, delta=W.delta, lanczos_tol=W.lanczos_tol, f_grav_z=W.f_grav_z,
              torque=W.torque, steric_u0=W.steric_u0, steric_b=W.steric_b, seed=0,
              precision="fp64", rfd_precision="fp64")
    out, iters = {}, []
    q = None
    for k in range(max(SNAPSHOTS) + 1):
        if k in SNAPSHOTS:
            q = host(state.pos).copy()
        iters.append(c.sab_step(state, **kw)[0])
        if k in SNAPSHOTS:
            out[k] = (q, host(state.u_prev).copy())
    c.close()
    z0, z1 = inp["pos"][:, 2].mean(), host(state.pos)[:, 2].mean()
    print(f"sheet16k: {len(iters)} steps, Lanczos m {min(iters)}..{max(iters)}, mean height "
          f"{z0:.4f} -> {z1:.4f}")
    return out


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_1612_00474_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("k", SNAPSHOTS)
def test_one_step_quantities_at_an_evolved_state(ctx, trajectory, k):
    q, u_gpu = trajectory[k]
    rows = np.random.default_rng(100 + k).choice(W.n, NROWS, replace=False)
    rows[0] = W.n - 1
    # forces at the state (all spheres: every one is a source of the product)
    F = forces.forces(q, 1.0, W.steric_u0, W.steric_b, W.f_grav_z)
    Fg = host(ctx.forces(dev(q), W.f_grav_z, W.steric_u0, W.steric_b))
    ef, mf = rel2(Fg, F), max_element(Fg, F)
    # the velocity the step stored
    T = np.tile(np.array(W.torque), (W.n, 1))
    u = mobility.matvec(q, F, T, rows=rows)
    eu, mu = rel2(u_gpu[rows], u), max_element(u_gpu[rows], u)
    # the drift at the state
    wt = np.random.default_rng(200 + k).standard_normal((W.n, 3))
    d = stochastic.rfd(q, wt, W.delta, rows=rows)
    dg = host(ctx.rfd(dev(q), dev(wt), W.delta, precision="fp64", rfd_precision="fp64"))[rows]
    ed, md = rel2(dg, d), max_element(dg, d)
    print(f"step {k}: forces {ef:.2e} ({mf:.2e}), u^n {eu:.2e} ({mu:.2e}), drift {ed:.2e} "
          f"({md:.2e}) [rel2 (max element)]")
    assert ef <= 1e-12 and mf <= 1e-11
    assert eu <= 1e-12 and mu <= 1e-11
    # product rounding (~1e-15 relative) divided by delta = 1e-4
    assert ed <= 1e-10 and md <= 1e-9
