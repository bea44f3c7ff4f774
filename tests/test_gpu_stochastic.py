"""GPU parity of rfd_drift, rpb_forces and rpb_normals against the oracle (through the C ABI)."""
import numpy as np
import pytest

from oracle import forces, philox, stochastic
from paper_1612_00474_amd import workloads as wl
from tests.gpu_util import awkward_config, dev, host, rel2, require_gpu

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
    return wl.make_inputs(wl.WORKLOADS["sheet256_rsa"], 0)


def test_rfd_fp64(ctx, c1):
    # the two products are O(1); their difference is divided by delta = 1e-4, so rounding
    # of ~1e-16 in each product shows up as ~1e-12 relative in the drift
    ref = stochastic.rfd(c1["pos"], c1["w_tilde"], 1e-4)
    d = host(ctx.rfd(dev(c1["pos"]), dev(c1["w_tilde"]), 1e-4))
    err = rel2(d, ref)
    print(f"rfd fp64: rel2 = {err:.3e}")
    assert err <= 1e-10


def test_rfd_one_sided_fp64(ctx, c1):
    # (kT/delta)[M(q + delta w~) w~ - M(q) w~]: same rounding amplification as the centred form
    for pos in (c1["pos"], awkward_config()):
        wt = np.random.default_rng(5).standard_normal(pos.shape)
        ref = stochastic.rfd_one_sided(pos, wt, 1e-4)
        d = host(ctx.rfd(dev(pos), dev(wt), 1e-4, rfd_scheme="one_sided"))
        assert rel2(d, ref) <= 1e-10


def test_rfd_awkward_config(ctx):
    pos = awkward_config()
    wt = np.random.default_rng(4).standard_normal(pos.shape)
    ref = stochastic.rfd(pos, wt, 1e-4)
    d = host(ctx.rfd(dev(pos), dev(wt), 1e-4))
    assert rel2(d, ref) <= 1e-10


def test_rfd_float32_products(ctx, c1):
    # float32 products: rounding u32 ~ 6e-8 of O(1) values divided by delta = 1e-4 gives
    # an a-priori relative error of order 4 u32 / delta ~ 2.4e-3 per component
    ref = stochastic.rfd(c1["pos"], c1["w_tilde"], 1e-4)
    d = host(ctx.rfd(dev(c1["pos"]), dev(c1["w_tilde"]), 1e-4, rfd_precision="mixed"))
    err = rel2(d, ref)
    print(f"rfd with float32 products: rel2 = {err:.3e}")
    assert err <= 5e-2


def test_forces(ctx, c1):
    for pos in (c1["pos"], awkward_config(), wl.sheet(3000, seed=4)):
        ref = forces.forces(pos, 1.0, 1.0, 0.1, -1.0)
        f = host(ctx.forces(dev(pos), -1.0, 1.0, 0.1))
        assert rel2(f, ref) <= 1e-12


def test_forces_full_size_sampled_rows(ctx):
    # the 65,536-sphere sheet: the sources are split over many workgroups; sampled rows
    # (first, last, random) against the oracle's row evaluation
    n = 65536
    pos = wl.sheet(n, seed=0)
    f = host(ctx.forces(dev(pos), -1.0, 1.0, 0.1))
    rows = np.concatenate([[0, 1, n - 1], np.random.default_rng(3).choice(n, 45, replace=False)])
    ref = forces.forces(pos, 1.0, 1.0, 0.1, -1.0, rows=rows)
    assert rel2(f[rows], ref) <= 1e-12


def test_normals_match_oracle_generator(ctx):
    for count, seed, stream, step in ((10, 0, 0, 0), (3 * 4097, 12345, 1, 77), (3, 2 ** 63 + 5, 0, 2 ** 40)):
        ref = philox.normals(count, seed, stream, step)
        got = host(ctx.normals(count, seed, stream, step))
        assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
