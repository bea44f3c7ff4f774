"""rpb_mobility_matvec_noalloc (the product that allocates nothing) against rpb_mobility_matvec and
the oracle, through the C ABI: two calls in a row, the second on a smaller system, then a larger
one again (the shared scratch array keeps the last call's contents)."""
import numpy as np
import pytest

from oracle import mobility
from paper_1612_00474_amd import workloads as wl
from tests.gpu_util import awkward_config, dev, host, rel2, require_gpu

pytestmark = pytest.mark.gpu

# against the existing entry point (same arithmetic, another summation order)
TOL = {"fp64": 1e-12, "mixed": 2e-6}
# against the oracle (relative 2-norm of the float64 and mixed paths)
ORACLE_TOL = {"fp64": 1e-12, "mixed": 1e-5}


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_1612_00474_amd import Context
    c = Context(0)
    yield c
    c.close()


def _inputs(n, seed):
    pos = wl.sheet(n, phi=0.4, seed=seed)
    rng = np.random.default_rng(seed + 100)
    return pos, rng.standard_normal((n, 3)), rng.standard_normal((n, 3))


def _compare(got, ref, tol, what):
    err = rel2(got, ref)
    emax = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"{what}: rel2 {err:.3e}, max element {emax:.3e}")
    assert err <= tol and emax <= 5 * tol, what


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_two_calls_in_a_row_match_the_allocating_product(ctx, precision):
    for n, seed in ((3000, 1), (700, 2), (4100, 3)):
        pos, F, T = _inputs(n, seed)
        u = host(ctx.matvec_noalloc(dev(pos), dev(F), dev(T), precision))
        ref = host(ctx.matvec(dev(pos), dev(F), dev(T), precision))
        _compare(u, ref, TOL[precision], f"{precision} n={n} vs rpb_mobility_matvec")
        if n == 700:
            exact = mobility.dense_matvec(pos, F, T)
            _compare(u, exact, ORACLE_TOL[precision], f"{precision} n={n} vs oracle")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_force_or_torque_alone_and_awkward_geometry(ctx, precision):
    pos = awkward_config(300, seed=7)
    rng = np.random.default_rng(8)
    F, T = rng.standard_normal((300, 3)), rng.standard_normal((300, 3))
    for f, t in ((F, None), (None, T)):
        u = host(ctx.matvec_noalloc(dev(pos), None if f is None else dev(f),
                                    None if t is None else dev(t), precision))
        exact = mobility.dense_matvec(pos, f, t)
        _compare(u, exact, ORACLE_TOL[precision], f"{precision} awkward, force={f is not None}")


def test_periodic_box_and_free_space():
    require_gpu()
    from paper_1612_00474_amd import Context
    pos, F, T = _inputs(600, 4)
    box = (40.0, 40.0)
    for kw, okw in (({"box": box}, {"box": box}), ({"wall": False}, {"wall": False})):
        c = Context(0, **kw)
        try:
            u = host(c.matvec_noalloc(dev(pos), dev(F), dev(T), "fp64"))
            exact = mobility.dense_matvec(pos, F, T, **okw)
            _compare(u, exact, ORACLE_TOL["fp64"], f"fp64 {kw}")
        finally:
            c.close()


def test_too_large_is_rejected(ctx):
    import torch
    from paper_1612_00474_amd import RpbError
    n = 500_000     # beyond the scratch array in both precisions; rejected before any launch
    pos = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    pos[:, 2] = 2.0
    F = torch.zeros_like(pos)
    for precision in ("fp64", "mixed"):
        with pytest.raises(RpbError) as e:
            ctx.matvec_noalloc(pos, F, None, precision)
        assert e.value.status == -1
        assert "scratch" in str(e.value)
