"""GPU parity of rpb_mobility_matvec against the FP64 oracle (through the C ABI)."""
import math

import numpy as np
import pytest

from oracle import mobility
from paper_1612_00474_amd import workloads as wl
from tests.gpu_util import max_element, close, awkward_config, dev, host, rel2, require_gpu

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12     # relative 2-norm, float64 path
MIXED_TOL = 1e-5     # relative 2-norm, float32 pair terms with Kahan sums


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


@pytest.fixture(scope="module")
def c1_ref(c1):
    return mobility.dense_matvec(c1["pos"], c1["force"], c1["torque"])


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_sheet256_parity(ctx, c1, c1_ref, precision, tol):
    u = host(ctx.matvec(dev(c1["pos"]), dev(c1["force"]), dev(c1["torque"]), precision))
    err = rel2(u, c1_ref)
    print(f"sheet256 {precision}: rel2 = {err:.3e}")
    assert err <= tol and max_element(u, c1_ref) <= 10 * tol
    assert np.abs(u - c1_ref).max() <= 10 * tol * np.abs(c1_ref).max()


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_coherent_forcing(ctx, precision, tol):
    # gravity-like F = (0, 0, -1) and the rollers' torque (0, 1, 0) on a wide sheet: the free
    # and image parts cancel to O(h^2/r^3) at large r, which exposes float32 cancellation
    pos = wl.sheet(2048, phi=0.4, seed=3)
    F = np.tile([0.0, 0.0, -1.0], (len(pos), 1))
    T = np.tile([0.0, 1.0, 0.0], (len(pos), 1))
    rows = np.arange(0, 2048, 16)
    ref = mobility.matvec(pos, F, T, rows=rows)
    u = host(ctx.matvec(dev(pos), dev(F), dev(T), precision))[rows]
    err = rel2(u, ref)
    print(f"coherent {precision}: rel2 = {err:.3e}")
    assert err <= tol and max_element(u, ref) <= 10 * tol


@pytest.mark.parametrize("n", [1, 2, 7, 255, 256, 257, 300])
def test_ragged_sizes_fp64(ctx, n):
    rng = np.random.default_rng(n)
    side = max(2.0, math.sqrt(n * math.pi / 0.4))
    pos = np.column_stack([rng.uniform(0, side, n), rng.uniform(0, side, n), rng.uniform(0.8, 3, n)])
    F = rng.standard_normal((n, 3))
    T = rng.standard_normal((n, 3))
    ref = mobility.dense_matvec(pos, F, T)
    u = host(ctx.matvec(dev(pos), dev(F), dev(T), "fp64"))
    assert close(u, ref, FP64_TOL)
    um = host(ctx.matvec(dev(pos), dev(F), dev(T), "mixed"))
    assert close(um, ref, MIXED_TOL)


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_wall_overlaps_and_coincident_spheres(ctx, precision, tol):
    pos = awkward_config()
    rng = np.random.default_rng(1)
    F = rng.standard_normal(pos.shape)
    T = rng.standard_normal(pos.shape)
    ref = mobility.dense_matvec(pos, F, T)
    u = host(ctx.matvec(dev(pos), dev(F), dev(T), precision))
    assert close(u, ref, tol)
    # spheres on / below the wall do not move (App. A)
    assert np.all(u[1] == 0.0) and np.all(u[2] == 0.0)


def test_force_only_and_torque_only(ctx, c1, c1_ref):
    pos = dev(c1["pos"])
    uf = host(ctx.matvec(pos, dev(c1["force"]), None, "fp64"))
    ut = host(ctx.matvec(pos, None, dev(c1["torque"]), "fp64"))
    assert close(uf, mobility.dense_matvec(c1["pos"], c1["force"], None), FP64_TOL)
    assert close(ut, mobility.dense_matvec(c1["pos"], None, c1["torque"]), FP64_TOL)
    assert close(uf + ut, c1_ref, FP64_TOL)


def test_row_shards_concatenate_bitwise(ctx):
    # row ranges use the ordered (target tile x source chunk) kernel, whose chunking depends on n
    # only; the whole product matches them bitwise when it takes that kernel too, and the
    # symmetric kernel's whole product within rounding
    from paper_1612_00474_amd import Context
    c = Context(0)
    pos = wl.sheet(5000, seed=2)
    rng = np.random.default_rng(2)
    F, T = dev(rng.standard_normal(pos.shape)), dev(rng.standard_normal(pos.shape))
    P = dev(pos)
    for precision in ("fp64", "mixed"):
        c.set_tuning(precision, symmetric=0)
        full = host(c.matvec(P, F, T, precision))
        cuts = [0, 1, 700, 2500, 4999, 5000]
        parts = [host(c.matvec(P, F, T, precision, rows=(a, b))) for a, b in zip(cuts[:-1], cuts[1:])]
        assert np.array_equal(np.vstack(parts), full)
        c.set_tuning(precision, symmetric=1)
        sym = host(c.matvec(P, F, T, precision))
        assert close(sym, full, (1e-13 if precision == "fp64" else 2e-6))
    c.close()


def test_deterministic(ctx, c1):
    P, F, T = dev(c1["pos"]), dev(c1["force"]), dev(c1["torque"])
    for precision in ("fp64", "mixed"):
        a = host(ctx.matvec(P, F, T, precision))
        b = host(ctx.matvec(P, F, T, precision))
        assert np.array_equal(a, b)


@pytest.mark.parametrize("name,nrows", [("sheet16k_fp64", 64), ("sheet64k_mixed", 256),
                                        ("sheet256k_mixed", 1024)])
def test_full_size_row_sampled(ctx, name, nrows):
    # the 16,384-sphere sheet against the oracle computed here; the two larger sheets against
    # the oracle's values stored by tests/golden/make_sheet_rows.py (256 and 1,024 rows)
    from tests.conftest import golden_sheet_rows
    w = wl.WORKLOADS[name]
    inp = wl.make_inputs(w, 0)
    if name == "sheet16k_fp64":
        rows = np.random.default_rng(9).choice(w.n, nrows, replace=False)
        rows[0] = w.n - 1                      # the last sphere (ragged last tile)
        ref = mobility.matvec(inp["pos"], inp["force"], inp["torque"], rows=rows)
    else:
        fname = {"sheet64k_mixed": "sheet64k_rows.txt", "sheet256k_mixed": "sheet256k_rows.txt"}
        rows, ref = golden_sheet_rows(fname[name], inp)["u"]
        assert len(rows) == nrows and rows[0] == w.n - 1
    P, F, T = dev(inp["pos"]), dev(inp["force"]), dev(inp["torque"])
    for precision, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL)):
        u = host(ctx.matvec(P, F, T, precision))[rows]
        err = rel2(u, ref)
        emax = max_element(u, ref)
        print(f"{name} {precision}: rel2 = {err:.3e}, max element {emax:.3e} over {nrows} rows")
        assert err <= tol and emax <= 10 * tol


def test_error_paths(ctx, c1):
    import torch
    from paper_1612_00474_amd._lib import RPB_EINVAL, RPB_ENONFINITE, RpbError
    P, F = dev(c1["pos"]), dev(c1["force"])
    with pytest.raises(RpbError) as e:
        ctx.matvec(P, None, None)
    assert e.value.status == RPB_EINVAL
    with pytest.raises(RpbError) as e:
        ctx.matvec(P, F, None, out=P)
    assert e.value.status == RPB_EINVAL
    bad = P.clone()
    bad[3, 1] = float("nan")
    with pytest.raises(RpbError) as e:
        ctx.matvec(bad, F, None)
    assert e.value.status == RPB_ENONFINITE
    ctx.a = -1.0
    try:
        with pytest.raises(RpbError) as e:
            ctx.matvec(P, F, None)
        assert e.value.status == RPB_EINVAL
    finally:
        ctx.a = 1.0
    empty = torch.empty((0, 3), dtype=torch.float64, device="cuda")
    assert ctx.matvec(empty, empty, None).shape == (0, 3)


@pytest.mark.parametrize("torque", [False, True])
@pytest.mark.parametrize("tpt", [1, 2, 4])
@pytest.mark.parametrize("n", [2, 63, 64, 65, 300, 513, 1100])
def test_symmetric_kernel_matches_oracle_and_ordered(ctx, n, tpt, torque):
    # whole-system products take the symmetric tile-pair kernel (each unordered pair evaluated
    # once; with torques both coupling directions come from the shared geometry); ragged tiles
    # and partial 64-source blocks included
    from paper_1612_00474_amd import Context
    c = Context(0)
    rng = np.random.default_rng(100 + n)
    side = max(2.0, math.sqrt(n * math.pi / 0.4))
    pos = np.column_stack([rng.uniform(0, side, n), rng.uniform(0, side, n), rng.uniform(0.8, 2.6, n)])
    F = rng.standard_normal((n, 3))
    T = rng.standard_normal((n, 3)) if torque else None
    ref = mobility.dense_matvec(pos, F, T)
    P, Fd, Td = dev(pos), dev(F), (dev(T) if torque else None)
    for precision, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL)):
        c.set_tuning(precision, tpt=tpt, symmetric=1)
        us = host(c.matvec(P, Fd, Td, precision))
        assert close(us, ref, tol), (precision, n, tpt)
        assert np.array_equal(us, host(c.matvec(P, Fd, Td, precision)))     # reproducible
        c.set_tuning(precision, symmetric=0)
        uo = host(c.matvec(P, Fd, Td, precision))
        assert close(us, uo, (1e-13 if precision == "fp64" else 2e-6))
    c.close()


def test_output_check(ctx, c1):
    # rpb_output_check_enable: results are scanned for NaN / Inf (only positions are checked
    # on input, so a NaN force is how a non-finite result arises)
    from paper_1612_00474_amd._lib import RPB_ENONFINITE, RpbError
    P, F, Wt = dev(c1["pos"]), dev(c1["force"]), dev(c1["w_tilde"])
    bad = F.clone()
    bad[7, 2] = float("nan")
    assert np.isnan(host(ctx.matvec(P, bad, None))).any()      # off by default
    ctx.output_check(True)
    try:
        for precision in ("fp64", "mixed"):
            assert np.isfinite(host(ctx.matvec(P, F, None, precision))).all()
            with pytest.raises(RpbError) as e:
                ctx.matvec(P, bad, None, precision)
            assert e.value.status == RPB_ENONFINITE
        n = P.shape[0]
        offs = np.array([0, 100, n], dtype=np.int64)
        ctx.matvec_batched(P, offs, F)
        with pytest.raises(RpbError) as e:
            ctx.matvec_batched(P, offs, bad)
        assert e.value.status == RPB_ENONFINITE
        assert np.isfinite(host(ctx.rfd(P, Wt, 1e-4))).all()
        badw = Wt.clone()
        badw[3, 0] = float("inf")
        with pytest.raises(RpbError) as e:
            ctx.rfd(P, badw, 1e-4)
        assert e.value.status == RPB_ENONFINITE
    finally:
        ctx.output_check(False)
    assert np.isnan(host(ctx.matvec(P, bad, None))).any()      # off again
