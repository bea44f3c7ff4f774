"""Errors of the mixed-precision path on the 65,536-sphere sheet (area fraction 0.4, heights in
[1.1a, 2.5a]) for the two stochastic outputs of a step: the Brownian increment M^{1/2}W
(Sec. II.C) and the RFD drift (Sec. II.A).  The velocity U = M F + M_C T at this size is checked
row by row against the oracle in test_gpu_matvec.py.

The drift is compared with the FP64 oracle on 64 sampled rows (values stored by
tests/golden/make_sheet_rows.py).  The oracle cannot run Lanczos at
this size (every iteration is a full product), so the mixed M^{1/2}W is compared with the FP64
GPU solve at the same number of iterations (the FP64 solve matches the oracle's Lanczos to 1e-12
at fixed m on smaller systems), and the tolerance run is checked against |g|^2 = w^T M w, which
holds for the symmetric root.
"""
import numpy as np
import pytest

from oracle import stochastic
from paper_1612_00474_amd import workloads as wl
from tests.gpu_util import dev, host, max_element, rel2, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_1612_00474_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def sheet():
    return wl.make_inputs(wl.WORKLOADS["sheet64k_mixed"], 0)


def test_drift_rows_against_oracle(ctx, sheet):
    # 64 rows of the oracle's drift, stored by tests/golden/make_sheet_rows.py
    from tests.conftest import golden_sheet_rows
    w = wl.WORKLOADS["sheet64k_mixed"]
    rows, ref = golden_sheet_rows("sheet64k_rows.txt", sheet)["drift"]
    assert len(rows) == 64 and rows[0] == w.n - 1    # the ragged last tile included
    P, Wt = dev(sheet["pos"]), dev(sheet["w_tilde"])
    # The step's default: float64 products for the difference.  The shifted positions
    # q +- (delta/2) w~ are rounded exactly as the oracle rounds them (product, then sum), so
    # the error is the products' own rounding (~4e-15 relative at this N) divided by delta:
    # ~4e-11 relative.
    d64 = host(ctx.rfd(P, Wt, w.delta, precision="mixed", rfd_precision="fp64"))[rows]
    # float32 products: rounding of ~u32 in each product amplified by 1/delta = 1e4
    d32 = host(ctx.rfd(P, Wt, w.delta, precision="mixed", rfd_precision="mixed"))[rows]
    e64, e32 = rel2(d64, ref), rel2(d32, ref)
    m64, m32 = max_element(d64, ref), max_element(d32, ref)
    print(f"sheet64k drift vs oracle ({len(rows)} rows): float64 products {e64:.2e} "
          f"(max element {m64:.2e}), float32 products {e32:.2e} (max element {m32:.2e})")
    assert e64 <= 1e-10 and m64 <= 1e-9
    assert e32 <= 5e-2 and m32 <= 5e-1


def test_brownian_increment_mixed(ctx, sheet):
    P, W = dev(sheet["pos"]), dev(sheet["w"])
    m = 12
    g64 = host(ctx.lanczos(P, W, 1e-300, max_iter=m, allow_noconv=True)[0])
    g32 = host(ctx.lanczos(P, W, 1e-300, max_iter=m, precision="mixed", allow_noconv=True)[0])
    e_fixed = rel2(g32, g64)
    g, it, eps, st = ctx.lanczos(P, W, 1e-3, precision="mixed")
    g = host(g)
    Mw = host(ctx.matvec(P, W, None, "fp64"))
    wMw = float(np.sum(sheet["w"] * Mw))
    e_norm = abs(float(np.sum(g * g)) / wMw - 1.0)
    print(f"sheet64k M^1/2 W: mixed vs float64 at m = {m}: {e_fixed:.2e}; tol 1e-3 run: "
          f"m = {it}, eps = {eps:.2e}, |g|^2 / w.Mw - 1 = {e_norm:.2e}")
    assert e_fixed <= 1e-5
    assert it <= 16 and eps < 1e-3
    assert e_norm <= 1e-3
