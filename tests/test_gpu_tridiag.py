"""GPU parity of lanczos_tridiag_sqrt (the tridiagonal square root of the Krylov method,
Sec. II.C) against the oracle's eigendecomposition, on matrices chosen to stress the
eigensolve: nearly equal eigenvalue pairs, negligible couplings, Toeplitz spectra, indefinite
matrices, a Krylov space that closes, and the Lanczos coefficients of the 256-sphere sheet up
to the largest Krylov space (64)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import lanczos, mobility
from paper_1612_00474_amd import workloads as wl
from tests.gpu_util import close, require_gpu

pytestmark = pytest.mark.gpu

TOL = 1e-12   # FP64 bar


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_1612_00474_amd import Context
    c = Context(0)
    yield c
    c.close()


def _lanczos_coefficients(M, w, its):
    """alpha, beta of `its` oracle-style Lanczos steps (full re-orthogonalisation, twice)."""
    V = [w / np.linalg.norm(w)]
    alpha, beta = [], []
    for k in range(its):
        v = V[-1]
        u = M @ v
        a = v @ u
        u = u - a * v
        if k > 0:
            u = u - beta[-1] * V[-2]
        Vm = np.array(V)
        u = u - Vm.T @ (Vm @ u)
        u = u - Vm.T @ (Vm @ u)
        b = np.linalg.norm(u)
        alpha.append(a)
        beta.append(b)
        V.append(u / b)
    return np.array(alpha), np.array(beta[:-1])


def _cases():
    rng = np.random.default_rng(2024)
    n = 21   # Wilkinson W21+: its largest eigenvalues come in pairs equal to ~1e-14
    yield "wilkinson21", np.abs(np.arange(n) - 10.0), np.ones(n - 1), 1.0
    n = 50   # second difference: eigenvalues 2 - 2 cos(k pi / 51), the smallest 3.8e-3
    yield "toeplitz50", np.full(n, 2.0), np.full(n - 1, -1.0), 2.5
    n = 40   # couplings from 1 down to 1e-13: most deflate
    yield "graded40", np.linspace(1.0, 2.0, n), 10.0 ** (-rng.integers(0, 14, n - 1)), 1.0
    n = 64
    yield "random64", 0.5 + rng.random(n), 0.5 * rng.random(n - 1) + 1e-3, 3.0
    n = 30   # indefinite, eigenvalues near +-(1..2), none near zero
    yield "indefinite30", np.where(np.arange(n) % 2 == 0, 1.0, -1.0) * (1.0 + rng.random(n)), \
        0.1 * rng.random(n - 1), 1.0
    yield "zero_couplings", np.array([3.0, 1.0, 4.0, 1.5, 9.0]), np.zeros(4), 1.0
    yield "one", np.array([0.7]), np.zeros(0), 2.0
    yield "two", np.array([2.5, 0.7]), np.array([0.9]), 3.0
    # two identical 30-dimensional blocks: the Krylov space has dimension 30
    A = rng.standard_normal((30, 30))
    A = A @ A.T / 30.0 + 0.1 * np.eye(30)
    a, b = _lanczos_coefficients(scipy.linalg.block_diag(A, A), rng.standard_normal(60), 28)
    yield "twin_blocks28", a, b, 1.0


CASES = list(_cases())


@pytest.mark.parametrize("name,alpha,beta,wnorm", CASES, ids=[c[0] for c in CASES])
def test_every_leading_block_matches_oracle(ctx, name, alpha, beta, wnorm):
    got = ctx.tridiag_sqrt(alpha, beta, wnorm)
    m = alpha.size
    for k in range(1, m + 1):
        ref = lanczos.tridiag_sqrt_e1(alpha[:k], beta[:k - 1], wnorm)
        close(got[k - 1, :k], ref, TOL)
        assert np.all(got[k - 1, k:] == 0.0)


def test_sheet256_lanczos_coefficients_up_to_64(ctx):
    inp = wl.make_inputs(wl.WORKLOADS["sheet256_rsa"], 0)
    M, _ = mobility.dense(inp["pos"])
    w = inp["w"].ravel()
    alpha, beta = _lanczos_coefficients(M, w, 64)
    got = ctx.tridiag_sqrt(alpha, beta, np.linalg.norm(w))
    for k in (1, 2, 3, 8, 25, 40, 64):
        ref = lanczos.tridiag_sqrt_e1(alpha[:k], beta[:k - 1], np.linalg.norm(w))
        close(got[k - 1, :k], ref, TOL)


def test_invalid_arguments_are_rejected(ctx):
    from paper_1612_00474_amd._lib import RPB_EINVAL
    lib = ctx.lib
    a = np.ones(65)
    b = np.ones(64)
    y = np.zeros(65 * 65)
    assert lib.lanczos_tridiag_sqrt(ctx.h, 65, a.ctypes.data, b.ctypes.data, 1.0,
                                    y.ctypes.data, None) == RPB_EINVAL
    assert lib.lanczos_tridiag_sqrt(ctx.h, 0, a.ctypes.data, b.ctypes.data, 1.0,
                                    y.ctypes.data, None) == RPB_EINVAL
    a[3] = np.nan
    assert lib.lanczos_tridiag_sqrt(ctx.h, 5, a.ctypes.data, b.ctypes.data, 1.0,
                                    y.ctypes.data, None) == RPB_EINVAL
    a[3] = 1.0
    assert lib.lanczos_tridiag_sqrt(ctx.h, 5, a.ctypes.data, b.ctypes.data, -1.0,
                                    y.ctypes.data, None) == RPB_EINVAL


def test_overflowing_coefficients_report_failure(ctx):
    """Coefficients whose squares overflow float64: the secular-equation roots cannot settle
    (every root loop is bounded), so the call reports the failure instead of returning
    non-finite values, and the context stays usable."""
    from paper_1612_00474_amd._lib import RPB_EDEVICE
    lib = ctx.lib
    a = np.array([1e300, 1e300])
    b = np.array([1e300])
    y = np.zeros(4)
    assert lib.lanczos_tridiag_sqrt(ctx.h, 2, a.ctypes.data, b.ctypes.data, 1.0,
                                    y.ctypes.data, None) == RPB_EDEVICE
    got = ctx.tridiag_sqrt(np.array([2.5, 0.7]), np.array([0.9]), 3.0)
    close(got[1], lanczos.tridiag_sqrt_e1(np.array([2.5, 0.7]), np.array([0.9]), 3.0), TOL)
