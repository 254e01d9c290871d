"""The whole-device engine's triangular solve R y = bt, on the GPU.

The test-only C-ABI entry ``lhdm_test_trsv`` runs the solver's chained
back substitution (the least-squares step of Algorithms 1 and 3) on a caller's
R: 64-row blocks from the bottom, the blocks far enough up the chain through
the inverse of their row-scaled diagonal block, the others by substitution.

The results are checked against a back substitution in extended precision
(numpy longdouble): the GPU's error may be at most ten times that of LAPACK's
substitution in double precision (plus a rounding-level floor), on R factors of
well- and ill-conditioned matrices, at sizes with and without inverted blocks
and with a ragged last block.  A block whose inverse overflows while the
substitution stays exact checks the fall-back to substitution.
"""
import ctypes

import numpy as np
import pytest
import scipy.linalg as sl
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2108_05345_amd import _lib
    lib = _lib.load()   # fails loudly if the HIP library is missing
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib


def _run(lib, R, bt):
    n = R.shape[0]
    d = torch.device("cuda:0")
    tR = torch.from_numpy(np.asfortranarray(R).ravel(order="F").copy()).to(d)
    tb = torch.from_numpy(bt.copy()).to(d)
    ty = torch.zeros(n, dtype=torch.float64, device=d)
    ninv = ctypes.c_int32(-1)
    print(f"[trsv] n={n}", flush=True)
    rc = lib.lhdm_test_trsv(torch.cuda.current_stream(d).cuda_stream, n, tR.data_ptr(), tb.data_ptr(),
                            ty.data_ptr(), ctypes.byref(ninv))
    assert rc == 0, rc
    return ty.cpu().numpy(), ninv.value


def _exact(R, b):
    # column-oriented back substitution in extended precision
    n = R.shape[0]
    Rl = R.astype(np.longdouble)
    y = b.astype(np.longdouble).copy()
    for i in range(n - 1, -1, -1):
        y[i] /= Rl[i, i]
        y[:i] -= Rl[:i, i] * y[i]
    return y


def _expected_inverted(n):
    # full 64-row blocks at least four places from the bottom of the chain
    nb, full = (n + 63) // 64, n // 64
    return sum(1 for g in range(4, nb) if nb - 1 - g < full)


def _r_factor(kind, n, rng):
    if kind == "gauss":
        return np.linalg.qr(rng.standard_normal((n + 64, n)), mode="r")
    # condition number 1e6 and a row range of 1e5, as the ill-conditioned workload
    m = n + 64
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (U * np.logspace(0, -6, n)) @ V.T
    A *= np.logspace(0, 5, m)[:, None]
    return np.linalg.qr(A, mode="r")


@pytest.mark.parametrize("n", [1, 63, 64, 65, 257, 320, 1000, 4096])
@pytest.mark.parametrize("kind", ["gauss", "illcond"])
def test_against_extended_precision(lib, n, kind):
    rng = np.random.default_rng(7 * n + (kind == "illcond"))
    R = _r_factor(kind, n, rng)
    b = rng.standard_normal(n)
    y, ninv = _run(lib, R, b)
    assert ninv == _expected_inverted(n)
    ye = _exact(R, b)
    scale = float(np.abs(ye).max())
    e_gpu = float(np.abs(y - ye).max()) / scale
    e_lapack = float(np.abs(sl.solve_triangular(R, b) - ye).max()) / scale
    print(f"[trsv] {kind} n={n} inverted blocks {ninv}: error {e_gpu:.2e} (LAPACK {e_lapack:.2e})", flush=True)
    assert np.isfinite(y).all()
    assert e_gpu <= 10.0 * e_lapack + 1e-15


def test_largest_size(lib):
    n = 8192
    rng = np.random.default_rng(8192)
    R = np.triu(rng.standard_normal((n, n))) * 0.01
    R[np.diag_indices(n)] = rng.uniform(1.0, 2.0, n)
    b = rng.standard_normal(n)
    y, ninv = _run(lib, R, b)
    assert ninv == _expected_inverted(n) == 124
    ye = _exact(R, b)
    e_gpu = float(np.abs(y - ye).max() / np.abs(ye).max())
    e_lapack = float(np.abs(sl.solve_triangular(R, b) - ye).max() / np.abs(ye).max())
    assert e_gpu <= 10.0 * e_lapack + 1e-15


def test_overflowing_inverse_falls_back(lib):
    # The top block of a 320-row identity gets R[0][1] = R[1][2] = 1e200, so
    # its inverse holds (1e200)^2 = inf, while with bt[1] = bt[2] = 0 the
    # substitution gives y = bt exactly (every product with 1e200 is by 0).
    # The block is five places from the bottom, so it is eligible for the
    # inverse form, and only the fall-back gets y right.
    n = 320
    R = np.eye(n)
    R[0, 1] = R[1, 2] = 1e200
    rng = np.random.default_rng(3)
    b = rng.standard_normal(n)
    b[1] = b[2] = 0.0
    y, ninv = _run(lib, R, b)
    assert ninv == 1
    assert np.array_equal(y, b)
