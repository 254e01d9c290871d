"""The small factorisations of the CholeskyQR2 panel, on the GPU.

The test-only C-ABI entry ``lhdm_test_cq_factors`` runs the one-wave
factorisations used by the whole-device engine on caller matrices:
- the Cholesky factor of a Gram matrix together with its inverse;
- the LU factorisation without pivoting of W - S = L U (the signs S chosen
  step by step), by row elimination (U and L^{-1}) and by column elimination
  (L and U^{-1}) side by side, which is how the Householder reflectors and
  their compact-WY factor are rebuilt from an orthonormal basis.

The results are checked against what defines them: R^T R = G, R R^{-1} = I,
L^{-1} (W - S) = U with L^{-1} unit lower and |U[t][t]| >= 1, the two
eliminations' signs equal and their factors each other's inverses.  They are
also checked against numpy's Cholesky and a plain LU with the same sign rule.
"""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2108_05345_amd import _lib
    lib = _lib.load()   # fails loudly if the HIP library is missing
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib


def _run(lib, G, W):
    n = G.shape[0]
    d = torch.device("cuda:0")
    tG = torch.from_numpy(np.asfortranarray(G).ravel(order="F").copy()).to(d)
    tW = torch.from_numpy(np.asfortranarray(W).ravel(order="F").copy()).to(d)
    outs = [torch.zeros(n * n, dtype=torch.float64, device=d) for _ in range(6)]
    sg = torch.zeros(n, dtype=torch.float64, device=d)
    sg2 = torch.zeros(n, dtype=torch.float64, device=d)
    sin2 = ctypes.c_double()
    rc = lib.lhdm_test_cq_factors(torch.cuda.current_stream(d).cuda_stream, n, tG.data_ptr(), tW.data_ptr(),
                                  *[o.data_ptr() for o in outs], sg.data_ptr(), sg2.data_ptr(), ctypes.byref(sin2))
    assert rc == 0, rc
    R, Ri, U, Li, L, Ui = [o.cpu().numpy().reshape(n, n, order="F") for o in outs]
    assert np.array_equal(sg.cpu().numpy(), sg2.cpu().numpy())
    return R, Ri, U, Li, L, Ui, sg.cpu().numpy(), sin2.value


def _lu_signed(W):
    # LU without pivoting of W - S, s_t = +1 for a negative pivot, else -1
    A = W.copy()
    n = A.shape[0]
    s = np.zeros(n)
    L = np.eye(n)
    for t in range(n):
        s[t] = 1.0 if A[t, t] < 0 else -1.0
        A[t, t] -= s[t]
        L[t + 1:, t] = A[t + 1:, t] / A[t, t]
        A[t + 1:, t + 1:] -= np.outer(L[t + 1:, t], A[t, t + 1:])
        A[t + 1:, t] = 0.0
    return L, np.triu(A), s


@pytest.mark.parametrize("n", [1, 2, 5, 16, 17, 31, 32])
def test_factors_against_their_definitions(lib, n):
    rng = np.random.default_rng(100 + n)
    X = rng.standard_normal((400, n)) * rng.uniform(0.5, 3.0, n)
    G = X.T @ X
    Q, _ = np.linalg.qr(rng.standard_normal((400, n)))
    W = Q[:n, :].copy()
    R, Ri, U, Li, L, Ui, sg, sin2 = _run(lib, G, W)
    # Cholesky and inverse
    assert np.array_equal(R, np.triu(R)) and (np.diag(R) > 0).all()
    assert np.abs(R.T @ R - G).max() <= 1e-14 * np.abs(G).max()
    assert np.abs(R @ Ri - np.eye(n)).max() <= 1e-13
    assert np.array_equal(Ri, np.triu(Ri))
    Rn = np.linalg.cholesky(G).T
    assert np.abs(R - Rn).max() <= 1e-13 * np.abs(Rn).max()
    assert sin2 == pytest.approx(float(np.min(np.diag(Rn) ** 2 / np.diag(G))), rel=1e-10)
    # LU of W - S with its signs, and L^{-1}
    Lr, Ur, sr = _lu_signed(W)
    assert np.array_equal(sg, sr)
    assert np.array_equal(Li, np.tril(Li)) and np.array_equal(np.diag(Li), np.ones(n))
    assert np.array_equal(U, np.triu(U))
    assert np.abs(Li @ (W - np.diag(sg)) - U).max() <= 1e-13
    assert (np.abs(np.diag(U)) >= 1.0 - 1e-12).all()
    assert np.abs(L - Lr).max() <= 1e-12 and np.abs(U - Ur).max() <= 1e-12
    # the column elimination: L unit lower, U^{-1} upper, each the other's inverse
    assert np.array_equal(L, np.tril(L)) and np.array_equal(np.diag(L), np.ones(n))
    assert np.array_equal(Ui, np.triu(Ui))
    assert np.abs(L @ Li - np.eye(n)).max() <= 1e-12
    assert np.abs(U @ Ui - np.eye(n)).max() <= 1e-12


def test_not_positive_definite(lib):
    # a Gram matrix with a negative eigenvalue: the factorisation reports -1
    n = 6
    rng = np.random.default_rng(5)
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    G = V @ np.diag([4.0, 3.0, 2.0, 1.0, 0.5, -0.5]) @ V.T
    *_, sin2 = _run(lib, G, np.eye(n))
    assert sin2 == -1.0
