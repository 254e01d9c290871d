"""Pins of the l1-NNLS front end (Section 3.3) in the oracle: the squared-l1
regularised least-squares problem min ||x||_1^2 + lam^2 ||A x - b||^2 written
as an NNLS problem on [1^T, 1^T; lam A, -lam A] and [0; lam b].

The checks come from the regularised problem itself, not from its NNLS form: a
closed form for one column, the optimality (subgradient) conditions derived by
hand, and the limit lam -> infinity (exact sparse recovery, Section 3.3)."""
import numpy as np
import pytest

import oracle
from workloads import make_signed


@pytest.mark.parametrize("sgn", [1.0, -1.0])
def test_l1_single_column_closed_form(sgn):
    # f(t) = t^2 + lam^2 ||a t - b||^2 is minimised at t = lam^2 a.b / (1 + lam^2 ||a||^2),
    # whose sign is that of a.b
    rng = np.random.default_rng(1)
    a = rng.standard_normal((7, 1))
    b = sgn * np.sign(float(a[:, 0] @ rng.standard_normal(7))) * rng.standard_normal(7)
    for lam in (0.5, 2.0, 10.0):
        x, info = oracle.oracle_l1nnls(a, b, lam)
        ab, aa = float(a[:, 0] @ b), float(a[:, 0] @ a[:, 0])
        ref = lam ** 2 * ab / (1.0 + lam ** 2 * aa)
        assert abs(x[0] - ref) <= 1e-13 * max(1.0, abs(ref))


def _l1_optimality(A, b, lam, x, tol):
    # 0 in 2 ||x||_1 d||x||_1 + 2 lam^2 A^T (A x - b): with g = lam^2 A^T (b - A x)
    # and s = ||x||_1, g_j = s sign(x_j) where x_j != 0 and |g_j| <= s where x_j = 0
    g = lam ** 2 * (A.T @ (b - A @ x))
    s = float(np.abs(x).sum())
    nz = x != 0.0
    assert np.all(np.abs(g[nz] - s * np.sign(x[nz])) <= tol * max(1.0, s))
    assert np.all(np.abs(g[~nz]) <= s + tol * max(1.0, s))


@pytest.mark.parametrize("method", ["lhdm", "lh"])
@pytest.mark.parametrize("lam", [0.3, 3.0, 30.0])
def test_l1_optimality_conditions(method, lam):
    inst = make_signed(40, 90, 6, 3, noise_std=1e-2)
    x, info = oracle.oracle_l1nnls(inst.A, inst.b, lam, method=method)
    assert info["status"] == oracle.STATUS_OK
    _l1_optimality(inst.A, inst.b, lam, x, 1e-8)
    z = info["z"]
    assert not np.any((z[:90] > 0) & (z[90:] > 0))       # never both parts of one entry


def test_l1_large_lambda_recovers_the_sparse_solution():
    # as lam grows the residual term dominates and the minimiser tends to the
    # minimum-l1 solution of A x = b, which is the planted sparse x here
    inst = make_signed(60, 150, 5, 4)
    errs = []
    for lam in (1.0, 10.0, 100.0, 1000.0):
        x, info = oracle.oracle_l1nnls(inst.A, inst.b, lam)
        errs.append(float(np.abs(x - inst.x_true).max()))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))
    assert errs[-1] <= 1e-4


def test_l1_matrix_layout():
    A = np.array([[1.0, 2.0], [3.0, 4.0]])
    M, rhs = oracle.l1nnls_matrix(A, np.array([5.0, 6.0]), 2.0)
    np.testing.assert_array_equal(M, [[1, 1, 1, 1], [2, 4, -2, -4], [6, 8, -6, -8]])
    np.testing.assert_array_equal(rhs, [0, 10, 12])
