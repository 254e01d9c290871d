"""Pins of the positivity trick (Section 3.2) and of its sign-flip inner loop
(Section 4.2) in the oracle.

The facts checked: negating one column of a triangular factor negates exactly
that component of the back-substitution solution and leaves the residual
unchanged (the identity Section 4.2 derives), brute force over all supports of
the 2n-column problem, the signed least-squares closed form for orthogonal A,
exact signed recovery of planted sparse solutions, and the KKT conditions of
Theorem 1 on [A, -A].
"""
import numpy as np
import pytest
from scipy.linalg import solve_triangular

import oracle
from oracle.nnls import _QRState, _sign_flip
from workloads import make_signed


def test_flipping_a_column_of_r_flips_that_component():
    # Section 4.2: R y = c and R' = R with column k negated give y' = (y1, -y_k, y2);
    # back substitution forms the same products, so the identity holds bitwise
    rng = np.random.default_rng(3)
    for k in (0, 3, 7):
        R = np.triu(rng.standard_normal((8, 8))) + 4 * np.eye(8)
        c = rng.standard_normal(8)
        y = solve_triangular(R, c)
        R2 = R.copy()
        R2[:, k] = -R2[:, k]
        y2 = solve_triangular(R2, c)
        expect = y.copy()
        expect[k] = -expect[k]
        np.testing.assert_array_equal(y2, expect)


def test_sign_flip_step_keeps_the_residual():
    # on a QR state of [B, -B] with three passive columns: flip the ones with a
    # negative least-squares component; y changes sign there, nothing else does,
    # the twins take their places, and A_P y (hence the residual) is unchanged
    rng = np.random.default_rng(5)
    B = rng.standard_normal((10, 4))
    A = np.concatenate([B, -B], axis=1)
    b = B @ np.array([1.0, -2.0, 0.5, -1.0])
    st = _QRState(A, b)
    for j in (0, 1, 3):
        st.append(j)
    y = st.solve()
    assert (y < 0).any() and (y > 0).any()
    x = np.zeros(8)
    x[[0, 1, 3]] = 1.0
    fit = A[:, st.P] @ y
    pairs = _sign_flip(st, x, y)
    assert pairs == [(j, j + 4) for c, j in enumerate([0, 1, 3]) if y[c] < 0]
    y2 = st.solve()
    np.testing.assert_array_equal(y2, np.abs(y))
    np.testing.assert_allclose(A[:, st.P] @ y2, fit, rtol=0, atol=1e-14)
    assert all(x[j] == 0.0 for j, _ in pairs)
    assert sorted(st.pos[st.pos >= 0].tolist()) == [0, 1, 2]


@pytest.mark.parametrize("method", ["lh", "lhdm"])
@pytest.mark.parametrize("flip", [True, False])
@pytest.mark.parametrize("seed", range(10))
def test_signed_brute_force_tiny(method, flip, seed):
    rng = np.random.default_rng(40 + seed)
    m = int(rng.integers(3, 9))
    n = int(rng.integers(2, 8))
    A = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    x, info = oracle.oracle_signed(A, b, method=method, sign_flip=flip)
    assert info["status"] == oracle.STATUS_OK
    A2 = np.concatenate([A, -A], axis=1)
    zb, objb = oracle.brute_force_nnls(A2, b)
    r = b - A @ x
    assert abs(float(r @ r) - objb) <= 1e-10 * max(1.0, objb)
    assert oracle.kkt_report(A2, b, info["z"])["kkt"] <= 1e-9
    # no column and its twin are passive together
    P = set(info["passive"])
    assert not any(j in P and (j + n) in P for j in range(n))
    if m >= n:   # full column rank: the signed least-squares solution is unique
        xls, *_ = np.linalg.lstsq(A, b, rcond=None)
        np.testing.assert_allclose(x, xls, rtol=0, atol=1e-9 * max(1.0, np.abs(xls).max()))


def test_signed_orthogonal_closed_form():
    # A with orthonormal columns: the signed least-squares solution is A^T b
    rng = np.random.default_rng(9)
    Q, _ = np.linalg.qr(rng.standard_normal((30, 12)))
    b = rng.standard_normal(30)
    for method in ("lh", "lhdm"):
        x, info = oracle.oracle_signed(Q, b, method=method)
        np.testing.assert_allclose(x, Q.T @ b, rtol=0, atol=1e-13)


@pytest.mark.parametrize("method", ["lh", "lhdm"])
@pytest.mark.parametrize("case", [(64, 128, 8, 1), (128, 512, 20, 2), (256, 1024, 40, 3)])
def test_signed_planted_recovery(method, case):
    # Section 3.2: a sparse signed solution of A x = b is recovered by the NNLS
    # problem on [A, -A]; with the sign flip as with the ordinary inner loop
    m, n, k, seed = case
    inst = make_signed(m, n, k, seed)
    x1, i1 = oracle.oracle_signed(inst.A, inst.b, method=method, sign_flip=True, record=True)
    x2, i2 = oracle.oracle_signed(inst.A, inst.b, method=method, sign_flip=False, record=True)
    np.testing.assert_allclose(x1, inst.x_true, rtol=0, atol=1e-12)
    np.testing.assert_allclose(x2, inst.x_true, rtol=0, atol=1e-12)
    # the sign-flip solve never downdates here (no exactly zero component)
    assert all(len(s["removed"]) == 0 for s in i1["trace"])


def test_sign_flip_replaces_inner_iterations():
    # an instance whose ordinary inner loop runs: the sign-flip solve flips
    # instead of downdating, and both reach the same signed solution
    inst = make_signed(128, 512, 20, 2)
    x1, i1 = oracle.oracle_signed(inst.A, inst.b, method="lhdm", sign_flip=True, record=True)
    x2, i2 = oracle.oracle_signed(inst.A, inst.b, method="lhdm", sign_flip=False, record=True)
    assert i2["inner_iters"] > 0
    assert sum(len(f) for s in i1["trace"] for f in s["flipped"]) > 0
    assert sum(len(r) for s in i1["trace"] for r in s["removed"]) == 0
    np.testing.assert_allclose(x1, x2, rtol=0, atol=1e-12)


def test_sign_flip_needs_the_twin_structure():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((6, 8))
    with pytest.raises(ValueError):
        oracle.oracle_lhdm(A, rng.standard_normal(6), sign_flip=True)
