"""Pins of the oracle's KKT report, of its numerical-dependence guard and of the
exact zero the step length gives (values fixed by hand from the KKT conditions
of Theorem 1 and from the inner loop of Algorithms 1 and 3).

Every expected value below is worked out by hand in the comments; none re-types
a formula of the oracle.
"""
import numpy as np
import pytest

import oracle
from workloads import make_c3, make_small


# ---------------------------------------------------------------------------
# kkt_report: scaled KKT residual max(max_Z w+, max_P |w|) / (max_j ||a_j|| ||b||)
# ---------------------------------------------------------------------------
def test_kkt_zero_iterate_with_positive_dual():
    # a0 = (3, 4, 0) (norm 5), a1 = (0, 0, 2) (norm 2), b = (1, 0, 0) (norm 1).
    # At x = 0 the dual is w = A^T b = (3, 0); P is empty, so the residual is
    # max w+ / (5 * 1) = 3 / 5.
    A = np.array([[3.0, 0.0], [4.0, 0.0], [0.0, 2.0]])
    b = np.array([1.0, 0.0, 0.0])
    rep = oracle.kkt_report(A, b, np.zeros(2))
    assert rep["kkt"] == pytest.approx(0.6, rel=1e-15)
    assert rep["dual_z"] == pytest.approx(0.6, rel=1e-15)
    assert rep["dual_p"] == 0.0
    assert rep["feasible"] and not rep["ok"]
    np.testing.assert_array_equal(rep["w"], [3.0, 0.0])
    assert rep["objective"] == 1.0


def test_kkt_zero_iterate_with_nonpositive_dual_is_optimal():
    # same A, b = (-1, 0, 0): w = (-3, 0) <= 0 on Z, so x = 0 satisfies KKT.
    A = np.array([[3.0, 0.0], [4.0, 0.0], [0.0, 2.0]])
    b = np.array([-1.0, 0.0, 0.0])
    rep = oracle.kkt_report(A, b, np.zeros(2))
    assert rep["kkt"] == 0.0 and rep["ok"]


def _orthonormal(m, k, seed):
    Qm, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((m, k)))
    return Qm


def test_kkt_perturbed_passive_entry_orthonormal():
    # A = Q with orthonormal columns (all norms 1), b = Q c with c = (1, 2, 2):
    # ||b|| = 3.  The optimum is x = c (w = 0).  With x_0 raised by 0.3 the
    # residual is r = -0.3 q_0, so w = A^T r = (-0.3, 0, 0); index 0 is passive
    # (x_0 > 0), so max_P |w| = 0.3 and the scaled residual is 0.3 / 3 = 0.1.
    Q = _orthonormal(12, 3, 1)
    c = np.array([1.0, 2.0, 2.0])
    b = Q @ c
    x = c + np.array([0.3, 0.0, 0.0])
    rep = oracle.kkt_report(Q, b, x)
    assert rep["kkt"] == pytest.approx(0.1, rel=1e-12)
    assert rep["dual_p"] == pytest.approx(0.1, rel=1e-12)
    assert rep["dual_z"] == 0.0
    assert not rep["ok"]
    # at the optimum itself the residual vanishes to rounding
    assert oracle.kkt_report(Q, b, c)["kkt"] <= 1e-15


def test_kkt_zero_set_entry_with_positive_dual_orthonormal():
    # same Q and b, x = (1, 2, 0): r = 2 q_2, w = (0, 0, 2); index 2 is in Z
    # with w_2 = 2 > 0, so the scaled residual is 2 / 3.
    Q = _orthonormal(12, 3, 1)
    c = np.array([1.0, 2.0, 2.0])
    b = Q @ c
    rep = oracle.kkt_report(Q, b, np.array([1.0, 2.0, 0.0]))
    assert rep["kkt"] == pytest.approx(2.0 / 3.0, rel=1e-12)
    assert rep["dual_z"] == pytest.approx(2.0 / 3.0, rel=1e-12)
    assert rep["dual_p"] <= 1e-15


def test_kkt_zero_rhs():
    # b = 0: the scale max||a|| ||b|| is 0 and is replaced by 1.  x = 0 is the
    # optimum (kkt 0).  x = e_0 with orthonormal columns: r = -q_0,
    # w = (-1, 0, 0), index 0 passive, so the residual is |w_0| / 1 = 1.
    Q = _orthonormal(9, 3, 2)
    b = np.zeros(9)
    assert oracle.kkt_report(Q, b, np.zeros(3))["kkt"] == 0.0
    rep = oracle.kkt_report(Q, b, np.array([1.0, 0.0, 0.0]))
    assert rep["kkt"] == pytest.approx(1.0, rel=1e-14)


def test_kkt_reports_infeasible_iterate():
    Q = _orthonormal(9, 3, 3)
    b = Q @ np.array([1.0, 1.0, 1.0])
    rep = oracle.kkt_report(Q, b, np.array([1.0, 1.0, -0.5]))
    assert not rep["feasible"] and not rep["ok"]


# ---------------------------------------------------------------------------
# numerical dependence: a column whose projected norm is rounding noise
# ---------------------------------------------------------------------------
DEP_CASES = [1, 16, 18]   # integer data, one column an exact combination of three others


def _dependent_instance(seed):
    rng = np.random.default_rng(seed)
    B = rng.integers(-3, 4, size=(8, 3)).astype(float)
    c = rng.integers(1, 3, size=3).astype(float)
    A = np.column_stack([B, B @ c, B[:, :1] * 3.0])   # columns 3 and 4 lie in range(B)
    b = rng.standard_normal(8)
    return A, b


def _in_span(A, cols, j):
    if not cols:
        return False
    coef, *_ = np.linalg.lstsq(A[:, cols], A[:, j], rcond=None)
    return np.linalg.norm(A[:, cols] @ coef - A[:, j]) <= 1e-12 * np.linalg.norm(A[:, j])


@pytest.mark.parametrize("solver", ["lh", "lhdm"])
@pytest.mark.parametrize("seed", DEP_CASES)
def test_dependent_columns_with_zero_tolerance(seed, solver):
    # With kkt_tol = 0 the dual of a column lying in the span of the passive
    # columns is rounding noise (it is exactly 0 for the least-squares residual).
    # Such a column must never enter P: the solve ends at the true minimum (the
    # brute-force objective over all supports), and it reports "no independent
    # column with positive dual left" exactly when a zero-set column with a
    # positive dual is left and every such column is dependent on P.
    A, b = _dependent_instance(seed)
    fn = oracle.oracle_lh if solver == "lh" else oracle.oracle_lhdm
    x, info = fn(A, b, kkt_tol=0.0)
    xb, objb = oracle.brute_force_nnls(A, b)
    assert info["status"] in (oracle.STATUS_OK, oracle.STATUS_RANK)
    assert abs(info["objective"] - objb) <= 1e-12 * max(1.0, objb)
    P = info["passive"]
    assert np.linalg.matrix_rank(A[:, P]) == len(P)          # P stays independent
    w = A.T @ (b - A @ x)
    Z = [j for j in range(A.shape[1]) if j not in P]
    pos = [j for j in Z if w[j] > 0.0]
    if info["status"] == oracle.STATUS_RANK:
        assert pos and all(_in_span(A, P, j) for j in pos)
    else:
        assert not pos


# ---------------------------------------------------------------------------
# the index attaining the step length leaves P (Algorithms 1 and 3, inner loop)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", [("uniform", 163), ("uniform", 171), ("gauss", 172), ("gauss", 164)])
def test_every_inner_iteration_removes_the_step_length_index(case):
    # alpha = min x_i / (x_i - y_i) over the nonpositive y_i makes the new x_i
    # exactly 0 for the minimising index (in exact arithmetic), so every inner
    # iteration removes at least that index, and its x stays 0.
    kind, seed = case
    if kind == "uniform":
        inst = make_small(40, 120, 12, seed, kind="uniform", noise_std=1e-2)
    else:
        inst = make_c3(5000 + seed, m=48, n=192, k=10)
    x, info = oracle.oracle_lhdm(inst.A, inst.b, record=True)
    assert info["status"] == oracle.STATUS_OK
    n_inner = 0
    for step in info["trace"]:
        for rm in step["removed"]:
            assert len(rm) >= 1
            n_inner += 1
    assert n_inner == info["inner_iters"] and n_inner > 0


# ---------------------------------------------------------------------------
# Theorem 4: tau1 = 1 and tau2 <= 1/2 make the feasibility loop on J idle
# ---------------------------------------------------------------------------
def tie_instance(seed, m=30, ntie=6, nweak=12):
    """Six columns with disjoint 3-row supports of ones (mutually orthogonal,
    norm sqrt(3)) and weak columns of U[0, 0.15] entries; b = ones.  The first
    dual vector is exactly 3 on the six (an exact tie; the weak columns' duals
    are smaller), so with tau1 = 1 the first block holds all six; later duals
    are continuous, so the rest of the path has no rounding-level ties."""
    rng = np.random.default_rng(seed)
    A = np.zeros((m, ntie + nweak))
    rows = rng.permutation(m)
    for i in range(ntie):
        A[rows[3 * i:3 * i + 3], i] = 1.0
    A[:, ntie:] = rng.uniform(0.0, 0.15, size=(m, nweak))
    assert (A[:, ntie:].sum(axis=0) < 3.0).all()
    return A, np.ones(m)


T4 = dict(tau1=1.0, tau2=0.5, kmax=8, delta=0.5 / 7)   # delta <= tau2 / (kmax - 1)


@pytest.mark.parametrize("seed", [11, 12, 13, 14, 15])
def test_theorem4_variant_takes_the_same_path(seed):
    # with tau1 = 1, tau2 <= 1/2 and delta <= tau2 / (kmax - 1), Theorem 4 says
    # the feasibility loop never drops a column, so skipping it must leave the
    # whole path unchanged
    A, b = tie_instance(seed)
    x1, i1 = oracle.oracle_lhdm(A, b, record=True, **T4)
    x2, i2 = oracle.oracle_lhdm(A, b, record=True, jloop=False, **T4)
    assert i1["jloop_drops"] == 0 and i2["jloop_drops"] == 0
    assert [s["J"] for s in i1["trace"]] == [s["J"] for s in i2["trace"]]
    assert i1["passive"] == i2["passive"]
    np.testing.assert_array_equal(x1, x2)
    assert len(i2["trace"][0]["J"]) == 6          # the tied orthogonal columns, in index order
    assert i2["trace"][0]["J"] == [0, 1, 2, 3, 4, 5]
    assert oracle.kkt_report(A, b, x2)["kkt"] <= 1e-9


def test_theorem4_variant_needs_its_thresholds():
    A, b = tie_instance(11)
    with pytest.raises(ValueError):
        oracle.oracle_lhdm(A, b, tau1=0.6, tau2=0.15, jloop=False)
    with pytest.raises(ValueError):
        oracle.oracle_lhdm(A, b, tau1=1.0, tau2=0.6, jloop=False)
    with pytest.raises(ValueError):
        oracle.oracle_lhdm(A, b, tau1=1.0, tau2=0.5, kmax=8, delta=0.9, jloop=False)


def test_zero_iterate_entry_limits_the_step_to_zero():
    # without the feasibility loop a new column can enter the inner loop with
    # x_j = 0 and y_j <= 0: its ratio is 0, so the step is 0 and it leaves P
    from oracle.nnls import _QRState, _inner_step
    A = np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]])
    st = _QRState(A, np.array([1.0, -1.0, 0.0]))
    st.append(0)
    st.append(1)
    x = np.array([0.5, 0.0])
    y = st.solve()                       # (1, -1): column 1 has y <= 0 and x = 0
    rm, alpha = _inner_step(st, x, y)
    assert alpha == 0.0 and rm == [1] and st.P == [0] and x[0] == 0.5
