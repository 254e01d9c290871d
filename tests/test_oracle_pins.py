"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests re-types a formula of ``oracle/nnls.py``: each checks a
defining property, a printed example, a closed form, brute force on tiny
inputs, planted recovery, a library routine, or a third-party solver run as a
black box.
"""
import os

import numpy as np
import pytest
import scipy.optimize

import oracle
from oracle.nnls import _QRState, _dm
from workloads import make_c1, make_small, make_c3, make_c4_batch

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# elementary transformations
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(5))
def test_house_defining_property(seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(7) * (10.0 ** rng.integers(-3, 4))
    v, beta, alpha = oracle.house(x)
    H = np.eye(7) - beta * np.outer(v, v)
    e1 = np.zeros(7)
    e1[0] = 1.0
    np.testing.assert_allclose(H @ x, alpha * e1, atol=1e-13 * np.linalg.norm(x))
    np.testing.assert_allclose(H.T @ H, np.eye(7), atol=1e-14)
    assert abs(abs(alpha) - np.linalg.norm(x)) <= 1e-14 * np.linalg.norm(x)


def test_house_zero_vector():
    v, beta, alpha = oracle.house(np.zeros(4))
    assert beta == 0.0 and alpha == 0.0


@pytest.mark.parametrize("a,b", [(3.0, 4.0), (-1.0, 2.0), (0.0, 5.0), (2.0, 0.0), (-1e-300, 1e-300)])
def test_givens_defining_property(a, b):
    c, s = oracle.givens(a, b)
    G = np.array([[c, s], [-s, c]])
    out = G @ np.array([a, b])
    assert abs(out[1]) <= 1e-15 * max(abs(a), abs(b), 1e-300)
    assert abs(c * c + s * s - 1.0) < 1e-15


# ---------------------------------------------------------------------------
# Algorithm 5: the worked example of Section 4.1
# ---------------------------------------------------------------------------
def _read_golden():
    rows = []
    meta = {}
    with open(os.path.join(GOLDEN, "downdate_example.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] in ("m", "n", "deleted"):
                meta[parts[0]] = [int(p) for p in parts[1:]]
            else:
                rows.append((int(parts[0]), int(parts[1])))
    return meta, rows


def test_downdate_worked_example_order():
    meta, expected = _read_golden()
    n = meta["n"][0]
    deleted0 = [d - 1 for d in meta["deleted"]]
    got = oracle.downdate_rotations(n, deleted0)
    got1 = [(r + 1, c + 1) for (r, c) in got]
    assert got1 == expected


def test_downdate_rotation_count_formula():
    # Section 4.1: a remaining column lying between the l-th and (l+1)-th deleted
    # columns has exactly l subdiagonal entries to annihilate.
    rng = np.random.default_rng(0)
    for _ in range(50):
        n = int(rng.integers(2, 30))
        q = int(rng.integers(1, n))
        dels = sorted(rng.choice(n, q, replace=False).tolist())
        expected = 0
        for l in range(1, q + 1):
            nxt = dels[l] if l < q else n
            expected += l * (nxt - dels[l - 1] - 1)
        assert len(oracle.downdate_rotations(n, dels)) == expected


def _r_equal_up_to_signs(R1, R2, tol):
    d1 = np.sign(np.diag(R1))
    d2 = np.sign(np.diag(R2))
    np.testing.assert_allclose(d1[:, None] * R1, d2[:, None] * R2, atol=tol)


@pytest.mark.parametrize("seed", range(6))
def test_append_and_remove_match_library_qr(seed):
    rng = np.random.default_rng(seed)
    m, n = 30, 40
    A = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    st = _QRState(A, b)
    order = rng.choice(n, 18, replace=False).tolist()
    for j in order:
        st.append(j)
    _, Rlib = np.linalg.qr(A[:, order])
    _r_equal_up_to_signs(st.R(), Rlib, 1e-12)
    y = st.solve()
    ylib, *_ = np.linalg.lstsq(A[:, order], b, rcond=None)
    np.testing.assert_allclose(y, ylib, rtol=1e-11, atol=1e-12)
    # delete a few positions (Algorithm 5) and compare again
    rm = sorted(rng.choice(18, int(rng.integers(1, 5)), replace=False).tolist())
    st.remove_positions(rm)
    keep = [j for c, j in enumerate(order) if c not in rm]
    assert st.P == keep
    _, Rlib2 = np.linalg.qr(A[:, keep])
    _r_equal_up_to_signs(st.R(), Rlib2, 1e-12)
    y2 = st.solve()
    ylib2, *_ = np.linalg.lstsq(A[:, keep], b, rcond=None)
    np.testing.assert_allclose(y2, ylib2, rtol=1e-11, atol=1e-12)
    # the trailing block keeps the projected column norms (u of Algorithm 3)
    Qk, _ = np.linalg.qr(A[:, keep])
    proj = A - Qk @ (Qk.T @ A)
    np.testing.assert_allclose(st.proj_norms(), np.linalg.norm(proj, axis=0), atol=1e-12)


# ---------------------------------------------------------------------------
# Algorithm 2 against its definition evaluated from scratch
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("delta", [0.2, 0.5, 0.9])
def test_dm_selection_matches_definition(delta):
    inst = make_c3(3001, m=96, n=384, k=19)
    A, b = inst.A, inst.b
    # follow an LHDM run and re-evaluate the selection at every outer step
    x, info = oracle.oracle_lhdm(A, b, delta=delta, record=True)
    st = _QRState(np.asarray(A), b)
    xcur = np.zeros(A.shape[1])
    anorm = np.linalg.norm(A, axis=0)
    checked = 0
    for step in info["trace"]:
        w = A.T @ (b - A @ xcur)
        u = st.proj_norms()
        excl = np.zeros(A.shape[1], bool)
        J = _dm(st, w, u, anorm, excl, 0.6, 0.15, delta, 32)
        Jref = oracle.dm_select_reference(A, b, st.P, xcur, 0.6, 0.15, delta, 32)
        assert J == Jref
        assert J[: len(step["J"])] == step["J"]
        checked += 1
        # replay the step on a fresh state: append J, drop to the accepted prefix, removals
        for j in J:
            st.append(j)
        for _ in range(len(J) - len(step["J"])):
            st.drop_last()
        for rm in step["removed"]:
            pos = [st.P.index(j) for j in rm]
            st.remove_positions(pos)
        xcur = np.zeros(A.shape[1])
        xcur[st.P] = st.solve()
    assert checked >= 2


# ---------------------------------------------------------------------------
# whole solves: brute force, closed forms, planted recovery, third party
# ---------------------------------------------------------------------------
SOLVERS = {
    "lh": lambda A, b, **k: oracle.oracle_lh(A, b, **k),
    "lhdm": lambda A, b, **k: oracle.oracle_lhdm(A, b, **k),
    "lhdm_k3_d05": lambda A, b, **k: oracle.oracle_lhdm(A, b, kmax=3, delta=0.5, **k),
}


@pytest.mark.parametrize("solver", list(SOLVERS))
@pytest.mark.parametrize("seed", range(12))
def test_brute_force_tiny(solver, seed):
    rng = np.random.default_rng(100 + seed)
    m = int(rng.integers(3, 12))
    n = int(rng.integers(2, 11))
    if seed % 3 == 0:
        A = rng.uniform(0, 1, (m, n))
    else:
        A = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    x, info = SOLVERS[solver](A, b)
    xb, objb = oracle.brute_force_nnls(A, b)
    assert info["status"] == oracle.STATUS_OK
    r = b - A @ x
    assert (x >= 0).all()
    assert abs(float(r @ r) - objb) <= 1e-10 * max(1.0, objb)
    rep = oracle.kkt_report(A, b, x)
    assert rep["kkt"] <= 1e-9
    if m >= n:   # full column rank almost surely: unique minimiser
        np.testing.assert_allclose(x, xb, atol=1e-9)


@pytest.mark.parametrize("solver", list(SOLVERS))
def test_closed_form_single_column(solver):
    rng = np.random.default_rng(7)
    for _ in range(10):
        a = rng.standard_normal((9, 1))
        b = rng.standard_normal(9)
        x, _ = SOLVERS[solver](a, b)
        ref = max(0.0, float(a[:, 0] @ b) / float(a[:, 0] @ a[:, 0]))
        assert abs(x[0] - ref) <= 1e-14 * max(1.0, abs(ref))


@pytest.mark.parametrize("solver", list(SOLVERS))
def test_closed_form_orthonormal_columns(solver):
    rng = np.random.default_rng(8)
    Qm, _ = np.linalg.qr(rng.standard_normal((40, 15)))
    b = rng.standard_normal(40)
    x, _ = SOLVERS[solver](Qm, b)
    np.testing.assert_allclose(x, np.maximum(Qm.T @ b, 0.0), atol=1e-13)


@pytest.mark.parametrize("solver", list(SOLVERS))
def test_closed_form_nonpositive_dual_gives_zero(solver):
    rng = np.random.default_rng(9)
    A = rng.uniform(0, 1, (20, 30))
    b = -rng.uniform(0, 1, 20)           # A^T b < 0 componentwise
    x, info = SOLVERS[solver](A, b)
    assert np.all(x == 0.0) and info["outer_iters"] == 0


@pytest.mark.parametrize("solver", list(SOLVERS))
def test_closed_form_interior_least_squares(solver):
    rng = np.random.default_rng(10)
    A = rng.standard_normal((50, 12))
    xt = rng.uniform(1, 2, 12)
    b = A @ xt + 1e-3 * rng.standard_normal(50)
    xls, *_ = np.linalg.lstsq(A, b, rcond=None)
    assert (xls > 0).all()
    x, _ = SOLVERS[solver](A, b)
    np.testing.assert_allclose(x, xls, rtol=1e-11)


@pytest.mark.parametrize("solver", list(SOLVERS))
@pytest.mark.parametrize("seed", [1000, 1001, 1002, 1003, 1004])
def test_planted_recovery_c1(solver, seed):
    inst = make_c1(seed)
    x, info = SOLVERS[solver](inst.A, inst.b)
    assert info["status"] == oracle.STATUS_OK
    np.testing.assert_allclose(x, inst.x_true, atol=1e-12)
    supp = np.nonzero(x > 1e-12 * x.max())[0]
    assert np.array_equal(supp, inst.support)


@pytest.mark.parametrize("seed", range(4))
def test_against_scipy_nnls_positive_residual(seed):
    inst = make_c4_batch(seed=4000 + seed, count=1, m_lo=40, m_hi=90)[0]
    xs, _ = scipy.optimize.nnls(inst.A, inst.b, maxiter=50 * inst.n)
    for name, solver in SOLVERS.items():
        x, info = solver(inst.A, inst.b)
        assert info["status"] == oracle.STATUS_OK
        rep = oracle.kkt_report(inst.A, inst.b, x)
        assert rep["kkt"] <= 1e-9
        rs = inst.b - inst.A @ xs
        assert abs(rep["objective"] - float(rs @ rs)) <= 1e-9 * float(rs @ rs)
        np.testing.assert_allclose(x, xs, atol=1e-8)


def test_lhdm_with_kmax_one_is_lh():
    inst = make_c3(3002, m=64, n=256, k=13)
    x1, i1 = oracle.oracle_lh(inst.A, inst.b, record=True)
    x2, i2 = oracle.oracle_lhdm(inst.A, inst.b, kmax=1, record=True)
    assert i1["passive"] == i2["passive"]
    assert [s["J"] for s in i1["trace"]] == [s["J"] for s in i2["trace"]]
    np.testing.assert_array_equal(x1, x2)


# ---------------------------------------------------------------------------
# invariants of the finite-convergence proof (Theorem 3) and Theorem 4
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed,delta", [(3003, 0.9), (3004, 0.5), (3005, 0.2)])
def test_convergence_invariants(seed, delta):
    inst = make_c3(seed, m=128, n=512, k=26)
    A, b = inst.A, inst.b
    x, info = oracle.oracle_lhdm(A, b, delta=delta, record=True)
    assert info["status"] == oracle.STATUS_OK
    objs = [float(b @ b)] + [s["obj"] for s in info["trace"]]
    assert all(objs[i + 1] < objs[i] for i in range(len(objs) - 1))      # strict decrease
    seen = set()
    P = []
    for s in info["trace"]:
        P = P + s["J"]
        if s["removed"]:
            # the block J survives the first inner iteration
            assert not (set(s["removed"][0]) & set(s["J"]))
        for rm in s["removed"]:
            P = [j for j in P if j not in rm]
        key = frozenset(P)
        assert key not in seen                                          # no passive set repeats
        seen.add(key)
        assert len(s["J"]) >= 1
    assert P == info["passive"]
    assert (x >= 0).all() and np.all(x[info["passive"]] > 0)
    assert oracle.kkt_report(A, b, x)["kkt"] <= 1e-9


def test_theorem4_tied_block_needs_no_feasibility_loop():
    # integer matrix, b = ones: the first dual vector A^T b has exact ties, so with
    # tau1 = 1 the candidate set is the tied columns; Theorem 4 says y_J > 0.
    rng = np.random.default_rng(11)
    base = rng.integers(0, 5, size=(24,)).astype(float)
    cols = [rng.permutation(base) for _ in range(6)]
    cols += [rng.integers(0, 3, size=(24,)).astype(float) for _ in range(10)]
    A = np.stack(cols, axis=1)
    b = np.ones(24)
    w0 = A.T @ b
    assert np.sum(w0 == w0.max()) >= 3
    x, info = oracle.oracle_lhdm(A, b, tau1=1.0, tau2=0.5, delta=0.9, kmax=8, record=True)
    assert len(info["trace"][0]["J"]) >= 2
    assert info["jloop_drops"] == 0
    assert oracle.kkt_report(A, b, x)["kkt"] <= 1e-9


# ---------------------------------------------------------------------------
# degenerate inputs
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("solver", list(SOLVERS))
def test_degenerate_inputs(solver):
    rng = np.random.default_rng(12)
    A = rng.standard_normal((10, 6))
    # b = 0
    x, info = SOLVERS[solver](A, np.zeros(10))
    assert np.all(x == 0) and info["status"] == oracle.STATUS_OK
    # non-finite input
    A2 = A.copy()
    A2[3, 2] = np.nan
    x, info = SOLVERS[solver](A2, rng.standard_normal(10))
    assert info["status"] == oracle.STATUS_NONFINITE and np.all(x == 0)
    # duplicate and zero columns
    A3 = np.concatenate([A, A[:, :2], np.zeros((10, 1))], axis=1)
    b3 = rng.standard_normal(10)
    x, info = SOLVERS[solver](A3, b3)
    assert info["status"] == oracle.STATUS_OK
    xb, objb = oracle.brute_force_nnls(A3, b3)
    assert abs(info["objective"] - objb) <= 1e-10 * max(1.0, objb)
    # m smaller than kmax, underdetermined
    A4 = rng.standard_normal((3, 12))
    b4 = rng.standard_normal(3)
    x, info = SOLVERS[solver](A4, b4)
    xb, objb = oracle.brute_force_nnls(A4, b4)
    assert abs(info["objective"] - objb) <= 1e-10 * max(1.0, objb)
    assert info["n_passive"] <= 3


def test_max_outer_reports_maxiter():
    inst = make_small(40, 120, 10, 5)
    x, info = oracle.oracle_lhdm(inst.A, inst.b, max_outer=1)
    assert info["status"] == oracle.STATUS_MAXITER
    assert (x >= 0).all()


# ---------------------------------------------------------------------------
# the derivative through the final passive set, against finite differences
# ---------------------------------------------------------------------------
def test_backward_reference_against_central_differences():
    rng = np.random.default_rng(13)
    m, n = 30, 12
    A = rng.standard_normal((m, n))
    xt = np.zeros(n)
    xt[[1, 4, 6, 9]] = [1.0, 2.0, 1.5, 0.7]
    b = A @ xt + 0.05 * rng.standard_normal(m)
    x, info = oracle.oracle_lhdm(A, b)
    t = rng.standard_normal(n)
    g = 2.0 * (x - t)
    gA, gb = oracle.nnls_grad_reference(A, b, x, info["passive"], g)

    def loss(AA, bb):
        xx, ii = oracle.oracle_lhdm(AA, bb)
        assert set(ii["passive"]) == set(info["passive"])
        return float(np.sum((xx - t) ** 2))

    h = 1e-6
    for _ in range(6):
        dA = rng.standard_normal((m, n))
        dA /= np.linalg.norm(dA)
        fd = (loss(A + h * dA, b) - loss(A - h * dA, b)) / (2 * h)
        assert abs(fd - float(np.sum(gA * dA))) <= 1e-6 * max(1.0, abs(fd))
        db = rng.standard_normal(m)
        db /= np.linalg.norm(db)
        fd = (loss(A, b + h * db) - loss(A, b - h * db)) / (2 * h)
        assert abs(fd - float(gb @ db)) <= 1e-6 * max(1.0, abs(fd))
    assert np.all(gA[:, [j for j in range(n) if j not in info["passive"]]] == 0)


# ---------------------------------------------------------------------------
# Algorithm 2 corner cases whose outcome the definition fixes by hand
# ---------------------------------------------------------------------------
def _first_block(A, b, **kw):
    x, info = oracle.oracle_lhdm(A, b, record=True, **kw)
    return info["trace"][0]["J"] if info["trace"] else []


def test_dm_ties_resolve_to_lowest_index():
    # six columns that are permutations of one integer vector, b = ones: their
    # first dual entries A^T b tie exactly; j1 is the lowest index and the
    # candidate list, ordered by (w desc, index asc) and cut to kmax-1 = 2, is [1, 2].
    rng = np.random.default_rng(21)
    base = np.arange(1, 17, dtype=float)
    A = np.stack([rng.permutation(base) for _ in range(6)], axis=1)
    b = np.ones(16)
    J = _first_block(A, b, kmax=3, delta=0.999, tau1=0.5, tau2=0.01)
    assert J[:1] == [0]
    assert J == [0, 1, 2]


def test_dm_block_size_is_at_most_kmax():
    # nearly orthogonal columns with equal duals: every candidate passes, so the
    # block is exactly kmax long (never kmax + 1)
    rng = np.random.default_rng(22)
    Qm, _ = np.linalg.qr(rng.standard_normal((64, 20)))
    b = Qm @ np.ones(20)
    for kmax in (2, 4, 7):
        J = _first_block(Qm, b, kmax=kmax, delta=0.5, tau1=0.1, tau2=0.01)
        assert len(J) == kmax


def test_dm_tau2_filter_excludes_short_columns():
    # column 0: unit norm, aligned with b (largest dual); column 1: norm 0.9 and
    # almost aligned with b (dual > tau1 * max) but u_1 = 0.9 < tau2 * max u
    # because column 2 has norm 100 and is orthogonal to b.
    # b = a0 + a1, so the least-squares coefficients on {0, 1} are (1, 1) > 0.
    m = 10
    e = np.eye(m)
    a0 = e[:, 0]
    a1 = 0.9 * (0.99 * e[:, 0] + np.sqrt(1 - 0.99 ** 2) * e[:, 1])
    a2 = 100.0 * e[:, 3]
    b = a0 + a1
    A = np.stack([a0, a1, a2], axis=1)
    assert _first_block(A, b, kmax=4, delta=0.999, tau1=0.6, tau2=0.15) == [0]
    # with a permissive tau2 the same column is accepted (cosine 0.99 < 0.999)
    assert _first_block(A, b, kmax=4, delta=0.999, tau1=0.6, tau2=0.001) == [0, 1]
