"""Plain float64 CPU implementation of Lawson-Hanson (LH) and Lawson-Hanson with
Deviation Maximization (LHDM) for  min ||A x - b||_2  s.t.  x >= 0.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Parity pins for every
function live in ``tests/test_oracle_*.py``; none of them re-types a formula of
this file.

State kept here follows the first of the two implementation options described at
the end of Section 4.1 (general case of updating/downdating the QR factors):
every orthogonal transformation is applied to the whole matrix, so
``M = Q^T [A | b]`` is held explicitly, the R factor of the passive columns is
``M[:n_P, P]`` and the trailing block ``C`` of the partial QR with column
pivoting (Section 2.1) is ``M[n_P:, Z]``.  No log of transformations is kept.

Readings of points where the paper is silent, ambiguous or garbled (the same
readings the device library implements):

* The termination test of the outer loop compares ``max_{j in Z} w_j`` against
  ``tol_w = kkt_tol * max_j ||a_j|| * ||b||`` instead of against 0.
* The dual vector after each outer step is ``w = A^T (b - A x)`` (Algorithm 3;
  the corresponding line of Algorithm 1 is garbled and is read the same way).
* ``argmax`` ties resolve to the lowest column index.
* In Deviation Maximization (Algorithm 2) the maxima of ``w`` and ``u`` are
  taken over ``Z``; the candidate set is ordered by ``w`` descending (ties by
  index ascending) and truncated to ``kmax - 1`` entries so that
  ``|J| <= kmax``; ``|J|`` is further capped at ``m - n_P``.  Cosines are those
  of the projected columns (the columns of ``C``), ``j1`` included; the
  acceptance test is the strict ``|theta| < delta`` against every column
  already accepted, visiting candidates in their order.
* ``u_j`` is the 2-norm of column ``j`` of ``C`` for the passive set at the top
  of the outer step.
* A column whose projected norm is at most ``DEP_TOL * ||a_j||`` is treated as
  numerically dependent and is not eligible for insertion.  If the feasibility
  loop on ``J`` removes every column (``y_{j1} <= 0``), ``j1`` is excluded for
  the rest of this outer step and the selection is repeated; if no eligible
  column with ``w_j > tol_w`` is left the solve stops with ``STATUS_RANK``.
* Removal set of an inner iteration: the indices attaining ``alpha`` are set to
  exactly 0, and every passive index with ``x_i <= 0`` after the update is
  removed; all of them are removed in one downdating sweep.
* Dropping the last column of ``J`` in the feasibility loop only shortens the
  R factor: the transformations already applied to the trailing rows are a
  valid orthogonal basis change of the complement, so nothing is undone.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

DEFAULTS = dict(tau1=0.6, tau2=0.15, delta=0.9, kmax=32, kkt_tol=1e-9)
DEP_TOL = 1e-12

STATUS_OK = 0
STATUS_MAXITER = 1
STATUS_NONFINITE = 2
STATUS_RANK = 3


# ---------------------------------------------------------------------------
# elementary transformations
# ---------------------------------------------------------------------------
def house(x):
    """Householder reflector ``H = I - beta v v^T`` with ``H x = alpha e_1``.

    Section 2.1 (rank-one update) and Algorithm 4 (``house``).  The sign of
    ``alpha`` is opposite to ``x[0]`` so that ``v[0] = x[0] - alpha`` involves no
    cancellation; the reflector as printed in Section 2.1 is garbled and is read
    as this standard form.
    """
    x = np.asarray(x, dtype=np.float64)
    normx = float(np.linalg.norm(x))
    v = x.copy()
    if normx == 0.0:
        return v, 0.0, 0.0
    alpha = -normx if x[0] >= 0.0 else normx
    v[0] = x[0] - alpha
    vtv = float(v @ v)
    beta = 2.0 / vtv
    return v, beta, alpha


def givens(a, b):
    """Rotation ``G = [[c, s], [-s, c]]`` with ``G [a, b]^T = [r, 0]^T`` (Algorithm 5)."""
    if b == 0.0:
        return 1.0, 0.0
    r = float(np.hypot(a, b))
    return a / r, b / r


def kkt_tolerance(A, b, kkt_tol):
    """Absolute dual tolerance ``kkt_tol * max_j ||a_j|| * ||b||`` (scaled KKT test)."""
    anorm = np.linalg.norm(A, axis=0)
    return kkt_tol * float(anorm.max(initial=0.0)) * float(np.linalg.norm(b))


# ---------------------------------------------------------------------------
# the transformed matrix M = Q^T [A | b]
# ---------------------------------------------------------------------------
class _QRState:
    """Partial QR with column pivoting of Section 2.1, kept as ``M = Q^T [A | b]``."""

    def __init__(self, A, b):
        m, n = A.shape
        self.m, self.n = m, n
        self.M = np.empty((m, n + 1), dtype=np.float64)   # row-major: rows are rotated
        self.M[:, :n] = A
        self.M[:, n] = b
        self.P = []                                        # ordered passive set
        self.pos = np.full(n, -1, dtype=np.int64)          # position in P or -1

    @property
    def nP(self):
        return len(self.P)

    def append(self, j):
        """Rank-one modification that appends column ``j`` (Section 2.1; Algorithm 4 loop body).

        The reflector of ``M[n_P:, j]`` is applied to the whole trailing row block
        of ``M`` (all columns and the right-hand side)."""
        r0 = self.nP
        v, beta, alpha = house(self.M[r0:, j])
        if beta != 0.0:
            blk = self.M[r0:, :]
            blk -= beta * np.outer(v, v @ blk)
        self.M[r0, j] = alpha
        self.M[r0 + 1:, j] = 0.0
        self.pos[j] = r0
        self.P.append(int(j))

    def drop_last(self):
        """Remove the most recently appended column (feasibility loop of Algorithm 3)."""
        j = self.P.pop()
        self.pos[j] = -1
        return j

    def solve(self):
        """``y_P`` from ``R y = (Q^T b)[:n_P]`` (Algorithm 3, least-squares step)."""
        k = self.nP
        if k == 0:
            return np.zeros(0)
        R = self.M[:k, :][:, self.P]
        return solve_triangular(R, self.M[:k, self.n], lower=False)

    def R(self):
        k = self.nP
        return self.M[:k, :][:, self.P].copy()

    def proj_norms(self):
        """Column norms of the trailing block ``C`` (``u`` of Algorithm 3)."""
        return np.linalg.norm(self.M[self.nP:, :self.n], axis=0)

    def remove_positions(self, positions):
        """Delete the passive columns at ``positions`` and re-triangularise (Algorithm 5).

        Column-major sweep: for every remaining column, in order, the entries
        below its new diagonal are annihilated bottom-up, each by a rotation of
        two adjacent rows of the whole of ``M``."""
        positions = sorted(int(p) for p in positions)
        rot = downdate_rotations(self.nP, positions)
        removed = set(positions)
        keep = [j for c, j in enumerate(self.P) if c not in removed]
        for (row, col) in rot:
            j = keep[col]
            a, bb = self.M[row - 1, j], self.M[row, j]
            c, s = givens(a, bb)
            r1 = self.M[row - 1, :].copy()
            r2 = self.M[row, :]
            self.M[row - 1, :] = c * r1 + s * r2
            self.M[row, :] = -s * r1 + c * r2
            self.M[row, j] = 0.0
        for c in removed:
            self.pos[self.P[c]] = -1
        self.P = keep
        for c, j in enumerate(self.P):
            self.pos[j] = c


def downdate_rotations(nP, positions):
    """Ordered list of ``(row, new_column)`` entries annihilated by Algorithm 5.

    Deleting the (0-based) positions ``positions`` from an upper triangular
    factor of order ``nP``: a remaining column that had ``l`` deleted columns
    before it has ``l`` subdiagonal entries; they are zeroed bottom-up, the
    entry ``(row, col)`` by a rotation of rows ``row-1`` and ``row``.  Columns
    are visited left to right."""
    positions = sorted(set(int(p) for p in positions))
    out = []
    newc = 0
    for oc in range(nP):
        if oc in positions:
            continue
        l = sum(1 for p in positions if p < oc)
        for row in range(newc + l, newc, -1):
            out.append((row, newc))
        newc += 1
    return out


# ---------------------------------------------------------------------------
# Deviation Maximization (Algorithm 2)
# ---------------------------------------------------------------------------
def _eligible(st, u, anorm, excluded):
    Z = st.pos < 0
    return Z & ~excluded & (u > DEP_TOL * anorm)


def _dm(st, w, u, anorm, excluded, tau1, tau2, delta, kmax):
    """Deviation Maximization column selection (Algorithm 2) on ``C = M[n_P:, Z]``."""
    Z = st.pos < 0
    elig = _eligible(st, u, anorm, excluded)
    if not elig.any():
        return []
    wz = np.where(elig, w, -np.inf)
    j1 = int(np.argmax(wz))                  # first maximiser = lowest index
    cap = st.m - st.nP
    if kmax <= 1 or cap <= 1:
        return [j1]
    maxw = w[j1]
    maxu = float(u[Z].max())
    cand = elig & (w >= tau1 * maxw) & (u >= tau2 * maxu)
    cand[j1] = False
    idx = np.nonzero(cand)[0]
    order = np.lexsort((idx, -w[idx]))       # w descending, index ascending
    I = [int(i) for i in idx[order][: kmax - 1]]
    if not I:
        return [j1]
    cols = [j1] + I
    C = st.M[st.nP:, cols]
    nrm = np.linalg.norm(C, axis=0)
    theta = (C.T @ C) / np.outer(nrm, nrm)   # cosine matrix, eq. (cosine matrix)
    acc = [0]
    for t in range(1, len(cols)):
        if len(acc) >= cap:
            break
        if all(abs(theta[t, a]) < delta for a in acc):
            acc.append(t)
    return [cols[a] for a in acc]


def dm_select_reference(A, b, P, x, tau1, tau2, delta, kmax, excluded=None):
    """Algorithm 2 evaluated from its definition, without any QR state.

    Projections onto ``range(A_P)^perp`` use ``numpy.linalg.qr`` of ``A_P``; ``w``
    is ``A^T (b - A x)``.  Used by the tests to pin ``_dm``."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    P = list(P)
    if P:
        Qp, _ = np.linalg.qr(A[:, P])
        Cfull = A - Qp @ (Qp.T @ A)
    else:
        Cfull = A.copy()
    u = np.linalg.norm(Cfull, axis=0)
    anorm = np.linalg.norm(A, axis=0)
    w = A.T @ (b - A @ x)
    Z = np.ones(n, bool)
    Z[P] = False
    excluded = np.zeros(n, bool) if excluded is None else excluded
    elig = Z & ~excluded & (u > DEP_TOL * anorm)
    if not elig.any():
        return []
    j1 = int(np.argmax(np.where(elig, w, -np.inf)))
    cap = m - len(P)
    if kmax <= 1 or cap <= 1:
        return [j1]
    cand = [i for i in range(n) if elig[i] and i != j1 and w[i] >= tau1 * w[j1]
            and u[i] >= tau2 * u[Z].max()]
    cand.sort(key=lambda i: (-w[i], i))
    cols = [j1] + cand[: kmax - 1]
    acc = [j1]
    for i in cols[1:]:
        if len(acc) >= cap:
            break
        ok = True
        for j in acc:
            cth = float(Cfull[:, i] @ Cfull[:, j]) / (u[i] * u[j])
            if not abs(cth) < delta:
                ok = False
                break
        if ok:
            acc.append(i)
    return acc


# ---------------------------------------------------------------------------
# the solvers
# ---------------------------------------------------------------------------
def _prep(A, b):
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    if A.ndim != 2 or A.shape[0] != b.shape[0]:
        raise ValueError("A must be (m, n) and b (m,)")
    return A, b


def _inner_step(st, x, y):
    """One inner iteration of Algorithms 1 and 3: step length, new iterate, removal set."""
    P = np.array(st.P, dtype=np.int64)
    xP = x[P]
    neg = np.nonzero(y <= 0.0)[0]
    # an entry whose iterate is exactly 0 (only a new column of J, in the
    # variant without the feasibility loop) limits the step to 0
    xn = xP[neg]
    ratios = np.zeros(len(neg))
    nz = xn != 0.0
    ratios[nz] = xn[nz] / (xn[nz] - y[neg][nz])
    alpha = float(ratios.min())
    xP = xP + alpha * (y - xP)
    xP[neg[ratios == alpha]] = 0.0
    rm = np.nonzero(xP <= 0.0)[0]
    xP[rm] = 0.0
    x[P] = xP
    st.remove_positions(rm)
    return [int(P[i]) for i in rm], alpha


def _sign_flip(st, x, y):
    """The inner iteration of the positivity-trick case (Section 4.2) on the
    matrix [B, -B]: every passive column with y_k < 0 is replaced, at the same
    position, by its twin (the negated column), so that column of R changes
    sign and y_k becomes -y_k > 0; the residual is unchanged.  Returns the
    (old, new) index pairs."""
    half = st.n // 2
    out = []
    for c in np.nonzero(y < 0.0)[0]:
        j = st.P[c]
        t = j + half if j < half else j - half
        st.M[:, t] = -st.M[:, j]          # Q^T (-a_j): the R column at position c, negated
        st.pos[j] = -1
        st.pos[t] = c
        st.P[c] = t
        x[j] = 0.0
        out.append((int(j), int(t)))
    return out


def _check_twins(A, sign_flip):
    if not sign_flip:
        return
    n = A.shape[1]
    if n % 2 or not np.array_equal(A[:, n // 2:], -A[:, :n // 2]):
        raise ValueError("the sign flip needs the positivity-trick matrix [B, -B]")


def _inner_iteration(st, x, y, sign_flip, step):
    """One pass of the inner loop: the sign flip of Section 4.2 when it applies
    (every nonpositive component strictly negative), else the step length and
    removal of Algorithms 1 and 3."""
    if sign_flip and not (y == 0.0).any():
        step["flipped"].append(_sign_flip(st, x, y))
    else:
        rm, _ = _inner_step(st, x, y)
        step["removed"].append(rm)


def _finish(st, A, b, x, w, status, outer, inner, jdrops, trace, tol_w):
    r = b - A @ x
    info = dict(status=status, outer_iters=outer, inner_iters=inner, jloop_drops=jdrops,
                n_passive=st.nP, passive=list(st.P), objective=float(r @ r),
                tol_w=tol_w, w=w, R=st.R(), trace=trace)
    return x, info


def oracle_lhdm(A, b, tau1=0.6, tau2=0.15, delta=0.9, kmax=32, kkt_tol=1e-9,
                max_outer=None, max_inner=None, record=False, jloop=True, sign_flip=False):
    """LHDM (Algorithm 3 with Deviation Maximization, Algorithm 2).

    ``jloop=False``: the variant of Theorem 4 (tau1 = 1 and tau2 <= 1/2, with
    the selection's delta <= tau2 / (kmax - 1) of Theorem 2 that makes the
    block's Gram matrix diagonally dominant), in which the least-squares
    components of every accepted block are positive and the feasibility loop
    on J is not evaluated; a violation by rounding is left to the inner loop (a
    zero iterate entry gives the step length 0).

    ``sign_flip=True`` (A must be the positivity-trick matrix [B, -B]): the
    inner loop of Section 4.2, which replaces each column with a negative
    least-squares component by its twin instead of stepping and downdating;
    an exactly zero component (the flip cannot make it positive) takes the
    ordinary inner iteration.

    Returns ``(x, info)``; ``info['passive']`` is the ordered passive set."""
    if not jloop and not (tau1 == 1.0 and tau2 <= 0.5 and (kmax <= 1 or delta <= tau2 / (kmax - 1))):
        raise ValueError("the variant without the feasibility loop needs tau1 = 1, tau2 <= 1/2 and "
                         "delta <= tau2 / (kmax - 1) (Theorems 2 and 4)")
    A, b = _prep(A, b)
    _check_twins(A, sign_flip)
    m, n = A.shape
    max_outer = 3 * n if max_outer is None else max_outer
    max_inner = 3 * n if max_inner is None else max_inner
    st = _QRState(A, b)
    x = np.zeros(n)
    if not (np.isfinite(A).all() and np.isfinite(b).all()):
        return _finish(st, A, b, x, np.zeros(n), STATUS_NONFINITE, 0, 0, 0, [], 0.0)
    anorm = np.linalg.norm(A, axis=0)
    tol_w = kkt_tol * float(anorm.max(initial=0.0)) * float(np.linalg.norm(b))
    w = A.T @ b                      # w^(0) = A^T b
    u = anorm.copy()                 # u^(0): column norms of A
    excluded = np.zeros(n, bool)
    outer = inner = jdrops = 0
    status = STATUS_OK
    trace = []
    while True:
        Z = st.pos < 0
        if not Z.any() or float(w[Z].max()) <= tol_w:
            break
        J = _dm(st, w, u, anorm, excluded, tau1, tau2, delta, kmax)
        if not J or w[J[0]] <= tol_w:
            status = STATUS_RANK
            break
        if outer >= max_outer:
            status = STATUS_MAXITER
            break
        n0 = st.nP
        j1 = J[0]
        for j in J:                  # block append: Algorithm 4 as k reflectors
            st.append(j)
        y = st.solve()
        drops = 0
        while jloop and len(J) > 0 and float(y[n0:].min()) <= 0.0:   # feasibility loop on J
            st.drop_last()
            J.pop()
            drops += 1
            if J:
                y = st.solve()
        jdrops += drops
        if not J:
            excluded[j1] = True      # safeguard: y_{j1} <= 0 only happens through rounding
            continue
        outer += 1
        excluded[:] = False
        step = dict(J=list(J), drops=drops, removed=[], flipped=[])
        while st.nP > 0 and float(y.min()) <= 0.0:          # inner loop
            if inner >= max_inner:
                status = STATUS_MAXITER
                break
            inner += 1
            _inner_iteration(st, x, y, sign_flip, step)
            y = st.solve()
        if status == STATUS_MAXITER:
            x[:] = np.maximum(x, 0.0)
            break
        x[:] = 0.0
        x[st.P] = y
        r = b - A @ x
        w = A.T @ r
        u = st.proj_norms()
        if record:
            step.update(nP=st.nP, obj=float(r @ r))
            trace.append(step)
    return _finish(st, A, b, x, w, status, outer, inner, jdrops, trace, tol_w)


def oracle_lh(A, b, kkt_tol=1e-9, max_outer=None, max_inner=None, record=False, sign_flip=False):
    """Plain Lawson-Hanson (Algorithm 1): one column per outer step, rank-one
    Householder append, inner loop with step length and Givens removal (or,
    with ``sign_flip`` on a positivity-trick matrix, the sign flip of Section
    4.2, as in ``oracle_lhdm``)."""
    A, b = _prep(A, b)
    _check_twins(A, sign_flip)
    m, n = A.shape
    max_outer = 3 * n if max_outer is None else max_outer
    max_inner = 3 * n if max_inner is None else max_inner
    st = _QRState(A, b)
    x = np.zeros(n)
    if not (np.isfinite(A).all() and np.isfinite(b).all()):
        return _finish(st, A, b, x, np.zeros(n), STATUS_NONFINITE, 0, 0, 0, [], 0.0)
    anorm = np.linalg.norm(A, axis=0)
    tol_w = kkt_tol * float(anorm.max(initial=0.0)) * float(np.linalg.norm(b))
    w = A.T @ b
    u = anorm.copy()
    excluded = np.zeros(n, bool)
    outer = inner = jdrops = 0
    status = STATUS_OK
    trace = []
    while True:
        Z = st.pos < 0
        if not Z.any() or float(w[Z].max()) <= tol_w:
            break
        elig = _eligible(st, u, anorm, excluded)
        if not elig.any():
            status = STATUS_RANK
            break
        j = int(np.argmax(np.where(elig, w, -np.inf)))       # pivoting step
        if w[j] <= tol_w:
            status = STATUS_RANK
            break
        if outer >= max_outer:
            status = STATUS_MAXITER
            break
        st.append(j)
        y = st.solve()
        if float(y[-1]) <= 0.0:       # safeguard of the same reading as in LHDM
            st.drop_last()
            jdrops += 1
            excluded[j] = True
            continue
        outer += 1
        excluded[:] = False
        step = dict(J=[j], drops=0, removed=[], flipped=[])
        while st.nP > 0 and float(y.min()) <= 0.0:           # inner loop
            if inner >= max_inner:
                status = STATUS_MAXITER
                break
            inner += 1
            _inner_iteration(st, x, y, sign_flip, step)
            y = st.solve()
        if status == STATUS_MAXITER:
            x[:] = np.maximum(x, 0.0)
            break
        x[:] = 0.0
        x[st.P] = y
        r = b - A @ x
        w = A.T @ r
        u = st.proj_norms()
        if record:
            step.update(nP=st.nP, obj=float(r @ r))
            trace.append(step)
    return _finish(st, A, b, x, w, status, outer, inner, jdrops, trace, tol_w)


def oracle_signed(A, b, method="lhdm", sign_flip=True, **kw):
    """Signed least squares by the positivity trick (Section 3.2): the NNLS
    problem min ||[A, -A] z - b||, z >= 0, solved by LHDM or LH (``method``)
    with the sign-flip inner loop of Section 4.2 (or the ordinary one);
    returns ``(x, info)`` with x = z[:n] - z[n:], and z in ``info['z']``."""
    A, b = _prep(A, b)
    n = A.shape[1]
    A2 = np.concatenate([A, -A], axis=1)
    if method == "lhdm":
        z, info = oracle_lhdm(A2, b, sign_flip=sign_flip, **kw)
    elif method == "lh":
        z, info = oracle_lh(A2, b, sign_flip=sign_flip, **kw)
    else:
        raise ValueError(method)
    info["z"] = z
    return z[:n] - z[n:], info


def l1nnls_matrix(A, b, lam):
    """The NNLS form of the squared-l1 regularised problem (Section 3.3): the
    matrix [1^T, 1^T; lam A, -lam A] and right-hand side [0; lam b]."""
    A, b = _prep(A, b)
    m, n = A.shape
    M = np.empty((m + 1, 2 * n))
    M[0, :] = 1.0
    M[1:, :n] = lam * A
    M[1:, n:] = -lam * A
    rhs = np.concatenate([[0.0], lam * b])
    return M, rhs


def oracle_l1nnls(A, b, lam, method="lhdm", **kw):
    """l1-NNLS (Section 3.3): min ||x||_1^2 + lam^2 ||A x - b||^2 written as the
    NNLS problem on [1^T, 1^T; lam A, -lam A], [0; lam b] with x = z+ - z-
    (the weight of the residual term is lam^2, as that matrix form gives),
    solved by LHDM or LH; returns ``(x, info)`` with z in ``info['z']``."""
    M, rhs = l1nnls_matrix(A, b, lam)
    n = M.shape[1] // 2
    if method == "lhdm":
        z, info = oracle_lhdm(M, rhs, **kw)
    elif method == "lh":
        z, info = oracle_lh(M, rhs, **kw)
    else:
        raise ValueError(method)
    info["z"] = z
    return z[:n] - z[n:], info


# ---------------------------------------------------------------------------
# checkers
# ---------------------------------------------------------------------------
def kkt_report(A, b, x, kkt_tol=1e-9):
    """Scaled KKT residual of Theorem 1 (KKT conditions for NNLS).

    ``kkt = max( max_{Z} w_j^+, max_{P} |w_j| ) / (max_j ||a_j|| ||b||)`` with
    ``P = {x_j > 0}``; also reports feasibility and the objective."""
    A, b = _prep(A, b)
    x = np.asarray(x, dtype=np.float64)
    r = b - A @ x
    w = A.T @ r
    scale = float(np.linalg.norm(A, axis=0).max(initial=0.0)) * float(np.linalg.norm(b))
    scale = scale if scale > 0 else 1.0
    P = x > 0
    vz = float(np.maximum(w[~P], 0.0).max(initial=0.0))
    vp = float(np.abs(w[P]).max(initial=0.0))
    return dict(kkt=max(vz, vp) / scale, dual_z=vz / scale, dual_p=vp / scale,
                feasible=bool((x >= 0).all()), objective=float(r @ r), w=w,
                ok=bool((x >= 0).all() and max(vz, vp) <= kkt_tol * scale))


def brute_force_nnls(A, b, neg_tol=1e-13):
    """Exact NNLS by enumerating all ``2^n`` supports (problem statement, Section 2).

    For every support ``S`` the unconstrained least-squares solution on ``A_S``
    is computed with ``numpy.linalg.lstsq``; among the nonnegative ones the
    smallest objective wins.  Only for ``n <= 14``."""
    A, b = _prep(A, b)
    m, n = A.shape
    if n > 14:
        raise ValueError("brute force limited to n <= 14")
    best_obj, best_x = float(b @ b), np.zeros(n)
    for mask in range(1, 1 << n):
        S = [j for j in range(n) if mask >> j & 1]
        xs, *_ = np.linalg.lstsq(A[:, S], b, rcond=None)
        if xs.min() < -neg_tol:
            continue
        x = np.zeros(n)
        x[S] = np.maximum(xs, 0.0)
        r = b - A @ x
        obj = float(r @ r)
        if obj < best_obj - 1e-14 * max(1.0, best_obj):
            best_obj, best_x = obj, x
    return best_x, best_obj


def nnls_grad_reference(A, b, x, P, g):
    """Derivative of the least-squares map on a fixed passive set ``P``.

    ``x_P = (A_P^T A_P)^{-1} A_P^T b`` (the subproblem of Section 2.1 at the final
    passive set); for a loss with gradient ``g`` in ``x``:
    ``lambda = (A_P^T A_P)^{-1} g_P``, ``grad_b = A_P lambda``,
    ``grad_A[:, P] = r lambda^T - (A_P lambda) x_P^T`` with ``r = b - A_P x_P``, and
    ``grad_A[:, Z] = 0``.  Dense reference with ``numpy.linalg.solve``."""
    A, b = _prep(A, b)
    P = np.asarray(list(P), dtype=np.int64)
    gA = np.zeros_like(A)
    if P.size == 0:
        return gA, np.zeros_like(b)
    AP = A[:, P]
    xP = np.asarray(x, dtype=np.float64)[P]
    r = b - AP @ xP
    lam = np.linalg.solve(AP.T @ AP, np.asarray(g, dtype=np.float64)[P])
    Al = AP @ lam
    gA[:, P] = np.outer(r, lam) - np.outer(Al, xP)
    return gA, Al
