"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar (from the requirements of the solver): identical passive set where the
minimiser is unique, x within 1e-10 relative (max-norm), KKT residual <= 1e-9.
Where the two follow the same path (no rounding-level near-ties) the ordered
passive set and the iteration counters agree as well.
"""
import numpy as np
import pytest
import torch

import oracle
from parity_util import KKT, XTOL, _check, _dev, _passive, _rel, _supp  # noqa: F401
from workloads import make_c1, make_c3, make_c4_batch, make_c5_batch, make_small

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lhdm():
    import paper_2108_05345_amd as mod
    from paper_2108_05345_amd import _lib
    _lib.load()   # fails loudly if the HIP library is missing
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return mod


ENGINES = ["workgroup", "device"]


def _lh(lhdm, A, b, engine):
    # plain LH: the C-ABI lh_solve (automatic engine) or LHDM with kmax = 1 on a forced engine
    if engine == "auto":
        return lhdm.lh_solve(A, b)
    return lhdm.solve(A, b, kmax=1, engine=engine)


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("seed", list(range(1000, 1012)))
def test_c1_lhdm_and_lh(lhdm, seed, engine):
    inst = make_c1(seed)
    A, b = _dev(inst.A, inst.b)
    xo, io = oracle.oracle_lhdm(inst.A, inst.b)
    assert _check(lhdm.solve(A, b, engine=engine), xo, io, tag=f"c1-lhdm-{seed}-{engine}") in ("path", "order")
    xo, io = oracle.oracle_lh(inst.A, inst.b)
    assert _check(_lh(lhdm, A, b, engine), xo, io, tag=f"c1-lh-{seed}-{engine}") == "path"
    # planted recovery
    np.testing.assert_allclose(lhdm.solve(A, b, engine=engine).x.cpu().numpy(), inst.x_true, atol=1e-12)


def test_c1_lh_entry_point(lhdm):
    inst = make_c1(1000)
    A, b = _dev(inst.A, inst.b)
    xo, io = oracle.oracle_lh(inst.A, inst.b)
    _check(lhdm.lh_solve(A, b), xo, io, tag="c1-lh-abi")


RAGGED = [
    # (m, n, k, kind, noise, seed): uniform A with noise -> positive residual (unique)
    (37, 91, 9, "uniform", 1e-2, 1),
    (64, 200, 20, "uniform", 1e-2, 2),
    (130, 333, 33, "uniform", 1e-2, 3),
    (200, 517, 52, "uniform", 1e-2, 4),
    (257, 300, 30, "uniform", 1e-2, 5),
    (300, 120, 40, "gauss", 1e-1, 6),     # overdetermined, full column rank
    (130, 333, 20, "gauss", 0.0, 7),      # noiseless planted sparse
    (71, 513, 7, "gauss", 0.0, 8),
]


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("case", RAGGED, ids=[f"{c[0]}x{c[1]}-{c[3]}" for c in RAGGED])
def test_ragged_unique_instances(lhdm, case, engine):
    m, n, k, kind, noise, seed = case
    inst = make_small(m, n, k, seed, kind=kind, noise_std=noise)
    A, b = _dev(inst.A, inst.b)
    for delta in (0.9, 0.5, 0.2):
        xo, io = oracle.oracle_lhdm(inst.A, inst.b, delta=delta)
        _check(lhdm.solve(A, b, delta=delta, engine=engine), xo, io, tag=f"{m}x{n}-d{delta}-{engine}")
    xo, io = oracle.oracle_lh(inst.A, inst.b)
    _check(_lh(lhdm, A, b, engine), xo, io, tag=f"{m}x{n}-lh-{engine}")


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("delta", [0.2, 0.5, 0.8])
def test_scaled_c3_delta_sweep(lhdm, delta, engine):
    # the large Gaussian family scaled down (k/n kept): zero-residual, non-unique
    # minimiser; both sides are compared on their path and the KKT conditions
    inst = make_c3(3000, m=160, n=640, k=32)
    A, b = _dev(inst.A, inst.b)
    xo, io = oracle.oracle_lhdm(inst.A, inst.b, delta=delta)
    # the oracle's solution is separated here (min x_P > 1e-8 max x), so the
    # whole path must be compared, not only its significant columns
    assert _check(lhdm.solve(A, b, delta=delta, engine=engine), xo, io, unique=False, same_path=True,
                  tag=f"c3s-d{delta}-{engine}") == "path"


@pytest.mark.parametrize("engine", ENGINES)
def test_kmax_variants(lhdm, engine):
    inst = make_small(90, 260, 25, 11, kind="uniform", noise_std=1e-2)
    A, b = _dev(inst.A, inst.b)
    for kmax in (1, 2, 5, 17, 64):
        xo, io = oracle.oracle_lhdm(inst.A, inst.b, kmax=kmax)
        _check(lhdm.solve(A, b, kmax=kmax, engine=engine), xo, io, tag=f"kmax{kmax}-{engine}")


def test_device_engine_multiblock_sizes(lhdm):
    # sizes spanning several row blocks of the chained triangular solve and
    # several column blocks of the chained downdate, with ragged tails
    for (m, n, k, seed) in ((333, 700, 60, 31), (517, 1100, 90, 32)):
        inst = make_small(m, n, k, seed, kind="uniform", noise_std=1e-2)
        A, b = _dev(inst.A, inst.b)
        xo, io = oracle.oracle_lhdm(inst.A, inst.b)
        _check(lhdm.solve(A, b, engine="device"), xo, io, same_path=False, tag=f"dev-{m}x{n}")
        xo, io = oracle.oracle_lh(inst.A, inst.b)
        _check(lhdm.solve(A, b, kmax=1, engine="device"), xo, io, same_path=False, tag=f"dev-lh-{m}x{n}")


def test_device_engine_many_candidates(lhdm):
    # uniform entries make almost every column pass the candidate filter of
    # Deviation Maximization at the first step (w_j >= tau1 max w and
    # ||a_j|| >= tau2 max ||a||): more than 256 of them, under the collected
    # list's capacity, so the first kmax - 1 are placed from the histogram's
    # short list rather than by sorting the whole list
    m, n = 300, 1800
    inst = make_small(m, n, 60, 51, kind="uniform", noise_std=1e-2)
    w = inst.A.T @ inst.b
    u = np.linalg.norm(inst.A, axis=0)
    cnt = int(np.count_nonzero((w >= 0.6 * w.max()) & (u >= 0.15 * u.max()))) - 1
    assert 256 < cnt <= 2048, cnt
    A, b = _dev(inst.A, inst.b)
    xo, io = oracle.oracle_lhdm(inst.A, inst.b)
    _check(lhdm.solve(A, b, engine="device"), xo, io, same_path=False, tag=f"cand-{m}x{n}")


def test_device_engine_tied_candidates(lhdm):
    # 600 exact copies of the column with the largest w (uniform entries,
    # that column scaled by 2): at the first step all of them pass the
    # candidate filter with equal w, so the histogram's deciding bucket holds
    # more than 256 candidates and the selection sorts the whole list; ties
    # are ordered by index, as in the oracle
    rng = np.random.default_rng(71)
    m, n, ndup = 128, 900, 600
    A = rng.uniform(0.0, 1.0, (m, n))
    A[:, 0] *= 2.0
    A[:, 1:1 + ndup] = A[:, [0]]
    xs = np.zeros(n)
    sup = rng.choice(np.arange(1 + ndup, n), 40, replace=False)
    xs[sup] = rng.uniform(1.0, 2.0, 40)
    xs[0] = 1.5
    b = A @ xs + 1e-2 * rng.standard_normal(m)
    w = A.T @ b
    u = np.linalg.norm(A, axis=0)
    assert int(np.argmax(w)) == 0
    assert int(np.count_nonzero((w >= 0.6 * w.max()) & (u >= 0.15 * u.max()))) - 1 > 256
    xo, io = oracle.oracle_lhdm(A, b)
    _check(lhdm.solve(*_dev(A, b), engine="device"), xo, io, unique=False, tag="tied-candidates")


def test_device_engine_long_downdate(lhdm, monkeypatch):
    # 1200 x 2400 Gaussian, 1100-sparse planted solution: one inner step
    # removes a single column more than 1024 positions before the end of the
    # passive set, so the compaction's scan of bt over the downdate's
    # rotations (16 chunks of 64 per sweep) takes more than one sweep.  The
    # oracle's removal positions are recorded to check that the instance
    # still has such a step.
    import oracle.nnls as onn
    inst = make_small(1200, 2400, 1100, 61, kind="gauss", noise_std=1e-3)
    seen = []
    step = onn._inner_step

    def recording_step(st, x, y):
        nP, P = st.nP, list(st.P)
        out = step(st, x, y)
        seen.append((nP, sorted(P.index(j) for j in out[0])))
        return out

    monkeypatch.setattr(onn, "_inner_step", recording_step)
    xo, io = oracle.oracle_lhdm(inst.A, inst.b)
    assert any(len(pos) == 1 and nP - 1 - pos[0] > 1024 for nP, pos in seen)
    A, b = _dev(inst.A, inst.b)
    _check(lhdm.solve(A, b, engine="device"), xo, io, unique=False, tag="long-downdate")


def test_device_engine_padded_leading_dimension(lhdm):
    # A given as a column-major view with a padded (even) leading dimension:
    # odd m with even lda takes the 16-byte-load column-block kernel for the
    # dual pass (its vector block then ends in a zero padding row), even m
    # with lda = m + 2 takes it with a column stride different from m
    for (m, n, k, seed, pad) in ((131, 420, 40, 41, 1), (257, 700, 70, 42, 1), (160, 500, 48, 43, 2)):
        inst = make_small(m, n, k, seed, kind="uniform", noise_std=1e-2)
        d = torch.device("cuda:0")
        store = torch.zeros((n, m + pad), dtype=torch.float64, device=d)
        store[:, :m] = torch.from_numpy(np.ascontiguousarray(inst.A.T)).to(d)
        A = store[:, :m].t()
        assert A.stride(0) == 1 and A.stride(1) == m + pad
        b = torch.from_numpy(np.ascontiguousarray(inst.b)).to(d)
        xo, io = oracle.oracle_lhdm(inst.A, inst.b)
        _check(lhdm.solve(A, b, engine="device"), xo, io, same_path=False, tag=f"lda-{m}x{n}+{pad}")
        xo, io = oracle.oracle_lh(inst.A, inst.b)
        _check(lhdm.solve(A, b, kmax=1, engine="device"), xo, io, same_path=False, tag=f"lda-lh-{m}x{n}+{pad}")


def test_c2_full_size(lhdm):
    # the 1024 x 4096 unit-column Gaussian instance, noiseless 128-sparse: unique
    from workloads import make_c2
    inst = make_c2(2000)
    A, b = _dev(inst.A, inst.b)
    xo, io = oracle.oracle_lhdm(inst.A, inst.b)
    r = lhdm.solve(A, b)
    assert _check(r, xo, io, tag="c2-lhdm") == "path"
    np.testing.assert_allclose(r.x.cpu().numpy(), inst.x_true, atol=1e-10)
    xo, io = oracle.oracle_lh(inst.A, inst.b)
    assert _check(lhdm.lh_solve(A, b), xo, io, tag="c2-lh") == "path"


@pytest.mark.parametrize("delta", [0.8])
def test_c3_full_size_properties(lhdm, delta):
    # 4096 x 16384: KKT at 1e-9, feasibility, and the final passive least-squares
    # subproblem re-solved by LAPACK on the returned passive set
    inst = make_c3(3000)
    A, b = _dev(inst.A, inst.b)
    for name, res in (("lhdm", lhdm.solve(A, b, delta=delta)),):
        print(f"[c3-{name}] {res.info}", flush=True)
        assert res.info["status"] == 0
        assert res.info["kkt_residual"] <= KKT
        x = res.x.cpu().numpy()
        P = _passive(res)
        assert (x >= 0).all() and all(x[j] > 0 for j in P)
        rep = oracle.kkt_report(inst.A, inst.b, x)
        assert rep["kkt"] <= KKT
        xs, *_ = np.linalg.lstsq(inst.A[:, P], inst.b, rcond=None)
        assert np.abs(xs - x[P]).max() <= 1e-8 * np.abs(xs).max()


def test_batched_c4_subset(lhdm):
    insts = make_c4_batch(count=48)
    As, bs = zip(*[_dev(i.A, i.b) for i in insts])
    for use_lh in (False, True):
        res = lhdm.solve_batched(list(As), list(bs), use_lh=use_lh)
        for inst, r in zip(insts, res):
            if use_lh:
                xo, io = oracle.oracle_lh(inst.A, inst.b)
            else:
                xo, io = oracle.oracle_lhdm(inst.A, inst.b)
            _check(r, xo, io, same_path=False, tag=f"c4-{inst.name}-lh{int(use_lh)}")


def test_backward_against_reference(lhdm):
    insts = make_c5_batch(count=3, m=96, n=192)
    for inst in insts:
        A, b = _dev(inst.A, inst.b)
        Ar = A.clone().requires_grad_(True)
        br = b.clone().requires_grad_(True)
        t = torch.from_numpy(inst.t).to(A.device)
        x, passive = lhdm.LHDMFunction.apply(Ar, br)
        ((x - t) ** 2).sum().backward()
        P = [int(j) for j in passive.cpu().numpy() if j >= 0]
        xn = x.detach().cpu().numpy()
        gA, gb = oracle.nnls_grad_reference(inst.A, inst.b, xn, P, 2 * (xn - inst.t))
        scale = max(np.abs(gA).max(), 1.0)
        assert np.abs(Ar.grad.cpu().numpy() - gA).max() <= 1e-8 * scale
        assert np.abs(br.grad.cpu().numpy() - gb).max() <= 1e-8 * max(np.abs(gb).max(), 1.0)


def test_degenerate_inputs(lhdm):
    rng = np.random.default_rng(5)
    A = rng.standard_normal((10, 6))
    Ad, bd = _dev(A, np.zeros(10))
    r = lhdm.solve(Ad, bd)
    assert r.info["status"] == 0 and r.info["n_passive"] == 0 and float(r.x.abs().max()) == 0.0
    A2 = A.copy()
    A2[3, 2] = np.nan
    r = lhdm.solve(*_dev(A2, rng.standard_normal(10)))
    assert r.info["status"] == oracle.STATUS_NONFINITE and float(r.x.abs().max()) == 0.0
    A3 = np.concatenate([A, A[:, :2], np.zeros((10, 1))], axis=1)
    b3 = rng.standard_normal(10)
    r = lhdm.solve(*_dev(A3, b3))
    xb, objb = oracle.brute_force_nnls(A3, b3)
    assert r.info["status"] == 0
    assert abs(r.info["objective"] - objb) <= 1e-10 * max(1.0, objb)
    A4 = rng.standard_normal((3, 12))
    b4 = rng.standard_normal(3)
    for fn in (lhdm.solve, lhdm.lh_solve):
        r = fn(*_dev(A4, b4))
        xb, objb = oracle.brute_force_nnls(A4, b4)
        assert abs(r.info["objective"] - objb) <= 1e-10 * max(1.0, objb)
    a1 = rng.standard_normal((9, 1))
    b1 = rng.standard_normal(9)
    r = lhdm.solve(*_dev(a1, b1))
    ref = max(0.0, float(a1[:, 0] @ b1) / float(a1[:, 0] @ a1[:, 0]))
    assert abs(float(r.x[0]) - ref) <= 1e-14 * max(1.0, ref)


def test_tiny_brute_force(lhdm):
    rng = np.random.default_rng(17)
    for t in range(12):
        m = int(rng.integers(3, 12))
        n = int(rng.integers(2, 11))
        A = rng.standard_normal((m, n))
        b = rng.standard_normal(m)
        xb, objb = oracle.brute_force_nnls(A, b)
        for fn in (lhdm.solve, lhdm.lh_solve):
            r = fn(*_dev(A, b))
            assert r.info["status"] == 0
            assert abs(r.info["objective"] - objb) <= 1e-10 * max(1.0, objb)


def test_deterministic(lhdm):
    inst = make_small(120, 400, 30, 21, kind="uniform", noise_std=1e-2)
    A, b = _dev(inst.A, inst.b)
    r1 = lhdm.solve(A, b)
    r2 = lhdm.solve(A, b)
    assert torch.equal(r1.x, r2.x) and torch.equal(r1.passive, r2.passive)


def test_device_engine_tall_panel_fallback(lhdm):
    # m large enough that a row chunk of the panel factorisation exceeds LDS:
    # the single-workgroup panel path; checked through KKT and the final LS subproblem
    inst = make_small(8256, 8400, 200, 41, kind="uniform", noise_std=1e-2)
    A, b = _dev(inst.A, inst.b)
    r = lhdm.solve(A, b, kmax=64)
    print(f"[tall] {r.info}", flush=True)
    assert r.info["status"] == 0 and r.info["kkt_residual"] <= KKT
    x = r.x.cpu().numpy()
    P = _passive(r)
    xs, *_ = np.linalg.lstsq(inst.A[:, P], inst.b, rcond=None)
    assert np.abs(xs - x[P]).max() <= 1e-8 * np.abs(xs).max()


def test_device_engine_more_than_4096_passive(lhdm):
    # the inner iteration keeps at most 4096 passive positions in registers (16
    # per thread); beyond that it takes the strided loop.  A dense planted
    # solution on a 4608-row instance ends with more than 4096 passive columns;
    # checked through KKT and the final LS subproblem
    inst = make_small(4608, 5200, 4400, 61, kind="uniform", noise_std=1e-2)
    A, b = _dev(inst.A, inst.b)
    r = lhdm.solve(A, b)
    print(f"[wide passive] {r.info}", flush=True)
    assert r.info["status"] == 0 and r.info["kkt_residual"] <= KKT
    P = _passive(r)
    assert len(P) > 4096
    x = r.x.cpu().numpy()
    xs, *_ = np.linalg.lstsq(inst.A[:, P], inst.b, rcond=None)
    assert np.abs(xs - x[P]).max() <= 1e-8 * np.abs(xs).max()
