"""Algorithm 5 (Givens downdating, Section 4.1) on the GPU against the oracle.

The solver's inner step deletes every position whose iterate reached zero in one
sweep.  On the parity instances an inner step almost always removes a single
column (several at once need an exact tie in the step length), so the
multi-removal branches of both engines are exercised here directly, through the
test-only C-ABI entry ``lhdm_test_downdate``: caller-given Q, R and Q^T b and a
set of removal positions go through the engines' own downdating kernels, and the
result is compared element by element with the oracle's ``remove_positions``
applied to the same state.

The oracle keeps ``M = Q^T [A | b]``; with the orthogonal factor carried as m
extra columns of ``M`` (``M[:, nP:nP+m] = Q^T``), the downdated Q, R and Q^T b
are all rows and columns of ``M`` after the sweep, so every entry of the three
is compared, which also pins the order and the signs of the rotations.
"""
import ctypes
import os

import numpy as np
import pytest
import torch

from oracle.nnls import _QRState

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = 1e-12


@pytest.fixture(scope="module")
def lib():
    from paper_2108_05345_amd import _lib
    lib = _lib.load()   # fails loudly if the HIP library is missing
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib


def _state(m, nP, seed):
    """A random QR state: orthogonal Q (library QR of a Gaussian matrix), upper
    triangular R with a well-conditioned diagonal, and Q^T b."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    R = np.triu(rng.standard_normal((nP, nP)))
    R[np.diag_indices(nP)] = np.sign(R.diagonal() + 0.5) * rng.uniform(0.5, 2.0, nP)
    bt = rng.standard_normal(m)
    return Q, R, bt


def _oracle(Q, R, bt, rm, per_sweep=None):
    """The oracle's Algorithm 5 on the same state; with per_sweep, the ascending
    positions are deleted in sweeps of at most that many (the lowest first), as
    the device engine does when one inner step removes more than it sweeps."""
    m, nP = Q.shape[0], R.shape[0]
    cols = np.zeros((m, nP + m))
    cols[:nP, :nP] = R
    cols[:, nP:] = Q.T
    st = _QRState(cols, bt)            # M = [R; 0 | Q^T | Q^T b] for the identity transform
    st.P = list(range(nP))
    st.pos[:nP] = np.arange(nP)
    step = per_sweep or len(rm)
    for k in range(0, len(rm), step):
        # positions below the current chunk are gone: renumber
        st.remove_positions([r - k for r in rm[k:k + step]])
    nk = nP - len(rm)
    Rk = np.triu(st.M[:nk][:, st.P])
    return st.M[:, nP:nP + m].T.copy(), Rk, st.M[:, -1].copy(), list(st.P)


def _gpu(lib, engine, Q, R, bt, rm):
    d = torch.device("cuda:0")
    m, nP = Q.shape[0], R.shape[0]
    nk = nP - len(rm)
    tQ = torch.from_numpy(np.asfortranarray(Q)).to(d)
    tR = torch.from_numpy(np.asfortranarray(R)).to(d)
    tb = torch.from_numpy(bt).to(d)
    oQ = torch.empty((m, m), dtype=torch.float64, device=d)
    oR = torch.zeros(max(1, nk * nk), dtype=torch.float64, device=d)
    ob = torch.empty(m, dtype=torch.float64, device=d)
    rmh = (ctypes.c_int32 * len(rm))(*rm)
    Ph = (ctypes.c_int32 * max(1, nk))()
    sw = ctypes.c_int32(0)
    print(f"downdate engine={engine} m={m} nP={nP} q={len(rm)}", flush=True)
    rc = lib.lhdm_test_downdate(torch.cuda.current_stream(d).cuda_stream, engine, m, nP, tQ.data_ptr(),
                                tR.data_ptr(), tb.data_ptr(), len(rm), rmh, oQ.data_ptr(), oR.data_ptr(),
                                ob.data_ptr(), Ph, ctypes.byref(sw))
    assert rc == 0, rc
    Qg = oQ.cpu().numpy().reshape(m, m).T          # column-major storage
    Rg = oR.cpu().numpy()[:nk * nk].reshape(nk, nk).T
    return Qg, Rg, ob.cpu().numpy(), list(Ph[:nk]), sw.value


def _compare(lib, engine, Q, R, bt, rm, want_sweeps=None, per_sweep=None):
    Qo, Ro, bo, Po = _oracle(Q, R, bt, rm, per_sweep)
    Qg, Rg, bg, Pg, sweeps = _gpu(lib, engine, Q, R, bt, rm)
    assert Pg == Po
    sR = max(1.0, float(np.abs(Ro).max(initial=0.0)))
    np.testing.assert_allclose(Rg, Ro, rtol=0, atol=TOL * sR)
    np.testing.assert_allclose(Qg, Qo, rtol=0, atol=TOL)
    np.testing.assert_allclose(bg, bo, rtol=0, atol=TOL * max(1.0, float(np.abs(bo).max())))
    if want_sweeps is not None:
        assert sweeps == want_sweeps
    return sweeps


def _golden_example():
    meta = {}
    with open(os.path.join(GOLDEN, "downdate_example.txt")) as f:
        for line in f:
            parts = line.split()
            if parts and parts[0] in ("m", "n", "deleted"):
                meta[parts[0]] = [int(p) for p in parts[1:]]
    return meta["m"][0], meta["n"][0], [d - 1 for d in meta["deleted"]]


@pytest.mark.parametrize("engine", [1, 2])
def test_section41_worked_example(lib, engine):
    # 8 x 7 factor, columns 2 and 5 (1-based) deleted: the example of Section 4.1
    m, n, rm = _golden_example()
    Q, R, bt = _state(m, n, 41)
    _compare(lib, engine, Q, R, bt, rm, want_sweeps=1)


CASES = [
    # (m, nP, positions spec, seed): several removals in one sweep
    (64, 50, "random:2", 1),
    (300, 300, "random:5", 2),
    (300, 257, "block:7@100", 3),          # consecutive positions
    (333, 200, "ends:3", 4),               # first and last positions
    (1024, 1000, "random:17", 5),
    (1024, 700, "random:64", 6),           # a full sweep of the device engine
    (2048, 2000, "random:40", 7),
    (100, 90, "tail:4", 13),               # only the last positions: nothing to rotate
    (40, 12, "random:12", 14),             # every position
]

SINGLE = [
    # one removal (every inner step of the large workloads): the whole-device
    # engine takes the closed form, chained over blocks of 64 new columns
    (1024, 1000, "block:1@0", 15),
    (1024, 1000, "block:1@300", 16),
    (300, 257, "block:1@190", 19),         # a ragged last block
    (700, 650, "block:1@649", 18),         # the last position: nothing to rotate
    # this triangle's forward substitution overflows (entries of O(1) above an
    # O(1) diagonal grow geometrically), so the closed form hands the removal
    # to the chained rotations
    (4096, 4000, "block:1@0", 17),
    # more new columns (4399) than the closed form keeps rotations for (4096):
    # the chained rotations again
    (5000, 4500, "block:1@100", 20),
]


def _positions(spec, nP, seed):
    kind, arg = spec.split(":")
    rng = np.random.default_rng(1000 + seed)
    if kind == "random":
        return sorted(rng.choice(nP, int(arg), replace=False).tolist())
    if kind == "block":
        cnt, start = (int(v) for v in arg.split("@"))
        return list(range(start, start + cnt))
    if kind == "tail":
        return list(range(nP - int(arg), nP))
    if kind == "ends":
        k = int(arg)
        return list(range(k)) + list(range(nP - k, nP))
    raise ValueError(spec)


@pytest.mark.parametrize("engine", [1, 2])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-{c[2]}" for c in CASES])
def test_multi_removal_sweep(lib, engine, case):
    m, nP, spec, seed = case
    Q, R, bt = _state(m, nP, seed)
    rm = _positions(spec, nP, seed)
    assert len(rm) >= 2
    _compare(lib, engine, Q, R, bt, rm, want_sweeps=1)


@pytest.mark.parametrize("engine", [1, 2])
@pytest.mark.parametrize("case", SINGLE, ids=[f"{c[0]}x{c[1]}-{c[2]}" for c in SINGLE])
def test_single_removal(lib, engine, case):
    m, nP, spec, seed = case
    if engine == 1 and m > 2048:
        pytest.skip("the one-workgroup engine holds m <= 2048")
    Q, R, bt = _state(m, nP, seed)
    _compare(lib, engine, Q, R, bt, _positions(spec, nP, seed), want_sweeps=1)


@pytest.mark.parametrize("case", [(4096, 4096, "random:64", 8), (4096, 3500, "random:33", 9)])
def test_multi_removal_sweep_full_size(lib, case):
    # the device engine at the size of the large instance (n_P up to m = 4096)
    m, nP, spec, seed = case
    Q, R, bt = _state(m, nP, seed)
    _compare(lib, 2, Q, R, bt, _positions(spec, nP, seed), want_sweeps=1)


@pytest.mark.parametrize("case", [(1500, 1200, 80, 10), (2048, 1800, 150, 11), (600, 500, 300, 12)])
def test_more_removals_than_one_sweep(lib, case):
    # more than 64 positions: the device engine sweeps the lowest 64 and
    # carries the rest to the next sweep (the solver's pending path), so it is
    # compared with the oracle deleting the same chunks in the same order; the
    # workgroup engine takes them all in one sweep.  (The two factorisations
    # differ: the kept columns' R and Q agree up to rounding and signs, the
    # freed columns of Q by an orthogonal change of basis.)
    m, nP, q, seed = case
    Q, R, bt = _state(m, nP, seed)
    rm = _positions(f"random:{q}", nP, seed)
    _compare(lib, 2, Q, R, bt, rm, want_sweeps=-(-q // 64), per_sweep=64)
    _compare(lib, 1, Q, R, bt, rm, want_sweeps=1)
