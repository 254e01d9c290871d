"""The whole-device engine's two factorisations of an appended block (Algorithm 4).

By default a block of 2 to 32 columns is factored by CholeskyQR2 on its Gram
matrix, and the Householder reflectors are rebuilt from the orthonormal factor.
The alternative (flag LHDM_FLAG_PANEL_HOUSEHOLDER, ``panel="householder"``)
factors the block column by column.  Both are compared with the oracle on their
path and with each other.  ``info["cq_panels"]`` counts the blocks that went the
CholeskyQR2 way, which shows which branch ran, including the fall-back for a
nearly dependent block.
"""
import numpy as np
import pytest
import torch

import oracle
from parity_util import XTOL, _check, _dev, _passive, _rel
from workloads import make_c3, make_small

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lhdm():
    import paper_2108_05345_amd as mod
    from paper_2108_05345_amd import _lib
    _lib.load()   # fails loudly if the HIP library is missing
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return mod


def _both(lhdm, A, b, **kw):
    r_cq = lhdm.solve(A, b, engine="device", **kw)
    r_hh = lhdm.solve(A, b, engine="device", panel="householder", **kw)
    assert r_hh.info["cq_panels"] == 0
    return r_cq, r_hh


def _agree(r_cq, r_hh, tag):
    # same passive set in the same order, same counters, x to the parity bar
    assert _passive(r_cq) == _passive(r_hh), tag
    for key in ("outer_iters", "inner_iters", "jloop_drops", "n_passive"):
        assert r_cq.info[key] == r_hh.info[key], (tag, key)
    assert _rel(r_cq.x.cpu().numpy(), r_hh.x.cpu().numpy()) <= XTOL, tag


@pytest.mark.parametrize("delta", [0.2, 0.5, 0.8])
def test_scaled_c3_both_panels(lhdm, delta):
    inst = make_c3(3000, m=160, n=640, k=32)
    A, b = _dev(inst.A, inst.b)
    xo, io = oracle.oracle_lhdm(inst.A, inst.b, delta=delta)
    r_cq, r_hh = _both(lhdm, A, b, delta=delta)
    assert r_cq.info["cq_panels"] > 0
    assert _check(r_cq, xo, io, unique=False, tag=f"cq-c3s-d{delta}") == "path"
    assert _check(r_hh, xo, io, unique=False, tag=f"hh-c3s-d{delta}") == "path"
    _agree(r_cq, r_hh, f"c3s-d{delta}")


@pytest.mark.parametrize("shape", [(333, 700, 60, 31), (517, 1100, 90, 32), (300, 1800, 60, 51)])
def test_uniform_instances_both_panels(lhdm, shape):
    # several row blocks of the CholeskyQR2 passes with ragged tails; the last
    # one has hundreds of candidates at the first step
    m, n, k, seed = shape
    inst = make_small(m, n, k, seed, kind="uniform", noise_std=1e-2)
    A, b = _dev(inst.A, inst.b)
    xo, io = oracle.oracle_lhdm(inst.A, inst.b)
    r_cq, r_hh = _both(lhdm, A, b)
    assert r_cq.info["cq_panels"] > 0
    _check(r_cq, xo, io, same_path=False, tag=f"cq-{m}x{n}")
    _check(r_hh, xo, io, same_path=False, tag=f"hh-{m}x{n}")
    _agree(r_cq, r_hh, f"{m}x{n}")


@pytest.mark.parametrize("kmax", [2, 17, 32, 48])
def test_block_widths(lhdm, kmax):
    # kmax = 48: blocks wider than 32 columns go column by column, narrower
    # ones (after the selection) may still take CholeskyQR2
    inst = make_small(200, 600, 40, 77, kind="uniform", noise_std=1e-2)
    A, b = _dev(inst.A, inst.b)
    xo, io = oracle.oracle_lhdm(inst.A, inst.b, kmax=kmax)
    r_cq, r_hh = _both(lhdm, A, b, kmax=kmax)
    _check(r_cq, xo, io, tag=f"cq-kmax{kmax}")
    _check(r_hh, xo, io, tag=f"hh-kmax{kmax}")
    if kmax <= 32:
        assert r_cq.info["cq_panels"] > 0


@pytest.mark.parametrize("eps, expect", [(1e-5, 0), (0.5, 1)])
def test_nearly_dependent_block(lhdm, eps, expect):
    # Unit columns u, v (orthogonal) and w = (u + v) / sqrt(2) + eps z,
    # normalised (z orthogonal to both), and b = u + v + w.  The three are the
    # first step's candidates.  Their pairwise cosines (about 0.71 and 0 for
    # eps = 1e-5, 0.63 and 0 for 0.5) are below delta = 0.8, so Algorithm 2
    # accepts all three as one block.  With eps = 1e-5, the squared sine of the
    # third column against the first two is about 1e-10: the block's Gram matrix
    # is nearly singular and the block goes column by column.  With eps = 0.5 it
    # is 1/3, and CholeskyQR2 factors the block.  The other five columns have
    # negative duals and never enter.
    m = 300
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.standard_normal((m, 8)))
    u, v, z = Q[:, 0], Q[:, 1], Q[:, 2]
    w = (u + v) / np.sqrt(2.0) + eps * z
    w /= np.linalg.norm(w)
    s = u + v + w
    neg = [-(s / np.linalg.norm(s)) * (1.0 - 0.01 * i) + 0.05 * Q[:, 3 + i] for i in range(5)]
    A = np.stack([u, v, w] + neg, axis=1)
    b = A[:, :3] @ np.ones(3)
    assert (A[:, 3:].T @ b < 0).all()
    Ad, bd = _dev(A, b)
    xo, io = oracle.oracle_lhdm(A, b, delta=0.8)
    assert io["outer_iters"] == 1 and sorted(io["passive"]) == [0, 1, 2]
    r_cq, r_hh = _both(lhdm, Ad, bd, delta=0.8)
    assert r_cq.info["cq_panels"] == expect, r_cq.info
    _check(r_cq, xo, io, tag=f"dep-cq-{eps}")
    _check(r_hh, xo, io, tag=f"dep-hh-{eps}")
    _agree(r_cq, r_hh, f"dep-{eps}")


def test_c3_full_size_both_panels(lhdm):
    # the 4096 x 16384 instance (delta = 0.8): both factorisations reach the
    # same passive set and x; the CholeskyQR2 one factors most blocks
    inst = make_c3(3000)
    A, b = _dev(inst.A, inst.b)
    r_cq, r_hh = _both(lhdm, A, b, delta=0.8)
    print(f"[c3-panels] cq {r_cq.info} | hh {r_hh.info}", flush=True)
    assert r_cq.info["status"] == 0 and r_hh.info["status"] == 0
    assert r_cq.info["cq_panels"] >= r_cq.info["outer_iters"] // 2
    _agree(r_cq, r_hh, "c3-full")
