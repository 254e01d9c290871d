"""The three batched engines (fused with one or two workgroups per compute unit,
phased with one kernel per stage replayed as a HIP graph) take the same steps in
the same order, so their results must agree bit for bit; the phased engine is
also compared with the oracle directly.

Workloads: uneven nonnegative instances of the NMF-subproblem kind (m from 32
to 512, n = m x U[2, 4]) and Gaussian differentiation instances (256 x 512)."""
import numpy as np
import pytest
import torch

import oracle
from parity_util import _check, _dev
from workloads import make_c4_batch, make_c5_batch

pytestmark = pytest.mark.gpu

ENGINES = ["fused", "fused2", "phased"]


@pytest.fixture(scope="module")
def lhdm():
    import paper_2108_05345_amd as mod
    from paper_2108_05345_amd import _lib
    _lib.load()   # fails loudly if the HIP library is missing
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return mod


def _pool(lhdm, insts):
    As = [torch.from_numpy(np.ascontiguousarray(i.A)).cuda() for i in insts]
    bs = [torch.from_numpy(i.b).cuda() for i in insts]
    return lhdm.pack(As, bs)


def _run(lhdm, pool, engine, use_lh):
    x, passive, infos = lhdm.solve_pooled(pool, use_lh=use_lh, engine=engine)
    torch.cuda.synchronize()
    return x.cpu().numpy(), passive.cpu().numpy(), infos


@pytest.mark.parametrize("use_lh", [False, True])
@pytest.mark.parametrize("which", ["c4", "c5"])
def test_engines_agree_bitwise(lhdm, which, use_lh):
    insts = make_c4_batch(4100, count=96) if which == "c4" else make_c5_batch(5100, count=40)
    pool = _pool(lhdm, insts)
    ref = _run(lhdm, pool, "fused", use_lh)
    assert all(i["status"] == 0 for i in ref[2])
    for eng in ENGINES[1:]:
        print(f"[engines] {which} lh={use_lh} {eng}", flush=True)
        got = _run(lhdm, pool, eng, use_lh)
        np.testing.assert_array_equal(got[0], ref[0])
        np.testing.assert_array_equal(got[1], ref[1])
        for a, b in zip(got[2], ref[2]):
            assert a == b
    auto = _run(lhdm, pool, "auto", use_lh)
    np.testing.assert_array_equal(auto[0], ref[0])


def test_phased_against_the_oracle(lhdm):
    insts = make_c4_batch(4200, count=24)
    As, bs = zip(*[_dev(i.A, i.b) for i in insts])
    for use_lh in (False, True):
        res = lhdm.solve_batched(list(As), list(bs), use_lh=use_lh, engine="phased")
        for inst, r in zip(insts, res):
            xo, io = (oracle.oracle_lh if use_lh else oracle.oracle_lhdm)(inst.A, inst.b)
            _check(r, xo, io, same_path=False, tag=f"phased-{inst.name}-lh{int(use_lh)}")


def test_phased_iteration_limit(lhdm):
    # a tiny outer limit ends every instance with the iteration-limit status,
    # with the same x in both engines
    insts = make_c4_batch(4300, count=16)
    pool = _pool(lhdm, insts)
    a = lhdm.solve_pooled(pool, max_outer=3, engine="fused")
    b = lhdm.solve_pooled(pool, max_outer=3, engine="phased")
    torch.cuda.synchronize()
    assert all(i["status"] == 1 for i in a[2])
    np.testing.assert_array_equal(a[0].cpu().numpy(), b[0].cpu().numpy())
    assert [i["status"] for i in a[2]] == [i["status"] for i in b[2]]
