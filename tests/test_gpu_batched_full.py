"""Batched parity at full size: every instance of the uneven nonnegative batch
(2000 instances, seed 4000) against the oracle's stored results, and the
backward at the differentiation shape (256 instances of 256 x 512).

The oracle's passive sets and counters for the 2000 instances were written by
``tests/golden/make_batch_golden.py`` (oracle and workloads only); on its final
passive set the oracle's x is the least-squares solution, recomputed here."""
import os

import numpy as np
import pytest
import torch

import oracle
from parity_util import KKT, SEP, SIG, XTOL, _rel
from workloads import make_c4_batch, make_c5_batch

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c4_seed4000_lhdm.npz")


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


@pytest.mark.parametrize("engine", ["auto", "fused2"])
def test_all_2000_uneven_instances_against_the_oracle(lhdm, engine):
    z = np.load(GOLDEN, allow_pickle=False)
    insts = make_c4_batch(4000)
    assert len(insts) == len(z["P_len"]) == 2000
    pool = _pool(lhdm, insts)
    x, passive, infos = lhdm.solve_pooled(pool, engine=engine)
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    passive = passive.cpu().numpy()
    offs = np.concatenate([[0], np.cumsum(z["P_len"])])
    kinds = {"path": 0, "order": 0}
    for i, inst in enumerate(insts):
        n = inst.A.shape[1]
        o = pool.x_off[i]
        xg = x[o:o + n]
        Pg = [int(j) for j in passive[o:o + n] if j >= 0]
        Po = [int(j) for j in z["P_flat"][offs[i]:offs[i + 1]]]
        st, outer, inner, jd, npas = (int(v) for v in z["counters"][i])
        info = infos[i]
        tag = f"c4-{i} m={inst.A.shape[0]} n={n}"
        assert st == 0 and info["status"] == 0, tag
        assert info["kkt_residual"] <= KKT, tag
        assert sorted(Pg) == sorted(Po), tag                     # identical support
        assert (xg >= 0).all() and np.count_nonzero(xg) == len(Pg), tag
        xo = np.zeros(n)
        xo[Po] = np.linalg.lstsq(inst.A[:, Po], inst.b, rcond=None)[0]
        assert _rel(xg, xo) <= XTOL, (tag, _rel(xg, xo))
        sep = len(Po) == 0 or (float(xo[Po].min()) > SEP * float(np.abs(xo).max())
                               and float(xg[Pg].min()) > SEP * float(np.abs(xg).max()))
        if sep:
            assert Pg == Po, tag
            assert (info["outer_iters"], info["inner_iters"], info["jloop_drops"]) == (outer, inner, jd), tag
            kinds["path"] += 1
        else:
            big = SIG * max(float(np.abs(xo).max()), float(np.abs(xg).max()))
            assert [j for j in Pg if xg[j] > big] == [j for j in Po if xo[j] > big], tag
            assert info["outer_iters"] == outer, tag
            kinds["order"] += 1
    print(f"[c4-all {engine}] compared: {kinds}", flush=True)
    assert kinds["path"] + kinds["order"] == 2000


def test_backward_at_the_differentiation_shape(lhdm):
    insts = make_c5_batch(5000)
    assert len(insts) == 256 and insts[0].A.shape == (256, 512)
    pool = _pool(lhdm, insts)
    x, passive, infos = lhdm.solve_pooled(pool)
    t = torch.from_numpy(np.concatenate([i.t for i in insts])).cuda()
    gx = 2.0 * (x - t)
    gA, gb = lhdm.backward_pooled(pool, x, passive, gx)
    torch.cuda.synchronize()
    assert all(i["status"] == 0 and i["kkt_residual"] <= KKT for i in infos)
    x, passive, gx = x.cpu().numpy(), passive.cpu().numpy(), gx.cpu().numpy()
    gA, gb = gA.cpu().numpy(), gb.cpu().numpy()
    for i in list(range(0, 256, 8)) + [255]:
        inst = insts[i]
        m, n = inst.A.shape
        o, ao, bo = pool.x_off[i], pool.a_off[i], pool.b_off[i]
        P = [int(j) for j in passive[o:o + n] if j >= 0]
        rA, rb = oracle.nnls_grad_reference(inst.A, inst.b, x[o:o + n], P, gx[o:o + n])
        gAi = gA[ao:ao + m * n].reshape(n, m).T      # column-major in the pool
        scale = max(np.abs(rA).max(), 1.0)
        assert np.abs(gAi - rA).max() <= 1e-8 * scale, i
        assert np.abs(gb[bo:bo + m] - rb).max() <= 1e-8 * max(np.abs(rb).max(), 1.0), i


C2_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_seeds2000-2019.npz")


@pytest.mark.parametrize("method", ["lhdm", "lh"])
def test_all_20_sparse_recovery_instances_against_the_oracle(lhdm, method):
    # m = 1024, n = 4096 (the whole-device engine): the ordered passive set,
    # the counters and x of every seed against the oracle's stored results,
    # and the planted solution recovered
    from parity_util import _dev
    from workloads import make_c2
    z = np.load(C2_GOLDEN, allow_pickle=False)
    offs = np.concatenate([[0], np.cumsum(z[f"{method}_P_len"])])
    for i, seed in enumerate(z["seeds"]):
        inst = make_c2(int(seed))
        A, b = _dev(inst.A, inst.b)
        r = lhdm.solve(A, b) if method == "lhdm" else lhdm.lh_solve(A, b)
        Po = [int(j) for j in z[f"{method}_P"][offs[i]:offs[i + 1]]]
        xo = np.zeros(inst.A.shape[1])
        xo[Po] = z[f"{method}_xP"][offs[i]:offs[i + 1]]
        st, outer, inner, jd, npas = (int(v) for v in z[f"{method}_counters"][i])
        x = r.x.cpu().numpy()
        Pg = [int(j) for j in r.passive.cpu().numpy() if j >= 0]
        tag = f"c2-{seed}-{method}"
        print(f"[{tag}] gpu {r.info} oracle outer={outer} inner={inner} jd={jd}", flush=True)
        assert st == 0 and r.info["status"] == 0, tag
        assert r.info["kkt_residual"] <= KKT, tag
        assert _rel(x, xo) <= XTOL, (tag, _rel(x, xo))
        if float(xo[Po].min()) > SEP * float(np.abs(xo).max()) and float(x[Pg].min()) > SEP * float(np.abs(x).max()):
            assert Pg == Po, tag
            assert (r.info["outer_iters"], r.info["inner_iters"], r.info["jloop_drops"]) == (outer, inner, jd), tag
        else:
            # a column entered with a rounding-level coefficient (zero residual):
            # the significant columns in the same order, the same outer steps
            big = SIG * max(float(np.abs(xo).max()), float(np.abs(x).max()))
            assert [j for j in Pg if x[j] > big] == [j for j in Po if xo[j] > big], tag
            assert r.info["outer_iters"] == outer, tag
        assert np.abs(x - inst.x_true).max() <= 1e-9 * np.abs(inst.x_true).max(), tag
