"""The 4096 x 16384 Gaussian instance (seed 3000) against the oracle's own path.

``tests/golden/c3_seed3000_delta<d>.npz`` hold what the CPU oracle computed on
this instance for delta in {0.2, 0.5, 0.8} (written by
``tests/golden/make_c3_golden.py``, which calls only the oracle and the input
generator): the final ordered passive set, x, the iteration counters, and the
accepted block J and the removal lists of every outer step.  The GPU solve must
follow the same path: identical ordered passive set and counters, x within
1e-10 relative (max-norm), KKT residual <= 1e-9.  When the final passive sets
differ, the first outer step after which the two passive sets differ is found by
re-running the GPU solve with an outer-step limit (bisection) and named in the
failure.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from parity_util import KKT, XTOL, _dev, _passive, _rel, oracle_passive_after
from workloads import make_c3

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def lhdm():
    import paper_2108_05345_amd as mod
    from paper_2108_05345_amd import _lib
    _lib.load()   # fails loudly if the HIP library is missing
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return mod


@pytest.fixture(scope="module")
def c3():
    inst = make_c3(3000)
    A, b = _dev(inst.A, inst.b)
    return inst, A, b


def _golden(delta):
    return np.load(os.path.join(GOLDEN, f"c3_seed3000_delta{delta:.1f}.npz"), allow_pickle=False)


def first_divergent_step(lhdm, A, b, delta, z):
    lo, hi = 0, int(z["counters"][1])   # P agrees after lo steps; disagrees after hi
    while hi - lo > 1:
        mid = (lo + hi) // 2
        r = lhdm.solve(A, b, delta=delta, max_outer=mid)
        if _passive(r) == oracle_passive_after(z, mid):
            lo = mid
        else:
            hi = mid
    return hi


@pytest.mark.parametrize("delta", [0.2, 0.5, 0.8])
def test_c3_full_size_follows_the_oracle_path(lhdm, c3, delta):
    inst, A, b = c3
    z = _golden(delta)
    st, outer, inner, jdrops, nP = (int(v) for v in z["counters"])
    print(f"c3 golden delta={delta}: oracle outer={outer} inner={inner} jd={jdrops} nP={nP}", flush=True)
    r = lhdm.solve(A, b, delta=delta)
    print(f"c3 gpu delta={delta}: {r.info}", flush=True)
    assert r.info["status"] == st == 0
    assert r.info["kkt_residual"] <= KKT
    P = _passive(r)
    Po = [int(j) for j in z["passive"]]
    if P != Po:
        s = first_divergent_step(lhdm, A, b, delta, z)
        pytest.fail(f"delta={delta}: the GPU's passive set first differs from the oracle's after outer step {s} "
                    f"of {outer}")
    assert (r.info["outer_iters"], r.info["inner_iters"], r.info["jloop_drops"], r.info["n_passive"]) == \
        (outer, inner, jdrops, nP)
    x = r.x.cpu().numpy()
    xo = z["x"]
    assert _rel(x, xo) <= XTOL, _rel(x, xo)
    assert (x >= 0).all() and np.count_nonzero(x) == len(P)
    # an independent check of the GPU's x: the oracle's KKT report on it
    assert oracle.kkt_report(inst.A, inst.b, x)["kkt"] <= KKT
