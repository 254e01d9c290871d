"""The stored oracle paths of the 4096 x 16384 instance (tests/golden/c3_*.npz)
checked against what the mathematics fixes, without a GPU: the step lists
rebuild the final passive set, the stored x satisfies the KKT conditions of
Theorem 1 at 1e-9 on the regenerated instance, and it is nonzero exactly on
the passive set."""
import os

import numpy as np
import pytest

import oracle
from parity_util import oracle_passive_after
from workloads import make_c3

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DELTAS = (0.2, 0.5, 0.8)


@pytest.fixture(scope="module")
def c3():
    return make_c3(3000)


@pytest.mark.parametrize("delta", DELTAS)
def test_golden_path_rebuilds_the_passive_set(delta):
    z = np.load(os.path.join(GOLDEN, f"c3_seed3000_delta{delta:.1f}.npz"), allow_pickle=False)
    st, outer, inner, jdrops, nP = (int(v) for v in z["counters"])
    assert st == 0 and float(z["delta"]) == delta and int(z["seed"]) == 3000
    assert len(z["J_len"]) == outer and int(z["rm_count"].sum()) == inner
    assert int(z["drops"].sum()) <= jdrops
    P = oracle_passive_after(z, outer)
    assert P == [int(j) for j in z["passive"]] and len(P) == nP
    # every step appends at least one column (Theorem 3: no empty step)
    assert (z["J_len"] >= 1).all() and (z["J_len"] <= 32).all()


@pytest.mark.parametrize("delta", DELTAS)
def test_golden_solution_satisfies_kkt(c3, delta):
    z = np.load(os.path.join(GOLDEN, f"c3_seed3000_delta{delta:.1f}.npz"), allow_pickle=False)
    x = z["x"]
    P = [int(j) for j in z["passive"]]
    assert (x >= 0).all() and np.count_nonzero(x) == len(P) and (x[P] > 0).all()
    rep = oracle.kkt_report(c3.A, c3.b, x)
    assert rep["kkt"] <= 1e-9 and rep["feasible"]
    assert abs(rep["kkt"] - float(z["kkt"])) <= 1e-12


def test_batch_fixture_matches_its_instances():
    # the stored passive sets index columns of the instances they were made for,
    # every stored solve converged, and instance i generated alone is instance i
    # of the batch
    import os
    import numpy as np
    from workloads import make_c4_batch, make_c4_instance
    z = np.load(os.path.join(os.path.dirname(__file__), "golden", "c4_seed4000_lhdm.npz"), allow_pickle=False)
    assert len(z["P_len"]) == 2000 and int(z["P_len"].sum()) == len(z["P_flat"])
    assert (z["counters"][:, 0] == 0).all()
    assert (z["counters"][:, 4] == z["P_len"]).all()
    batch = make_c4_batch(4000, count=2000)
    offs = np.concatenate([[0], np.cumsum(z["P_len"])])
    for i in (0, 1, 999, 1999):
        one = make_c4_instance(i, 4000)
        assert np.array_equal(one.A, batch[i].A) and np.array_equal(one.b, batch[i].b)
        P = z["P_flat"][offs[i]:offs[i + 1]]
        assert len(set(P.tolist())) == len(P) and P.min() >= 0 and P.max() < one.A.shape[1]
        assert len(P) <= min(one.A.shape)


def test_c2_fixture_is_the_planted_solution():
    # noiseless sparse recovery: the stored oracle solutions are the planted x
    # (the unique NNLS solution); the passive set holds its support, plus at
    # most a column whose coefficient is rounding noise (zero residual)
    import os
    import numpy as np
    from workloads import make_c2
    z = np.load(os.path.join(os.path.dirname(__file__), "golden", "c2_seeds2000-2019.npz"), allow_pickle=False)
    for method in ("lhdm", "lh"):
        offs = np.concatenate([[0], np.cumsum(z[f"{method}_P_len"])])
        assert (z[f"{method}_counters"][:, 0] == 0).all()
        for i, seed in enumerate(z["seeds"][:4]):
            inst = make_c2(int(seed))
            P = z[f"{method}_P"][offs[i]:offs[i + 1]]
            x = np.zeros(inst.A.shape[1])
            x[P] = z[f"{method}_xP"][offs[i]:offs[i + 1]]
            supp = sorted(np.nonzero(x > 1e-12)[0].tolist())
            assert supp == sorted(np.nonzero(inst.x_true)[0].tolist())
            assert set(supp) <= set(P.tolist())
            np.testing.assert_allclose(x, inst.x_true, rtol=0, atol=1e-10)
