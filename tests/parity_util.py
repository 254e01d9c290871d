"""Helpers shared by the GPU parity tests (not a test module).

Bar (from the requirements of the solver): identical passive set where the
minimiser is unique, x within 1e-10 relative (max-norm), KKT residual <= 1e-9.
Where the two follow the same path (no rounding-level near-ties) the ordered
passive set and the iteration counters agree as well.
"""
import numpy as np
import torch

XTOL = 1e-10
KKT = 1e-9


def _dev(A, b):
    d = torch.device("cuda:0")
    return (torch.from_numpy(np.asfortranarray(A)).to(d), torch.from_numpy(np.ascontiguousarray(b)).to(d))


def _rel(x, xo):
    return float(np.abs(x - xo).max() / max(np.abs(xo).max(), 1e-300))


def _passive(res):
    P = res.passive.cpu().numpy()
    return [int(j) for j in P if j >= 0]


SUPP_THR = 1e-12   # support = entries above this fraction of max|x| (rounding-level entries excluded)
SEP = 1e-8         # a solution is well separated when every passive entry exceeds SEP * max|x|
SIG = 1e-12        # significant entries (above rounding level) for the order comparison


def _supp(x):
    return sorted(int(j) for j in np.nonzero(x > SUPP_THR * np.abs(x).max(initial=0.0))[0])


def _check(res, x_o, info_o, *, same_path=True, unique=True, tag=""):
    """Compare one GPU result with the oracle's; returns what was compared.

    In zero-residual instances an appended column can have an exactly-zero
    least-squares coefficient; its sign, and so the decisions of the feasibility
    loops, is then set by rounding and legitimately differs between summation
    orders.  Path identity (ordered P, iteration counters) is therefore required
    when both solutions are well separated from zero ("path"); otherwise the
    significant columns must enter P in the same order and the outer steps agree
    ("order").  "none": same_path was not asked for."""
    x = res.x.cpu().numpy()
    print(f"[{tag}] gpu info {res.info} | oracle outer={info_o['outer_iters']} inner={info_o['inner_iters']} "
          f"jd={info_o['jloop_drops']} nP={info_o['n_passive']}", flush=True)
    assert res.info["status"] == info_o["status"] == 0
    assert (x >= 0).all()
    assert res.info["kkt_residual"] <= KKT
    P = _passive(res)
    assert res.info["n_passive"] == len(P)
    assert all(x[j] > 0 for j in P)
    assert np.count_nonzero(x) == len(P)
    if unique:
        assert _supp(x) == _supp(x_o), tag
        assert _rel(x, x_o) <= XTOL, (tag, _rel(x, x_o))
    Po = info_o["passive"]

    def sep(xx, PP):
        return len(PP) == 0 or float(np.min(xx[PP])) > SEP * float(np.abs(xx).max())

    separated = sep(x_o, Po) and sep(x, P)
    if not same_path:
        return "none"
    if separated:
        assert P == Po, tag
        for key in ("outer_iters", "inner_iters", "jloop_drops"):
            assert res.info[key] == info_o[key], (tag, key)
        return "path"
    # rounding-level entries (a column appended with an exactly-zero
    # coefficient): their fate is set by rounding, so only the order of the
    # significant columns and the number of accepted outer steps are compared
    big = SIG * max(float(np.abs(x_o).max()), float(np.abs(x).max()))
    assert [j for j in P if x[j] > big] == [j for j in Po if x_o[j] > big], tag
    assert res.info["outer_iters"] == info_o["outer_iters"], tag
    return "order"




def oracle_passive_after(z, steps):
    """The oracle's ordered passive set after `steps` accepted outer steps."""
    P = []
    jo = ro = ri = 0
    for s in range(steps):
        P = P + [int(j) for j in z["J_flat"][jo:jo + z["J_len"][s]]]
        jo += int(z["J_len"][s])
        for _ in range(int(z["rm_count"][s])):
            rm = set(int(j) for j in z["rm_flat"][ro:ro + z["rm_len"][ri]])
            ro += int(z["rm_len"][ri])
            ri += 1
            P = [j for j in P if j not in rm]
    return P
