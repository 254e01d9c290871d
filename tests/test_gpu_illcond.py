"""Parity on moderately ill-conditioned instances (condition number about 1e5 to
1e7), the regime of the paper's experiments with modified condition numbers.

``make_illcond``: nonnegative uniform matrices with rows scaled over 4 or 5
decades.  Row scaling keeps the set {x >= 0: A x = b}, so the sparse planted
solution stays the unique one, while the triangular factors, the Givens
downdates and the norm downdating of the projected column norms work with
entries spread over many orders of magnitude.  Noiseless instances must
recover the planted solution; noisy ones (positive residual) are compared with
the oracle's solution.
"""
import numpy as np
import pytest
import torch

import oracle
from parity_util import _check, _dev
from workloads import make_illcond

pytestmark = pytest.mark.gpu

ENGINES = ["workgroup", "device"]

CASES = [
    # (m, n, k, row_range, noise, seed)
    (128, 512, 8, 1e5, 0.0, 1),
    (128, 512, 13, 1e6, 0.0, 2),
    (256, 1024, 26, 1e5, 0.0, 4),
    (256, 1024, 26, 1e5, 1e-6, 5),
    (300, 900, 30, 1e6, 1e-7, 6),
]


@pytest.fixture(scope="module")
def lhdm():
    import paper_2108_05345_amd as mod
    from paper_2108_05345_amd import _lib
    _lib.load()   # fails loudly if the HIP library is missing
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return mod


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-r{c[3]:.0e}-n{c[4]:.0e}" for c in CASES])
def test_illconditioned_parity(lhdm, case, engine):
    m, n, k, rr, noise, seed = case
    inst = make_illcond(m, n, k, rr, seed, noise_std=noise)
    cond = np.linalg.cond(inst.A)
    assert 1e5 <= cond <= 1e8, cond
    A, b = _dev(inst.A, inst.b)
    # noiseless: the passive set ends with columns of rounding-level
    # coefficients, and with condition numbers near 1e6 the feasibility
    # decisions on them are set by rounding, so only the result is compared
    # (support, x, KKT); noisy (positive residual, separated): the whole path
    same = noise > 0.0
    for delta in (0.9, 0.5):
        xo, io = oracle.oracle_lhdm(inst.A, inst.b, delta=delta)
        r = lhdm.solve(A, b, delta=delta, engine=engine)
        got = _check(r, xo, io, same_path=same, tag=f"ill-{m}x{n}-d{delta}-{engine}")
        assert got == ("path" if same else "none")
        if noise == 0.0:
            np.testing.assert_allclose(r.x.cpu().numpy(), inst.x_true, rtol=0, atol=1e-9)
    xo, io = oracle.oracle_lh(inst.A, inst.b)
    r = lhdm.solve(A, b, kmax=1, engine=engine)
    _check(r, xo, io, same_path=same, tag=f"ill-{m}x{n}-lh-{engine}")


def test_illconditioned_large_device(lhdm):
    # several row blocks of the chained kernels, condition number ~1e6
    inst = make_illcond(1024, 4096, 80, 1e5, 7)
    A, b = _dev(inst.A, inst.b)
    xo, io = oracle.oracle_lhdm(inst.A, inst.b)
    r = lhdm.solve(A, b, engine="device")
    _check(r, xo, io, same_path=False, tag="ill-1024x4096")
    np.testing.assert_allclose(r.x.cpu().numpy(), inst.x_true, rtol=0, atol=1e-9)
