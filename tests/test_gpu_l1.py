"""l1-NNLS (Section 3.3) on the GPU against the oracle: the squared-l1
regularised least squares min ||x||_1^2 + lam^2 ||A x - b||^2 solved through
its NNLS form (assembled on the device).  Compared: z = (x+, x-), the passive
set and the counters (path identity where separated), the signed x, and the
optimality conditions of the regularised problem on the GPU's x."""
import types

import numpy as np
import pytest
import torch

import oracle
from parity_util import _check, _dev
from test_oracle_pins_l1 import _l1_optimality
from workloads import make_signed

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lhdm():
    import paper_2108_05345_amd as mod
    from paper_2108_05345_amd import _lib
    _lib.load()   # fails loudly if the HIP library is missing
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return mod


CASES = [(40, 90, 6, 1e-2, 3), (100, 300, 12, 1e-2, 7), (257, 700, 25, 1e-3, 8)]


@pytest.mark.parametrize("engine", ["workgroup", "device"])
@pytest.mark.parametrize("lam", [0.3, 3.0, 30.0])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}" for c in CASES])
def test_l1nnls_parity(lhdm, case, lam, engine):
    m, n, k, noise, seed = case
    inst = make_signed(m, n, k, seed, noise_std=noise)
    A, b = _dev(inst.A, inst.b)
    for method, kmax in (("lhdm", 32), ("lh", 1)):
        x_o, io = oracle.oracle_l1nnls(inst.A, inst.b, lam, method=method)
        r = lhdm.solve_l1(A, b, lam, kmax=kmax, engine=engine)
        res = types.SimpleNamespace(x=r.z, passive=r.passive, info=r.info)
        _check(res, io["z"], io, tag=f"l1-{m}x{n}-lam{lam}-{method}-{engine}")
        x = r.x.cpu().numpy()
        assert np.abs(x - x_o).max() <= 1e-10 * max(1.0, np.abs(x_o).max())
        _l1_optimality(inst.A, inst.b, lam, x, 1e-8)


def test_l1nnls_rejects_bad_lambda(lhdm):
    from paper_2108_05345_amd import LhdmError
    inst = make_signed(20, 40, 3, 1)
    A, b = _dev(inst.A, inst.b)
    for lam in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(LhdmError):
            lhdm.solve_l1(A, b, lam)
