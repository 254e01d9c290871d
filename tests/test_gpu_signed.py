"""The positivity trick (Section 3.2) on the GPU against the oracle, with the
sign-flip inner loop of Section 4.2 and with the ordinary one, both engines.

The GPU never forms -A: column j >= n of [A, -A] is read as -a_{j-n}.  Compared
with the oracle's solve on the explicit [A, -A]: the 2n-vector z = (x+, x-), its
passive set and iteration counters (path identity where the solution is
separated), and the signed x = x+ - x-; noiseless sparse instances must recover
the planted signed solution.
"""
import types

import numpy as np
import pytest
import torch

import oracle
from parity_util import _check, _dev
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


CASES = [
    # (m, n, k, noise, seed)
    (64, 128, 8, 0.0, 1),
    (128, 512, 20, 0.0, 2),
    (256, 1024, 40, 0.0, 3),
    (200, 150, 40, 1e-2, 4),     # overdetermined, noisy: unique signed least-squares solution
]


def _compare(r, inst, method, flip, tag):
    kw = {} if method == "lhdm" else {}
    x_o, io = oracle.oracle_signed(inst.A, inst.b, method=method, sign_flip=flip)
    res = types.SimpleNamespace(x=r.z, passive=r.passive, info=r.info)
    got = _check(res, io["z"], io, unique=False, tag=tag)
    x = r.x.cpu().numpy()
    np.testing.assert_allclose(x, r.z.cpu().numpy()[:inst.n] - r.z.cpu().numpy()[inst.n:], rtol=0, atol=0)
    assert np.abs(x - x_o).max() <= 1e-10 * max(1.0, np.abs(x_o).max()), tag
    return got


@pytest.mark.parametrize("engine", ["workgroup", "device"])
@pytest.mark.parametrize("flip", [True, False])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-k{c[2]}-n{c[3]:.0e}" for c in CASES])
def test_signed_parity(lhdm, case, flip, engine):
    m, n, k, noise, seed = case
    inst = make_signed(m, n, k, seed, noise_std=noise)
    A, b = _dev(inst.A, inst.b)
    r = lhdm.solve_signed(A, b, sign_flip=flip, engine=engine)
    assert _compare(r, inst, "lhdm", flip, f"signed-{m}x{n}-f{int(flip)}-{engine}") in ("path", "order")
    rl = lhdm.solve_signed(A, b, sign_flip=flip, kmax=1, engine=engine)
    assert _compare(rl, inst, "lh", flip, f"signed-lh-{m}x{n}-f{int(flip)}-{engine}") in ("path", "order")
    if noise == 0.0:
        for rr in (r, rl):
            np.testing.assert_allclose(rr.x.cpu().numpy(), inst.x_true, rtol=0, atol=1e-11)


def test_sign_flips_counted_as_inner_iterations(lhdm):
    # an instance whose ordinary inner loop runs several times: with the flip the
    # GPU's inner iterations are the oracle's flips, and no column is removed
    inst = make_signed(128, 512, 20, 2)
    A, b = _dev(inst.A, inst.b)
    x1, i1 = oracle.oracle_signed(inst.A, inst.b, sign_flip=True, record=True)
    assert sum(len(f) for s in i1["trace"] for f in s["flipped"]) > 0
    r = lhdm.solve_signed(A, b, sign_flip=True, engine="device")
    assert r.info["inner_iters"] == i1["inner_iters"]
    assert r.info["n_passive"] == i1["n_passive"]


def test_signed_large_device(lhdm):
    # several row blocks of the chained kernels; the sign flip on the device engine
    inst = make_signed(1024, 4096, 200, 5)   # 4 sign-flip inner iterations in the oracle
    A, b = _dev(inst.A, inst.b)
    for flip in (True, False):
        r = lhdm.solve_signed(A, b, sign_flip=flip)
        _compare(r, inst, "lhdm", flip, f"signed-1024x4096-f{int(flip)}")
        np.testing.assert_allclose(r.x.cpu().numpy(), inst.x_true, rtol=0, atol=1e-11)
