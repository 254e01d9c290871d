"""The variant of Theorem 4 on the GPU: tau1 = 1, tau2 <= 1/2 and delta <=
tau2 / (kmax - 1), with the feasibility loop on J not evaluated
(LHDM_FLAG_NO_JLOOP), against the oracle run the same way and against the
oracle with the loop (Theorem 4: the paths coincide)."""
import numpy as np
import pytest
import torch

import oracle
from parity_util import _check, _dev
from test_oracle_pins_kkt import T4, tie_instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lhdm():
    import paper_2108_05345_amd as mod
    from paper_2108_05345_amd import _lib
    _lib.load()   # fails loudly if the HIP library is missing
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return mod


@pytest.mark.parametrize("engine", ["workgroup", "device"])
@pytest.mark.parametrize("seed", [11, 12, 13, 14, 15])
def test_theorem4_variant_parity(lhdm, seed, engine):
    A, b = tie_instance(seed)
    xo, io = oracle.oracle_lhdm(A, b, jloop=False, **T4)
    xj, ij = oracle.oracle_lhdm(A, b, **T4)
    assert io["passive"] == ij["passive"] and ij["jloop_drops"] == 0
    r = lhdm.solve(*_dev(A, b), engine=engine, no_jloop=True, **T4)
    assert r.info["jloop_drops"] == 0
    assert _check(r, xo, io, unique=False, tag=f"t4-{seed}-{engine}") in ("path", "order")


def test_theorem4_flag_needs_its_thresholds(lhdm):
    from paper_2108_05345_amd import LhdmError
    A, b = tie_instance(11)
    with pytest.raises(LhdmError):
        lhdm.solve(*_dev(A, b), no_jloop=True)            # tau1 = 0.6
    with pytest.raises(LhdmError):
        lhdm.solve(*_dev(A, b), no_jloop=True, tau1=1.0, tau2=0.5, kmax=8, delta=0.9)
