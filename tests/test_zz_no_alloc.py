"""The allocation-free batched solve (lhdm_solve_batched_noalloc) against the
batched solve with a workspace (lhdm_solve_batched), through the C ABI.

Same instances, same parameters: the two entry points run the same kernels on
the same data, so x, the passive sets and the iteration counters must be
identical; the noalloc call differs only in where its buffers live (the
library's fixed device scratch) and in the queue order.  Two calls in a row,
the second with a smaller batch, check that the scratch left by the first call
does not leak into the second.
"""
import ctypes

import numpy as np
import pytest
import torch

from workloads import make_c1, make_c4_batch, make_small

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2108_05345_amd import _lib
    lib = _lib.load()   # fails loudly if the HIP library is missing
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib


def _pool(insts):
    import paper_2108_05345_amd as lhdm
    d = torch.device("cuda:0")
    As = [torch.from_numpy(np.ascontiguousarray(i.A)).to(d) for i in insts]
    bs = [torch.from_numpy(i.b).to(d) for i in insts]
    return lhdm.pack(As, bs)


def _noalloc(lib, pool, use_lh=False):
    from paper_2108_05345_amd import _lib
    import paper_2108_05345_amd as lhdm
    d = pool.A.device
    B = len(pool.m)
    mm, nn, ao, bo, xo = pool.arrays()
    p = lhdm.default_params()
    x = torch.full((pool.nx,), -7.0, dtype=torch.float64, device=d)
    passive = torch.full((pool.nx,), -7, dtype=torch.int32, device=d)
    infos = torch.zeros(B * _lib.INFO_BYTES, dtype=torch.uint8, device=d)
    print(f"noalloc batch={B} use_lh={use_lh}", flush=True)
    rc = lib.lhdm_solve_batched_noalloc(torch.cuda.current_stream(d).cuda_stream, B, mm, nn, ao,
                                        pool.A.data_ptr(), bo, pool.b.data_ptr(), xo, x.data_ptr(),
                                        passive.data_ptr(), ctypes.byref(p), 1 if use_lh else 0,
                                        infos.data_ptr())
    assert rc == 0, rc
    return x, passive, lhdm._info_dicts(infos, B)


def _same(lib, insts, use_lh=False):
    import paper_2108_05345_amd as lhdm
    pool = _pool(insts)
    x0, p0, i0 = lhdm.solve_pooled(pool, use_lh=use_lh)
    x1, p1, i1 = _noalloc(lib, pool, use_lh)
    assert torch.equal(x0, x1)
    assert torch.equal(p0, p1)
    for a, b in zip(i0, i1):
        assert a == b
        assert a["status"] == 0
    return i1


def test_two_calls_in_a_row_second_smaller(lib):
    big = [make_c1(1000 + s) for s in range(300)] + [make_small(97, 301, 20, s, kind="uniform", noise_std=1e-2)
                                                      for s in range(40)]
    _same(lib, big)
    small = [make_c1(2000 + s) for s in range(17)]
    _same(lib, small)


def test_uneven_batch_and_plain_lh(lib):
    insts = make_c4_batch(4000, count=60)
    _same(lib, insts)
    _same(lib, insts[:9], use_lh=True)


def test_fewer_slots_than_instances(lib):
    # 2048 x 4096: one slot (Q and R of 32 MiB each) is beyond the 64 MiB
    # scratch -> rejected before any device work; 1024 x 1536 (~17 MB a slot)
    # fits three slots, so six instances go through three workgroups in turn
    from paper_2108_05345_amd import _lib
    insts = [make_small(1024, 1536, 60, s, kind="uniform", noise_std=1e-2) for s in range(6)]
    _same(lib, insts)
    big = [make_small(2048, 4096, 10, 0, kind="uniform", noise_std=1e-2)]
    pool = _pool(big)
    mm, nn, ao, bo, xo = pool.arrays()
    import paper_2108_05345_amd as lhdm
    p = lhdm.default_params()
    x = torch.empty(pool.nx, dtype=torch.float64, device=pool.A.device)
    rc = lib.lhdm_solve_batched_noalloc(None, 1, mm, nn, ao, pool.A.data_ptr(), bo, pool.b.data_ptr(), xo,
                                        x.data_ptr(), None, ctypes.byref(p), 0, None)
    assert rc == _lib.LHDM_EUNSUPPORTED
