"""MI355X (gfx950) nonnegative least squares: Lawson-Hanson and Lawson-Hanson with
Deviation Maximization (Dessole, Dell'Orto, Marcuzzi, arXiv 2108.05345).

Thin PyTorch binding over the C ABI of ``liblhdm.so`` (``include/lhdm.h``):
argument checking and marshalling only -- every step of the solve runs in the
library's HIP kernels.  Tensors must be float64 on the current ROCm device; the
call is enqueued on torch's current stream and returns after the result is
written.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import torch

from . import _lib
from ._lib import (LhdmError, LhdmInfo, LhdmParams, STATUS_MAXITER, STATUS_NONFINITE, STATUS_OK,  # noqa: F401
                   STATUS_RANK)

__all__ = [
    "solve", "lh_solve", "solve_signed", "solve_l1", "solve_batched", "solve_pooled", "backward_pooled", "LHDMFunction",
    "default_params", "Result", "pack", "LhdmError",
]


def default_params(**overrides) -> LhdmParams:
    p = LhdmParams()
    _lib.load().lhdm_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if v is None:
            continue
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


@dataclass
class Result:
    x: torch.Tensor            # (n,) float64
    w: torch.Tensor            # (n,) float64, dual A^T (b - A x)
    passive: torch.Tensor      # (n,) int32, P in insertion order, -1 padded
    info: dict


def _check_dev_tensor(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device.type != "cuda":
        raise TypeError(f"{name} must be a float64 tensor on a ROCm device")


def _colmajor(A: torch.Tensor) -> Tuple[torch.Tensor, int]:
    """Column-major view (or copy) of an (m, n) tensor and its leading dimension."""
    if A.dim() != 2:
        raise ValueError("A must be 2-D (m, n)")
    m = A.shape[0]
    if A.stride(0) == 1 and A.stride(1) >= max(1, m):
        return A, A.stride(1)
    return A.t().contiguous().t(), m


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class _Workspace:
    def __init__(self, nbytes: int, device):
        self.buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
        self.ptr = (self.buf.data_ptr() + 255) & ~255
        self.nbytes = int(nbytes)


def _info_dicts(buf: torch.Tensor, count: int) -> List[dict]:
    raw = bytes(buf.cpu().numpy().tobytes())
    out = []
    for i in range(count):
        inf = LhdmInfo.from_buffer_copy(raw[i * _lib.INFO_BYTES:(i + 1) * _lib.INFO_BYTES])
        out.append({f: getattr(inf, f) for f, _ in LhdmInfo._fields_})
    return out


def _single(A, b, method: str, params: LhdmParams) -> Result:
    _check_dev_tensor(A, "A")
    _check_dev_tensor(b, "b")
    Acm, lda = _colmajor(A)
    m, n = A.shape
    b = b.reshape(-1).contiguous()
    if b.numel() != m:
        raise ValueError("b must have m entries")
    dev = A.device
    lib = _lib.load()
    x = torch.empty(n, dtype=torch.float64, device=dev)
    w = torch.empty(n, dtype=torch.float64, device=dev)
    passive = torch.empty(n, dtype=torch.int32, device=dev)
    info = torch.empty(_lib.INFO_BYTES, dtype=torch.uint8, device=dev)
    ws = _Workspace(lib.lhdm_workspace_bytes(m, n, ctypes.byref(params)), dev)
    with torch.cuda.device(dev):
        s = _stream(dev)
        if method == "lhdm":
            rc = lib.lhdm_solve(s, m, n, Acm.data_ptr(), lda, b.data_ptr(), ctypes.byref(params), x.data_ptr(),
                                w.data_ptr(), passive.data_ptr(), info.data_ptr(), ws.ptr, ws.nbytes)
        else:
            rc = lib.lh_solve(s, m, n, Acm.data_ptr(), lda, b.data_ptr(), params.kkt_tol, params.max_outer,
                              x.data_ptr(), w.data_ptr(), passive.data_ptr(), info.data_ptr(), ws.ptr, ws.nbytes)
    _lib.check(rc)
    return Result(x, w, passive, _info_dicts(info, 1)[0])


ENGINES = {"auto": 0, "workgroup": 1, "device": 2}


FLAG_NO_JLOOP = 4
FLAG_PANEL_HOUSEHOLDER = 64


def solve(A: torch.Tensor, b: torch.Tensor, *, tau1=0.6, tau2=0.15, delta=0.9, kmax=32, kkt_tol=1e-9,
          max_outer=0, max_inner=0, engine="auto", no_jloop=False, panel="auto") -> Result:
    """LHDM solve of min ||A x - b|| s.t. x >= 0 (Algorithm 3 with Algorithm 2).

    ``engine``: "auto", "workgroup" (one workgroup per instance, m <= 2048) or
    "device" (one instance over the whole GPU).  ``no_jloop``: the variant of
    Theorem 4 without the feasibility loop on J (needs tau1 = 1, tau2 <= 1/2).
    ``panel`` (whole-device engine): "auto" factors blocks of 2 to 32 columns by
    CholeskyQR2 with rebuilt reflectors, "householder" every block column by
    column (Algorithm 4's steps)."""
    if panel not in ("auto", "householder"):
        raise ValueError(f"panel must be 'auto' or 'householder', not {panel!r}")
    flags = ENGINES[engine] | (FLAG_NO_JLOOP if no_jloop else 0)
    flags |= FLAG_PANEL_HOUSEHOLDER if panel == "householder" else 0
    p = default_params(tau1=tau1, tau2=tau2, delta=delta, kmax=kmax, kkt_tol=kkt_tol, max_outer=max_outer,
                       max_inner=max_inner, flags=flags)
    return _single(A, b, "lhdm", p)


@dataclass
class SignedResult:
    x: torch.Tensor            # (n,) float64, signed solution x+ - x-
    z: torch.Tensor            # (2n,) float64, (x+, x-)
    passive: torch.Tensor      # (2n,) int32, P over the columns of [A, -A], -1 padded
    info: dict


def solve_signed(A: torch.Tensor, b: torch.Tensor, *, sign_flip=True, tau1=0.6, tau2=0.15, delta=0.9, kmax=32,
                 kkt_tol=1e-9, max_outer=0, max_inner=0, engine="auto") -> SignedResult:
    """Signed least squares by the positivity trick (Section 3.2): NNLS on [A, -A]
    (never formed) by LHDM, or LH with ``kmax=1``; ``sign_flip`` selects the
    inner loop of Section 4.2."""
    _check_dev_tensor(A, "A")
    _check_dev_tensor(b, "b")
    Acm, lda = _colmajor(A)
    m, n = A.shape
    b = b.reshape(-1).contiguous()
    if b.numel() != m:
        raise ValueError("b must have m entries")
    dev = A.device
    lib = _lib.load()
    p = default_params(tau1=tau1, tau2=tau2, delta=delta, kmax=kmax, kkt_tol=kkt_tol, max_outer=max_outer,
                       max_inner=max_inner, flags=ENGINES[engine])
    x = torch.empty(n, dtype=torch.float64, device=dev)
    z = torch.empty(2 * n, dtype=torch.float64, device=dev)
    passive = torch.empty(2 * n, dtype=torch.int32, device=dev)
    info = torch.empty(_lib.INFO_BYTES, dtype=torch.uint8, device=dev)
    ws = _Workspace(lib.lhdm_signed_workspace_bytes(m, n, ctypes.byref(p)), dev)
    with torch.cuda.device(dev):
        rc = lib.lhdm_solve_signed(_stream(dev), m, n, Acm.data_ptr(), lda, b.data_ptr(), ctypes.byref(p),
                                   1 if sign_flip else 0, x.data_ptr(), z.data_ptr(), passive.data_ptr(),
                                   info.data_ptr(), ws.ptr, ws.nbytes)
    _lib.check(rc)
    return SignedResult(x, z, passive, _info_dicts(info, 1)[0])


def solve_l1(A: torch.Tensor, b: torch.Tensor, lam: float, *, tau1=0.6, tau2=0.15, delta=0.9, kmax=32,
             kkt_tol=1e-9, max_outer=0, max_inner=0, engine="auto") -> SignedResult:
    """l1-NNLS (Section 3.3): min ||x||_1^2 + lam^2 ||A x - b||^2 through the NNLS
    problem on [1^T, 1^T; lam A, -lam A], [0; lam b], solved by LHDM (LH with
    ``kmax=1``)."""
    _check_dev_tensor(A, "A")
    _check_dev_tensor(b, "b")
    Acm, lda = _colmajor(A)
    m, n = A.shape
    b = b.reshape(-1).contiguous()
    if b.numel() != m:
        raise ValueError("b must have m entries")
    dev = A.device
    lib = _lib.load()
    p = default_params(tau1=tau1, tau2=tau2, delta=delta, kmax=kmax, kkt_tol=kkt_tol, max_outer=max_outer,
                       max_inner=max_inner, flags=ENGINES[engine])
    x = torch.empty(n, dtype=torch.float64, device=dev)
    z = torch.empty(2 * n, dtype=torch.float64, device=dev)
    passive = torch.empty(2 * n, dtype=torch.int32, device=dev)
    info = torch.empty(_lib.INFO_BYTES, dtype=torch.uint8, device=dev)
    ws = _Workspace(lib.lhdm_l1_workspace_bytes(m, n, ctypes.byref(p)), dev)
    with torch.cuda.device(dev):
        rc = lib.lhdm_solve_l1(_stream(dev), m, n, Acm.data_ptr(), lda, b.data_ptr(), float(lam), ctypes.byref(p),
                               x.data_ptr(), z.data_ptr(), passive.data_ptr(), info.data_ptr(), ws.ptr, ws.nbytes)
    _lib.check(rc)
    return SignedResult(x, z, passive, _info_dicts(info, 1)[0])


def lh_solve(A: torch.Tensor, b: torch.Tensor, *, kkt_tol=1e-9, max_outer=0) -> Result:
    """Plain Lawson-Hanson solve (Algorithm 1)."""
    p = default_params(kkt_tol=kkt_tol, max_outer=max_outer, kmax=1)
    return _single(A, b, "lh", p)


# ---------------------------------------------------------------------------
# pooled (batched) interface
# ---------------------------------------------------------------------------
@dataclass
class Pool:
    m: List[int]
    n: List[int]
    a_off: List[int]
    b_off: List[int]
    x_off: List[int]
    A: torch.Tensor     # flat float64: column-major A_i at a_off[i]
    b: torch.Tensor     # flat float64
    nx: int             # total x entries

    def arrays(self):
        B = len(self.m)
        return ((ctypes.c_int32 * B)(*self.m), (ctypes.c_int32 * B)(*self.n), (ctypes.c_int64 * B)(*self.a_off),
                (ctypes.c_int64 * B)(*self.b_off), (ctypes.c_int64 * B)(*self.x_off))


def pack(As: Sequence[torch.Tensor], bs: Sequence[torch.Tensor]) -> Pool:
    """Pack (m_i x n_i) matrices (column-major) and right-hand sides into flat pools."""
    if len(As) != len(bs) or not As:
        raise ValueError("need matching non-empty lists")
    m, n, ao, bo, xo = [], [], [], [], []
    a = bb = xx = 0
    for A, b in zip(As, bs):
        _check_dev_tensor(A, "A")
        _check_dev_tensor(b, "b")
        mi, ni = A.shape
        m.append(mi)
        n.append(ni)
        ao.append(a)
        bo.append(bb)
        xo.append(xx)
        a += mi * ni
        bb += mi
        xx += ni
    Apool = torch.cat([A.t().contiguous().reshape(-1) for A in As])
    bpool = torch.cat([b.reshape(-1) for b in bs]).contiguous()
    return Pool(m, n, ao, bo, xo, Apool, bpool, xx)


BATCH_ENGINES = {"auto": 0, "fused": 8, "fused2": 16, "phased": 32}


def solve_pooled(pool: Pool, *, use_lh=False, tau1=0.6, tau2=0.15, delta=0.9, kmax=32, kkt_tol=1e-9,
                 max_outer=0, max_inner=0, engine="auto"):
    """Batched solve over a packed pool; returns (x_pool, passive_pool, infos).

    ``engine``: "auto" (the library's tuning table), "fused", "fused2" or
    "phased" (LHDM_FLAG_BATCH_* in lhdm.h)."""
    lib = _lib.load()
    dev = pool.A.device
    if engine not in BATCH_ENGINES:
        raise ValueError(f"engine must be one of {sorted(BATCH_ENGINES)}")
    p = default_params(tau1=tau1, tau2=tau2, delta=delta, kmax=kmax, kkt_tol=kkt_tol, max_outer=max_outer,
                       max_inner=max_inner)
    p.flags |= BATCH_ENGINES[engine]
    B = len(pool.m)
    mm, nn, ao, bo, xo = pool.arrays()
    x = torch.empty(pool.nx, dtype=torch.float64, device=dev)
    passive = torch.empty(pool.nx, dtype=torch.int32, device=dev)
    infos = torch.empty(B * _lib.INFO_BYTES, dtype=torch.uint8, device=dev)
    ws = _Workspace(lib.lhdm_batched_workspace_bytes(B, mm, nn, ctypes.byref(p)), dev)
    with torch.cuda.device(dev):
        rc = lib.lhdm_solve_batched(_stream(dev), B, mm, nn, ao, pool.A.data_ptr(), bo, pool.b.data_ptr(), xo,
                                    x.data_ptr(), passive.data_ptr(), ctypes.byref(p), 1 if use_lh else 0,
                                    infos.data_ptr(), ws.ptr, ws.nbytes)
    _lib.check(rc)
    return x, passive, _info_dicts(infos, B)


def solve_batched(As, bs, **kw) -> List[Result]:
    pool = pack(As, bs)
    x, passive, infos = solve_pooled(pool, **kw)
    out = []
    for i in range(len(pool.m)):
        o, ni = pool.x_off[i], pool.n[i]
        out.append(Result(x[o:o + ni], torch.empty(0), passive[o:o + ni], infos[i]))
    return out


def backward_pooled(pool: Pool, x: torch.Tensor, passive: torch.Tensor, grad_x: torch.Tensor):
    """Adjoint through the final passive sets: returns (grad_A_pool, grad_b_pool)."""
    lib = _lib.load()
    dev = pool.A.device
    B = len(pool.m)
    mm, nn, ao, bo, xo = pool.arrays()
    for t, nm in ((x, "x"), (grad_x, "grad_x")):
        _check_dev_tensor(t, nm)
    gA = torch.empty_like(pool.A)
    gb = torch.empty_like(pool.b)
    ws = _Workspace(lib.lhdm_backward_workspace_bytes(B, mm, nn), dev)
    x = x.contiguous()
    grad_x = grad_x.contiguous()
    passive = passive.to(torch.int32).contiguous()
    with torch.cuda.device(dev):
        rc = lib.lhdm_backward(_stream(dev), B, mm, nn, ao, pool.A.data_ptr(), bo, pool.b.data_ptr(), xo,
                               x.data_ptr(), passive.data_ptr(), grad_x.data_ptr(), gA.data_ptr(), gb.data_ptr(),
                               ws.ptr, ws.nbytes)
    _lib.check(rc)
    return gA, gb


class LHDMFunction(torch.autograd.Function):
    """x = argmin_{x >= 0} ||A x - b||, differentiable through the final passive set.

    ``LHDMFunction.apply(A, b)`` for one (m, n) instance; ``A`` and ``b`` are
    float64 device tensors.  Solver parameters take their defaults.  The forward
    runs the one-workgroup engine and the backward one workgroup per instance, so
    both need m <= 2048 (the backward min(m, n) <= 2048): larger instances raise
    ``LhdmError`` (LHDM_EUNSUPPORTED)."""

    @staticmethod
    def forward(ctx, A, b):
        pool = pack([A.detach()], [b.detach()])
        x, passive, infos = solve_pooled(pool)
        ctx.save_for_backward(x, passive)
        ctx.pool = pool
        ctx.shape = A.shape
        ctx.mark_non_differentiable(passive)
        return x, passive

    @staticmethod
    def backward(ctx, grad_x, grad_passive=None):
        x, passive = ctx.saved_tensors
        if grad_x is None:
            return None, None
        gA, gb = backward_pooled(ctx.pool, x, passive, grad_x.to(torch.float64).contiguous())
        m, n = ctx.shape
        return gA.reshape(n, m).t(), gb.reshape(m)
