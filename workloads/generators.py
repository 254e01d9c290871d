"""Seeded generators for the synthetic NNLS workloads.

Every instance is drawn with ``numpy.random.Generator(PCG64(seed))`` in a fixed
order: the matrix ``A``, the support ``S`` of the planted solution, its values,
the measurement noise, and (differentiation workload only) the target ``t``.
``A`` is returned column-major (Fortran order), which is the layout the device
library reads; ``b = A @ x_true + noise`` is formed once here so that the oracle
and the HIP path see identical bytes.

The paper's experiments use a third-party matrix database that is not available
here and whose instance sizes the paper does not state; these synthetic
families stand in for it (planted sparse nonnegative solutions of dense
Gaussian and uniform matrices, the setting of the paper's sparse-recovery
experiments).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Instance:
    name: str
    seed: object
    A: np.ndarray            # (m, n) float64, Fortran order
    b: np.ndarray            # (m,) float64
    x_true: np.ndarray       # (n,) float64, planted nonnegative solution
    support: np.ndarray      # sorted indices of the planted nonzeros
    t: Optional[np.ndarray] = None   # differentiation target (n,)
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.SeedSequence):
        return np.random.Generator(np.random.PCG64(seed))
    return np.random.Generator(np.random.PCG64(int(seed)))


def _planted(rng, A, k, draw_vals, noise_std, name, seed, meta=None):
    m, n = A.shape
    S = np.sort(rng.choice(n, size=k, replace=False))
    x = np.zeros(n)
    x[S] = draw_vals(rng, k)
    b = A @ x
    if noise_std > 0.0:
        b = b + noise_std * rng.standard_normal(m)
    return Instance(name=name, seed=seed, A=np.asfortranarray(A), b=np.ascontiguousarray(b),
                    x_true=x, support=S, meta=dict(meta or {}))


def make_gaussian_planted(m, n, k, seed, *, vals=(1.0, 2.0), noise_std=0.0,
                          unit_columns=False, name="gauss"):
    """A ~ N(0, 1/m) i.i.d.; x_true k-sparse with U[vals] entries; b = A x + noise."""
    rng = _rng(seed)
    A = rng.standard_normal((m, n)) / np.sqrt(m)
    if unit_columns:
        A = A / np.linalg.norm(A, axis=0, keepdims=True)
    lo, hi = vals
    return _planted(rng, A, k, lambda r, kk: r.uniform(lo, hi, kk), noise_std, name, seed,
                    {"m": m, "n": n, "k": k, "noise_std": noise_std})


def make_small(m, n, k, seed, *, kind="gauss", noise_std=0.0, vals=(1.0, 2.0)):
    """Small generic instance for tests: Gaussian N(0,1/m) or uniform U[0,1] entries."""
    rng = _rng(seed)
    if kind == "gauss":
        A = rng.standard_normal((m, n)) / np.sqrt(m)
    elif kind == "uniform":
        A = rng.uniform(0.0, 1.0, (m, n))
    else:
        raise ValueError(kind)
    lo, hi = vals
    return _planted(rng, A, k, lambda r, kk: r.uniform(lo, hi, kk), noise_std,
                    f"small-{kind}", seed, {"m": m, "n": n, "k": k, "noise_std": noise_std})


def make_c1(seed: int = 1000) -> Instance:
    """m=64, n=128, A ~ N(0,1/m), 8-sparse planted x with U[1,2] values, b = A x."""
    return make_gaussian_planted(64, 128, 8, seed, vals=(1.0, 2.0), name="c1-gauss-64x128")


def make_c2(seed: int = 2000) -> Instance:
    """m=1024, n=4096, unit-norm Gaussian columns, 128-sparse U[0.5,1.5], noiseless."""
    return make_gaussian_planted(1024, 4096, 128, seed, vals=(0.5, 1.5), unit_columns=True,
                                 name="c2-gauss-unitcol-1024x4096")


def make_c3(seed: int = 3000, m: int = 4096, n: int = 16384, k: int = 820) -> Instance:
    """m=4096, n=16384, A ~ N(0,1/m), 820-sparse |N(0,1)|+0.1 values, noise std 1e-3.

    ``m``, ``n`` and ``k`` may be scaled down (keeping k/n) for oracle-sized tests.
    """
    rng = _rng(seed)
    A = rng.standard_normal((m, n)) / np.sqrt(m)
    return _planted(rng, A, k, lambda r, kk: np.abs(r.standard_normal(kk)) + 0.1, 1e-3,
                    f"c3-gauss-{m}x{n}", seed, {"m": m, "n": n, "k": k, "noise_std": 1e-3})


def _c4_from_child(child, i, seed, m_lo, m_hi):
    rng = _rng(child)
    m = int(rng.integers(m_lo, m_hi + 1))
    n = int(round(m * rng.uniform(2.0, 4.0)))
    A = rng.uniform(0.0, 1.0, (m, n))
    k = int(round(0.1 * n))
    return _planted(rng, A, k, lambda r, kk: r.uniform(0.0, 1.0, kk), 1e-2,
                    f"c4-uniform-{i}", (seed, i), {"m": m, "n": n, "k": k})


def make_c4_batch(seed: int = 4000, count: int = 2000, m_lo: int = 32, m_hi: int = 512):
    """Uneven batch: m ~ U{m_lo..m_hi}, n = round(m U[2,4]), A ~ U[0,1], 10%-dense U[0,1]
    nonnegative x, noise std 1e-2.  Child seeds come from SeedSequence(seed).spawn(count)."""
    return [_c4_from_child(child, i, seed, m_lo, m_hi)
            for i, child in enumerate(np.random.SeedSequence(seed).spawn(count))]


def make_c4_instance(i: int, seed: int = 4000, count: int = 2000, m_lo: int = 32, m_hi: int = 512):
    """Instance i of make_c4_batch(seed, count, m_lo, m_hi), generated alone."""
    child = np.random.SeedSequence(seed).spawn(count)[i]
    return _c4_from_child(child, i, seed, m_lo, m_hi)


def make_c5_batch(seed: int = 5000, count: int = 256, m: int = 256, n: int = 512):
    """Differentiation batch: m=256, n=512, A ~ N(0,1/m), 32-sparse U[1,2], noise 1e-3,
    target t ~ N(0,1)^n for the loss ||x*(A,b) - t||^2."""
    out = []
    for i, child in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = _rng(child)
        A = rng.standard_normal((m, n)) / np.sqrt(m)
        inst = _planted(rng, A, 32, lambda r, kk: r.uniform(1.0, 2.0, kk), 1e-3,
                        f"c5-gauss-{i}", (seed, i), {"m": m, "n": n, "k": 32})
        inst.t = rng.standard_normal(n)
        out.append(inst)
    return out


def make_illcond(m, n, k, row_range, seed, *, vals=(1.0, 2.0), noise_std=0.0, name="illcond"):
    """A = diag(d) U with U ~ U[0, 1]^(m x n) and row scales d log-spaced from 1
    down to 1 / row_range; x_true k-sparse with U[vals] entries; b = A x + noise.

    Row scaling leaves the set {x >= 0 : A x = b} unchanged (it is the set of
    the unscaled system), so a sparse planted solution of the nonnegative
    matrix U stays the unique one, while the condition number of A grows to
    about 10 * row_range (1e4 -> ~5e5, 1e5 -> ~5e6).  Stands in for the
    moderately ill-conditioned matrices (condition number 1e5 to 1e6) of the
    paper's experiments, whose dataset is not available here."""
    rng = _rng(seed)
    U = rng.uniform(0.0, 1.0, (m, n))
    d = np.logspace(0.0, -np.log10(row_range), m)
    A = d[:, None] * U
    lo, hi = vals
    return _planted(rng, A, k, lambda r, kk: r.uniform(lo, hi, kk), noise_std, name, seed,
                    {"m": m, "n": n, "k": k, "row_range": row_range, "noise_std": noise_std})


def make_signed(m, n, k, seed, *, noise_std=0.0, name="signed"):
    """Signed sparse recovery (the positivity-trick problem): A ~ N(0, 1/m),
    x_true k-sparse with random signs and magnitudes U[1, 2]; b = A x + noise.
    ``x_true`` is signed here (the nonnegative variable of the trick is
    (x+, x-))."""
    rng = _rng(seed)
    A = rng.standard_normal((m, n)) / np.sqrt(m)
    S = np.sort(rng.choice(n, size=k, replace=False))
    x = np.zeros(n)
    x[S] = rng.uniform(1.0, 2.0, k) * rng.choice([-1.0, 1.0], size=k)
    b = A @ x
    if noise_std > 0.0:
        b = b + noise_std * rng.standard_normal(m)
    return Instance(name=name, seed=seed, A=np.asfortranarray(A), b=np.ascontiguousarray(b), x_true=x,
                    support=S, meta={"m": m, "n": n, "k": k, "noise_std": noise_std})


CONFIGS = {
    "c1": make_c1,
    "c2": make_c2,
    "c3": make_c3,
    "c4": make_c4_batch,
    "c5": make_c5_batch,
}
