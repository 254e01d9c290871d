"""CPU oracle for the LH / LHDM nonnegative least-squares solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (``paper_2108_05345_amd``); the only module both sides read is the input
generator package ``workloads``.

Plain, slow, float64 numpy.  Every function cites the passage of the paper
(Dessole, Dell'Orto, Marcuzzi, "The Lawson-Hanson Algorithm with Deviation
Maximization: Finite Convergence and Sparse Recovery", arXiv 2108.05345) it
follows.
"""
from .nnls import (  # noqa: F401
    DEFAULTS,
    STATUS_OK,
    STATUS_MAXITER,
    STATUS_NONFINITE,
    STATUS_RANK,
    DEP_TOL,
    house,
    givens,
    oracle_lh,
    oracle_lhdm,
    oracle_signed,
    oracle_l1nnls,
    l1nnls_matrix,
    dm_select_reference,
    downdate_rotations,
    kkt_report,
    brute_force_nnls,
    nnls_grad_reference,
    kkt_tolerance,
)
