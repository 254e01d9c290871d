/*
 * lhdm_testing.h -- test-only entry points of liblhdm.so.
 *
 * These calls expose single steps of the solvers so that tests can compare
 * them with a reference implementation on inputs that the whole solve rarely
 * produces.  They are not part of the solver API: they allocate and free their
 * own device memory, synchronise the stream and are not tuned for speed.
 * Conventions as in lhdm.h (float64, column-major, [dev] / [host] pointers,
 * negative LHDM_E* return codes on failure).
 */
#ifndef LHDM_TESTING_H
#define LHDM_TESTING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Algorithm 5 (Section 4.1, "Downdating"): delete the columns at the ascending
 * positions rm[0..q) from the triangular factor of a QR factorisation of nP
 * columns and restore the triangle with Givens rotations -- columns left to
 * right, each column's subdiagonal entries annihilated bottom-up, every
 * rotation acting on two adjacent rows -- applying the same rotations to Q^T b
 * and to the columns of the orthogonal factor, exactly as one inner iteration
 * of the solvers does.
 *   engine 1: the one-workgroup engine (one sweep over all q positions);
 *   engine 2: the whole-device engine (the solver's inner-step kernels, in
 *             sweeps of at most 64 positions, the rest carried to the next
 *             sweep as in the solver).
 *   Q  [dev] m x m, column-major (ld m): the orthogonal factor.
 *   R  [dev] nP x nP, column-major (ld nP): upper triangular factor (entries
 *      below the diagonal are ignored).
 *   bt [dev] m: Q^T b.
 *   rm [host] q strictly ascending positions in [0, nP), 1 <= q <= nP.
 *   Q_out [dev] m x m, R_out [dev] (nP-q) x (nP-q) (ld nP-q, zeros below the
 *   diagonal), bt_out [dev] m: the downdated factors.
 *   P_out [host, may be NULL] nP-q: the kept positions, in their new order.
 *   sweeps [host, may be NULL]: downdating sweeps run.
 * Returns LHDM_EINVAL on bad sizes, pointers or positions, LHDM_EUNSUPPORTED
 * for nP > m or, with engine 1, m > 2048. */
int lhdm_test_downdate(void* stream, int32_t engine, int32_t m, int32_t nP, const double* Q,
                       const double* R, const double* bt, int32_t q, const int32_t* rm,
                       double* Q_out, double* R_out, double* bt_out, int32_t* P_out,
                       int32_t* sweeps);

/* The least-squares step of Algorithms 1 and 3: the back substitution R y =
 * bt of the whole-device engine, exactly as the solver runs it (64-row blocks
 * chained across workgroups from the bottom; a full block far enough up the
 * chain is solved through the inverse of its row-scaled diagonal block, formed
 * while it waits, the others by substitution).
 *   R  [dev] n x n, column-major (ld n), upper triangular with a nonzero
 *      diagonal (entries below the diagonal are ignored).
 *   bt [dev] n: the right-hand side.
 *   y  [dev] n: the solution.
 *   inv_blocks [host, may be NULL]: how many blocks are eligible for the
 *      inverse form (one whose inverse has a non-finite entry falls back to
 *      substitution).
 * 1 <= n <= 8192.  Returns LHDM_EINVAL on bad sizes or pointers,
 * LHDM_EUNSUPPORTED for n > 8192, LHDM_EHIP when a block's wait timed out. */
int lhdm_test_trsv(void* stream, int32_t n, const double* R, const double* bt, double* y,
                   int32_t* inv_blocks);

/* The small factorisations of the whole-device engine's CholeskyQR2 panel
 * (Householder reconstruction from an orthonormal basis), each run by one wave
 * as in the solver:
 *   G [dev] n x n, column-major (ld n), symmetric positive definite (upper
 *     triangle read): R [dev] n x n upper (R^T R = G) and Ri [dev] n x n = R^{-1};
 *     sin2 [host]: the smallest R[t][t]^2 / G[t][t], or -1 when a pivot is not a
 *     positive finite number.
 *   W [dev] n x n, column-major: LU without pivoting of W - S = L U with S =
 *     diag(sg), sg[t] = +1 when step t's pivot is negative and -1 otherwise,
 *     by row elimination (U [dev] n x n upper, Li [dev] n x n = L^{-1}, unit
 *     lower, sg [dev] n) and, on a second wave at the same time, by column
 *     elimination (L [dev] n x n unit lower, Ui [dev] n x n = U^{-1}, sg2 [dev]
 *     n), as the solver runs both.
 * 1 <= n <= 32.  Returns LHDM_EINVAL on bad sizes or pointers. */
int lhdm_test_cq_factors(void* stream, int32_t n, const double* G, const double* W, double* R, double* Ri,
                         double* U, double* Li, double* L, double* Ui, double* sg, double* sg2,
                         double* sin2);

#ifdef __cplusplus
}
#endif

#endif /* LHDM_TESTING_H */
