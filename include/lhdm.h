/*
 * lhdm.h -- C ABI of the MI355X (gfx950) nonnegative least-squares library.
 *
 * Problem (Section 2, problem (NNLS)): given a dense A (m x n) and b (m),
 *     minimise ||A x - b||_2  subject to  x >= 0.
 * Solvers: Lawson-Hanson (Algorithm 1, `lh_solve`) and Lawson-Hanson with
 * Deviation Maximization (Algorithm 3 with the column selection of Algorithm 2,
 * `lhdm_solve`, `lhdm_solve_batched`), both returning the primal x, the dual
 * w = A^T (b - A x) and the ordered passive set P (Theorem 1, KKT conditions).
 * `lhdm_backward` differentiates x*(A, b) through the final passive set.
 *
 * Conventions shared by every entry point
 *   - All matrices are float64, column-major, with leading dimension lda >= m.
 *   - Pointers marked [dev] are device pointers on the current HIP device,
 *     pointers marked [host] are host pointers.  The caller owns every buffer it
 *     passes; the library never frees caller memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All device work is
 *     enqueued on it.  Every entry point returns after its results are written
 *     (it synchronises `stream`).
 *   - Workspace: `ws` [dev] of at least the size returned by the matching
 *     *_workspace_bytes query, aligned to 256 bytes.  If ws is NULL the library
 *     allocates a workspace itself and keeps it cached per device until
 *     lhdm_release() is called.  A workspace (the caller's or the cached one)
 *     serves one call at a time: calls that overlap in time (from several host
 *     threads, or on several streams) must use distinct workspaces, and the
 *     cached workspace must then not be used by more than one of them.
 *   - Return value: 0 on success, a negative LHDM_E* code if the call itself
 *     failed (nothing was solved; outputs are unspecified).  The per-instance
 *     outcome is reported in lhdm_info.status (LHDM_STATUS_*).
 *   - No exception crosses this interface.
 */
#ifndef LHDM_H
#define LHDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* call-level errors (negative return values) */
#define LHDM_EINVAL     (-1)   /* bad size, pointer or parameter */
#define LHDM_EWORKSPACE (-2)   /* workspace too small or misaligned */
#define LHDM_EHIP       (-3)   /* a HIP runtime call failed; see lhdm_last_hip_error() */
#define LHDM_EUNSUPPORTED (-4) /* size beyond what this build supports */

/* per-instance outcome (lhdm_info.status) */
#define LHDM_STATUS_OK        0  /* KKT conditions hold at kkt_tol */
#define LHDM_STATUS_MAXITER   1  /* iteration limit reached; x is the last feasible iterate */
#define LHDM_STATUS_NONFINITE 2  /* A or b holds a NaN or Inf; x = 0 */
#define LHDM_STATUS_RANK      3  /* no numerically independent column with positive dual left */

/* lhdm_params.flags: engine selection (default 0 = automatic). */
#define LHDM_FLAG_ENGINE_WORKGROUP 1  /* one workgroup per instance (m <= 2048) */
#define LHDM_FLAG_ENGINE_DEVICE    2  /* one instance over the whole GPU */
/* Theorem 4 (Section 3): with tau1 = 1 and tau2 <= 1/2 (and the selection's
 * delta <= tau2 / (kmax - 1) of Theorem 2, which makes the block's Gram matrix
 * diagonally dominant) the least-squares components of every accepted block J
 * are positive, so the feasibility loop on J is not evaluated (the block is
 * taken whole).  Requires tau1 == 1, tau2 <= 0.5 and delta <= tau2 / (kmax - 1),
 * else LHDM_EINVAL.  A violation by rounding (excluded in exact
 * arithmetic) is left to the inner loop, where a zero iterate entry with a
 * nonpositive least-squares component gives the step length 0. */
#define LHDM_FLAG_NO_JLOOP         4
/* Batched solves (lhdm_solve_batched and lhdm_batched_workspace_bytes, which
   must be given the same flags): the engine.  Without any of these the library
   takes it from its tuning table (written by the package's autotuner from
   timings on the target GPU) by instances per compute unit and largest m.
     FUSED:  one persistent kernel runs whole solves, one workgroup per compute
             unit, instances taken largest first from a device queue;
     FUSED2: the same kernel compiled for two workgroups per compute unit;
     PHASED: one kernel launch per stage of the outer step (append, inner loop,
             accept) over every unfinished instance, the rounds replayed as a
             HIP graph; every instance's state stays in the workspace, which is
             therefore the sum of the instances' own sizes.
   All three take the same steps in the same order: results are identical. */
#define LHDM_FLAG_BATCH_FUSED      8
#define LHDM_FLAG_BATCH_FUSED2     16
#define LHDM_FLAG_BATCH_PHASED     32
/* Whole-device engine: factor every appended block column by column
   (Algorithm 4's Householder steps, one cross-workgroup exchange per column)
   instead of by default, for blocks of 2 to 32 columns, through CholeskyQR2 on
   the block's Gram matrix with the Householder reflectors rebuilt from the
   orthonormal factor.  Both produce the R, reflectors and compact-WY factor of
   Algorithm 4 (up to rounding); the default falls back to the column-by-column
   factorisation by itself when the block's Gram matrix is poorly conditioned. */
#define LHDM_FLAG_PANEL_HOUSEHOLDER 64

/* Solver parameters [host].  tau1, tau2, delta and kmax are the thresholds of
 * Algorithm 2 (delta is the tau_c of the Algorithm 3 signature); the defaults are
 * the values used throughout the paper's experiments (Section 5): tau1 = 0.6,
 * tau2 = 0.15, delta = 0.9, kmax = 32.  kkt_tol scales the outer-loop stopping
 * test: stop when max_{j in Z} w_j <= kkt_tol * max_j ||a_j||_2 * ||b||_2.
 * max_outer / max_inner <= 0 select 3n (per instance in lhdm_solve_batched).  flags: LHDM_FLAG_* (0 = automatic engine:
 * the one-workgroup engine for m <= 2048 and m*n <= 2^18, the whole-device
 * engine otherwise; lhdm_solve_batched always uses the one-workgroup engine). */
typedef struct lhdm_params {
    double  tau1;
    double  tau2;
    double  delta;
    double  kkt_tol;
    int32_t kmax;        /* 1 <= kmax <= 64 */
    int32_t max_outer;
    int32_t max_inner;
    int32_t flags;
} lhdm_params;

/* Per-instance result, written to device memory [dev]. */
typedef struct lhdm_info {
    int32_t status;        /* LHDM_STATUS_* */
    int32_t outer_iters;   /* accepted outer steps */
    int32_t inner_iters;   /* inner (feasibility) iterations */
    int32_t jloop_drops;   /* columns dropped by the feasibility loop on J */
    int32_t n_passive;     /* |P| at exit */
    int32_t cq_panels;     /* whole-device engine: appended blocks factored by CholeskyQR2
                              (the rest column by column); 0 on the one-workgroup engine */
    double  kkt_residual;  /* max(max_Z w+, max_P |w|) / (max_j ||a_j|| ||b||) */
    double  objective;     /* ||b - A x||^2 */
} lhdm_info;

/* Fill p with the defaults above (kkt_tol = 1e-9). */
void lhdm_default_params(lhdm_params* p);

/* Bytes of workspace needed by lhdm_solve / lh_solve for an m x n instance. */
size_t lhdm_workspace_bytes(int32_t m, int32_t n, const lhdm_params* p);

/* LHDM solve of one instance (Algorithm 3; selection by Algorithm 2; block
 * append by the Householder updating of Algorithm 4 in compact-WY form; removal
 * by the Givens downdating of Algorithm 5).
 *   A [dev] m x n, lda >= m;  b [dev] m.
 *   x [dev] n (out): the solution, exactly 0 outside P.
 *   w [dev] n (out, may be NULL): the dual A^T (b - A x) at exit.
 *   passive [dev] n (out, may be NULL): P in insertion order, padded with -1.
 *   info [dev] (out, may be NULL).
 * Returns LHDM_EINVAL for m < 1, n < 1, lda < m, NULL A/b/x, tau1 or tau2
 * outside (0, 1], delta outside (0, 1], kmax outside [1, 64]. */
int lhdm_solve(void* stream, int32_t m, int32_t n, const double* A, int64_t lda,
               const double* b, const lhdm_params* p, double* x, double* w,
               int32_t* passive, lhdm_info* info, void* ws, size_t ws_bytes);

/* Signed least squares by the positivity trick (Section 3.2, problem
 * (positivity trick)): min ||[A, -A] z - b||_2 s.t. z >= 0 with z = (x+, x-),
 * solved by LHDM (or LH with kmax = 1) on the 2n columns of [A, -A] without
 * forming -A: column j >= n is the caller's column j - n negated, and its dual
 * is -w_{j-n}, so each outer step still reads A once.
 *   sign_flip != 0: the inner loop of the positivity-trick case (Section 4.2):
 *     each passive column whose least-squares component is negative is
 *     replaced, at the same position, by its twin, which negates that column
 *     of R and the component, leaves the residual unchanged and ends the inner
 *     loop without a downdate; an exactly zero component takes the ordinary
 *     inner iteration.  sign_flip == 0: the ordinary inner loop (step length
 *     and Givens downdating) on [A, -A].
 *   x [dev] n (out): the signed solution x+ - x-.
 *   z [dev] 2n (out, may be NULL): (x+, x-).
 *   passive [dev] 2n (out, may be NULL): P over the 2n columns, insertion
 *     order, -1 padded.
 *   info: as lhdm_solve (outer, inner iterations over the 2n-column problem;
 *     a sign flip counts as one inner iteration).
 * Other arguments, workspace and errors as lhdm_solve (workspace size from
 * lhdm_signed_workspace_bytes). */
size_t lhdm_signed_workspace_bytes(int32_t m, int32_t n, const lhdm_params* p);
int lhdm_solve_signed(void* stream, int32_t m, int32_t n, const double* A, int64_t lda,
                      const double* b, const lhdm_params* p, int32_t sign_flip, double* x,
                      double* z, int32_t* passive, lhdm_info* info, void* ws, size_t ws_bytes);

/* l1-NNLS (Section 3.3, problem (l1-NNLS)): the squared-l1 regularised least
 * squares min ||x||_1^2 + lambda^2 ||A x - b||_2^2 in its NNLS form
 *     min || [1^T, 1^T; lambda A, -lambda A] z - [0; lambda b] ||_2,  z >= 0,
 * x = z[:n] - z[n:].  The (m + 1) x 2n matrix and the right-hand side are
 * assembled in the workspace (8 (m + 1) 2n bytes) and solved by LHDM, or LH
 * with kmax = 1.  lambda > 0 and finite, else LHDM_EINVAL.
 *   x [dev] n (out): the signed solution.
 *   z [dev] 2n (out, may be NULL);  passive [dev] 2n (out, may be NULL).
 * Other arguments, workspace (lhdm_l1_workspace_bytes) and errors as
 * lhdm_solve; the engine is chosen for the (m + 1) x 2n problem. */
size_t lhdm_l1_workspace_bytes(int32_t m, int32_t n, const lhdm_params* p);
int lhdm_solve_l1(void* stream, int32_t m, int32_t n, const double* A, int64_t lda,
                  const double* b, double lambda, const lhdm_params* p, double* x, double* z,
                  int32_t* passive, lhdm_info* info, void* ws, size_t ws_bytes);

/* Plain Lawson-Hanson (Algorithm 1): one column per outer step with a rank-one
 * Householder append.  Same arguments and outputs as lhdm_solve. */
int lh_solve(void* stream, int32_t m, int32_t n, const double* A, int64_t lda,
             const double* b, double kkt_tol, int32_t max_outer, double* x,
             double* w, int32_t* passive, lhdm_info* info, void* ws, size_t ws_bytes);

/* Bytes of workspace for lhdm_solve_batched over `batch` instances with the
 * given sizes (m, n are [host] arrays of length batch). */
size_t lhdm_batched_workspace_bytes(int32_t batch, const int32_t* m, const int32_t* n,
                                    const lhdm_params* p);

/* Many independent instances of uneven size in one persistent launch: one
 * workgroup solves one instance at a time, instances are taken largest-first
 * from a device work queue.
 *   m, n, a_off, b_off, x_off: [host] arrays of length batch.  Instance i reads
 *   A_pool + a_off[i] (column-major, lda = m[i]) and b_pool + b_off[i], and writes
 *   x_pool + x_off[i] (n[i] values) and passive_pool + x_off[i] (n[i] values,
 *   may be NULL).  use_lh = 1 runs plain LH instead of LHDM.
 *   infos [dev] batch entries (may be NULL). */
int lhdm_solve_batched(void* stream, int32_t batch, const int32_t* m, const int32_t* n,
                       const int64_t* a_off, const double* A_pool,
                       const int64_t* b_off, const double* b_pool,
                       const int64_t* x_off, double* x_pool, int32_t* passive_pool,
                       const lhdm_params* p, int32_t use_lh, lhdm_info* infos,
                       void* ws, size_t ws_bytes);

/* Size of the fixed device scratch of lhdm_solve_batched_noalloc (per device). */
#define LHDM_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the batched
 * solve of lhdm_solve_batched without a workspace argument and without any
 * allocation.  Arguments and results as in lhdm_solve_batched.  Every buffer
 * beyond the caller's inputs and outputs lives in a fixed scratch array of
 * LHDM_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on
 * until the process ends.  The scratch keeps the bookkeeping of the batch
 * (about 90 bytes per instance) and as many instance slots as fit (a slot is
 * the state of one instance of the largest m and n: about 8 (m^2 + min(m,n)^2
 * + 4 m kmax) bytes plus a few vectors of length m and n), so fewer instances
 * may be in flight at once than
 * with lhdm_solve_batched; instances are taken in the given order (no
 * largest-first reordering).  Returns LHDM_EUNSUPPORTED, before any device
 * work, when the bookkeeping plus one slot exceeds the scratch, and for m > 2048.
 * All calls on one device share its scratch and every call overwrites it (what
 * must start at zero is cleared by the call itself): calls that overlap in time
 * on one device race, so serialise them (one host thread, one stream). */
int lhdm_solve_batched_noalloc(void* stream, int32_t batch, const int32_t* m, const int32_t* n,
                               const int64_t* a_off, const double* A_pool,
                               const int64_t* b_off, const double* b_pool,
                               const int64_t* x_off, double* x_pool, int32_t* passive_pool,
                               const lhdm_params* p, int32_t use_lh, lhdm_info* infos);

/* Bytes of workspace for lhdm_backward. */
size_t lhdm_backward_workspace_bytes(int32_t batch, const int32_t* m, const int32_t* n);

/* Derivative of x*(A, b) through the final passive set (not in the paper: the
 * least-squares map x_P = argmin ||A_P y - b|| of Section 2.1 at the returned P,
 * with x_Z = 0, differentiated exactly).  For upstream gradient g = dL/dx:
 *   lambda = (A_P^T A_P)^{-1} g_P          (via a Householder QR of A_P)
 *   grad_b = A_P lambda
 *   grad_A[:, P] = r lambda^T - (A_P lambda) x_P^T,  r = b - A_P x_P
 *   grad_A[:, Z] = 0.
 * Layout as in lhdm_solve_batched: [host] size/offset arrays, [dev] pools.
 * passive_pool holds each instance's P (as returned by the forward call, -1
 * padded); grad_A_pool is fully overwritten (lda = m[i]); grad_b_pool gets m[i]
 * values at b_off[i].  Each instance is handled by one workgroup, which keeps
 * its QR in the workspace and its multipliers in LDS: a batch holding an
 * instance with min(m, n) > 2048 returns LHDM_EUNSUPPORTED (nothing is
 * written). */
int lhdm_backward(void* stream, int32_t batch, const int32_t* m, const int32_t* n,
                  const int64_t* a_off, const double* A_pool,
                  const int64_t* b_off, const double* b_pool,
                  const int64_t* x_off, const double* x_pool, const int32_t* passive_pool,
                  const double* grad_x_pool, double* grad_A_pool, double* grad_b_pool,
                  void* ws, size_t ws_bytes);

/* Timing of the dominant kernel: the dual w = A^T r fused with the projected-
 * norm update in the whole-device engine (lg_dual_ws for up to 32 update
 * directions, lg_colmat2 for 33 to 48, lg_colmat_dot when A is not 16-byte
 * aligned).  When enabled, every launch of it records a start and a stop event
 * on the solve's stream (the launch records them itself where it can); the
 * elapsed times are collected at the library's own stream synchronisations.
 * lhdm_profile_enable(1) resets the counters.  lhdm_profile_read reports the
 * summed kernel time [ms], the number of launches and the algorithmic bytes
 * those launches move (8 m n for A plus the vectors read and written). */
void lhdm_profile_enable(int on);
int lhdm_profile_read(double* total_ms, int64_t* launches, double* bytes);

/* Text for a status or error code. */
const char* lhdm_status_string(int code);

/* The last hipError_t seen by a call that returned LHDM_EHIP (0 if none). */
int lhdm_last_hip_error(void);

/* Free workspaces the library allocated itself (ws == NULL calls). */
void lhdm_release(void);

#ifdef __cplusplus
}
#endif

#endif /* LHDM_H */
