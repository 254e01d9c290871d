// Shared device-side definitions of the gfx950 LH / LHDM library.
//
// Problem: min ||A x - b||_2 s.t. x >= 0 (Section 2).  State kept on the device
// for one instance (the design differs from the paper's Matlab code: see the
// per-field comments):
//   Q   m x m, column-major: the full orthogonal factor, kept explicitly.  Its
//       first n_P columns span range(A_P); blocked Householder appends update it
//       by compact-WY products and Givens removals rotate pairs of its columns.
//   R   n_P x n_P upper triangular, column-major, leading dimension kc = min(m,n);
//       logical column c (the passive column P[c]) lives in physical column
//       slot[c], so removals never move data; rows are positional.
//   bt  Q^T b (m entries).
//   u2  squared norms of the projections of the columns of A onto range(A_P)^perp
//       (the vector u of Algorithm 3, squared), maintained incrementally.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lhdm.h"

namespace lhdm {

constexpr int WG = 256;              // threads per workgroup in every kernel
constexpr int NW = WG / 64;          // waves per workgroup
constexpr int KM = 64;               // largest supported kmax
constexpr double DEP_TOL = 1e-12;    // projected norm <= DEP_TOL ||a_j||: numerically dependent
constexpr double RECOMP_FRAC = 1e-4; // u2 below this fraction of ||a_j||^2: recompute exactly
constexpr int YMAX = 2048;           // largest min(m, n) of the workgroup engine
constexpr int MMAX_WG = 2048;        // largest m of the workgroup engine
constexpr int DVL = 64;              // vectors per row of the workgroup engine's vector block

struct DevParams {
    double tau1, tau2, delta, kkt_tol;
    int kmax, max_outer, max_inner, lh;
    int nojloop;   // feasibility loop on J not evaluated (Theorem 4 regime)
    int twin;      // positivity trick: the matrix is [A, -A], -A never formed
    int signflip;  // inner loop by the sign flip of the positivity-trick case
    int panel_hh;  // whole-device engine: every panel column by column (no CholeskyQR2)
};

// One instance: caller buffers plus its workspace slice.
struct Prob {
    const double* A;
    long long lda;
    const double* b;
    double* x;
    double* w;
    int* passive;      // may be null
    lhdm_info* info;   // may be null
    int m, n, kc, kq;  // kc = min(m, n); kq = columns of the panel buffers (>= 2)
    int nph;           // columns of the caller's A: n, or n / 2 for the positivity trick
                       // (column j >= nph is the negated caller column j - nph)
    double* Q;         // m * m
    double* R;         // kc * kc
    double* bt;        // m
    double* r;         // m
    double* u2;        // n
    double* an2;       // n
    double* G;         // m * kq : projected candidates / Householder panel
    double* V;         // m * kq : explicit Householder vectors (zeros above the unit diagonal)
    double* W;         // m * kq : WY scratch
    double* Qadd;      // m * kq : the columns of Q appended in this outer step
    double* T;         // kq * kq : compact-WY factor, also the Gram matrix of the candidates
    double* rot;       // 2 * kc  : rotations of one column of the downdate
    int* P;            // kc : ordered passive set
    int* pos;          // n  : position in P, or -1
    int* excl;         // n  : excluded for the current outer step
    int* rm;           // kc : removal positions of an inner iteration
    int* slot;         // kc : physical column of R holding logical column c (a permutation;
                       //      slots [n_P, kc) are the free ones)
    double* ybuf;      // kc : least-squares solution by position (large-instance engine)
    double* Vt;        // m * kq : V stored row-major (large-instance engine)
    int* itmp;         // 2 * kc : scratch of the passive-set compaction
    double* Dv;        // m * DVL, row-major: vector block of the workgroup engine's products
};

// Bytes of one instance's workspace slice (each array padded to 256 bytes).
__host__ __device__ inline size_t pad256(size_t b) { return (b + 255) & ~size_t(255); }

__host__ __device__ inline int panel_cols(int kmax) { return kmax < 2 ? 2 : kmax; }

__host__ __device__ inline size_t slot_bytes(int m, int n, int kmax) {
    const size_t kc = (size_t)(m < n ? m : n);
    const size_t kq = (size_t)panel_cols(kmax);
    size_t s = 0;
    s += pad256(sizeof(double) * (size_t)m * m);       // Q
    s += pad256(sizeof(double) * kc * kc);             // R
    s += 2 * pad256(sizeof(double) * (size_t)m);       // bt, r
    s += 2 * pad256(sizeof(double) * (size_t)n);       // u2, an2
    s += 4 * pad256(sizeof(double) * (size_t)m * kq);  // G, V, W, Qadd
    s += pad256(sizeof(double) * kq * kq);             // T
    s += pad256(sizeof(double) * 2 * kc);              // rot
    s += 3 * pad256(sizeof(int) * kc);                 // P, rm, slot
    s += pad256(sizeof(int) * 2 * kc);                 // itmp
    s += 2 * pad256(sizeof(int) * (size_t)n);          // pos, excl
    s += pad256(sizeof(double) * (size_t)m * DVL);     // Dv
    return s;
}

__host__ __device__ inline void carve_slot(Prob& p, char* base, int m, int n, int kmax) {
    const size_t kc = (size_t)(m < n ? m : n);
    const size_t kq = (size_t)panel_cols(kmax);
    p.m = m;
    p.n = n;
    p.kc = (int)kc;
    p.kq = (int)kq;
    char* c = base;
    auto take = [&](size_t bytes) { char* r = c; c += pad256(bytes); return r; };
    p.Q = (double*)take(sizeof(double) * (size_t)m * m);
    p.R = (double*)take(sizeof(double) * kc * kc);
    p.bt = (double*)take(sizeof(double) * m);
    p.r = (double*)take(sizeof(double) * m);
    p.u2 = (double*)take(sizeof(double) * n);
    p.an2 = (double*)take(sizeof(double) * n);
    p.G = (double*)take(sizeof(double) * (size_t)m * kq);
    p.V = (double*)take(sizeof(double) * (size_t)m * kq);
    p.W = (double*)take(sizeof(double) * (size_t)m * kq);
    p.Qadd = (double*)take(sizeof(double) * (size_t)m * kq);
    p.T = (double*)take(sizeof(double) * kq * kq);
    p.rot = (double*)take(sizeof(double) * 2 * kc);
    p.P = (int*)take(sizeof(int) * kc);
    p.rm = (int*)take(sizeof(int) * kc);
    p.slot = (int*)take(sizeof(int) * kc);
    p.itmp = (int*)take(sizeof(int) * 2 * kc);
    p.pos = (int*)take(sizeof(int) * n);
    p.excl = (int*)take(sizeof(int) * n);
    p.Dv = (double*)take(sizeof(double) * (size_t)m * DVL);
    p.ybuf = nullptr;
    p.Vt = nullptr;
    p.nph = n;
}

// Global-memory view of a buffer.  Loads and stores through it are global_*
// instructions: the compiler tracks their completion one by one (a flat
// instruction may also address LDS, so flat loads are waited for all at once)
// and knows they cannot alias private copies of the instance descriptor, so
// the hot loops hoist those fields and keep many loads in flight.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* x) {
    return (__attribute__((address_space(1))) T*)x;
}

// The instance's buffers as global-memory views (see gmem).
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) int gint;
struct GProb {
    const gdouble* A;
    const gdouble* b;
    gdouble *x, *w, *Q, *R, *bt, *r, *u2, *an2, *G, *V, *W, *Qadd, *T, *rot, *Dv;
    gint *passive, *P, *pos, *excl, *rm, *slot, *itmp;
};

__device__ inline GProb gview(const Prob& p) {
    GProb g;
    g.A = gmem(p.A);
    g.b = gmem(p.b);
    g.x = gmem(p.x);
    g.w = gmem(p.w);
    g.Q = gmem(p.Q);
    g.R = gmem(p.R);
    g.bt = gmem(p.bt);
    g.r = gmem(p.r);
    g.u2 = gmem(p.u2);
    g.an2 = gmem(p.an2);
    g.G = gmem(p.G);
    g.V = gmem(p.V);
    g.W = gmem(p.W);
    g.Qadd = gmem(p.Qadd);
    g.T = gmem(p.T);
    g.rot = gmem(p.rot);
    g.Dv = gmem(p.Dv);
    g.passive = gmem(p.passive);
    g.P = gmem(p.P);
    g.pos = gmem(p.pos);
    g.excl = gmem(p.excl);
    g.rm = gmem(p.rm);
    g.slot = gmem(p.slot);
    g.itmp = gmem(p.itmp);
    return g;
}

// Column j of the instance's matrix: the caller's column j or, in the
// positivity-trick mode (n = 2 nph, Section 3.2), the caller's column j - nph
// negated (sign -1) for j >= nph.
__host__ __device__ inline const double* col_ptr(const Prob& p, int j, double& sign) {
    if (j >= p.nph) {
        sign = -1.0;
        return p.A + (size_t)(j - p.nph) * p.lda;
    }
    sign = 1.0;
    return p.A + (size_t)j * p.lda;
}

// The twin of column j in the positivity-trick mode (its negation).
__host__ __device__ inline int twin_of(const Prob& p, int j) { return j >= p.nph ? j - p.nph : j + p.nph; }

// A column whose twin is passive lies in range(A_P): its projected norm is 0
// in exact arithmetic, so it is not eligible (positivity-trick mode only).
__device__ __forceinline__ bool twin_passive(const Prob& p, int j) {
    return p.n != p.nph && p.pos[twin_of(p, j)] >= 0;
}

// ---------------------------------------------------------------------------
// wave / workgroup reductions (fixed association order: results are identical
// in every lane and reproducible run to run)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return __shfl(v, 0, 64);
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    return __shfl(v, 0, 64);
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_down(v, o, 64));
    return __shfl(v, 0, 64);
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return __shfl(v, 0, 64);
}

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_down(v, o, 64));
    return __shfl(v, 0, 64);
}

// larger value first, lower index on ties
__device__ __forceinline__ bool better(double va, int ia, double vb, int ib) {
    return va > vb || (va == vb && ia < ib);
}

__device__ __forceinline__ void wave_argmax(double& v, int& i) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_down(v, o, 64);
        const int oi = __shfl_down(i, o, 64);
        if (better(ov, oi, v, i)) {
            v = ov;
            i = oi;
        }
    }
    v = __shfl(v, 0, 64);
    i = __shfl(i, 0, 64);
}

// Index of this thread's wave in the workgroup, as a scalar: the compiler then
// treats conditions on it as uniform (scalar branches, no exec masking).
__device__ __forceinline__ int wave_index() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Orders this wave's LDS accesses at a point where its lanes exchange data
// through LDS (emits no instruction: the LDS operations of one wave complete
// in order; this only keeps the compiler from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Value of lane `l` (wave-uniform, normally a compile-time constant) of a
// double, through the scalar unit rather than the LDS crossbar.
__device__ __forceinline__ double readlane_d(double v, int l) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)bits, l);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Step-length ratio x_i / (x_i - y_i) of an inner iteration for a passive
// entry with y_i <= 0; an entry whose iterate is exactly 0 gives 0 (it can only
// arise in the variant without the feasibility loop on J).
__device__ __forceinline__ double step_ratio(double xc, double yc) {
    return (xc == 0.0) ? 0.0 : xc / (xc - yc);
}

// Rotation G = [[c, s], [-s, c]] with G [a, b]^T = [r, 0]^T (Algorithm 5's givens).
__device__ __forceinline__ void givens(double a, double b, double& c, double& s, double& r) {
    if (b == 0.0) {
        c = 1.0;
        s = 0.0;
        r = a;
        return;
    }
    r = hypot(a, b);
    c = a / r;
    s = b / r;
}

// The same rotation with one reciprocal square root instead of a scaled
// hypot and two divisions (a few ulp from the correctly rounded c, s, r), for
// the latency-bound chain of the downdate; inputs whose squares could leave
// the normal range take the scaled path.
__device__ __forceinline__ void givens_fast(double a, double b, double& c, double& s, double& r) {
    const double mx = fmax(fabs(a), fabs(b));
    if (b != 0.0 && mx > 0x1p-480 && mx < 0x1p480) {
        const double q = fma(a, a, b * b);
        const double y = rsqrt(q);
        c = a * y;
        s = b * y;
        r = q * y;
        return;
    }
    givens(a, b, c, s, r);
}

}  // namespace lhdm
