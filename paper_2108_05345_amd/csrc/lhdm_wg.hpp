// Workgroup engine: one workgroup of WG threads runs a whole LH / LHDM solve of
// one instance (Algorithms 1 and 3).  Every control decision is made from LDS
// values after a barrier, so control flow is uniform across the workgroup.
//
// The same step functions serve the batched persistent kernel (one instance per
// workgroup at a time) and the small single-instance path.
#pragma once

#include <climits>

#include "lhdm_device.hpp"

namespace lhdm {

// Control state of one solve.  The workgroup engine keeps it in LDS for the
// whole solve; the large-instance engine keeps it in global memory between
// launches and copies it into LDS inside each single-workgroup kernel.
// Stages of an outer step (Wg::stage_*).
enum { ST_APPEND = 0, ST_INNER = 1, ST_ACCEPT = 2, ST_DONE = 3 };

struct Ctl {
    double tol_w, anmax, bnorm;
    int nP, nP0, nPa, status, outer, inner, jdrops, ncol, k, kr, done, q, any_excl, j1, stage;
    int J[KM];
    double tau[KM];          // Householder scalars of the panel
    double beta[KM];         // diagonal of the new R block
};

struct WgShared : Ctl {
    double rd[NW];
    int ri[NW];
    double mr[KM + 1][NW];   // per-wave partial sums of a vector of dot products
    double vec[KM + 1];      // reduced vector of dot products
    double y[YMAX];          // least-squares solution by passive position
    double c[YMAX];          // right-hand side being reduced by the triangular solve
    int cnt[WG];             // prefix counts for compaction
};

typedef double wd4 __attribute__((ext_vector_type(4)));
typedef double wd2 __attribute__((ext_vector_type(2)));

// LDS work area of the phases that stage tiles (triangular solve, downdate,
// matrix-core products); the phases are separated by barriers, so one area
// serves them all.  It is reached only through LDS-typed pointers (ds_*
// instructions).  The control block WgShared, which the step functions reach
// through a generic reference (flat instructions), must lie in the first
// 64 KiB of the workgroup's LDS: flat accesses above that offset are not
// routed to LDS.  Kernels therefore declare both in one WgLds, the control
// block first.
typedef __attribute__((address_space(3))) double lds_double;
typedef __attribute__((address_space(3))) int lds_int;
constexpr int WG_TS = 64;                          // triangular-solve block
constexpr int WG_DB = 64;                          // downdate window
constexpr int WG_LX = WG_TS * (WG_TS + 1) + YMAX / 2;
static_assert(WG_LX >= NW * 16 * 65, "colmat tile staging");
static_assert(WG_LX >= (WG_DB + 1) * WG_DB + 2 * WG_DB, "downdate window and its rotations");
static_assert(WG_LX >= WG_TS * (WG_TS + 1) + YMAX / 2, "triangular-solve block and slot indices");
static_assert(WG_LX >= NW * KM * 17, "Q-update tiles");
struct WgLds {
    WgShared sh;
    double x[WG_LX];
    int sidx;
};
static_assert(sizeof(WgShared) <= 65536, "flat accesses to the control block stay below 64 KiB");

struct Wg {
    static constexpr int LB = 8;   // gathered loads issued together per thread
    Prob& p;
    const DevParams& prm;
    __attribute__((address_space(3))) WgShared& s;   // LDS: ds_* instructions
    int tid, lane, wid;
    double* yv;   // least-squares solution by position: LDS (workgroup engine) or global
    lds_double* lx;   // LDS work area of trsv, downdate and colmat (WG_LX doubles)
    GProb gp;         // the instance's buffers as global-memory views

    __device__ Wg(Prob& p_, const DevParams& prm_, WgShared& s_, lds_double* x_ = nullptr)
        : p(p_), prm(prm_), s(*(__attribute__((address_space(3))) WgShared*)&s_), tid(threadIdx.x), lane(threadIdx.x & 63), wid(wave_index()),
          yv(p_.ybuf ? p_.ybuf : s_.y), lx(x_), gp(gview(p_)) {}

    // ---------------- workgroup reductions ----------------
    __device__ __forceinline__ double sum(double v) {
        v = wave_sum(v);
        __syncthreads();
        if (lane == 0) s.rd[wid] = v;
        __syncthreads();
        double t = s.rd[0];
#pragma unroll
        for (int i = 1; i < NW; ++i) t += s.rd[i];
        return t;
    }
    __device__ __forceinline__ double vmax(double v) {
        v = wave_max(v);
        __syncthreads();
        if (lane == 0) s.rd[wid] = v;
        __syncthreads();
        double t = s.rd[0];
#pragma unroll
        for (int i = 1; i < NW; ++i) t = fmax(t, s.rd[i]);
        return t;
    }
    __device__ __forceinline__ double vmin(double v) {
        v = wave_min(v);
        __syncthreads();
        if (lane == 0) s.rd[wid] = v;
        __syncthreads();
        double t = s.rd[0];
#pragma unroll
        for (int i = 1; i < NW; ++i) t = fmin(t, s.rd[i]);
        return t;
    }
    __device__ __forceinline__ int imax(int v) {
        v = wave_max_int(v);
        __syncthreads();
        if (lane == 0) s.ri[wid] = v;
        __syncthreads();
        int t = s.ri[0];
#pragma unroll
        for (int i = 1; i < NW; ++i) t = max(t, s.ri[i]);
        return t;
    }
    __device__ __forceinline__ void argmax(double& v, int& i) {
        wave_argmax(v, i);
        __syncthreads();
        if (lane == 0) {
            s.rd[wid] = v;
            s.ri[wid] = i;
        }
        __syncthreads();
        v = s.rd[0];
        i = s.ri[0];
#pragma unroll
        for (int w = 1; w < NW; ++w)
            if (better(s.rd[w], s.ri[w], v, i)) {
                v = s.rd[w];
                i = s.ri[w];
            }
    }
    // Per-thread partial of dot product t is written by the caller into
    // s.mr via push(); finish(cnt) leaves the sums in s.vec[0..cnt).
    __device__ __forceinline__ void push(int t, double part) {
        part = wave_sum(part);
        if (lane == 0) s.mr[t][wid] = part;
    }
    __device__ __forceinline__ void finish(int cnt) {
        __syncthreads();
        if (tid < cnt) {
            double a = s.mr[tid][0];
#pragma unroll
            for (int w = 1; w < NW; ++w) a += s.mr[tid][w];
            s.vec[tid] = a;
        }
        __syncthreads();
    }

    __device__ __forceinline__ gdouble& Qat(int i, int j) { return gp.Q[(size_t)j * p.m + i]; }
    __device__ __forceinline__ gdouble& Rat(int i, int j) { return gp.R[(size_t)gp.slot[j] * p.kc + i]; }
    __device__ __forceinline__ const gdouble* Acol(int j) { return gp.A + (size_t)j * p.lda; }
    // column j of the instance's matrix and its sign (as col_ptr)
    __device__ __forceinline__ const gdouble* gcol(int j, double& sign) {
        if (j >= p.nph) {
            sign = -1.0;
            return gp.A + (size_t)(j - p.nph) * p.lda;
        }
        sign = 1.0;
        return gp.A + (size_t)j * p.lda;
    }
    // twin of column j passive (positivity-trick mode only, as twin_passive)
    __device__ __forceinline__ bool gtwin_passive(int j) { return p.n != p.nph && gp.pos[twin_of(p, j)] >= 0; }

    // ---------------- a0: initialisation (Algorithm 3, first lines) ----------------
    __device__ __forceinline__ void init() {
        const int m = p.m, nph = p.nph;
        double anmax = 0.0;
        int bad = 0;
        for (int j = wid; j < nph; j += NW) {
            const gdouble* a = Acol(j);
            double ab = 0.0, aa = 0.0;
            for (int i = lane; i < m; i += 64) {
                const double v = a[i];
                ab += v * gp.b[i];
                aa += v * v;
            }
            ab = wave_sum(ab);
            aa = wave_sum(aa);
            if (lane == 0) {
                gp.w[j] = ab;          // w^(0) = A^T b
                gp.an2[j] = aa;
                gp.u2[j] = aa;         // u^(0) = column norms of A
                gp.pos[j] = -1;
                gp.excl[j] = 0;
                gp.x[j] = 0.0;
                if (nph != p.n) {     // the twin -a_j of the positivity trick
                    const int t = j + nph;
                    gp.w[t] = -ab;
                    gp.an2[t] = aa;
                    gp.u2[t] = aa;
                    gp.pos[t] = -1;
                    gp.excl[t] = 0;
                    gp.x[t] = 0.0;
                }
            }
            if (!isfinite(ab) || !isfinite(aa)) bad = 1;
            anmax = fmax(anmax, aa);
        }
        double bb = 0.0;
        for (int i = tid; i < m; i += WG) {
            const double v = gp.b[i];
            bb += v * v;
            gp.bt[i] = v;
            gp.r[i] = v;
        }
        bb = sum(bb);
        anmax = vmax(anmax);
        bad = imax(bad);
        const size_t mm = (size_t)m * m;
        for (size_t e = tid; e < mm; e += WG) gp.Q[e] = ((e % m) == (e / m)) ? 1.0 : 0.0;
        for (int c = tid; c < p.kc; c += WG) gp.slot[c] = c;
        if (tid == 0) {
            s.anmax = sqrt(anmax);
            s.bnorm = sqrt(bb);
            s.tol_w = prm.kkt_tol * s.anmax * s.bnorm;
            s.nP = 0;
            s.status = (bad || !isfinite(bb)) ? LHDM_STATUS_NONFINITE : LHDM_STATUS_OK;
            s.outer = s.inner = s.jdrops = 0;
            s.any_excl = 0;
            s.done = 0;
        }
        __syncthreads();
    }

    // ---------------- a1 + a2: termination test and Deviation Maximization ----------------
    // Leaves s.done = 1 to stop (status set), else s.J[0..s.ncol) = [j1, candidates...].
    __device__ __forceinline__ void select() {
        const int n = p.n;
        double mwz = -INFINITY, mu = 0.0, bv = -INFINITY;
        int bi = INT_MAX;
        for (int j = tid; j < n; j += WG) {
            if (gp.pos[j] >= 0) continue;
            const double wj = gp.w[j];
            const double u = sqrt(fmax(gp.u2[j], 0.0));
            mwz = fmax(mwz, wj);
            mu = fmax(mu, u);
            if (!gp.excl[j] && u > DEP_TOL * sqrt(gp.an2[j]) && !gtwin_passive(j) && better(wj, j, bv, bi)) {
                bv = wj;
                bi = j;
            }
        }
        mwz = vmax(mwz);
        mu = vmax(mu);
        argmax(bv, bi);
        const int cap = p.m - s.nP;
        __syncthreads();
        if (tid == 0) {
            s.done = 0;
            s.ncol = 1;
            s.J[0] = bi;
            if (mwz == -INFINITY || mwz <= s.tol_w) {
                s.done = 1;   // converged: Z empty or max_Z w <= tol
            } else if (bi == INT_MAX || bv <= s.tol_w) {
                s.done = 1;
                s.status = LHDM_STATUS_RANK;
            } else if (s.outer >= prm.max_outer) {
                s.done = 1;
                s.status = LHDM_STATUS_MAXITER;
            }
        }
        __syncthreads();
        if (s.done || prm.lh || prm.kmax <= 1 || cap <= 1) return;
        // candidates: w_i >= tau1 * max w, u_i >= tau2 * max u, ordered by (w desc, index asc)
        const double tw = prm.tau1 * bv, tu = prm.tau2 * mu;
        double pv = bv;
        int pi = bi;
        for (int t = 1; t < prm.kmax; ++t) {
            double cv = -INFINITY;
            int ci = INT_MAX;
            for (int j = tid; j < n; j += WG) {
                if (gp.pos[j] >= 0 || gp.excl[j] || j == bi) continue;
                const double wj = gp.w[j];
                if (!(wj >= tw)) continue;
                const double u = sqrt(fmax(gp.u2[j], 0.0));
                if (!(u >= tu) || !(u > DEP_TOL * sqrt(gp.an2[j])) || gtwin_passive(j)) continue;
                if (!(wj < pv || (wj == pv && j > pi))) continue;   // strictly after the previous pick
                if (better(wj, j, cv, ci)) {
                    cv = wj;
                    ci = j;
                }
            }
            argmax(cv, ci);
            if (ci == INT_MAX) break;
            if (tid == 0) {
                s.J[t] = ci;
                s.ncol = t + 1;
            }
            pv = cv;
            pi = ci;
        }
        __syncthreads();
    }

    // out(j, t) = X[:, j] . Dv[:, t] for j < ncols, t < nv <= 16 NT, on the FP64
    // matrix cores (v_mfma_f64_16x16x4f64).  X is column-major (ld ldx, rows
    // [0, m)); Dv is the slot's row-major vector block (ld DVL).  Each wave
    // takes 16-column tiles in turn and walks down them in 32-row steps: lane
    // (c, g) feeds column c of the tile with rows 8 g .. 8 g + 7 of the step
    // (16-byte loads where X allows them), the s-th product of a step taking
    // row 8 g + s.  A finished tile goes through LDS: lane c < 16 then calls
    // put(j0 + c, vals, nv) with vals[t] = out(j0 + c, t) (an LDS row).
    template <int NT, int TB, typename Put>
    __device__ __forceinline__ void colmat(const gdouble* X, long long ldx, int ncols, int nv, Put put) {
        lds_double(*ct)[16][16 * 4 + 1] = reinterpret_cast<lds_double(*)[16][16 * 4 + 1]>(lx);
        const int m = p.m;
        const gdouble* __restrict__ D = gp.Dv;
        const bool al16 = ((((uintptr_t)X) & 15) == 0) && ((ldx & 1) == 0);
        const int ntile = (ncols + 15) / 16, g = lane >> 4, cl = lane & 15;
        // TB tiles per wave at a time: they share the vector-block loads, and
        // their column loads are in flight together
        for (int tile = wid * TB; tile < ntile; tile += NW * TB) {
            const gdouble* xc[TB];
#pragma unroll
            for (int b = 0; b < TB; ++b) xc[b] = X + (size_t)min((tile + b) * 16 + cl, ncols - 1) * ldx;
            wd4 acc[TB][NT];
#pragma unroll
            for (int b = 0; b < TB; ++b)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[b][t] = wd4{0.0, 0.0, 0.0, 0.0};
            // product s = 2 h + e of a 32-row step takes row r0 + 8 h + 2 g + e for
            // K index g: the four lanes of a column read 64 contiguous bytes per
            // load (16-byte loads where X allows them)
            for (int r0 = 0; r0 < m; r0 += 32) {
                double av[TB][8];
                if (r0 + 32 <= m && al16) {
#pragma unroll
                    for (int b = 0; b < TB; ++b)
#pragma unroll
                        for (int h = 0; h < 4; ++h) {
                            const wd2 x = *reinterpret_cast<const __attribute__((address_space(1))) wd2*>(
                                xc[b] + r0 + 8 * h + 2 * g);
                            av[b][2 * h] = x[0];
                            av[b][2 * h + 1] = x[1];
                        }
                } else {
#pragma unroll
                    for (int b = 0; b < TB; ++b)
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int row = r0 + 8 * (u >> 1) + 2 * g + (u & 1);
                            const double x = xc[b][min(row, m - 1)];
                            av[b][u] = (row < m) ? x : 0.0;
                        }
                }
                double bv[NT][8];
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int row = r0 + 8 * (u >> 1) + 2 * g + (u & 1);
                        const double x = D[(size_t)min(row, m - 1) * DVL + 16 * t + cl];
                        bv[t][u] = (row < m) ? x : 0.0;
                    }
#pragma unroll
                for (int b = 0; b < TB; ++b)
#pragma unroll
                    for (int t = 0; t < NT; ++t)
#pragma unroll
                        for (int u = 0; u < 8; ++u)
                            acc[b][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[b][u], bv[t][u], acc[b][t], 0, 0, 0);
            }
#pragma unroll
            for (int b = 0; b < TB; ++b) {
                const int j0 = (tile + b) * 16;
                if (j0 >= ncols) break;
                // lane l, register v: column 4 v + l / 16 of the tile, vector 16 t + l % 16
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) ct[wid][4 * v + g][16 * t + cl] = acc[b][t][v];
                wave_lds_sync();
                if (lane < 16 && j0 + lane < ncols) put(j0 + lane, ct[wid][lane], nv);
                wave_lds_sync();
            }
        }
        __syncthreads();
    }

    template <typename Put>
    __device__ __forceinline__ void colmat_any(const gdouble* X, long long ldx, int ncols, int nv, Put put) {
        if (nv <= 16) colmat<1, 4>(X, ldx, ncols, nv, put);
        else if (nv <= 32) colmat<2, 2>(X, ldx, ncols, nv, put);
        else if (nv <= 48) colmat<3, 2>(X, ldx, ncols, nv, put);
        else colmat<4, 1>(X, ldx, ncols, nv, put);
    }

    // G[:, t] = Q^T a_{J[t]} for t < cnt (full projection: rows < n_P are Q_P^T a,
    // rows >= n_P the coordinates of the projected column in the trailing basis),
    // as one product of the columns of Q with the gathered candidate columns.
    __device__ __forceinline__ void project(int cnt) {
        const int m = p.m, nvp = (cnt + 15) & ~15;   // columns colmat reads
        // consecutive threads take consecutive rows of a column; eight loads in flight
        for (int e0 = tid; e0 < m * nvp; e0 += WG * LB) {
            double v[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int e = e0 + WG * u, t = e / m, i = e - t * m;
                v[u] = 0.0;
                if (e < m * nvp && t < cnt) {
                    double sg;
                    const gdouble* a = gcol(s.J[t], sg);
                    v[u] = sg * a[i];
                }
            }
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int e = e0 + WG * u, t = e / m, i = e - t * m;
                if (e < m * nvp) gp.Dv[(size_t)i * DVL + t] = v[u];
            }
        }
        __syncthreads();
        colmat_any(gp.Q, m, m, cnt, [&](int i, const lds_double* c, int nv) {
            for (int t = 0; t < nv; ++t) gp.G[(size_t)t * m + i] = c[t];
        });
    }

    // Gram matrix of the projected candidates G[n_P:m, 0:ncol] into T (ld kq).
    __device__ __forceinline__ void candidate_gram() {
        const int m = p.m, c = s.ncol, r0 = s.nP, kq = p.kq;
        const int npair = c * (c + 1) / 2;
        for (int pr = wid; pr < npair; pr += NW) {
            int a = 0, rem = pr;
            while (rem > a) {
                rem -= a + 1;
                ++a;
            }
            const int bcol = rem;   // pair (a, bcol), bcol <= a
            const gdouble* ga = gp.G + (size_t)a * m;
            const gdouble* gb = gp.G + (size_t)bcol * m;
            double acc = 0.0;
            for (int i = r0 + lane; i < m; i += 64) acc += ga[i] * gb[i];
            acc = wave_sum(acc);
            if (lane == 0) {
                gp.T[(size_t)a * kq + bcol] = acc;
                gp.T[(size_t)bcol * kq + a] = acc;
            }
        }
        __syncthreads();
    }

    // Cosines of the projected candidates (eq. of the cosine matrix) from the
    // Gram matrix in T, and the greedy acceptance of Algorithm 2.  Compacts G
    // to the accepted columns.
    __device__ __forceinline__ void greedy_from_gram() {
        const int m = p.m, c = s.ncol, kq = p.kq;
        if (tid == 0) {
            const int cap = p.m - s.nP;
            int acc[KM];
            int na = 1;
            acc[0] = 0;
            for (int t = 1; t < c; ++t) {
                if (na >= cap) break;
                const double nt = sqrt(gp.T[(size_t)t * kq + t]);
                bool ok = true;
                for (int q = 0; q < na; ++q) {
                    const int a = acc[q];
                    const double th = gp.T[(size_t)a * kq + t] / (nt * sqrt(gp.T[(size_t)a * kq + a]));
                    if (!(fabs(th) < prm.delta)) {
                        ok = false;
                        break;
                    }
                }
                if (ok) acc[na++] = t;
            }
            for (int q = 0; q < na; ++q) {
                s.vec[q] = (double)acc[q];
                s.J[q] = s.J[acc[q]];
            }
            s.k = na;
        }
        __syncthreads();
        // compact G columns (acc is increasing, so in-place forward copy is safe)
        const int k = s.k;
        for (int q = 1; q < k; ++q) {
            const int from = (int)s.vec[q];
            if (from != q)
                for (int i = tid; i < m; i += WG) gp.G[(size_t)q * m + i] = gp.G[(size_t)from * m + i];
            __syncthreads();
        }
    }

    __device__ __forceinline__ void deviation_maximization() {
        candidate_gram();
        greedy_from_gram();
    }

    // a3: Householder QR of the panel G[n_P:m, 0:k] with bt[n_P:m] carried as an
    // extra column (Algorithm 4); G keeps the reflectors below the diagonal,
    // s.beta the new diagonal of R, s.tau the reflector scalars.  Per column:
    // one pass for all dot products with the reflector, one pass for the update
    // that also accumulates the norm of the next column.
    __device__ __forceinline__ void panel_qr() {
        const int m = p.m, k = s.kr, r0 = s.nP;
        double part0 = 0.0;
        for (int i = r0 + tid; i < m; i += WG) part0 += gp.G[i] * gp.G[i];
        double nrm2 = sum(part0);
        for (int t = 0; t < k; ++t) {
            const int rt = r0 + t;
            gdouble* g = gp.G + (size_t)t * m;
            const double x0 = g[rt];
            const double normx = sqrt(nrm2);
            double tau = 0.0, beta = x0, scal = 0.0;
            if (normx > 0.0) {
                beta = (x0 >= 0.0) ? -normx : normx;
                tau = (beta - x0) / beta;
                scal = 1.0 / (x0 - beta);
            }
            __syncthreads();
            for (int i = rt + 1 + tid; i < m; i += WG) g[i] *= scal;
            if (tid == 0) {
                g[rt] = 1.0;
                s.tau[t] = tau;
                s.beta[t] = beta;
            }
            __syncthreads();
            // dot products of the reflector with columns t+1..k-1 and bt, 16 at a time
            const int nrest = k - t;
            for (int q0 = 0; q0 < nrest; q0 += 16) {
                double pd[16];
#pragma unroll
                for (int qq = 0; qq < 16; ++qq) pd[qq] = 0.0;
                for (int i = rt + tid; i < m; i += WG) {
                    const double vi = g[i];
#pragma unroll
                    for (int qq = 0; qq < 16; ++qq) {
                        const int q = q0 + qq;
                        if (q < nrest) {
                            const gdouble* col = (q < nrest - 1) ? gp.G + (size_t)(t + 1 + q) * m : gp.bt;
                            pd[qq] += vi * col[i];
                        }
                    }
                }
#pragma unroll
                for (int qq = 0; qq < 16; ++qq)
                    if (q0 + qq < nrest) push(q0 + qq, pd[qq]);
            }
            finish(nrest);
            // update, and the squared norm of column t+1 from row rt+1
            double nn = 0.0;
            for (int i = rt + tid; i < m; i += WG) {
                const double vi = g[i];
                for (int q = 0; q < nrest; ++q) {
                    gdouble* col = (q < nrest - 1) ? gp.G + (size_t)(t + 1 + q) * m : gp.bt;
                    const double nv = col[i] - (tau * s.vec[q]) * vi;
                    col[i] = nv;
                    if (q == 0 && i > rt && t + 1 < k) nn += nv * nv;
                }
            }
            if (t + 1 < k) nrm2 = sum(nn);
            else __syncthreads();
        }
    }

    // Explicit V (zeros above the unit diagonal, rows >= n_P).
    __device__ __forceinline__ void explicit_v() {
        const int m = p.m, k = s.kr, r0 = s.nP;
        for (int t = 0; t < k; ++t) {
            const gdouble* g = gp.G + (size_t)t * m;
            gdouble* v = gp.V + (size_t)t * m;
            for (int i = tid; i < m; i += WG) v[i] = (i < r0 + t) ? 0.0 : g[i];
        }
        __syncthreads();
    }

    // V^T V, strictly upper part, into W (k x k, column-major ld kq).
    __device__ __forceinline__ void vtv() {
        const int m = p.m, k = s.kr, r0 = s.nP, kq = p.kq;
        const int npair = k * (k - 1) / 2;
        for (int pr = wid; pr < npair; pr += NW) {
            int a = 1, rem = pr;
            while (rem >= a) {
                rem -= a;
                ++a;
            }
            const int b = rem;   // pair (b, a), b < a
            const gdouble* va = gp.V + (size_t)a * m;
            const gdouble* vb = gp.V + (size_t)b * m;
            double acc = 0.0;
            for (int i = r0 + a + lane; i < m; i += 64) acc += vb[i] * va[i];
            acc = wave_sum(acc);
            if (lane == 0) gp.W[(size_t)a * kq + b] = acc;
        }
        __syncthreads();
    }

    // Compact-WY factor T with H_0 H_1 ... H_{k-1} = I - V T V^T (forward,
    // columnwise) from s.tau and V^T V in W.
    __device__ __forceinline__ void form_t() {
        const int k = s.kr, kq = p.kq;
        if (tid == 0) {
            gdouble* T = gp.T;
            for (int t = 0; t < k; ++t) {
                T[(size_t)t * kq + t] = s.tau[t];
                double z[KM];
                for (int i = 0; i < t; ++i) z[i] = -s.tau[t] * gp.W[(size_t)t * kq + i];
                for (int i = 0; i < t; ++i) {
                    double acc = 0.0;
                    for (int l = i; l < t; ++l) acc += T[(size_t)l * kq + i] * z[l];
                    T[(size_t)t * kq + i] = acc;
                }
                for (int i = t + 1; i < k; ++i) T[(size_t)t * kq + i] = 0.0;
            }
        }
        __syncthreads();
    }

    __device__ __forceinline__ void form_wy() {
        explicit_v();
        vtv();
        form_t();
    }

    // New R columns: [Q_P^T a_J ; R_JJ].
    __device__ __forceinline__ void append_r() {
        const int m = p.m, k = s.kr, r0 = s.nP;
        for (int t = 0; t < k; ++t) {
            const gdouble* g = gp.G + (size_t)t * m;
            for (int i = tid; i < r0 + t + 1; i += WG) {
                double v;
                if (i < r0 + t) v = g[i];
                else v = s.beta[t];
                Rat(i, r0 + t) = v;
            }
        }
        __syncthreads();
    }

    // Q[:, n_P:m] <- Q[:, n_P:m] (I - V T V^T) on the FP64 matrix cores.  Rows
    // of Q are independent, so each wave owns 16-row tiles of Q in turn:
    //   W^T  = V^T Q_t^T   (k x 16, K = the trailing columns, 32 at a time),
    //   W2^T = T^T W^T     (T upper triangular),
    //   Q_t^T -= V W2^T    (16 trailing columns of Q per product, K = k),
    // with W^T and then W2^T in the wave's part of the LDS work area.
    template <int NT>
    __device__ __forceinline__ void update_q_tiles() {
        const int m = p.m, k = s.kr, r0 = s.nP, kq = p.kq;
        const int g = lane >> 4, cl = lane & 15;
        auto* __restrict__ Q = gmem(gp.Q);
        const auto* __restrict__ V = gmem(gp.V);
        const auto* __restrict__ T = gmem(gp.T);
        lds_double* wt = lx + wid * (KM * 17);   // [KM][17]: row t = column t of W (16 rows of Q)
        const int ntile = (m + 15) / 16;
        for (int tile = wid; tile < ntile; tile += NW) {
            const int i0 = tile * 16;
            const int ic = min(i0 + cl, m - 1);
            wd4 acc[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = wd4{0.0, 0.0, 0.0, 0.0};
            // W^T(t, i) = sum_l V(l, t) Q(i, l): lane (c, g) feeds V column 16 t + c and
            // Q row i0 + c; product s = 2 h + e of a 32-row step takes l = l0 + 8 h + 2 g + e
            // HS 32-row steps per trip, all their loads before their products
            constexpr int HS = NT <= 2 ? 2 : 1;
            for (int l0 = r0; l0 < m; l0 += 32 * HS) {
                double bq[HS][8], av[HS][NT][8];
#pragma unroll
                for (int h = 0; h < HS; ++h) {
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int l = l0 + 32 * h + 8 * (u >> 1) + 2 * g + (u & 1);
                        const double x = Q[(size_t)min(l, m - 1) * m + ic];
                        bq[h][u] = (l < m) ? x : 0.0;
                    }
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const int tc = 16 * t + cl;
                        const auto* vc = V + (size_t)min(tc, k - 1) * m;
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int l = l0 + 32 * h + 8 * (u >> 1) + 2 * g + (u & 1);
                            const double x = vc[min(l, m - 1)];
                            av[h][t][u] = (tc < k && l < m) ? x : 0.0;
                        }
                    }
                }
#pragma unroll
                for (int h = 0; h < HS; ++h)
#pragma unroll
                    for (int t = 0; t < NT; ++t)
#pragma unroll
                        for (int u = 0; u < 8; ++u)
                            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[h][t][u], bq[h][u], acc[t], 0, 0, 0);
            }
            // result lane l, register v: W^T(16 t + 4 v + l / 16, i0 + l % 16)
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) wt[(16 * t + 4 * v + g) * 17 + cl] = acc[t][v];
            wave_lds_sync();
            // W2^T(t', i) = sum_{t <= t'} T(t, t') W^T(t, i); all operands loaded first
            wd4 acc2[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) acc2[t] = wd4{0.0, 0.0, 0.0, 0.0};
            {
                double at[4 * NT][NT], bw[4 * NT];
#pragma unroll
                for (int ks = 0; ks < 4 * NT; ++ks) {
                    const int kk = 4 * ks + g;
                    const double wv = wt[min(kk, KM - 1) * 17 + cl];
                    bw[ks] = (kk < k) ? wv : 0.0;
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const int tc = 16 * t + cl;
                        const double tv = T[(size_t)min(tc, k - 1) * kq + min(kk, k - 1)];
                        at[ks][t] = (kk < k && tc < k) ? tv : 0.0;
                    }
                }
#pragma unroll
                for (int ks = 0; ks < 4 * NT; ++ks)
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        acc2[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(at[ks][t], bw[ks], acc2[t], 0, 0, 0);
            }
            wave_lds_sync();
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) wt[(16 * t + 4 * v + g) * 17 + cl] = acc2[t][v];
            wave_lds_sync();
            // Q(i, l) -= sum_t V(l, t) W2^T(t, i), HQ 16-column tiles of Q at a time,
            // every operand of a group loaded before its products
            double bw[4 * NT];
#pragma unroll
            for (int ks = 0; ks < 4 * NT; ++ks) {
                const int kk = 4 * ks + g;
                const double wv = wt[min(kk, KM - 1) * 17 + cl];
                bw[ks] = (kk < k) ? wv : 0.0;
            }
            constexpr int HQ = NT <= 2 ? 4 : 2;
            for (int l0 = r0; l0 < m; l0 += 16 * HQ) {
                wd4 d[HQ];
#pragma unroll
                for (int h = 0; h < HQ; ++h) d[h] = wd4{0.0, 0.0, 0.0, 0.0};
                // Q entries of the group first: lane l, register v of tile h holds
                // (Q column l0 + 16 h + 4 v + l / 16, row i0 + l % 16)
                double qv[HQ][4];
#pragma unroll
                for (int h = 0; h < HQ; ++h)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int l = l0 + 16 * h + 4 * v + g;
                        const double x = Q[(size_t)min(l, m - 1) * m + min(i0 + cl, m - 1)];
                        qv[h][v] = (l < m && i0 + cl < m) ? x : 0.0;
                    }
                double av[4 * NT][HQ];
#pragma unroll
                for (int ks = 0; ks < 4 * NT; ++ks) {
                    const int kk = 4 * ks + g;
                    const auto* vk = V + (size_t)min(kk, k - 1) * m;
#pragma unroll
                    for (int h = 0; h < HQ; ++h) {
                        const int lc = l0 + 16 * h + cl;
                        const double x = vk[min(lc, m - 1)];
                        av[ks][h] = (kk < k && lc < m) ? x : 0.0;
                    }
                }
#pragma unroll
                for (int ks = 0; ks < 4 * NT; ++ks)
#pragma unroll
                    for (int h = 0; h < HQ; ++h) d[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks][h], bw[ks], d[h], 0, 0, 0);
                // result lane l, register v: the same Q entry as qv[h][v]
                if (i0 + cl < m) {
#pragma unroll
                    for (int h = 0; h < HQ; ++h)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int l = l0 + 16 * h + 4 * v + g;
                            if (l < m) Q[(size_t)l * m + i0 + cl] = qv[h][v] - d[h][v];
                        }
                }
            }
            wave_lds_sync();   // wt is rewritten by the next tile
        }
        __syncthreads();
    }

    __device__ __forceinline__ void update_q() {
        const int k = s.kr;
        if (k <= 16) update_q_tiles<1>();
        else if (k <= 32) update_q_tiles<2>();
        else if (k <= 48) update_q_tiles<3>();
        else update_q_tiles<4>();
    }

    // a5: feasibility loop on J (Algorithm 3): keep the longest prefix of J whose
    // own least-squares components are all positive.
    __device__ __forceinline__ void jloop() {
        if (prm.nojloop) {   // Theorem 4: the block is taken whole
            if (tid == 0) s.k = s.kr;
            __syncthreads();
            return;
        }
        if (tid == 0) {
            const int r0 = s.nP;
            int k = s.kr;
            while (k > 0) {
                double yy[KM];
                for (int i = 0; i < k; ++i) yy[i] = gp.bt[r0 + i];
                double mn = INFINITY;
                for (int j = k - 1; j >= 0; --j) {
                    const double yj = yy[j] / Rat(r0 + j, r0 + j);
                    yy[j] = yj;
                    mn = fmin(mn, yj);
                    for (int i = 0; i < j; ++i) yy[i] -= yj * Rat(r0 + i, r0 + j);
                }
                if (mn > 0.0) break;
                --k;
                s.jdrops += 1;
            }
            s.k = k;
        }
        __syncthreads();
    }

    // a4: y = R^{-1} bt[0:n_P], by blocks of TS rows from the bottom.  The slot
    // indices of all passive positions are staged in LDS once.  The diagonal
    // block is staged in LDS with coalesced loads; wave 0 takes its row,
    // scaled by the inverse diagonal, into registers and back-substitutes
    // (lane i holds row i, entry j is broadcast from lane j through the scalar
    // unit when step j reaches it); then every thread subtracts the block's
    // contribution from its rows above, with 32 columns' loads in flight.
    static constexpr int TS = WG_TS;
    __device__ __forceinline__ void trsv() {
        lds_double(*Rd)[TS + 1] = reinterpret_cast<lds_double(*)[TS + 1]>(lx);
        lds_int* sl = reinterpret_cast<lds_int*>(lx + TS * (TS + 1));   // slot of every position
        const int nP = s.nP;
        for (int i = tid; i < nP; i += WG) {
            s.c[i] = gp.bt[i];
            sl[i] = gp.slot[i];
        }
        for (int r0 = ((nP - 1) / TS) * TS; r0 >= 0 && nP > 0; r0 -= TS) {
            const int nr = min(nP, r0 + TS) - r0;
            __syncthreads();   // rows >= r0 of c are final; Rd is free
            for (int e = tid; e < TS * TS; e += WG) {
                const int j = e / TS, i = e % TS;   // consecutive threads: consecutive rows of a column
                Rd[i][j] = (j < nr && i <= j) ? gp.R[(size_t)sl[r0 + j] * p.kc + r0 + i] : 0.0;
            }
            __syncthreads();
            if (wid == 0) {
                const bool ok = lane < nr;
                const double rinv = ok ? 1.0 / Rd[lane][lane] : 0.0;
                double row[TS];
#pragma unroll
                for (int j = 0; j < TS; ++j) row[j] = Rd[lane][j] * rinv;
                double v = ok ? s.c[r0 + lane] * rinv : 0.0;
#pragma unroll
                for (int j = TS - 1; j >= 0; --j) {
                    const double yj = readlane_d(v, j);
                    v = (lane < j) ? fma(-row[j], yj, v) : v;
                }
                if (ok) yv[r0 + lane] = v;
            }
            __syncthreads();
            for (int i = tid; i < r0; i += WG) {
                double acc = 0.0;
                for (int j0 = 0; j0 < nr; j0 += 32) {
                    double rv[32];
#pragma unroll
                    for (int k = 0; k < 32; ++k)
                        rv[k] = (j0 + k < nr) ? gp.R[(size_t)sl[r0 + j0 + k] * p.kc + i] : 0.0;
#pragma unroll
                    for (int k = 0; k < 32; ++k)
                        if (j0 + k < nr) acc = fma(rv[k], yv[r0 + j0 + k], acc);
                }
                s.c[i] -= acc;
            }
        }
        __syncthreads();
    }

    // a6: one inner iteration: step length, new iterate, removal set.  Leaves
    // the ascending removal positions in gp.rm[0..s.q).  have_al: the step
    // length al_in was already taken (the minimum of the same ratios).
    __device__ __forceinline__ void inner_step(bool have_al = false, double al_in = 0.0) {
#pragma clang fp contract(off)
        const int nP = s.nP;
        double al = al_in;
        if (!have_al) {
            al = INFINITY;
            for (int c = tid; c < nP; c += WG) {
                const double yc = yv[c];
                if (yc <= 0.0) {
                    const double xc = gp.x[gp.P[c]];
                    al = fmin(al, step_ratio(xc, yc));
                }
            }
            al = vmin(al);
        }
        const int chunk = (nP + WG - 1) / WG;
        const int c0 = tid * chunk, c1 = min(nP, c0 + chunk);
        // the removal flags are taken from the new iterates as they are written
        int mine = 0;
        unsigned long long mask = 0;
        // the positions of a chunk are distinct columns, so a batch's loads all
        // go out before its stores (a store per position would order every
        // later gathered load behind it)
        for (int cb = c0; cb < c1; cb += LB) {
            int j[LB];
            double xc[LB], yc[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int c = min(cb + u, c1 - 1);
                j[u] = gp.P[c];
                yc[u] = yv[c];
            }
#pragma unroll
            for (int u = 0; u < LB; ++u) xc[u] = gp.x[j[u]];
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                if (cb + u < c1) {
                    double xn = xc[u] + al * (yc[u] - xc[u]);
                    if (yc[u] <= 0.0 && step_ratio(xc[u], yc[u]) == al) xn = 0.0;
                    if (xn <= 0.0) {
                        xn = 0.0;
                        ++mine;
                        if (cb + u - c0 < 64) mask |= 1ull << (cb + u - c0);
                    }
                    gp.x[j[u]] = xn;
                }
            }
        }
        place_positions(mine, mask, chunk, c0, c1, [&](int c, int j) { return gp.x[j] <= 0.0; });
    }

    // gp.rm[0..s.q) = ascending passive positions whose x is <= 0.
    __device__ __forceinline__ void collect_removals() {
        collect_positions([&](int c, int j) { return gp.x[j] <= 0.0; });
    }

    // gp.rm[0..s.q) = ascending passive positions c (column j = P[c]) for which
    // pick(c, j) holds.
    template <typename Pick>
    __device__ __forceinline__ void collect_positions(Pick pick) {
        const int nP = s.nP;
        const int chunk = (nP + WG - 1) / WG;
        const int c0 = tid * chunk, c1 = min(nP, c0 + chunk);
        // flags of the chunk in batches of gathered loads; kept as a bit mask
        // when the chunk has at most 64 positions
        int mine = 0;
        unsigned long long mask = 0;
        for (int cb = c0; cb < c1; cb += LB) {
            int j[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) j[u] = gp.P[min(cb + u, c1 - 1)];
            bool hit[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) hit[u] = pick(min(cb + u, c1 - 1), j[u]);
#pragma unroll
            for (int u = 0; u < LB; ++u)
                if (cb + u < c1 && hit[u]) {
                    ++mine;
                    if (cb + u - c0 < 64) mask |= 1ull << (cb + u - c0);
                }
        }
        place_positions(mine, mask, chunk, c0, c1, pick);
    }

    // gp.rm[0..s.q) from each thread's count of picked positions in its chunk
    // c0..c1 and, for chunks of at most 64 positions, their bit mask (longer
    // chunks are scanned again with pick).
    template <typename Pick>
    __device__ __forceinline__ void place_positions(int mine, unsigned long long mask, int chunk, int c0, int c1,
                                                    Pick pick) {
        // exclusive prefix sum of the counts in thread order: a scan within
        // each wave, then the totals of the waves before it
        int incl = mine;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(incl, d, 64);
            if (lane >= d) incl += v;
        }
        __syncthreads();
        if (lane == 63) s.cnt[wid] = incl;
        __syncthreads();
        int o = incl - mine;
        for (int w = 0; w < wid; ++w) o += s.cnt[w];
        if (tid == WG - 1) s.q = o + mine;
        if (chunk <= 64) {
            while (mask) {
                gp.rm[o++] = c0 + __builtin_ctzll(mask);
                mask &= mask - 1;
            }
        } else {
            for (int c = c0; c < c1; ++c)
                if (pick(c, gp.P[c])) gp.rm[o++] = c;
        }
        __syncthreads();
    }

    // The inner iteration of the positivity-trick case (Section 4.2): every
    // passive position with y < 0 takes the twin of its column (the negated
    // column), whose R column is the negated one and whose least-squares
    // component is -y > 0; the residual is unchanged, so the inner loop ends.
    // Returns false, changing nothing, when a component is exactly 0 (the
    // ordinary inner iteration then runs).
    __device__ __forceinline__ bool sign_flip() {
        const int nP = s.nP;
        int zero = 0;
        for (int c = tid; c < nP; c += WG) zero |= (yv[c] == 0.0) ? 1 : 0;
        if (imax(zero)) return false;
        collect_positions([&](int c, int j) { return yv[c] < 0.0; });
        const int q = s.q;
        for (int t = 0; t < q; ++t) {
            const int c = gp.rm[t];
            gdouble* col = gp.R + (size_t)gp.slot[c] * p.kc;
            for (int i = tid; i <= c; i += WG) col[i] = -col[i];
        }
        for (int t = tid; t < q; t += WG) {
            const int c = gp.rm[t], j = gp.P[c], tw = twin_of(p, j);
            gp.P[c] = tw;
            gp.pos[j] = -1;
            gp.pos[tw] = c;
            gp.x[j] = 0.0;
            yv[c] = -yv[c];
        }
        __syncthreads();
        return true;
    }

    // Algorithm 5 for a single removal (position first = rm[0]): every kept
    // column after it carries one rotation, on the rows of its new and old
    // positions, so rotation e acts on rows (first + e, first + e + 1).  Wave 0
    // takes the kept columns in blocks of 64 (lane t: kept column 64 b + t).
    // For each earlier block it applies that block's 64 rotations to the 65
    // rows they touch, staged in an LDS window (one column per lane), with the
    // running entry in a register; then it generates the block's own
    // rotations in a chain along the lanes: rotation t is computed by lane t
    // from its two entries and broadcast through the scalar unit, and every
    // lane applies it (for the columns left of t those rows are below the
    // diagonal, and the entry each lane's own rotation zeroes is stored as 0
    // afterwards).  The rotations then go to bt and to the columns of Q (one
    // thread per row, loads sixteen columns ahead).  Same rotations, in the
    // same order, as the general sweep.
    static constexpr int DB = WG_DB;
    __device__ __forceinline__ void downdate_unit() {
        lds_double(*win)[DB] = reinterpret_cast<lds_double(*)[DB]>(lx);
        lds_double* rl = lx + (DB + 1) * DB;   // rotations of the window being applied
        gdouble* rot = gp.rot;                 // (c, s) of rotation e at 2 e, 2 e + 1
        const int nP = s.nP, first = gp.rm[0], m = p.m;
        const int nd = nP - 1 - first;
        if (wid == 0 && nd > 0) {
            const int nb = (nd + DB - 1) / DB;
            for (int b = 0; b < nb; ++b) {
                const int e = b * DB + lane;
                const bool valid = e < nd;
                gdouble* col = gp.R + (size_t)gp.slot[first + 1 + (valid ? e : nd - 1)] * p.kc;
                double run = 0.0;   // entry carried from one window to the next
                for (int bb = 0; bb <= b; ++bb) {
                    const int rlo = first + DB * bb;
                    const int nw = min(DB, nd - DB * bb);   // rotations of block bb
                    // the window's rows 1 .. nw (row 0 is the carried entry), sixteen
                    // loads in flight per lane
                    for (int r1 = 1; r1 <= nw; r1 += 16) {
                        double t16[16];
#pragma unroll
                        for (int u = 0; u < 16; ++u) t16[u] = (r1 + u <= nw) ? col[rlo + r1 + u] : 0.0;
#pragma unroll
                        for (int u = 0; u < 16; ++u)
                            if (r1 + u <= nw) win[r1 + u][lane] = t16[u];
                    }
                    if (bb == 0) run = col[rlo];
                    wave_lds_sync();
                    if (bb < b) {
                        // block bb's rotations (written by this wave) into LDS
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int q = 64 * h + lane;
                            const double v = rot[2 * DB * bb + min(q, 2 * nw - 1)];
                            rl[q] = v;
                        }
                        wave_lds_sync();
                        for (int k = 0; k < nw; ++k) {
                            const double cs = rl[2 * k], sn = rl[2 * k + 1];
                            const double y = win[k + 1][lane];
                            win[k][lane] = cs * run + sn * y;
                            run = -sn * run + cs * y;
                        }
                    } else {
                        for (int k = 0; k < nw; ++k) {
                            const double y = win[k + 1][lane];
                            double cs, sn, rr;
                            givens(run, y, cs, sn, rr);
                            cs = readlane_d(cs, k);
                            sn = readlane_d(sn, k);
                            if (lane == 0) {
                                rot[2 * (DB * bb + k)] = cs;
                                rot[2 * (DB * bb + k) + 1] = sn;
                            }
                            wave_lds_sync();
                            win[k][lane] = cs * run + sn * y;
                            run = -sn * run + cs * y;
                        }
                    }
                    win[nw][lane] = run;
                    // the rotations stored above are read back by this wave in later windows
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                    wave_lds_sync();
                    if (valid) {
                        const int top = (bb < b) ? nw - 1 : nw;   // the carried row goes to the next window
                        for (int r = 0; r <= top; ++r) col[rlo + r] = win[r][lane];
                        if (bb == b) col[rlo + lane + 1] = 0.0;   // the entry this lane's rotation zeroed
                    }
                    wave_lds_sync();
                }
            }
        }
        __syncthreads();   // rotations in rot, R updated
        if (nd > 0) {
            // bt and the columns of Q: row `row` of [Q; bt^T], running entry in a register
            for (int row = tid; row <= m; row += WG) {
                gdouble* base = (row < m) ? gp.Q + row : gp.bt;
                const size_t stride = (row < m) ? (size_t)m : 1;
                double x = base[(size_t)first * stride];
                for (int e0 = 0; e0 < nd; e0 += 16) {
                    double y[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) y[u] = (e0 + u < nd) ? base[(size_t)(first + e0 + u + 1) * stride] : 0.0;
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        if (e0 + u < nd) {
                            const double cs = rot[2 * (e0 + u)], sn = rot[2 * (e0 + u) + 1];
                            base[(size_t)(first + e0 + u) * stride] = cs * x + sn * y[u];
                            x = -sn * x + cs * y[u];
                        }
                    }
                }
                base[(size_t)(first + nd) * stride] = x;
            }
        }
        __syncthreads();
        compact();
    }

    // Algorithm 5: delete the passive positions gp.rm[0..q) from R and restore the
    // triangle with Givens rotations, column by column, bottom-up within a
    // column; rotations are applied to R, bt and the columns of Q.
    __device__ __forceinline__ void downdate() {
        if (s.q == 1) {
            downdate_unit();
            return;
        }
        const int q = s.q, nP = s.nP, m = p.m;
        const int first = gp.rm[0];
        int ri = 0;
        for (int oc = first; oc < nP; ++oc) {
            if (ri < q && gp.rm[ri] == oc) {
                ++ri;
                continue;
            }
            const int l = ri;          // deleted columns before this one
            const int c = oc - l;      // its new position
            if (tid == 0) {
                for (int i = oc, g = 0; i > c; --i, ++g) {
                    const double a = Rat(i - 1, oc), bb = Rat(i, oc);
                    double cs, sn, rr;
                    givens(a, bb, cs, sn, rr);
                    Rat(i - 1, oc) = cs * a + sn * bb;
                    Rat(i, oc) = 0.0;
                    gp.rot[2 * g] = cs;
                    gp.rot[2 * g + 1] = sn;
                }
            }
            __syncthreads();
            // later kept columns: rows c..oc
            {
                int rj = ri;
                for (int oc2 = oc + 1 + tid; oc2 < nP; oc2 += WG) {
                    // is oc2 deleted?  (rm is ascending; scan from ri)
                    bool del = false;
                    for (int t = rj; t < q; ++t) {
                        if (gp.rm[t] == oc2) {
                            del = true;
                            break;
                        }
                        if (gp.rm[t] > oc2) break;
                    }
                    if (del) continue;
                    for (int i = oc, g = 0; i > c; --i, ++g) {
                        const double cs = gp.rot[2 * g], sn = gp.rot[2 * g + 1];
                        const double a = Rat(i - 1, oc2), bb = Rat(i, oc2);
                        Rat(i - 1, oc2) = cs * a + sn * bb;
                        Rat(i, oc2) = -sn * a + cs * bb;
                    }
                }
            }
            if (tid == 0) {
                for (int i = oc, g = 0; i > c; --i, ++g) {
                    const double cs = gp.rot[2 * g], sn = gp.rot[2 * g + 1];
                    const double a = gp.bt[i - 1], bb = gp.bt[i];
                    gp.bt[i - 1] = cs * a + sn * bb;
                    gp.bt[i] = -sn * a + cs * bb;
                }
            }
            for (int row = tid; row < m; row += WG) {
                for (int i = oc, g = 0; i > c; --i, ++g) {
                    const double cs = gp.rot[2 * g], sn = gp.rot[2 * g + 1];
                    const double a = Qat(row, i - 1), bb = Qat(row, i);
                    Qat(row, i - 1) = cs * a + sn * bb;
                    Qat(row, i) = -sn * a + cs * bb;
                }
            }
            __syncthreads();
        }
        compact();
    }

    // Drop the removed positions from P; their R slots move behind the kept ones
    // (slot stays a permutation, free slots at [n_P, kc)).  Kept position c
    // moves to c - #{removed < c}; the t-th removed slot goes to n_P - q + t.
    __device__ __forceinline__ void compact() {
        const int q = s.q, nP = s.nP;
        if (q == 0) return;
        gint* oldP = gp.itmp;
        gint* oldS = gp.itmp + p.kc;
        // the int arrays may alias as far as the compiler knows: each batch's
        // loads go out before its stores, instead of one round trip per position
        for (int c0 = tid; c0 < nP; c0 += WG * LB) {
            int pv[LB], sv[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int c = min(c0 + WG * u, nP - 1);
                pv[u] = gp.P[c];
                sv[u] = gp.slot[c];
            }
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int c = c0 + WG * u;
                if (c < nP) {
                    oldP[c] = pv[u];
                    oldS[c] = sv[u];
                }
            }
        }
        __syncthreads();
        for (int c0 = tid; c0 < nP; c0 += WG * LB) {
            int pv[LB], sv[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int c = min(c0 + WG * u, nP - 1);
                pv[u] = oldP[c];
                sv[u] = oldS[c];
            }
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int c = c0 + WG * u;
                if (c >= nP) continue;
                int lo = 0, hi = q;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (gp.rm[mid] < c) lo = mid + 1;
                    else hi = mid;
                }
                const int j = pv[u];
                if (lo < q && gp.rm[lo] == c) {
                    gp.pos[j] = -1;
                    gp.slot[nP - q + lo] = sv[u];
                } else {
                    const int w = c - lo;
                    gp.P[w] = j;
                    gp.slot[w] = sv[u];
                    gp.pos[j] = w;
                }
            }
        }
        __syncthreads();
        if (tid == 0) s.nP = nP - q;
        __syncthreads();
    }

    // a7: r = b - A_P x_P.  P is staged in LDS and each thread keeps sixteen
    // columns' loads in flight; the sum still runs over the positions in order.
    __device__ __forceinline__ void residual() {
        const int m = p.m, nP = s.nP;
        lds_int* Pl = reinterpret_cast<lds_int*>(lx);
        for (int c = tid; c < nP; c += WG) Pl[c] = gp.P[c];
        __syncthreads();
        for (int i = tid; i < m; i += WG) {
            double acc = gp.b[i];
            for (int c0 = 0; c0 < nP; c0 += 16) {
                double av[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    double sg;
                    const gdouble* a = gcol(Pl[min(c0 + u, nP - 1)], sg);
                    av[u] = sg * a[i];
                }
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    if (c0 + u < nP) acc -= av[u] * yv[c0 + u];
            }
            gp.r[i] = acc;
        }
        __syncthreads();
    }

    // a7: w = A^T r and the update of u2 = ||Q_perp^T a_j||^2:
    //   u2 <- u2 - sum_added (q^T a)^2 + sum_dropped (q^T a)^2,
    // or exactly from the trailing columns of Q when they are fewer.  The vectors
    // (r, then the added and dropped columns of Q, or the trailing ones) go
    // through the matrix-core product DVL at a time, so A is read once per
    // chunk instead of once per vector.
    __device__ __forceinline__ void dual_and_norms(int kadd) {
        const int m = p.m, nph = p.nph, nP = s.nP, nPa = s.nPa;
        const int ndrop = nPa - nP;
        const bool exact = (m - nP) <= kadd + ndrop;
        const bool tw = nph != p.n;
        const int nvec = 1 + (exact ? m - nP : kadd + ndrop);
        for (int c0 = 0; c0 < nvec; c0 += DVL) {
            const int nv = min(DVL, nvec - c0), nvp = (nv + 15) & ~15;
            // consecutive threads take consecutive rows of a vector; eight loads in flight
            for (int e0 = tid; e0 < m * nvp; e0 += WG * LB) {
                double val[LB];
#pragma unroll
                for (int u = 0; u < LB; ++u) {
                    const int e = e0 + WG * u, t = e / m, i = e - t * m, v = c0 + t;
                    val[u] = 0.0;
                    if (e < m * nvp && t < nv) {
                        if (v == 0) val[u] = gp.r[i];
                        else if (exact) val[u] = Qat(i, nP + v - 1);
                        else if (v <= kadd) val[u] = gp.Qadd[(size_t)(v - 1) * m + i];
                        else val[u] = Qat(i, nP + v - 1 - kadd);
                    }
                }
#pragma unroll
                for (int u = 0; u < LB; ++u) {
                    const int e = e0 + WG * u, t = e / m, i = e - t * m;
                    if (e < m * nvp) gp.Dv[(size_t)i * DVL + t] = val[u];
                }
            }
            __syncthreads();
            colmat_any(gp.A, p.lda, nph, nv, [&](int j, const lds_double* c, int nvv) {
                double u2;
                int t = 0;
                if (c0 == 0) {
                    gp.w[j] = c[0];
                    if (tw) gp.w[j + nph] = -c[0];
                    u2 = exact ? 0.0 : gp.u2[j];
                    t = 1;
                } else {
                    u2 = gp.u2[j];
                }
                for (; t < nvv; ++t) {
                    const double d = c[t];
                    if (exact || c0 + t > kadd) u2 += d * d;
                    else u2 -= d * d;
                }
                gp.u2[j] = u2;
            });
        }
        // clamp; columns whose updated norm lost most of its digits are
        // recomputed from the trailing columns of Q, one wave per column
        for (int base = wid * 64; base < nph; base += WG) {
            const int j = base + lane;
            bool flag = false;
            double u2 = 0.0;
            if (j < nph) {
                u2 = gp.u2[j];
                if (!exact) {
                    u2 = fmax(u2, 0.0);
                    flag = gp.pos[j] < 0 && !gtwin_passive(j) && u2 < RECOMP_FRAC * gp.an2[j];
                }
                if (!flag) {
                    gp.u2[j] = u2;
                    if (tw) gp.u2[j + nph] = u2;
                }
            }
            unsigned long long mask = __ballot(flag);
            while (mask) {
                const int jj = base + __ffsll((long long)mask) - 1;
                mask &= mask - 1;
                const gdouble* a = Acol(jj);
                double r2 = 0.0;
                for (int t = nP; t < m; ++t) {
                    double d = 0.0;
                    for (int i = lane; i < m; i += 64) d += a[i] * Qat(i, t);
                    d = wave_sum(d);
                    r2 += d * d;
                }
                if (lane == 0) {
                    gp.u2[jj] = r2;
                    if (tw) gp.u2[jj + nph] = r2;
                }
            }
        }
        __syncthreads();
    }

    // r and w for the current x (used when the loop stops inside an inner loop)
    __device__ __forceinline__ void refresh_dual() {
        const int m = p.m, nph = p.nph;
        for (int i = tid; i < m; i += WG) {
            double acc = gp.b[i];
            for (int c = 0; c < s.nP; ++c) {
                const int j = gp.P[c];
                double sg;
                const gdouble* a = gcol(j, sg);
                acc -= (sg * a[i]) * gp.x[j];
            }
            gp.r[i] = acc;
        }
        __syncthreads();
        for (int j = wid; j < nph; j += NW) {
            const gdouble* a = Acol(j);
            double acc = 0.0;
            for (int i = lane; i < m; i += 64) acc += a[i] * gp.r[i];
            acc = wave_sum(acc);
            if (lane == 0) {
                gp.w[j] = acc;
                if (nph != p.n) gp.w[j + nph] = -acc;
            }
        }
        __syncthreads();
    }

    __device__ __forceinline__ void finalize() {
        const int n = p.n, m = p.m, nP = s.nP;
        double vz = 0.0, vp = 0.0;
        for (int j = tid; j < n; j += WG) {
            const double wj = gp.w[j];
            if (gp.pos[j] >= 0) vp = fmax(vp, fabs(wj));
            else vz = fmax(vz, fmax(wj, 0.0));
            if (gp.passive) gp.passive[j] = (j < nP) ? gp.P[j] : -1;
        }
        vz = vmax(vz);
        vp = vmax(vp);
        double rr = 0.0;
        for (int i = tid; i < m; i += WG) rr += gp.r[i] * gp.r[i];
        rr = sum(rr);
        if (tid == 0 && p.info) {
            double scale = s.anmax * s.bnorm;
            if (!(scale > 0.0)) scale = 1.0;
            lhdm_info inf;
            inf.status = s.status;
            inf.outer_iters = s.outer;
            inf.inner_iters = s.inner;
            inf.jloop_drops = s.jdrops;
            inf.n_passive = nP;
            inf.cq_panels = 0;
            inf.kkt_residual = fmax(vz, vp) / scale;
            inf.objective = rr;
            *p.info = inf;
        }
        __syncthreads();
    }

    // ---------------- stages of an outer step ----------------
    // One outer step in three stages, so that a solve runs either in one loop
    // (run) or as one kernel launch per stage over many instances (the phased
    // batched engine); the stage and everything the next stage needs live in
    // the control block and the instance's workspace.
    //   APPEND: selection, projection, deviation maximization, Householder
    //           panel, compact-WY Q update, feasibility loop on J, y = R^-1 bt;
    //   INNER:  the inner loop (step length, removals, downdate) until y > 0;
    //   ACCEPT: x = y, residual, dual and projected-norm update.
    __device__ __forceinline__ void stage_append() {
        select();
        if (s.done) {
            if (tid == 0) s.stage = ST_DONE;
            __syncthreads();
            return;
        }
        const int ncol = s.ncol;
        project(ncol);
        if (ncol > 1) {
            deviation_maximization();
        } else {
            if (tid == 0) s.k = 1;
            __syncthreads();
        }
        if (tid == 0) {
            s.kr = s.k;
            s.j1 = s.J[0];
        }
        __syncthreads();
        panel_qr();
        if (s.kr > 1) form_wy();
        else {
            // one reflector: V = [0; 1; v], T = tau
            const int m = p.m, r0 = s.nP;
            for (int i = tid; i < m; i += WG) gp.V[i] = (i < r0) ? 0.0 : gp.G[i];
            if (tid == 0) gp.T[0] = s.tau[0];
            __syncthreads();
        }
        append_r();
        update_q();
        jloop();
        const int k = s.k;
        if (k == 0) {
            if (tid == 0) {
                gp.excl[s.j1] = 1;
                s.any_excl = 1;
                s.stage = ST_APPEND;
            }
            __syncthreads();
            return;
        }
        if (s.any_excl) {
            for (int j = tid; j < p.n; j += WG) gp.excl[j] = 0;
            __syncthreads();
            if (tid == 0) s.any_excl = 0;
        }
        // passive set grows by J, in order
        const int m = p.m, r0 = s.nP;
        for (int t = 0; t < k; ++t)
            for (int i = tid; i < m; i += WG) gp.Qadd[(size_t)t * m + i] = Qat(i, r0 + t);
        if (tid == 0) {
            for (int t = 0; t < k; ++t) {
                gp.P[r0 + t] = s.J[t];
                gp.pos[s.J[t]] = r0 + t;
            }
            s.nP = r0 + k;
            s.nPa = r0 + k;
            s.outer += 1;
            s.stage = ST_INNER;
        }
        __syncthreads();
        trsv();
    }

    __device__ __forceinline__ void stage_inner() {
        bool stop = false;
        while (true) {
            double mn = INFINITY;
            for (int c = tid; c < s.nP; c += WG) mn = fmin(mn, yv[c]);
            mn = vmin(mn);
            if (mn > 0.0) break;
            if (s.inner >= prm.max_inner) {
                stop = true;
                break;
            }
            __syncthreads();
            if (tid == 0) s.inner += 1;
            if (prm.signflip && sign_flip()) break;   // y > 0 now: the inner loop ends
            inner_step();
            downdate();
            trsv();
        }
        __syncthreads();
        if (stop) {
            if (tid == 0) {
                s.status = LHDM_STATUS_MAXITER;
                s.stage = ST_DONE;
            }
            __syncthreads();
            refresh_dual();
            return;
        }
        if (tid == 0) s.stage = ST_ACCEPT;
        __syncthreads();
    }

    __device__ __forceinline__ void stage_accept() {
        for (int c = tid; c < s.nP; c += WG) gp.x[gp.P[c]] = yv[c];
        __syncthreads();
        residual();
        dual_and_norms(s.k);
        if (tid == 0) s.stage = ST_APPEND;
        __syncthreads();
    }

    // a0 and the first stage; false when the solve is already finished
    __device__ __forceinline__ bool start() {
        init();
        if (tid == 0) s.stage = (s.status == LHDM_STATUS_NONFINITE) ? ST_DONE : ST_APPEND;
        __syncthreads();
        return s.stage != ST_DONE;
    }

    __device__ __forceinline__ void step() {
        const int st = s.stage;
        if (st == ST_APPEND) stage_append();
        else if (st == ST_INNER) stage_inner();
        else if (st == ST_ACCEPT) stage_accept();
    }

    // ---------------- the whole solve ----------------
    __device__ __forceinline__ void run() {
        if (start())
            while (s.stage != ST_DONE) step();
        finalize();
    }
};

}  // namespace lhdm
