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
struct Ctl {
    double tol_w, anmax, bnorm;
    int nP, nP0, nPa, status, outer, inner, jdrops, ncol, k, kr, done, q, any_excl, j1;
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

struct Wg {
    static constexpr int LB = 8;   // gathered loads issued together per thread
    Prob& p;
    const DevParams& prm;
    WgShared& s;
    int tid, lane, wid;
    double* yv;   // least-squares solution by position: LDS (workgroup engine) or global

    __device__ Wg(Prob& p_, const DevParams& prm_, WgShared& s_)
        : p(p_), prm(prm_), s(s_), tid(threadIdx.x), lane(threadIdx.x & 63), wid(wave_index()),
          yv(p_.ybuf ? p_.ybuf : s_.y) {}

    // ---------------- workgroup reductions ----------------
    __device__ double sum(double v) {
        v = wave_sum(v);
        __syncthreads();
        if (lane == 0) s.rd[wid] = v;
        __syncthreads();
        double t = s.rd[0];
#pragma unroll
        for (int i = 1; i < NW; ++i) t += s.rd[i];
        return t;
    }
    __device__ double vmax(double v) {
        v = wave_max(v);
        __syncthreads();
        if (lane == 0) s.rd[wid] = v;
        __syncthreads();
        double t = s.rd[0];
#pragma unroll
        for (int i = 1; i < NW; ++i) t = fmax(t, s.rd[i]);
        return t;
    }
    __device__ double vmin(double v) {
        v = wave_min(v);
        __syncthreads();
        if (lane == 0) s.rd[wid] = v;
        __syncthreads();
        double t = s.rd[0];
#pragma unroll
        for (int i = 1; i < NW; ++i) t = fmin(t, s.rd[i]);
        return t;
    }
    __device__ int imax(int v) {
        v = wave_max_int(v);
        __syncthreads();
        if (lane == 0) s.ri[wid] = v;
        __syncthreads();
        int t = s.ri[0];
#pragma unroll
        for (int i = 1; i < NW; ++i) t = max(t, s.ri[i]);
        return t;
    }
    __device__ void argmax(double& v, int& i) {
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
    __device__ void push(int t, double part) {
        part = wave_sum(part);
        if (lane == 0) s.mr[t][wid] = part;
    }
    __device__ void finish(int cnt) {
        __syncthreads();
        if (tid < cnt) {
            double a = s.mr[tid][0];
#pragma unroll
            for (int w = 1; w < NW; ++w) a += s.mr[tid][w];
            s.vec[tid] = a;
        }
        __syncthreads();
    }

    __device__ double& Qat(int i, int j) { return p.Q[(size_t)j * p.m + i]; }
    __device__ double& Rat(int i, int j) { return p.R[(size_t)p.slot[j] * p.kc + i]; }
    __device__ const double* Acol(int j) { return p.A + (size_t)j * p.lda; }

    // ---------------- a0: initialisation (Algorithm 3, first lines) ----------------
    __device__ void init() {
        const int m = p.m, nph = p.nph;
        double anmax = 0.0;
        int bad = 0;
        for (int j = wid; j < nph; j += NW) {
            const double* a = Acol(j);
            double ab = 0.0, aa = 0.0;
            for (int i = lane; i < m; i += 64) {
                const double v = a[i];
                ab += v * p.b[i];
                aa += v * v;
            }
            ab = wave_sum(ab);
            aa = wave_sum(aa);
            if (lane == 0) {
                p.w[j] = ab;          // w^(0) = A^T b
                p.an2[j] = aa;
                p.u2[j] = aa;         // u^(0) = column norms of A
                p.pos[j] = -1;
                p.excl[j] = 0;
                p.x[j] = 0.0;
                if (nph != p.n) {     // the twin -a_j of the positivity trick
                    const int t = j + nph;
                    p.w[t] = -ab;
                    p.an2[t] = aa;
                    p.u2[t] = aa;
                    p.pos[t] = -1;
                    p.excl[t] = 0;
                    p.x[t] = 0.0;
                }
            }
            if (!isfinite(ab) || !isfinite(aa)) bad = 1;
            anmax = fmax(anmax, aa);
        }
        double bb = 0.0;
        for (int i = tid; i < m; i += WG) {
            const double v = p.b[i];
            bb += v * v;
            p.bt[i] = v;
            p.r[i] = v;
        }
        bb = sum(bb);
        anmax = vmax(anmax);
        bad = imax(bad);
        const size_t mm = (size_t)m * m;
        for (size_t e = tid; e < mm; e += WG) p.Q[e] = ((e % m) == (e / m)) ? 1.0 : 0.0;
        for (int c = tid; c < p.kc; c += WG) p.slot[c] = c;
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
    __device__ void select() {
        const int n = p.n;
        double mwz = -INFINITY, mu = 0.0, bv = -INFINITY;
        int bi = INT_MAX;
        for (int j = tid; j < n; j += WG) {
            if (p.pos[j] >= 0) continue;
            const double wj = p.w[j];
            const double u = sqrt(fmax(p.u2[j], 0.0));
            mwz = fmax(mwz, wj);
            mu = fmax(mu, u);
            if (!p.excl[j] && u > DEP_TOL * sqrt(p.an2[j]) && !twin_passive(p, j) && better(wj, j, bv, bi)) {
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
                if (p.pos[j] >= 0 || p.excl[j] || j == bi) continue;
                const double wj = p.w[j];
                if (!(wj >= tw)) continue;
                const double u = sqrt(fmax(p.u2[j], 0.0));
                if (!(u >= tu) || !(u > DEP_TOL * sqrt(p.an2[j])) || twin_passive(p, j)) continue;
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

    // G[:, t] = Q^T a_{J[t]} for t < cnt (full projection: rows < n_P are Q_P^T a,
    // rows >= n_P the coordinates of the projected column in the trailing basis).
    __device__ void project(int cnt) {
        const int m = p.m;
        for (int i = tid; i < m; i += WG) {
            const double* q = &Qat(0, i);
            for (int t = 0; t < cnt; ++t) {
                double sg;
                const double* a = col_ptr(p, s.J[t], sg);
                double acc = 0.0;
                for (int l = 0; l < m; ++l) acc += q[l] * a[l];
                p.G[(size_t)t * m + i] = sg * acc;
            }
        }
        __syncthreads();
    }

    // Gram matrix of the projected candidates G[n_P:m, 0:ncol] into T (ld kq).
    __device__ void candidate_gram() {
        const int m = p.m, c = s.ncol, r0 = s.nP, kq = p.kq;
        const int npair = c * (c + 1) / 2;
        for (int pr = wid; pr < npair; pr += NW) {
            int a = 0, rem = pr;
            while (rem > a) {
                rem -= a + 1;
                ++a;
            }
            const int bcol = rem;   // pair (a, bcol), bcol <= a
            const double* ga = p.G + (size_t)a * m;
            const double* gb = p.G + (size_t)bcol * m;
            double acc = 0.0;
            for (int i = r0 + lane; i < m; i += 64) acc += ga[i] * gb[i];
            acc = wave_sum(acc);
            if (lane == 0) {
                p.T[(size_t)a * kq + bcol] = acc;
                p.T[(size_t)bcol * kq + a] = acc;
            }
        }
        __syncthreads();
    }

    // Cosines of the projected candidates (eq. of the cosine matrix) from the
    // Gram matrix in T, and the greedy acceptance of Algorithm 2.  Compacts G
    // to the accepted columns.
    __device__ void greedy_from_gram() {
        const int m = p.m, c = s.ncol, kq = p.kq;
        if (tid == 0) {
            const int cap = p.m - s.nP;
            int acc[KM];
            int na = 1;
            acc[0] = 0;
            for (int t = 1; t < c; ++t) {
                if (na >= cap) break;
                const double nt = sqrt(p.T[(size_t)t * kq + t]);
                bool ok = true;
                for (int q = 0; q < na; ++q) {
                    const int a = acc[q];
                    const double th = p.T[(size_t)a * kq + t] / (nt * sqrt(p.T[(size_t)a * kq + a]));
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
                for (int i = tid; i < m; i += WG) p.G[(size_t)q * m + i] = p.G[(size_t)from * m + i];
            __syncthreads();
        }
    }

    __device__ void deviation_maximization() {
        candidate_gram();
        greedy_from_gram();
    }

    // a3: Householder QR of the panel G[n_P:m, 0:k] with bt[n_P:m] carried as an
    // extra column (Algorithm 4); G keeps the reflectors below the diagonal,
    // s.beta the new diagonal of R, s.tau the reflector scalars.  Per column:
    // one pass for all dot products with the reflector, one pass for the update
    // that also accumulates the norm of the next column.
    __device__ void panel_qr() {
        const int m = p.m, k = s.kr, r0 = s.nP;
        double part0 = 0.0;
        for (int i = r0 + tid; i < m; i += WG) part0 += p.G[i] * p.G[i];
        double nrm2 = sum(part0);
        for (int t = 0; t < k; ++t) {
            const int rt = r0 + t;
            double* g = p.G + (size_t)t * m;
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
                            const double* col = (q < nrest - 1) ? p.G + (size_t)(t + 1 + q) * m : p.bt;
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
                    double* col = (q < nrest - 1) ? p.G + (size_t)(t + 1 + q) * m : p.bt;
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
    __device__ void explicit_v() {
        const int m = p.m, k = s.kr, r0 = s.nP;
        for (int t = 0; t < k; ++t) {
            const double* g = p.G + (size_t)t * m;
            double* v = p.V + (size_t)t * m;
            for (int i = tid; i < m; i += WG) v[i] = (i < r0 + t) ? 0.0 : g[i];
        }
        __syncthreads();
    }

    // V^T V, strictly upper part, into W (k x k, column-major ld kq).
    __device__ void vtv() {
        const int m = p.m, k = s.kr, r0 = s.nP, kq = p.kq;
        const int npair = k * (k - 1) / 2;
        for (int pr = wid; pr < npair; pr += NW) {
            int a = 1, rem = pr;
            while (rem >= a) {
                rem -= a;
                ++a;
            }
            const int b = rem;   // pair (b, a), b < a
            const double* va = p.V + (size_t)a * m;
            const double* vb = p.V + (size_t)b * m;
            double acc = 0.0;
            for (int i = r0 + a + lane; i < m; i += 64) acc += vb[i] * va[i];
            acc = wave_sum(acc);
            if (lane == 0) p.W[(size_t)a * kq + b] = acc;
        }
        __syncthreads();
    }

    // Compact-WY factor T with H_0 H_1 ... H_{k-1} = I - V T V^T (forward,
    // columnwise) from s.tau and V^T V in W.
    __device__ void form_t() {
        const int k = s.kr, kq = p.kq;
        if (tid == 0) {
            double* T = p.T;
            for (int t = 0; t < k; ++t) {
                T[(size_t)t * kq + t] = s.tau[t];
                double z[KM];
                for (int i = 0; i < t; ++i) z[i] = -s.tau[t] * p.W[(size_t)t * kq + i];
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

    __device__ void form_wy() {
        explicit_v();
        vtv();
        form_t();
    }

    // New R columns: [Q_P^T a_J ; R_JJ].
    __device__ void append_r() {
        const int m = p.m, k = s.kr, r0 = s.nP;
        for (int t = 0; t < k; ++t) {
            const double* g = p.G + (size_t)t * m;
            for (int i = tid; i < r0 + t + 1; i += WG) {
                double v;
                if (i < r0 + t) v = g[i];
                else v = s.beta[t];
                Rat(i, r0 + t) = v;
            }
        }
        __syncthreads();
    }

    // Q[:, n_P:m] <- Q[:, n_P:m] (I - V T V^T)  (rows of Q are independent).
    __device__ void update_q() {
        const int m = p.m, k = s.kr, r0 = s.nP, kq = p.kq;
        for (int i = tid; i < m; i += WG) {
            double wrow[KM];
#pragma unroll
            for (int t = 0; t < KM; ++t) wrow[t] = 0.0;
            for (int l = r0; l < m; ++l) {
                const double q = Qat(i, l);
#pragma unroll
                for (int t = 0; t < KM; ++t)
                    if (t < k) wrow[t] += q * p.V[(size_t)t * m + l];
            }
            double w2[KM];
#pragma unroll
            for (int t = 0; t < KM; ++t) {
                double acc = 0.0;
                if (t < k)
                    for (int l = 0; l <= t; ++l) acc += wrow[l] * p.T[(size_t)t * kq + l];
                w2[t] = acc;
            }
            for (int l = r0; l < m; ++l) {
                double acc = 0.0;
#pragma unroll
                for (int t = 0; t < KM; ++t)
                    if (t < k) acc += w2[t] * p.V[(size_t)t * m + l];
                Qat(i, l) -= acc;
            }
        }
        __syncthreads();
    }

    // a5: feasibility loop on J (Algorithm 3): keep the longest prefix of J whose
    // own least-squares components are all positive.
    __device__ void jloop() {
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
                for (int i = 0; i < k; ++i) yy[i] = p.bt[r0 + i];
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

    // a4: y = R^{-1} bt[0:n_P] (column-oriented back substitution).
    __device__ void trsv() {
        const int nP = s.nP;
        for (int i = tid; i < nP; i += WG) s.c[i] = p.bt[i];
        for (int j = nP - 1; j >= 0; --j) {
            __syncthreads();
            const double yj = s.c[j] / Rat(j, j);
            if (tid == 0) yv[j] = yj;
            for (int i = tid; i < j; i += WG) s.c[i] -= yj * Rat(i, j);
        }
        __syncthreads();
    }

    // a6: one inner iteration: step length, new iterate, removal set.  Leaves
    // the ascending removal positions in p.rm[0..s.q).
    __device__ void inner_step() {
#pragma clang fp contract(off)
        const int nP = s.nP;
        double al = INFINITY;
        for (int c = tid; c < nP; c += WG) {
            const double yc = yv[c];
            if (yc <= 0.0) {
                const double xc = p.x[p.P[c]];
                al = fmin(al, step_ratio(xc, yc));
            }
        }
        al = vmin(al);
        const int chunk = (nP + WG - 1) / WG;
        const int c0 = tid * chunk, c1 = min(nP, c0 + chunk);
        // the positions of a chunk are distinct columns, so a batch's loads all
        // go out before its stores (a store per position would order every
        // later gathered load behind it)
        for (int cb = c0; cb < c1; cb += LB) {
            int j[LB];
            double xc[LB], yc[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int c = min(cb + u, c1 - 1);
                j[u] = p.P[c];
                yc[u] = yv[c];
            }
#pragma unroll
            for (int u = 0; u < LB; ++u) xc[u] = p.x[j[u]];
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                if (cb + u < c1) {
                    double xn = xc[u] + al * (yc[u] - xc[u]);
                    if (yc[u] <= 0.0 && step_ratio(xc[u], yc[u]) == al) xn = 0.0;
                    if (xn <= 0.0) xn = 0.0;
                    p.x[j[u]] = xn;
                }
            }
        }
        collect_removals();
    }

    // p.rm[0..s.q) = ascending passive positions whose x is <= 0.
    __device__ void collect_removals() {
        collect_positions([&](int c, int j) { return p.x[j] <= 0.0; });
    }

    // p.rm[0..s.q) = ascending passive positions c (column j = P[c]) for which
    // pick(c, j) holds.
    template <typename Pick>
    __device__ void collect_positions(Pick pick) {
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
            for (int u = 0; u < LB; ++u) j[u] = p.P[min(cb + u, c1 - 1)];
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
                p.rm[o++] = c0 + __builtin_ctzll(mask);
                mask &= mask - 1;
            }
        } else {
            for (int c = c0; c < c1; ++c)
                if (pick(c, p.P[c])) p.rm[o++] = c;
        }
        __syncthreads();
    }

    // The inner iteration of the positivity-trick case (Section 4.2): every
    // passive position with y < 0 takes the twin of its column (the negated
    // column), whose R column is the negated one and whose least-squares
    // component is -y > 0; the residual is unchanged, so the inner loop ends.
    // Returns false, changing nothing, when a component is exactly 0 (the
    // ordinary inner iteration then runs).
    __device__ bool sign_flip() {
        const int nP = s.nP;
        int zero = 0;
        for (int c = tid; c < nP; c += WG) zero |= (yv[c] == 0.0) ? 1 : 0;
        if (imax(zero)) return false;
        collect_positions([&](int c, int j) { return yv[c] < 0.0; });
        const int q = s.q;
        for (int t = 0; t < q; ++t) {
            const int c = p.rm[t];
            double* col = p.R + (size_t)p.slot[c] * p.kc;
            for (int i = tid; i <= c; i += WG) col[i] = -col[i];
        }
        for (int t = tid; t < q; t += WG) {
            const int c = p.rm[t], j = p.P[c], tw = twin_of(p, j);
            p.P[c] = tw;
            p.pos[j] = -1;
            p.pos[tw] = c;
            p.x[j] = 0.0;
            yv[c] = -yv[c];
        }
        __syncthreads();
        return true;
    }

    // Algorithm 5: delete the passive positions p.rm[0..q) from R and restore the
    // triangle with Givens rotations, column by column, bottom-up within a
    // column; rotations are applied to R, bt and the columns of Q.
    __device__ void downdate() {
        const int q = s.q, nP = s.nP, m = p.m;
        const int first = p.rm[0];
        int ri = 0;
        for (int oc = first; oc < nP; ++oc) {
            if (ri < q && p.rm[ri] == oc) {
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
                    p.rot[2 * g] = cs;
                    p.rot[2 * g + 1] = sn;
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
                        if (p.rm[t] == oc2) {
                            del = true;
                            break;
                        }
                        if (p.rm[t] > oc2) break;
                    }
                    if (del) continue;
                    for (int i = oc, g = 0; i > c; --i, ++g) {
                        const double cs = p.rot[2 * g], sn = p.rot[2 * g + 1];
                        const double a = Rat(i - 1, oc2), bb = Rat(i, oc2);
                        Rat(i - 1, oc2) = cs * a + sn * bb;
                        Rat(i, oc2) = -sn * a + cs * bb;
                    }
                }
            }
            if (tid == 0) {
                for (int i = oc, g = 0; i > c; --i, ++g) {
                    const double cs = p.rot[2 * g], sn = p.rot[2 * g + 1];
                    const double a = p.bt[i - 1], bb = p.bt[i];
                    p.bt[i - 1] = cs * a + sn * bb;
                    p.bt[i] = -sn * a + cs * bb;
                }
            }
            for (int row = tid; row < m; row += WG) {
                for (int i = oc, g = 0; i > c; --i, ++g) {
                    const double cs = p.rot[2 * g], sn = p.rot[2 * g + 1];
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
    __device__ void compact() {
        const int q = s.q, nP = s.nP;
        if (q == 0) return;
        int* oldP = p.itmp;
        int* oldS = p.itmp + p.kc;
        // the int arrays may alias as far as the compiler knows: each batch's
        // loads go out before its stores, instead of one round trip per position
        for (int c0 = tid; c0 < nP; c0 += WG * LB) {
            int pv[LB], sv[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int c = min(c0 + WG * u, nP - 1);
                pv[u] = p.P[c];
                sv[u] = p.slot[c];
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
                    if (p.rm[mid] < c) lo = mid + 1;
                    else hi = mid;
                }
                const int j = pv[u];
                if (lo < q && p.rm[lo] == c) {
                    p.pos[j] = -1;
                    p.slot[nP - q + lo] = sv[u];
                } else {
                    const int w = c - lo;
                    p.P[w] = j;
                    p.slot[w] = sv[u];
                    p.pos[j] = w;
                }
            }
        }
        __syncthreads();
        if (tid == 0) s.nP = nP - q;
        __syncthreads();
    }

    // a7: r = b - A_P x_P
    __device__ void residual() {
        const int m = p.m, nP = s.nP;
        for (int i = tid; i < m; i += WG) {
            double acc = p.b[i];
            for (int c = 0; c < nP; ++c) {
                double sg;
                const double* a = col_ptr(p, p.P[c], sg);
                acc -= (sg * a[i]) * yv[c];
            }
            p.r[i] = acc;
        }
        __syncthreads();
    }

    // a7: w = A^T r and the update of u2 = ||Q_perp^T a_j||^2:
    //   u2 <- u2 - sum_added (q^T a)^2 + sum_dropped (q^T a)^2,
    // or exactly from the trailing columns of Q when they are fewer.
    __device__ void dual_and_norms(int kadd) {
        const int m = p.m, nph = p.nph, nP = s.nP, nPa = s.nPa;
        const int ndrop = nPa - nP;
        const bool exact = (m - nP) <= kadd + ndrop;
        const bool tw = nph != p.n;
        for (int j = wid; j < nph; j += NW) {
            const double* a = Acol(j);
            double acc = 0.0;
            for (int i = lane; i < m; i += 64) acc += a[i] * p.r[i];
            const double wj = wave_sum(acc);
            double u2;
            if (exact) {
                u2 = 0.0;
                for (int t = nP; t < m; ++t) {
                    double d = 0.0;
                    for (int i = lane; i < m; i += 64) d += a[i] * Qat(i, t);
                    d = wave_sum(d);
                    u2 += d * d;
                }
            } else {
                u2 = p.u2[j];
                for (int t = 0; t < kadd; ++t) {
                    double d = 0.0;
                    const double* qa = p.Qadd + (size_t)t * m;
                    for (int i = lane; i < m; i += 64) d += a[i] * qa[i];
                    d = wave_sum(d);
                    u2 -= d * d;
                }
                for (int t = nP; t < nPa; ++t) {
                    double d = 0.0;
                    for (int i = lane; i < m; i += 64) d += a[i] * Qat(i, t);
                    d = wave_sum(d);
                    u2 += d * d;
                }
                u2 = fmax(u2, 0.0);
                if (p.pos[j] < 0 && !twin_passive(p, j) && u2 < RECOMP_FRAC * p.an2[j]) {
                    u2 = 0.0;
                    for (int t = nP; t < m; ++t) {
                        double d = 0.0;
                        for (int i = lane; i < m; i += 64) d += a[i] * Qat(i, t);
                        d = wave_sum(d);
                        u2 += d * d;
                    }
                }
            }
            if (lane == 0) {
                p.w[j] = wj;
                p.u2[j] = u2;
                if (tw) {
                    p.w[j + nph] = -wj;
                    p.u2[j + nph] = u2;
                }
            }
        }
        __syncthreads();
    }

    // r and w for the current x (used when the loop stops inside an inner loop)
    __device__ void refresh_dual() {
        const int m = p.m, nph = p.nph;
        for (int i = tid; i < m; i += WG) {
            double acc = p.b[i];
            for (int c = 0; c < s.nP; ++c) {
                const int j = p.P[c];
                double sg;
                const double* a = col_ptr(p, j, sg);
                acc -= (sg * a[i]) * p.x[j];
            }
            p.r[i] = acc;
        }
        __syncthreads();
        for (int j = wid; j < nph; j += NW) {
            const double* a = Acol(j);
            double acc = 0.0;
            for (int i = lane; i < m; i += 64) acc += a[i] * p.r[i];
            acc = wave_sum(acc);
            if (lane == 0) {
                p.w[j] = acc;
                if (nph != p.n) p.w[j + nph] = -acc;
            }
        }
        __syncthreads();
    }

    __device__ void finalize() {
        const int n = p.n, m = p.m, nP = s.nP;
        double vz = 0.0, vp = 0.0;
        for (int j = tid; j < n; j += WG) {
            const double wj = p.w[j];
            if (p.pos[j] >= 0) vp = fmax(vp, fabs(wj));
            else vz = fmax(vz, fmax(wj, 0.0));
            if (p.passive) p.passive[j] = (j < nP) ? p.P[j] : -1;
        }
        vz = vmax(vz);
        vp = vmax(vp);
        double rr = 0.0;
        for (int i = tid; i < m; i += WG) rr += p.r[i] * p.r[i];
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
            inf.reserved = 0;
            inf.kkt_residual = fmax(vz, vp) / scale;
            inf.objective = rr;
            *p.info = inf;
        }
        __syncthreads();
    }

    // ---------------- the whole solve ----------------
    __device__ void run() {
        init();
        if (s.status == LHDM_STATUS_NONFINITE) {
            finalize();
            return;
        }
        while (true) {
            select();
            if (s.done) break;
            const int ncol = s.ncol;
            project(ncol);
            if (ncol > 1) {
                deviation_maximization();
            } else {
                if (tid == 0) s.k = 1;
                __syncthreads();
            }
            if (tid == 0) s.kr = s.k;
            __syncthreads();
            panel_qr();
            if (s.kr > 1) form_wy();
            else {
                // one reflector: V = [0; 1; v], T = tau
                const int m = p.m, r0 = s.nP;
                for (int i = tid; i < m; i += WG) p.V[i] = (i < r0) ? 0.0 : p.G[i];
                if (tid == 0) p.T[0] = s.tau[0];
                __syncthreads();
            }
            append_r();
            update_q();
            const int j1 = s.J[0];
            jloop();
            const int k = s.k;
            if (k == 0) {
                if (tid == 0) {
                    p.excl[j1] = 1;
                    s.any_excl = 1;
                }
                __syncthreads();
                continue;
            }
            if (s.any_excl) {
                for (int j = tid; j < p.n; j += WG) p.excl[j] = 0;
                __syncthreads();
                if (tid == 0) s.any_excl = 0;
            }
            // passive set grows by J, in order
            const int m = p.m, r0 = s.nP;
            for (int t = 0; t < k; ++t)
                for (int i = tid; i < m; i += WG) p.Qadd[(size_t)t * m + i] = Qat(i, r0 + t);
            if (tid == 0) {
                for (int t = 0; t < k; ++t) {
                    p.P[r0 + t] = s.J[t];
                    p.pos[s.J[t]] = r0 + t;
                }
                s.nP = r0 + k;
                s.nPa = r0 + k;
                s.outer += 1;
            }
            __syncthreads();
            trsv();
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
            if (stop) {
                if (tid == 0) s.status = LHDM_STATUS_MAXITER;
                __syncthreads();
                refresh_dual();
                break;
            }
            for (int c = tid; c < s.nP; c += WG) p.x[p.P[c]] = yv[c];
            __syncthreads();
            residual();
            dual_and_norms(k);
        }
        finalize();
    }
};

}  // namespace lhdm
