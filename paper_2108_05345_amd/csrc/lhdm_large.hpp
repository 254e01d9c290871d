// Large-instance engine: one instance spread over the whole GPU.
//
// The outer/inner loops of Algorithm 3 run on the host; every step runs in a
// kernel.  Bandwidth- and FLOP-heavy steps are multi-workgroup kernels:
//   * lg_colmat_dot  -- X^T D for a column-major X and a few vectors D, on the
//                       FP64 matrix cores (v_mfma_f64_16x16x4f64).  Used for the
//                       dual w = A^T r fused with the update of the projected
//                       column norms, and for the candidate projection Q^T A_J.
//   * lg_qup1/2      -- Q[:, n_P:m] <- Q[:, n_P:m] (I - V T V^T) (compact WY).
//   * lg_trsv        -- R y = (Q^T b)[:n_P], row blocks chained by device flags.
//   * lg_givens      -- Algorithm 5 on R: column blocks chained by device flags.
//   * lg_qrot        -- the same rotations applied to the columns of Q.
//   * lg_residual    -- r = b - A_P x_P.
// The selection, deviation maximization, panel factorisation, feasibility
// loop on J and the step length run in single-workgroup kernels that reuse
// the workgroup engine's step functions on the shared control block Ctl.
#pragma once

#include <climits>
#include <cstddef>
#include <type_traits>
#include <vector>

#include "lhdm_device.hpp"
#include "lhdm_host.hpp"
#include "lhdm_wg.hpp"

namespace lhdm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef unsigned long long u64;

constexpr int TB = 64;          // rows per block of the chained triangular solve
constexpr int GB = 64;          // new columns per block of the chained downdate
constexpr int RQ = 64;          // largest number of removals handled in one downdating sweep
constexpr int RES_CHUNKS = 64;  // column chunks of the residual kernel
constexpr long long SPIN_LIMIT = 1LL << 21;   // bounded waits: ~2 s of polling, far beyond any chain

struct LgExtra {
    int inner_done;   // set by lg_inner: no more inner iterations this outer step
    int restart;      // the outer step appended nothing (feasibility loop emptied J)
    int err;          // a chained kernel gave up waiting (should never happen)
    int first;        // first removed position of the current downdate
    int ndown;        // number of new columns from `first` on
    int totrot;       // rotations of the current downdate
    int cfok;         // epoch of the last downdate done in closed form
    int nrecomp;      // columns flagged for an exact norm recomputation
    int nvec;         // vectors of the dual update (r, added, dropped or trailing)
    int kadd;         // added directions in the dual update
    int exact;        // 1: norms recomputed from the trailing columns of Q
    int pending;      // removals left over from a sweep capped at RQ positions
    int gident;       // 1: every candidate of the outer step was accepted
    int ccount;       // candidates collected by the selection (may exceed CAND_CAP)
    int cq_ok;        // 1: this outer step's panel is factored by CholeskyQR2 (lg_cq_*)
    int ncq;          // panels factored by CholeskyQR2 so far
    int gmap[KM];     // candidate panel column of accepted column q
    int seg_start[RQ + 1];
    int seg_off[RQ + 1];
};

// Host copy of the control block and of the head of LgExtra.  The kernels
// that end with a host decision write it into fine-grained pinned host memory
// and then store `seq`, which the host polls.
constexpr size_t CTL_SPAN = (sizeof(Ctl) + 255) / 256 * 256;
constexpr int EX_HEAD = 16;   // ints of LgExtra mirrored (inner_done .. gident and more)
struct Mirror {
    union {
        Ctl ctl;
        char raw[CTL_SPAN];
    };
    int ex_head[EX_HEAD];
    int seq;
};
static_assert(sizeof(LgExtra) >= EX_HEAD * sizeof(int), "mirrored head of LgExtra");

struct LgArgs {
    Prob p;
    DevParams prm;
    Ctl* ctl;
    LgExtra* ex;
    double* Dt;       // m x 64 row-major vectors for lg_colmat_dot
    double* rotbuf;   // 2 * kc * RQ rotation pairs
    int* ocol;        // kc: old logical column of each new column of the downdate
    int* lcnt;        // kc: rotations of each new column
    int* roff;        // kc: offset of its rotations
    u64* yll;         // 2 * kc : y published by the chained triangular solve
    u64* rotll;       // 4 * kc * RQ : rotations published by the chained downdate
    int* recomp;      // n: columns whose projected norm is recomputed exactly
    double* rpart;    // RES_CHUNKS * m residual partial sums
    double* gpart;    // partial Gram matrices (max(ceil(m / GRAM_ROWS), PNW) blocks of 64 x 64)
    double* selv;     // 3 * NSEL partial maxima of the selection
    int* seli;        // NSEL partial argmax indices
    double* candw;    // CAND_CAP: collected candidates' dual values
    int* candi;       // CAND_CAP: and column indices
    u64* pll;         // 2 * (2 PNW + 2) x (KM + 1) : panel partials (dots, pivot row)
    double* wpart;    // ceil(m / QCB) x kq x m : pass-1 partial products of the Q update
    double* cq;       // CQ_DOUBLES: small factors of the CholeskyQR2 panel (R1, U R2, Y1, z)
    Mirror* hmir;     // device view of the host mirror
};

// --------------------------------------------------------------------------
// helpers
// --------------------------------------------------------------------------
__device__ inline void ctl_load(WgShared& s, const Ctl* g) {
    int* d = reinterpret_cast<int*>(static_cast<Ctl*>(&s));
    const int* src = reinterpret_cast<const int*>(g);
    constexpr int NI = (int)(sizeof(Ctl) / sizeof(int));
    const int bd = blockDim.x;
    // two words per thread and step, both loads before either store: one
    // memory round trip for the whole block at 256 threads
    for (int i = threadIdx.x; i < NI; i += 2 * bd) {
        const bool two = i + bd < NI;
        const int v0 = src[i], v1 = two ? src[i + bd] : 0;
        d[i] = v0;
        if (two) d[i + bd] = v1;
    }
    __syncthreads();
}

__device__ inline void ctl_store(const WgShared& s, Ctl* g) {
    __syncthreads();
    const int* src = reinterpret_cast<const int*>(static_cast<const Ctl*>(&s));
    int* d = reinterpret_cast<int*>(g);
    for (int i = threadIdx.x; i < (int)(sizeof(Ctl) / sizeof(int)); i += blockDim.x) d[i] = src[i];
    __syncthreads();
}

// Copy the scalar head of the control block (the fields before its arrays,
// all the host reads) and the head of LgExtra to the host mirror with
// system-scope stores, then store the sequence number `seq` (release, system
// scope).  Called by every thread of a single-workgroup kernel as its last step.
__device__ inline void publish(const LgArgs& a, int seq) {
    __syncthreads();
    __threadfence();   // the workgroup's global writes of ctl and ex, before the reads below
    constexpr int NC = (int)(offsetof(Ctl, J) / sizeof(int));
    const int* sc = reinterpret_cast<const int*>(a.ctl);
    const int* se = reinterpret_cast<const int*>(a.ex);
    int* dc = reinterpret_cast<int*>(&a.hmir->ctl);
    int* de = a.hmir->ex_head;
    for (int i = threadIdx.x; i < NC + EX_HEAD; i += blockDim.x) {
        if (i < NC) __hip_atomic_store(dc + i, sc[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        else __hip_atomic_store(de + (i - NC), se[i - NC], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(&a.hmir->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Low-latency hand-off: a double travels as two 8-byte words {32-bit half,
// epoch}, each stored and loaded as one single-copy-atomic system-scope access.
// A consumer polls the data itself until both halves carry the current epoch,
// so no separate flag, store-completion wait or atomic counter is needed.
// Epochs start at 1 and never repeat on a buffer (buffers are cleared when a
// workspace is first used).
__device__ inline void ll_put(u64* slot, double v, int epoch) {
    const u64 bits = (u64)__double_as_longlong(v);
    const u64 e = ((u64)(unsigned)epoch) << 32;
    __hip_atomic_store(slot, e | (bits & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(slot + 1, e | (bits >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ inline bool ll_try(const u64* slot, int epoch, double& v) {
    const u64 w0 = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    const u64 w1 = __hip_atomic_load(slot + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    const unsigned e = (unsigned)epoch;
    if ((unsigned)(w0 >> 32) != e || (unsigned)(w1 >> 32) != e) return false;
    v = __longlong_as_double((long long)((w1 << 32) | (w0 & 0xffffffffull)));
    return true;
}

// Wave-uniform: every lane with `need` waits for its value (bounded wait).
// A wave whose value is not yet on the critical path (URGENT false) polls
// eight times less often, which keeps the many consumers of one published
// block from crowding out the one that is waiting for it next.
template <bool URGENT = true>
__device__ inline double ll_get(const u64* slot, bool need, int epoch, int* err) {
    double v = 0.0;
    bool ok = !need;
    long long it = 0;
    while (true) {
        if (!ok) ok = ll_try(slot, epoch, v);
        if (__all(ok)) break;
        if (++it > SPIN_LIMIT) {
            if ((threadIdx.x & 63) == 0) atomicExch(err, 1);
            break;
        }
        if (URGENT) __builtin_amdgcn_s_sleep(1);
        else __builtin_amdgcn_s_sleep(8);
    }
    return v;
}

__device__ inline double ll_get_u(const u64* slot, bool need, int epoch, int* err, bool urgent) {
    return urgent ? ll_get<true>(slot, need, epoch, err) : ll_get<false>(slot, need, epoch, err);
}

// Wave-uniform: one lane polls a single word (the last one a producer writes)
// until it carries `epoch`, at a low rate (bounded wait).  Consumers that are
// not on the critical path wait here before reading the whole block, so that
// the uncached polling traffic of many waiting waves stays small.
__device__ inline void ll_wait_word(const u64* word, int epoch, int* err) {
    long long it = 0;
    while (true) {
        bool ok = true;
        if ((threadIdx.x & 63) == 0)
            ok = (unsigned)(__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) >> 32) ==
                 (unsigned)epoch;
        if (__all(ok)) break;
        if (++it > SPIN_LIMIT) {
            if ((threadIdx.x & 63) == 0) atomicExch(err, 1);
            break;
        }
        __builtin_amdgcn_s_sleep(8);
    }
}

// --------------------------------------------------------------------------
// initialisation
// --------------------------------------------------------------------------
// w = A^T b, ||a_j||^2, and the per-column state; one wave per column of the
// caller's A (with its twin -a_j in the positivity-trick mode).
__global__ __launch_bounds__(WG) void lg_init_cols(LgArgs a, unsigned long long* anmax_bits, int* bad) {
    const Prob& p = a.p;
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * NW + wave_index();
    if (j >= p.nph) return;
    const double* col = p.A + (size_t)j * p.lda;
    double ab = 0.0, aa = 0.0;
    for (int i = lane; i < p.m; i += 64) {
        const double v = col[i];
        ab += v * p.b[i];
        aa += v * v;
    }
    ab = wave_sum(ab);
    aa = wave_sum(aa);
    if (lane == 0) {
        p.w[j] = ab;
        p.an2[j] = aa;
        p.u2[j] = aa;
        p.pos[j] = -1;
        p.excl[j] = 0;
        p.x[j] = 0.0;
        if (p.nph != p.n) {
            const int t = j + p.nph;
            p.w[t] = -ab;
            p.an2[t] = aa;
            p.u2[t] = aa;
            p.pos[t] = -1;
            p.excl[t] = 0;
            p.x[t] = 0.0;
        }
        if (!isfinite(ab) || !isfinite(aa)) atomicOr(bad, 1);
        else atomicMax(anmax_bits, (unsigned long long)__double_as_longlong(aa));
    }
}

__global__ __launch_bounds__(WG) void lg_fill_identity(double* Q, int m) {
    const size_t mm = (size_t)m * m;
    for (size_t e = (size_t)blockIdx.x * WG + threadIdx.x; e < mm; e += (size_t)gridDim.x * WG)
        Q[e] = ((e % m) == (e / m)) ? 1.0 : 0.0;
}

__global__ __launch_bounds__(WG) void lg_init_ctl(LgArgs a, const unsigned long long* anmax_bits, const int* bad) {
    __shared__ WgShared s;
    Prob p = a.p;
    Wg wg(p, a.prm, s);
    double bb = 0.0;
    for (int i = threadIdx.x; i < p.m; i += WG) {
        const double v = p.b[i];
        bb += v * v;
        p.bt[i] = v;
        p.r[i] = v;
    }
    bb = wg.sum(bb);
    for (int c = threadIdx.x; c < p.kc; c += WG) p.slot[c] = c;
    if (threadIdx.x == 0) {
        const double anmax = __longlong_as_double((long long)*anmax_bits);
        s.anmax = sqrt(anmax);
        s.bnorm = sqrt(bb);
        s.tol_w = a.prm.kkt_tol * s.anmax * s.bnorm;
        s.nP = 0;
        s.status = (*bad || !isfinite(bb)) ? LHDM_STATUS_NONFINITE : LHDM_STATUS_OK;
        s.outer = s.inner = s.jdrops = 0;
        s.any_excl = 0;
        s.done = (s.status != LHDM_STATUS_OK);
        s.k = 0;
        s.kr = 0;
        a.ex->err = 0;
        a.ex->nrecomp = 0;
        a.ex->cq_ok = 0;
        a.ex->ncq = 0;
        a.ex->cfok = 0;
    }
    ctl_store(s, a.ctl);
}

// --------------------------------------------------------------------------
// single-workgroup steps
// --------------------------------------------------------------------------
// Selection, pass 1: per-workgroup partial maxima over a slice of the columns
// (max_Z w, max_Z u, best eligible (w, index)).
constexpr int NSEL = 64;   // workgroups of the first selection pass

__global__ __launch_bounds__(WG) void lg_sel_part(LgArgs a, double* pv, int* pi) {
    const Prob& p = a.p;
    __shared__ double sd[3][NW];
    __shared__ int si[NW];
    const int n = p.n, lane = threadIdx.x & 63, wv = wave_index();
    const int per = (n + NSEL - 1) / NSEL;
    const int j0 = blockIdx.x * per, j1 = min(n, j0 + per);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ex->ccount = 0;
    double mwz = -INFINITY, mu = 0.0, bv = -INFINITY;
    int bi = INT_MAX;
    for (int j = j0 + threadIdx.x; j < j1; j += WG) {
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
    mwz = wave_max(mwz);
    mu = wave_max(mu);
    wave_argmax(bv, bi);
    if (lane == 0) {
        sd[0][wv] = mwz;
        sd[1][wv] = mu;
        sd[2][wv] = bv;
        si[wv] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NW; ++w) {
            mwz = fmax(mwz, sd[0][w]);
            mu = fmax(mu, sd[1][w]);
            if (better(sd[2][w], si[w], bv, bi)) {
                bv = sd[2][w];
                bi = si[w];
            }
        }
        mwz = fmax(sd[0][0], mwz);
        mu = fmax(sd[1][0], mu);
        if (better(sd[2][0], si[0], bv, bi)) {
            bv = sd[2][0];
            bi = si[0];
        }
        pv[3 * blockIdx.x + 0] = mwz;
        pv[3 * blockIdx.x + 1] = mu;
        pv[3 * blockIdx.x + 2] = bv;
        pi[blockIdx.x] = bi;
    }
}

// Selection, pass 2 (NSEL workgroups): Deviation Maximization's candidate
// filter (a2).  Every workgroup reduces the partial maxima of pass 1 (the same
// exact maxima everywhere), then appends the columns of its range passing
// w_j >= tau1 max w and u_j >= tau2 max u to a global list (order immaterial:
// pass 3 ranks them).
constexpr int CAND_CAP = 2048;

__global__ __launch_bounds__(WG) void lg_sel_cand(LgArgs a, const double* pv, const int* pi) {
    const Prob& p = a.p;
    const DevParams& prm = a.prm;
    __shared__ double red[2];
    __shared__ int redi;
    const int tid = threadIdx.x, lane = tid & 63;
    if (tid < 64) {
        double mu = 0.0, bv = -INFINITY;
        int bi = INT_MAX;
        for (int g = lane; g < NSEL; g += 64) {
            mu = fmax(mu, pv[3 * g + 1]);
            if (better(pv[3 * g + 2], pi[g], bv, bi)) {
                bv = pv[3 * g + 2];
                bi = pi[g];
            }
        }
        mu = wave_max(mu);
        wave_argmax(bv, bi);
        if (lane == 0) {
            red[0] = mu;
            red[1] = bv;
            redi = bi;
        }
    }
    __syncthreads();
    const double mu = red[0], bv = red[1];
    const int bi = redi;
    if (bi == INT_MAX || p.m - a.ctl->nP <= 1) return;
    const double tw = prm.tau1 * bv, tu = prm.tau2 * mu;
    const int per = (p.n + NSEL - 1) / NSEL;
    const int j0 = blockIdx.x * per, j1 = min(p.n, j0 + per);
    for (int j = j0 + tid; j < j1; j += WG) {
        const int ps = p.pos[j], ex = p.excl[j];
        const double wj = p.w[j], u2 = p.u2[j], an2 = p.an2[j];
        if (ps >= 0 || ex || j == bi || !(wj >= tw)) continue;
        const double u = sqrt(fmax(u2, 0.0));
        if (!(u >= tu) || !(u > DEP_TOL * sqrt(an2)) || twin_passive(p, j)) continue;
        const int slot = atomicAdd(&a.ex->ccount, 1);
        if (slot < CAND_CAP) {
            a.candw[slot] = wj;
            a.candi[slot] = j;
        }
    }
}

// The first kmax - 1 of cnt (> 256) collected candidates in (w desc, index
// asc) order without sorting them all: w is mapped to SEL_NBK buckets by a map
// that is monotone in w (rounding included), a histogram gives the first
// bucket at which the running count reaches kmax - 1, and only the candidates
// in that bucket and above are ranked.  Every wanted candidate, and every
// candidate better than one of them, lies there, so the ranks within that
// short list are the ranks among all.  Returns false (nothing placed) when
// the short list would exceed SEL_SL (clustered values) or the map is
// degenerate; the caller then sorts the whole list.
constexpr int SEL_NBK = 256;
constexpr int SEL_SL = 256;

__device__ __forceinline__ int sel_bucket(double w, double bv, double scale) {
    const double z = (bv - w) * scale;
    return (z >= (double)(SEL_NBK - 1)) ? SEL_NBK - 1 : ((z > 0.0) ? (int)z : 0);
}

__device__ bool top_by_histogram(const LgArgs& a, WgShared& s, double* cw, int* ci, int cnt, double bv) {
    __shared__ int hist[SEL_NBK];
    __shared__ double lw[SEL_SL];
    __shared__ int li[SEL_SL];
    __shared__ int shB, shN;
    const int K = a.prm.kmax - 1, tid = threadIdx.x;
    const double scale = SEL_NBK / (bv - a.prm.tau1 * bv);
    if (!(K < cnt && K <= SEL_SL && scale > 0.0 && scale < INFINITY)) return false;   // uniform
    for (int e = tid; e < cnt; e += WG) {
        cw[e] = a.candw[e];
        ci[e] = a.candi[e];
    }
    for (int t = tid; t < SEL_NBK; t += WG) hist[t] = 0;
    if (tid == 0) shN = 0;
    __syncthreads();
    for (int e = tid; e < cnt; e += WG) atomicAdd(&hist[sel_bucket(cw[e], bv, scale)], 1);
    __syncthreads();
    if (tid < 64) {
        constexpr int PL = SEL_NBK / 64;   // buckets per lane
        int h[PL], sum = 0;
#pragma unroll
        for (int u = 0; u < PL; ++u) {
            h[u] = hist[tid * PL + u];
            sum += h[u];
        }
        int inc = sum;   // inclusive scan of the lane sums (every lane takes part)
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int o = __shfl_up(inc, d, 64);
            if (tid >= d) inc += o;
        }
        int run = inc - sum, bk = SEL_NBK;
#pragma unroll
        for (int u = 0; u < PL; ++u) {
            run += h[u];
            if (run >= K && bk == SEL_NBK) bk = tid * PL + u;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) bk = min(bk, __shfl_xor(bk, o, 64));
        if (tid == 0) shB = bk;   // < SEL_NBK: all cnt > K candidates are counted
    }
    __syncthreads();
    const int B = shB;
    for (int e = tid; e < cnt; e += WG) {
        if (sel_bucket(cw[e], bv, scale) <= B) {
            const int sl = atomicAdd(&shN, 1);
            if (sl < SEL_SL) {
                lw[sl] = cw[e];
                li[sl] = ci[e];
            }
        }
    }
    __syncthreads();
    const int nl = shN;
    if (nl > SEL_SL) return false;   // uniform
    for (int e = tid; e < nl; e += WG) {
        const double we = lw[e];
        const int je = li[e];
        int r = 0;
        for (int f = 0; f < nl; ++f) r += better(lw[f], li[f], we, je) ? 1 : 0;
        if (r < K) s.J[1 + r] = je;
    }
    return true;
}

// Selection, pass 3 (one workgroup): termination test (a1) and the first
// kmax - 1 collected candidates in (w desc, index asc) order, each placed by
// its rank among the collected ones.  More than CAND_CAP candidates falls back
// to passes over memory.
__global__ __launch_bounds__(WG) void lg_sel_main(LgArgs a, const double* pv, const int* pi, int pub) {
    __shared__ WgShared s;
    __shared__ double cw[CAND_CAP];
    __shared__ int ci[CAND_CAP];
    ctl_load(s, a.ctl);
    Wg wg(a.p, a.prm, s);
    const Prob& p = a.p;
    const DevParams& prm = a.prm;
    double mwz = -INFINITY, mu = 0.0, bv = -INFINITY;
    int bi = INT_MAX;
    for (int g = threadIdx.x; g < NSEL; g += WG) {
        mwz = fmax(mwz, pv[3 * g]);
        mu = fmax(mu, pv[3 * g + 1]);
        if (better(pv[3 * g + 2], pi[g], bv, bi)) {
            bv = pv[3 * g + 2];
            bi = pi[g];
        }
    }
    mwz = wg.vmax(mwz);
    mu = wg.vmax(mu);
    wg.argmax(bv, bi);
    const int cap = p.m - s.nP;
    __syncthreads();
    if (threadIdx.x == 0) {
        s.done = 0;
        s.ncol = 1;
        s.J[0] = bi;
        s.nP0 = s.nP;
        if (mwz == -INFINITY || mwz <= s.tol_w) {
            s.done = 1;
        } else if (bi == INT_MAX || bv <= s.tol_w) {
            s.done = 1;
            s.status = LHDM_STATUS_RANK;
        } else if (s.outer >= prm.max_outer) {
            s.done = 1;
            s.status = LHDM_STATUS_MAXITER;
        }
    }
    __syncthreads();
    if (!(s.done || prm.lh || prm.kmax <= 1 || cap <= 1)) {
        const int cnt = a.ex->ccount;
        if (cnt > CAND_CAP) {
            wg.select();   // rare: many candidates -> passes over memory
        } else {
            if (cnt <= 256) {
                for (int e = threadIdx.x; e < cnt; e += WG) {
                    cw[e] = a.candw[e];
                    ci[e] = a.candi[e];
                }
                __syncthreads();
                for (int e = threadIdx.x; e < cnt; e += WG) {
                    const double we = cw[e];
                    const int je = ci[e];
                    int r = 0;
                    for (int f = 0; f < cnt; ++f) r += better(cw[f], ci[f], we, je) ? 1 : 0;
                    if (r < prm.kmax - 1) s.J[1 + r] = je;
                }
            } else if (!top_by_histogram(a, s, cw, ci, cnt, bv)) {
                // bitonic sort of the padded list, best first
                int nn = 512;
                while (nn < cnt) nn <<= 1;
                for (int e = threadIdx.x; e < nn; e += WG) {
                    cw[e] = (e < cnt) ? a.candw[e] : -INFINITY;
                    ci[e] = (e < cnt) ? a.candi[e] : INT_MAX;
                }
                __syncthreads();
                for (int k = 2; k <= nn; k <<= 1) {
                    for (int jj = k >> 1; jj > 0; jj >>= 1) {
                        for (int e = threadIdx.x; e < nn; e += WG) {
                            const int l = e ^ jj;
                            if (l > e) {
                                const bool first_better = better(cw[e], ci[e], cw[l], ci[l]);
                                const bool want_first = (e & k) == 0;   // this run sorts best first
                                if (first_better != want_first) {
                                    const double tw = cw[e];
                                    const int ti = ci[e];
                                    cw[e] = cw[l];
                                    ci[e] = ci[l];
                                    cw[l] = tw;
                                    ci[l] = ti;
                                }
                            }
                        }
                        __syncthreads();
                    }
                }
                for (int r = threadIdx.x; r < min(cnt, prm.kmax - 1); r += WG) s.J[1 + r] = ci[r];
            }
            if (threadIdx.x == 0) s.ncol = 1 + min(cnt, prm.kmax - 1);
        }
    }
    if (threadIdx.x == 0) s.nP0 = s.nP;
    ctl_store(s, a.ctl);
    publish(a, pub);
}

// Dt[row * 64 + t] = A[row, J[t]] (t < ncol), zero-padded to 64 columns.
// Vector block element (row, t) -> Dt index: row-major (ldd 64) or the pair
// layout of the pipelined column-block kernel.
__device__ __forceinline__ void dt_coords(size_t e, int pair, int& row, int& t) {
    if (pair) {
        row = (int)(e / 128) * 2 + (int)(e & 1);
        t = (int)((e / 2) % 64);
    } else {
        row = (int)(e / 64);
        t = (int)(e % 64);
    }
}
__global__ __launch_bounds__(WG) void lg_gather_cand(LgArgs a, int pair) {
    if (a.ctl->done) return;   // launched before the host reads the selection
    const Prob& p = a.p;
    const int nc = a.ctl->ncol, m = p.m;
    const size_t tot = (size_t)(pair ? (m + 1) / 2 * 2 : m) * 64;
    for (size_t e = (size_t)blockIdx.x * WG + threadIdx.x; e < tot; e += (size_t)gridDim.x * WG) {
        int row, t;
        dt_coords(e, pair, row, t);
        double v = 0.0;
        if (t < nc && row < m) {
            double sg;
            const double* col = col_ptr(p, a.ctl->J[t], sg);
            v = sg * col[row];
        }
        a.Dt[e] = v;
    }
}

// Partial Gram matrix of X[r0:m, 0:c] (column-major, ld m) over row blocks of
// GRAM_ROWS rows, on the matrix cores; symmetric tiles ti <= tj only.  which = 0: the
// projected candidates (G, c = ncol); which = 1: the reflectors (V, c = kr).
constexpr int GRAM_ROWS = 128;   // rows per workgroup of the partial Gram
// Layout of a partial Gram block (at most 64 x 64, symmetric): its upper 16 x
// 16 tiles (ti <= tj), each stored whole and row-major in 256 consecutive
// doubles, tile (ti, tj) at position tj (tj + 1) / 2 + ti, so a matrix of up
// to 16 c columns occupies the first c (c + 1) / 2 tiles.
constexpr int GP_TILE = 256;
constexpr int GP_STRIDE = 10 * GP_TILE;   // doubles per block (64 columns: ten tiles)
__device__ __forceinline__ int gp_tile(int ti, int tj) { return tj * (tj + 1) / 2 + ti; }

// Partial Gram X^T X over one block of GRAM_ROWS rows of the trailing part
// (rows >= n_P): X = G (projected candidates, which = 0) or V (reflectors,
// which = 1), c columns.  The block is staged in LDS with coalesced loads
// (columns past c are zero); each wave takes upper 16 x 16 tiles and runs two
// independent MFMA accumulators over the block.  Block blk writes its tiles
// to part + blk GP_STRIDE in the partial-Gram layout.
__global__ __launch_bounds__(WG) void lg_gram_part(LgArgs a, int which, double* part) {
    __shared__ double xs[GRAM_ROWS][KM + 1];
    const Ctl* ctl = a.ctl;
    const Prob& p = a.p;
    const int r0 = ctl->nP, m = p.m;
    const int c = which ? ctl->kr : ctl->ncol;
    const double* X = which ? p.V : p.G;
    const int rs = r0 + blockIdx.x * GRAM_ROWS;
    if (rs >= m || c <= 0) return;
    const int nr = min(m, rs + GRAM_ROWS) - rs;
    const int tid = threadIdx.x, lane = tid & 63, wv = wave_index();
    const int nt = (c + 15) / 16;
    for (int e = tid; e < GRAM_ROWS * nt * 16; e += WG) {
        const int q = e / GRAM_ROWS, i = e % GRAM_ROWS;
        xs[i][q] = (i < nr && q < c) ? X[(size_t)q * m + rs + i] : 0.0;
    }
    __syncthreads();
    double* out = part + (size_t)blockIdx.x * GP_STRIDE;
    int tile = 0;
    for (int ti = 0; ti < nt; ++ti)
        for (int tj = ti; tj < nt; ++tj, ++tile) {
            if ((tile % NW) != wv) continue;
            d4 acc0 = d4{0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
            const int ca = ti * 16 + (lane & 15), cb = tj * 16 + (lane & 15), g = lane >> 4;
#pragma unroll 4
            for (int r = 0; r < GRAM_ROWS; r += 8) {
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[r + g][ca], xs[r + g][cb], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[r + 4 + g][ca], xs[r + 4 + g][cb], acc1, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v)
                out[gp_tile(ti, tj) * GP_TILE + (4 * v + (lane >> 4)) * 16 + (lane & 15)] = acc0[v] + acc1[v];
        }
}

// The upper triangle (i <= j < n, n <= 64) of an n x n Gram matrix from its
// nblk partial blocks (the partial-Gram layout, GP_STRIDE apart), each entry
// the sum of the blocks in block order (from 0.0, block 0 first), handed to
// put(i, j, value).  Thread p takes position p of every tile: GU_T tiles of
// GU_B blocks are loaded together (coalesced, one memory round trip), so n <=
// 32 with nblk <= 32 takes one round trip.
constexpr int GU_T = 3, GU_B = 32;
template <typename Put>
__device__ inline void gram_upper(const double* part, int nblk, int n, Put put) {
    const int p = threadIdx.x, pr = p >> 4, pc = p & 15;
    const int nt = (n + 15) / 16, ntile = nt * (nt + 1) / 2;
    for (int k0 = 0; k0 < ntile; k0 += GU_T) {
        double acc[GU_T];
#pragma unroll
        for (int e = 0; e < GU_T; ++e) acc[e] = 0.0;
        for (int b0 = 0; b0 < nblk; b0 += GU_B) {
            double v[GU_T][GU_B];
#pragma unroll
            for (int e = 0; e < GU_T; ++e)
#pragma unroll
                for (int bb = 0; bb < GU_B; ++bb)
                    v[e][bb] = (k0 + e < ntile && b0 + bb < nblk)
                                   ? part[(size_t)(b0 + bb) * GP_STRIDE + (k0 + e) * GP_TILE + p]
                                   : 0.0;
#pragma unroll
            for (int e = 0; e < GU_T; ++e)
#pragma unroll
                for (int bb = 0; bb < GU_B; ++bb)
                    if (b0 + bb < nblk) acc[e] += v[e][bb];
        }
#pragma unroll
        for (int e = 0; e < GU_T; ++e) {
            const int k = k0 + e;
            if (k < ntile) {
                int tj = 0;
                while ((tj + 1) * (tj + 2) / 2 <= k) ++tj;
                const int ti = k - tj * (tj + 1) / 2;
                const int i = 16 * ti + pr, j = 16 * tj + pc;
                if (i <= j && j < n) put(i, j, acc[e]);
            }
        }
    }
}

// --------------------------------------------------------------------------
// Panel factorisation by CholeskyQR2 with Householder reconstruction
// --------------------------------------------------------------------------
// The accepted block's projected columns X = G[n_P:m, J] (2 <= kr <= CQ_MAX)
// are factored as X = Q R from Gram matrices: R1 is the Cholesky factor of
// X^T X (whose entries lg_greedy already holds), Q1 = X R1^{-1}, R2 the
// Cholesky factor of Q1^T Q1, Q = Q1 R2^{-1} and R = R2 R1 (CholeskyQR2,
// Fukaya, Nakatsukasa, Yanagisawa and Yamamoto, 2014).  The reflectors of
// Algorithm 4 are then rebuilt from Q (Ballard, Demmel, Grigori, Jacquelin,
// Nguyen and Solomonik, 2015): an LU factorisation without pivoting of Q's
// top kr x kr block minus S, S = diag(s_t) with s_t the opposite of the sign
// of step t's pivot (so every pivot of U is at least 1 in magnitude), gives
// Q - [S; 0] = Y U with Y unit lower trapezoidal.  Y is the matrix of
// reflectors with unit diagonal, S R the new diagonal block of R (the signs of
// the column-by-column factorisation), and the rows of Y below the top block
// are y = q U^{-1} = q1 (U R2)^{-1}.  The compact-WY factor is T = -U S
// Y1^{-T}.  The LU runs twice side by side on two waves, as row operations on
// [Q_top - S, I] (leaving U and Y1^{-1}, so T is one product) and as column
// operations on [Q_top - S; I] (leaving Y1 and U^{-1}); both form the same
// Schur complements with the same products, so their pivots and signs agree
// bit for bit.  The row passes multiply 16-row tiles by the explicit inverses
// R1^{-1} and (U R2)^{-1} on the matrix cores; the small factors are formed by
// one wave each with the matrices in registers (one column or row per lane).  Two row passes over the panel and two one-workgroup steps
// replace the per-column exchange; a block whose Gram matrix is far from well
// conditioned goes the column-by-column way.
constexpr int CQ_MAX = 32;          // widest panel (one column per lane of a wave)
constexpr int CQ_ROWS = 128;        // panel rows per workgroup of the row passes
constexpr int CQ_XW = 49;           // LDS row of the row passes: three 16-column tiles and a pad
constexpr double CQ_SIN2 = 1e-6;    // smallest squared sine of a column against the earlier ones
constexpr double CQ_ORTH = 1e-4;    // largest |Q1^T Q1 - I| entry taken by the second pass
constexpr double CQ_SER = 1e-8;     // up to this |Q1^T Q1 - I| entry, R2 and R2^{-1} by series
constexpr int CQ_SQ = CQ_MAX * CQ_MAX;
constexpr int CQ_R1 = 0;            // R1 (row-major, CQ_MAX x CQ_MAX, zero outside kr x kr)
constexpr int CQ_R1I = CQ_SQ;       // R1^{-1}
constexpr int CQ_M2I = 2 * CQ_SQ;   // (U R2)^{-1}
constexpr int CQ_Y1 = 3 * CQ_SQ;    // top block of Y (unit lower)
constexpr int CQ_R22 = 4 * CQ_SQ;   // the new diagonal block S R of R
constexpr int CQ_Z = 5 * CQ_SQ;     // z = T^T (Y^T bt)
constexpr int CQ_DOUBLES = 5 * CQ_SQ + CQ_MAX;
// dynamic LDS of the second row pass (inside lg_panel_mw): the row block,
// (U R2)^{-1} and eight partial column sums
constexpr size_t CQ_P2_LDS = sizeof(double) * (CQ_ROWS * CQ_XW + CQ_MAX * (CQ_MAX + 1) + 8 * CQ_MAX);
static_assert(WG == 2 * CQ_ROWS && NW == 4, "row passes: two threads per row, four waves");
typedef lds_double CqRow[CQ_MAX + 1];   // a row of a small matrix in LDS
typedef lds_double CqX[CQ_XW];          // a row of a row block in LDS

// Cholesky factor and its inverse in one pass, by one wave.  G: an n x n
// symmetric positive definite matrix in LDS (n <= CQ_MAX, upper triangle
// read).  The elimination runs on blockdiag(G, I) (steps past n are identity
// steps, so no step needs a guard) augmented by the identity: lane j < 32
// holds column j of the matrix (its upper triangle), lane 32 + c column c of
// the identity.  Step t scales row t by the inverse square root of its pivot
// and subtracts R[t][i] times it from row i > t (the multipliers are the
// scaled row's entries, broadcast through rowbuf, 64 doubles of LDS).  The
// matrix lanes end with R (R^T R = G), the identity lanes with R^{-T}.  R and
// Ri (= R^{-1}) are written whole, zero outside the n x n triangle.  Returns
// the smallest R[t][t]^2 / G[t][t] over t < n (the squared sine of column t's
// angle with the span of the columns before it), or -1 when a pivot is not a
// positive finite number.  All lanes of one wave call it.
// 1 / sqrt(d) and 1 / u: the hardware estimates refined by two Newton steps
// each (every step squares the relative error).
__device__ __forceinline__ double rsqrt_nr(double d) {
    double y = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 2; ++it) y = fma(0.5 * y, fma(-(d * y), y, 1.0), y);
    return y;
}
__device__ __forceinline__ double rcp_nr(double u) {
    double y = __builtin_amdgcn_rcp(u);
#pragma unroll
    for (int it = 0; it < 2; ++it) y = fma(y, fma(-u, y, 1.0), y);
    return y;
}

__device__ __forceinline__ double chol_inv_wave(const CqRow* G, int n, CqRow* R, CqRow* Ri, lds_double* rowbuf) {
    const int lane = threadIdx.x & 63, j = lane & 31;
    const bool mat = lane < 32;
    double g[CQ_MAX];
#pragma unroll
    for (int i = 0; i < CQ_MAX; ++i) {
        const double gij = G[i][j];
        g[i] = (mat && j < n) ? ((i <= j) ? gij : 0.0) : (i == j ? 1.0 : 0.0);
    }
    // the next pivot is taken ahead of the broadcast: lane t + 1's own
    // multiplier is its own entry of the scaled row
    double dn = readlane_d(g[0], 0);
#pragma unroll
    for (int t = 0; t < CQ_MAX; ++t) {
        const double ri = rsqrt_nr(dn);
        const double v = (lane == t) ? dn * ri : g[t] * ri;
        g[t] = v;
        rowbuf[lane] = v;
        if (t + 1 < CQ_MAX) dn = readlane_d(fma(-v, v, g[t + 1]), t + 1);
        wave_lds_sync();   // the other lanes' entries of the row are read below
        // all multipliers in one LDS round trip, then the updates
        double mu[CQ_MAX];
#pragma unroll
        for (int i = t + 1; i < CQ_MAX; ++i) mu[i] = rowbuf[i];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = t + 1; i < CQ_MAX; ++i) g[i] = fma(-mu[i], v, g[i]);
        wave_lds_sync();   // before the next step overwrites the row
    }
    // pivot test: lane t < n holds R[t][t] in g[t]
    double rtt = 0.0;
#pragma unroll
    for (int t = 0; t < CQ_MAX; ++t) rtt = (lane == t) ? g[t] : rtt;
    double q = 1.0;
    if (mat && j < n) {
        const double ratio = rtt * rtt / G[j][j];
        q = (rtt > 0.0 && rtt < INFINITY && ratio == ratio) ? ratio : -1.0;
    }
    for (int o = 32; o > 0; o >>= 1) q = fmin(q, __shfl_xor(q, o, 64));
    const bool live = j < n;
#pragma unroll
    for (int i = 0; i < CQ_MAX; ++i) {
        if (mat) R[i][j] = (live && i <= j) ? g[i] : 0.0;
        else Ri[j][i] = (live && i >= j && i < n) ? g[i] : 0.0;
    }
    return q;
}

// LU factorisation without pivoting of W - S and the inverse of its L in one
// pass, by one wave (the reconstruction's LU).  W: n x n in LDS (n <= CQ_MAX,
// zero outside n x n); S = diag(s_t), s_t = +1 when step t's pivot is
// negative and -1 otherwise, so every pivot of U is at least 1 in magnitude.
// Row elimination on [W, I]: lane c < 32 holds column c of W, lane 32 + c
// column c of the identity; step t takes the pivot from lane t, modifies it by
// -s_t and subtracts l_i = W[i][t] / pivot times row t from each row i > t
// (the multipliers are column t's entries, read from lane t through the
// scalar unit).  Steps past n meet a zero column and act as identity steps.
// The matrix lanes end with U (W - S = L U), the identity lanes with L^{-1}
// (unit lower).  U and Li are written whole (zero outside n x n); sg[t] = s_t.
__device__ __forceinline__ void lu_rows_wave(const CqRow* W, int n, CqRow* U, CqRow* Li, lds_double* sg) {
    const int lane = threadIdx.x & 63, c = lane & 31;
    const bool mat = lane < 32;
    double w[CQ_MAX];
#pragma unroll
    for (int i = 0; i < CQ_MAX; ++i) {
        const double wic = W[i][c];
        w[i] = mat ? wic : (i == c ? 1.0 : 0.0);
    }
    // the next pivot is taken ahead of the update
    double pn = readlane_d(w[0], 0);
#pragma unroll
    for (int t = 0; t < CQ_MAX; ++t) {
        const double piv = pn;
        const double st = (piv < 0.0) ? 1.0 : -1.0;
        const double u = piv - st;
        const double ru = rcp_nr(u);
        if (lane == 0) sg[t] = st;
        if (lane == t) w[t] = u;
        const double wt = w[t];   // row t of this lane's column
        if (t + 1 < CQ_MAX) pn = readlane_d(fma(-(readlane_d(w[t + 1], t) * ru), wt, w[t + 1]), t + 1);
#pragma unroll
        for (int i = t + 1; i < CQ_MAX; ++i) w[i] = fma(-(readlane_d(w[i], t) * ru), wt, w[i]);
    }
    const bool live = c < n;
#pragma unroll
    for (int i = 0; i < CQ_MAX; ++i) {
        if (mat) U[i][c] = (live && i <= c) ? w[i] : 0.0;
        else Li[i][c] = (live && i < n && i >= c) ? ((i == c) ? 1.0 : w[i]) : 0.0;
    }
}

// LU factorisation without pivoting of W - S and the inverse of U in one
// pass, by one wave (the reconstruction's LU).  W: n x n in LDS (n <= CQ_MAX,
// zero outside n x n); S = diag(s_t), s_t = +1 when step t's pivot is negative
// and -1 otherwise, so every pivot of U is at least 1 in magnitude.  Column
// elimination on [W; I]: lane r < 32 holds row r of W, lane 32 + q row q of
// the identity; step t takes the pivot from lane t, scales column t by its
// inverse and subtracts U[t][c] times it from column c > t (row t of U, read
// from lane t through the scalar unit).  Steps past n meet a zero row and act as
// identity steps.  The matrix lanes end with the unit lower L (W - S = L U),
// the identity lanes with U^{-1}.  L and Ui are written whole (zero outside n x
// n, L with its unit diagonal); sg[t] = s_t.
__device__ __forceinline__ void lu_inv_wave(const CqRow* W, int n, CqRow* L, CqRow* Ui, lds_double* sg) {
    const int lane = threadIdx.x & 63, r = lane & 31;
    const bool mat = lane < 32;
    double w[CQ_MAX];
#pragma unroll
    for (int c = 0; c < CQ_MAX; ++c) {
        const double wrc = W[r][c];
        w[c] = mat ? wrc : (c == r ? 1.0 : 0.0);
    }
    // the next pivot is taken ahead of the update
    double pn = readlane_d(w[0], 0);
#pragma unroll
    for (int t = 0; t < CQ_MAX; ++t) {
        const double piv = pn;
        const double st = (piv < 0.0) ? 1.0 : -1.0;
        const double ru = rcp_nr(piv - st);
        if (lane == 0) sg[t] = st;
        const double wt = (lane == t) ? 1.0 : w[t] * ru;
        w[t] = wt;
        if (t + 1 < CQ_MAX) pn = readlane_d(fma(-readlane_d(w[t + 1], t), wt, w[t + 1]), t + 1);
        // row t of U from lane t (its entries past t are not changed by this step)
#pragma unroll
        for (int c = t + 1; c < CQ_MAX; ++c) w[c] = fma(-readlane_d(w[c], t), wt, w[c]);
    }
    const bool live = r < n;
#pragma unroll
    for (int c = 0; c < CQ_MAX; ++c) {
        if (mat) L[r][c] = (live && c < n) ? ((c < r) ? w[c] : (c == r) ? 1.0 : 0.0) : 0.0;
        else Ui[r][c] = (live && c >= r && c < n) ? w[c] : 0.0;
    }
}


// C = A B for 32 x 32 matrices in LDS on the matrix cores, one 16 x 16 tile
// of C per wave (all four waves call it); C must not alias A or B.
__device__ __forceinline__ void mm32(const CqRow* A, const CqRow* B, CqRow* C) {
    const int lane = threadIdx.x & 63, wv = wave_index();
    const int ti = wv >> 1, tj = wv & 1, r = lane & 15, g = lane >> 4;
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < CQ_MAX; kk += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[16 * ti + r][kk + g], B[kk + g][16 * tj + r], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) C[16 * ti + 4 * v + g][16 * tj + r] = acc[v];
}

// C = A B^T, as mm32.
__device__ __forceinline__ void mm32t(const CqRow* A, const CqRow* B, CqRow* C) {
    const int lane = threadIdx.x & 63, wv = wave_index();
    const int ti = wv >> 1, tj = wv & 1, r = lane & 15, g = lane >> 4;
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < CQ_MAX; kk += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[16 * ti + r][kk + g], B[16 * tj + r][kk + g], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) C[16 * ti + 4 * v + g][16 * tj + r] = acc[v];
}


// Deviation maximization's greedy test (Algorithm 2) on the candidates' Gram
// matrix, or the single column of Lawson-Hanson.  The pairwise cosines are
// evaluated in parallel into bit masks (bit a of bad[t]: |cos(a, t)| >= delta);
// the greedy scan in candidate order is then one mask test per candidate.
// Accepted candidates' panel columns go to gmap; the panel factorisation
// reads the candidate panel through it.
// With cq set (and 2 <= k <= CQ_MAX accepted) it also factors the accepted
// columns' Gram matrix for the CholeskyQR2 panel (R1 into a.cq) and sets
// ex->cq_ok when every column keeps a squared sine of at least CQ_SIN2 against
// the ones before it; otherwise ex->cq_ok = 0.
__global__ __launch_bounds__(WG, 1) void lg_greedy(LgArgs a, const double* part, int cq) {
    __shared__ WgShared s;
    __shared__ double Tl[KM][KM + 1];
    __shared__ double Gs_[CQ_MAX][CQ_MAX + 1], R1s_[CQ_MAX][CQ_MAX + 1], R1is_[CQ_MAX][CQ_MAX + 1];
    __shared__ double rowbuf_[64];
    __shared__ double sq[KM];
    __shared__ unsigned long long bad[KM];
    __shared__ int gm[KM];
    __shared__ double sin2s;
    __shared__ int gid;
    ctl_load(s, a.ctl);
    const Prob& p = a.p;
    LgExtra* ex = a.ex;
    const int c = s.ncol, tid = threadIdx.x, lane = tid & 63, wv = wave_index();
    CqRow* Gs = (CqRow*)Gs_;
    CqRow* R1s = (CqRow*)R1s_;
    CqRow* R1is = (CqRow*)R1is_;
    // while wave 0 runs the selection, wave 1 factors the Gram matrix of all
    // candidates in their order: the accepted block's when the scan keeps
    // every candidate, which is the common case
    const bool spec = cq && c > 1 && c <= CQ_MAX;
    if (c > 1) {
        // the candidates' Gram matrix from the partial blocks (upper part)
        const int nblk = (p.m - s.nP + GRAM_ROWS - 1) / GRAM_ROWS;
        gram_upper(part, nblk, c, [&](int ra, int t, double v) { Tl[ra][t] = v; });
        __syncthreads();
        if (wv == 0) {
            // c <= 64: one candidate per lane
            const int t = lane;
            if (t < c) sq[t] = sqrt(Tl[t][t]);
            wave_lds_sync();
            if (t < c) {
                const double nt = sq[t];
                unsigned long long msk = 0;
                for (int ra = 0; ra < t; ++ra) {
                    const double th = Tl[ra][t] / (nt * sq[ra]);
                    if (!(fabs(th) < a.prm.delta)) msk |= 1ull << ra;
                }
                bad[t] = msk;
            }
            wave_lds_sync();
            if (lane == 0) {
                const int cap = p.m - s.nP;
                unsigned long long acc = 1ull;
                int na = 1;
                gm[0] = 0;
                for (int t2 = 1; t2 < c; ++t2) {
                    if (na >= cap) break;
                    if ((bad[t2] & acc) == 0ull) {
                        acc |= 1ull << t2;
                        gm[na++] = t2;
                    }
                }
                for (int q = 0; q < na; ++q) s.J[q] = s.J[gm[q]];
                s.k = na;
                gid = (na == c);
                ex->gident = (na == c);
            }
        } else if (wv == 1 && spec) {
            for (int e = lane; e < CQ_SQ; e += 64) {
                const int q = e / CQ_MAX, r = e % CQ_MAX;
                Gs[q][r] = (q <= r && r < c) ? Tl[q][r] : 0.0;
            }
            wave_lds_sync();
            const double q2 = chol_inv_wave(Gs, c, R1s, R1is, (lds_double*)rowbuf_);
            if (lane == 0) sin2s = q2;
        }
    } else {
        if (tid == 0) {
            s.k = 1;
            gm[0] = 0;
            gid = 1;
            ex->gident = 1;
        }
    }
    __syncthreads();
    if (tid < s.k) ex->gmap[tid] = gm[tid];
    const int na = s.k;
    if (cq && c > 1 && na >= 2 && na <= CQ_MAX) {
        if (!(spec && gid)) {
            // R1 and R1^{-1} of the accepted columns (one wave)
            for (int e = tid; e < CQ_SQ; e += WG) {
                const int q = e / CQ_MAX, r = e % CQ_MAX;
                Gs[q][r] = (q <= r && r < na) ? Tl[gm[q]][gm[r]] : 0.0;
            }
            __syncthreads();
            if (wv == 0) {
                const double q2 = chol_inv_wave(Gs, na, R1s, R1is, (lds_double*)rowbuf_);
                if (lane == 0) sin2s = q2;
            }
            __syncthreads();
        }
        if (tid == 0) ex->cq_ok = (sin2s >= CQ_SIN2) ? 1 : 0;
        for (int e = tid; e < CQ_SQ; e += WG) {
            a.cq[CQ_R1 + e] = R1s[e / CQ_MAX][e % CQ_MAX];
            a.cq[CQ_R1I + e] = R1is[e / CQ_MAX][e % CQ_MAX];
        }
    } else if (tid == 0) {
        ex->cq_ok = 0;
    }
    if (tid == 0) s.kr = s.k;
    ctl_store(s, a.ctl);
}

// G[row, q] = G[row, gmap[q]] for q < kr on the rows this thread owns; the
// whole row is read before any of it is written.
__device__ inline void compact_panel_row(const Prob& p, const int* gmap, int kr, int row) {
    double v[KM];
#pragma unroll
    for (int q = 0; q < KM; ++q) v[q] = (q < kr) ? p.G[(size_t)gmap[q] * p.m + row] : 0.0;
#pragma unroll
    for (int q = 0; q < KM; ++q)
        if (q < kr) p.G[(size_t)q * p.m + row] = v[q];
}

// Stage a CQ_ROWS x 48 row block into xs: xs[i][q] = src(q, i) for i < nr
// and q < nc, else 0 (column 48, the pad, is not touched).  Each thread owns
// one row and every other column, and issues all its loads before its first
// LDS store.
template <typename F>
__device__ __forceinline__ void cq_stage(CqX* xs, int nr, int nc, F src) {
    const int i = threadIdx.x % CQ_ROWS, h = threadIdx.x / CQ_ROWS;
    double v[24];
#pragma unroll
    for (int u = 0; u < 24; ++u) {
        const int q = h + 2 * u;
        v[u] = (i < nr && q < nc) ? src(q, i) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 24; ++u) xs[i][h + 2 * u] = v[u];
}

// xs[:, 0:ncol] = (xs[:, 0:32] M)[:, 0:ncol] for the row block in LDS (M 32 x
// 32 in LDS) on the matrix cores.  Wave w takes the 16-row tiles w and w + 4
// whole (both column tiles), so it overwrites only rows no other wave reads.
__device__ __forceinline__ void cq_rows_times(CqX* xs, const CqRow* M, int ncol) {
    const int lane = threadIdx.x & 63, wv = wave_index(), r = lane & 15, g = lane >> 4;
    for (int rb = wv; rb < CQ_ROWS / 16; rb += NW) {
        d4 a0 = d4{0.0, 0.0, 0.0, 0.0}, a1 = a0;
#pragma unroll
        for (int kk = 0; kk < CQ_MAX; kk += 4) {
            const double x = xs[16 * rb + r][kk + g];
            a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, M[kk + g][r], a0, 0, 0, 0);
            a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, M[kk + g][16 + r], a1, 0, 0, 0);
        }
        wave_lds_sync();
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * rb + 4 * v + g;
            if (r < ncol) xs[row][r] = a0[v];
            if (16 + r < ncol) xs[row][16 + r] = a1[v];
        }
    }
}

// Partial Gram X^T X of the row block xs (nc columns; its columns nc .. 47
// and its rows past the panel zero) into out (the partial-Gram layout), on
// the matrix cores.
__device__ __forceinline__ void cq_gram_tiles(const CqX* xs, int nc, double* out) {
    const int lane = threadIdx.x & 63, wv = wave_index(), g = lane >> 4;
    const int nt = (nc + 15) / 16;
    int tile = 0;
    for (int ti = 0; ti < nt; ++ti)
        for (int tj = ti; tj < nt; ++tj, ++tile) {
            if ((tile % NW) != wv) continue;
            d4 acc0 = d4{0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
            const int ca = ti * 16 + (lane & 15), cb = tj * 16 + (lane & 15);
#pragma unroll 4
            for (int r = 0; r < CQ_ROWS; r += 8) {
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[r + g][ca], xs[r + g][cb], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[r + 4 + g][ca], xs[r + 4 + g][cb], acc1, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v)
                out[gp_tile(ti, tj) * GP_TILE + (4 * v + (lane >> 4)) * 16 + (lane & 15)] = acc0[v] + acc1[v];
        }
}

// CholeskyQR2 panel, first row pass.  Workgroup w < nb = ceil((m - n_P) /
// CQ_ROWS) takes panel rows n_P + w CQ_ROWS ...: Q1 = X R1^{-1} for its rows,
// Q1 into W (column-major) and the block's partial Q1^T Q1 into slot w of
// gpart.  The workgroups past nb copy the accepted candidates' rows above the
// panel into the new columns of R.
__global__ __launch_bounds__(WG) void lg_cq_p1(LgArgs a) {
    __shared__ double xs_[CQ_ROWS][CQ_XW];
    __shared__ double Mi_[CQ_MAX][CQ_MAX + 1];
    __shared__ int gml[CQ_MAX];
    const LgExtra* ex = a.ex;
    if (!ex->cq_ok) return;
    const Ctl* ctl = a.ctl;
    const Prob& p = a.p;
    const int r0 = ctl->nP, kr = ctl->kr, m = p.m, tid = threadIdx.x;
    const int nb = (m - r0 + CQ_ROWS - 1) / CQ_ROWS;
    if ((int)blockIdx.x >= nb) {
        const int row = ((int)blockIdx.x - nb) * WG + tid;
        int gm[CQ_MAX], sl[CQ_MAX];
#pragma unroll
        for (int t = 0; t < CQ_MAX; ++t) {
            gm[t] = (t < kr) ? ex->gmap[t] : 0;
            sl[t] = (t < kr) ? p.slot[r0 + t] : 0;
        }
        if (row < r0) {
            double v[CQ_MAX];
#pragma unroll
            for (int t = 0; t < CQ_MAX; ++t) v[t] = (t < kr) ? p.G[(size_t)gm[t] * m + row] : 0.0;
#pragma unroll
            for (int t = 0; t < CQ_MAX; ++t)
                if (t < kr) p.R[(size_t)sl[t] * p.kc + row] = v[t];
        }
        return;
    }
    CqX* xs = (CqX*)xs_;
    CqRow* Mi = (CqRow*)Mi_;
    const int rs = r0 + (int)blockIdx.x * CQ_ROWS, nr = min(m - rs, CQ_ROWS);
    if (tid < CQ_MAX) gml[tid] = (tid < kr) ? ex->gmap[tid] : 0;
    double mr[CQ_SQ / WG];
#pragma unroll
    for (int u = 0; u < CQ_SQ / WG; ++u) mr[u] = a.cq[CQ_R1I + tid + WG * u];
    __syncthreads();
    cq_stage(xs, nr, kr, [&](int q, int i) { return p.G[(size_t)gml[q] * m + rs + i]; });
#pragma unroll
    for (int u = 0; u < CQ_SQ / WG; ++u) {
        const int e = tid + WG * u;
        Mi[e / CQ_MAX][e % CQ_MAX] = mr[u];
    }
    __syncthreads();
    cq_rows_times(xs, Mi, CQ_MAX);   // columns >= kr stay zero (R1^{-1} is zero there)
    __syncthreads();
    {
        const int i = tid % CQ_ROWS, h = tid / CQ_ROWS;
#pragma unroll
        for (int u = 0; u < CQ_MAX / 2; ++u) {
            const int q = h + 2 * u;
            if (q < kr && i < nr) p.W[(size_t)q * m + rs + i] = xs[i][q];
        }
    }
    cq_gram_tiles(xs, kr, a.gpart + (size_t)blockIdx.x * GP_STRIDE);
}

// CholeskyQR2 panel, the small factors (one workgroup): R2 from the summed
// Q1^T Q1 (ex->cq_ok = 0 when an entry of Q1^T Q1 - I exceeds CQ_ORTH or a
// pivot fails: the column-by-column panel then runs), R = R2 R1, Q's top block
// Q1_top R2^{-1}, its LU with signs (S, U, Y1 and their inverses, on two
// waves), T = -U S Y1^{-T} into p.T, the new columns' rows n_P .. n_P + t of
// R (S R, also in a.cq, diagonal into ctl->beta), and (U R2)^{-1} and Y1 for
// the second row pass.  The serial parts (Cholesky, LU) run on one wave each
// with the matrices in registers; the products on the matrix cores.
__global__ __launch_bounds__(WG, 1) void lg_cq_b(LgArgs a) {
    // lifetimes: G2 then Q_top in A0; R1 then U S in A1; Q1_top then T in A2;
    // R2^{-1} then U R2 in R2i_
    __shared__ double A0_[CQ_MAX][CQ_MAX + 1], A1_[CQ_MAX][CQ_MAX + 1], A2_[CQ_MAX][CQ_MAX + 1];
    __shared__ double R2_[CQ_MAX][CQ_MAX + 1], R2i_[CQ_MAX][CQ_MAX + 1], Rr_[CQ_MAX][CQ_MAX + 1];
    __shared__ double L_[CQ_MAX][CQ_MAX + 1], Li_[CQ_MAX][CQ_MAX + 1];
    __shared__ double Lc_[CQ_MAX][CQ_MAX + 1], Ui_[CQ_MAX][CQ_MAX + 1], M2i_[CQ_MAX][CQ_MAX + 1];
    __shared__ double sg_[CQ_MAX], sg2_[CQ_MAX], rowbuf_[64];
    __shared__ int mode;
    LgExtra* ex = a.ex;
    if (!ex->cq_ok) return;
    Ctl* ctl = a.ctl;
    const Prob& p = a.p;
    const int r0 = ctl->nP, kr = ctl->kr, m = p.m, kq = p.kq, tid = threadIdx.x, lane = tid & 63,
              wv = wave_index();
    const int nb = (m - r0 + CQ_ROWS - 1) / CQ_ROWS;
    CqRow* G2 = (CqRow*)A0_;
    CqRow* Qt = (CqRow*)A0_;
    CqRow* R1 = (CqRow*)A1_;
    CqRow* US = (CqRow*)A1_;
    CqRow* Q1t = (CqRow*)A2_;
    CqRow* Tm = (CqRow*)A2_;
    CqRow* R2 = (CqRow*)R2_;
    CqRow* R2i = (CqRow*)R2i_;
    CqRow* Rr = (CqRow*)Rr_;
    CqRow* L = (CqRow*)L_;   // scratch of the series for R2, then U
    CqRow* U = (CqRow*)L_;
    CqRow* Li = (CqRow*)Li_;
    CqRow* Lc = (CqRow*)Lc_;
    CqRow* Ui = (CqRow*)Ui_;
    CqRow* M2i = (CqRow*)M2i_;
    lds_double* sg = (lds_double*)sg_;
    lds_double* sg2 = (lds_double*)sg2_;
    // R1, Q1's top rows and the new columns' slots are loaded together with
    // the partial Gram blocks (their LDS stores follow the reduction)
    double lr[CQ_SQ / WG], lw[CQ_SQ / WG];
    int sl[CQ_SQ / WG];
#pragma unroll
    for (int u = 0; u < CQ_SQ / WG; ++u) {
        const int e = tid + WG * u, i = e / CQ_MAX, t = e % CQ_MAX;
        lr[u] = a.cq[CQ_R1 + e];
        lw[u] = (i < kr && t < kr) ? p.W[(size_t)t * m + r0 + i] : 0.0;
        sl[u] = (t < kr) ? p.slot[r0 + t] : 0;
        G2[i][t] = 0.0;
    }
    __syncthreads();
    gram_upper(a.gpart, nb, kr, [&](int i, int t, double v) { G2[i][t] = v; });
#pragma unroll
    for (int u = 0; u < CQ_SQ / WG; ++u) {
        const int e = tid + WG * u, i = e / CQ_MAX, t = e % CQ_MAX;
        R1[i][t] = lr[u];
        Q1t[i][t] = lw[u];
    }
    __syncthreads();
    if (wv == 0) {
        // largest deviation of Q1^T Q1 from the identity (upper triangle)
        const int c = lane & 31;
        double dev = 0.0;
#pragma unroll
        for (int i = 0; i < CQ_MAX; ++i) {
            const double e = fabs(G2[i][c] - (i == c ? 1.0 : 0.0));
            dev = (i <= c && lane < kr) ? fmax(dev, e) : dev;
        }
        if (!(dev == dev)) dev = INFINITY;
        for (int o = 32; o > 0; o >>= 1) dev = fmax(dev, __shfl_xor(dev, o, 64));
        if (lane == 0) mode = (dev <= CQ_SER) ? 2 : (dev <= CQ_ORTH) ? 1 : 0;
    }
    __syncthreads();
    if (mode == 2) {
        // Q1^T Q1 = I + E with |E| <= CQ_SER: R2 = I + F, F upper triangular
        // with F + F^T + F^T F = E, to second order F = Phi(E) - Phi(F0^T F0)
        // with F0 = Phi(E) (Phi: strict upper triangle plus half the
        // diagonal); R2^{-1} = I - F + F^2.  The neglected terms are of third
        // order in |E| <= CQ_MAX CQ_SER.
        CqRow* F0 = R2;
        CqRow* F0t = R2i;
        CqRow* P = Rr;
        CqRow* F = L;
        for (int e = tid; e < CQ_SQ; e += WG) {
            const int i = e / CQ_MAX, j = e % CQ_MAX;
            const bool in = j < kr;
            const double eij = (i < j) ? G2[i][j] : (i == j) ? 0.5 * (G2[i][i] - 1.0) : 0.0;
            F0[i][j] = in ? eij : 0.0;
            F0t[j][i] = in ? eij : 0.0;
        }
        __syncthreads();
        mm32(F0t, F0, P);   // F0^T F0 (symmetric)
        __syncthreads();
        for (int e = tid; e < CQ_SQ; e += WG) {
            const int i = e / CQ_MAX, j = e % CQ_MAX;
            const double pij = (i < j) ? P[i][j] : (i == j) ? 0.5 * P[i][i] : 0.0;
            F[i][j] = F0[i][j] - pij;
        }
        __syncthreads();
        mm32(F, F, P);      // F^2
        __syncthreads();
        for (int e = tid; e < CQ_SQ; e += WG) {
            const int i = e / CQ_MAX, j = e % CQ_MAX;
            const bool in = i < kr && j < kr;
            const double id = (i == j) ? 1.0 : 0.0;
            R2[i][j] = in ? id + F[i][j] : 0.0;
            R2i[i][j] = in ? (id - F[i][j]) + P[i][j] : 0.0;
        }
    } else if (mode == 1) {
        __shared__ int ok;
        if (wv == 0) {
            const double piv = chol_inv_wave(G2, kr, R2, R2i, (lds_double*)rowbuf_);
            if (lane == 0) ok = (piv > 0.0) ? 1 : 0;
        }
        __syncthreads();
        if (!ok) mode = 0;   // read by every thread below after the barrier
    }
    __syncthreads();
    if (mode == 0) {
        if (tid == 0) ex->cq_ok = 0;
        return;
    }
    mm32(R2, R1, Rr);     // R = R2 R1
    mm32(Q1t, R2i, Qt);   // Q's top block (G2 is no longer needed)
    __syncthreads();
    if (wv == 0) lu_rows_wave(Qt, kr, U, Li, sg);
    else if (wv == 1) lu_inv_wave(Qt, kr, Lc, Ui, sg2);
    __syncthreads();
    if (tid < kr && sg[tid] != sg2[tid]) mode = 0;   // cannot happen: the two take the same pivots
    for (int e = tid; e < CQ_SQ; e += WG) {   // U S (R1 is no longer needed)
        const int i = e / CQ_MAX, j = e % CQ_MAX;
        US[i][j] = U[i][j] * sg[j];
    }
    __syncthreads();
    if (mode == 0) {
        if (tid == 0) ex->cq_ok = 0;
        return;
    }
    mm32t(US, Li, Tm);    // U S Y1^{-T} = -T (Q1_top is no longer needed)
    mm32(R2i, Ui, M2i);   // (U R2)^{-1} = R2^{-1} U^{-1}
    __syncthreads();
    {
#pragma unroll
        for (int u = 0; u < CQ_SQ / WG; ++u) {
            const int e = tid + WG * u, i = e / CQ_MAX, j = e % CQ_MAX;
            const double rh = (i <= j && j < kr) ? sg[i] * Rr[i][j] : 0.0;
            a.cq[CQ_M2I + e] = M2i[i][j];
            a.cq[CQ_Y1 + e] = Lc[i][j];
            a.cq[CQ_R22 + e] = rh;
            if (i <= j && j < kr) p.R[(size_t)sl[u] * p.kc + r0 + i] = rh;
        }
    }
    // T (column-major, ld kq; zero below the diagonal and past kr rows)
    for (int e = tid; e < kr * kq; e += WG) {
        const int t = e / kq, i = e % kq;
        p.T[(size_t)t * kq + i] = (i < kr) ? -Tm[i][t] : 0.0;
    }
    if (tid < kr) {
        ctl->beta[tid] = sg[tid] * Rr[tid][tid];
        ctl->tau[tid] = -Tm[tid][tid];
    }
}

// CholeskyQR2 panel, second row pass (run by lg_panel_mw's workgroups w <
// nb = ceil((m - n_P) / CQ_ROWS)): the reflectors.  Rows n_P .. n_P + kr - 1
// take Y1 (unit diagonal, zeros above), the others y = q1 (U R2)^{-1}; y into
// V (column-major) and V^T (row-major), and the block's partial Y^T bt (kr
// values, summed over its rows in row order) into slot w of gpart.  dyn:
// CQ_P2_LDS bytes of LDS.
__device__ inline void cq_second_pass(const LgArgs& a, lds_double* dyn) {
    const Ctl* ctl = a.ctl;
    const Prob& p = a.p;
    const int r0 = ctl->nP, kr = ctl->kr, m = p.m, kq = p.kq, tid = threadIdx.x;
    const int nb = (m - r0 + CQ_ROWS - 1) / CQ_ROWS;
    if ((int)blockIdx.x >= nb) return;
    CqX* xs = (CqX*)dyn;
    CqRow* Mi = (CqRow*)(dyn + CQ_ROWS * CQ_XW);
    lds_double* part8 = dyn + CQ_ROWS * CQ_XW + CQ_MAX * (CQ_MAX + 1);   // 8 x CQ_MAX
    const int rs = r0 + (int)blockIdx.x * CQ_ROWS, nr = min(m - rs, CQ_ROWS);
    double mr[CQ_SQ / WG], yr[CQ_SQ / WG];
#pragma unroll
    for (int u = 0; u < CQ_SQ / WG; ++u) {
        mr[u] = a.cq[CQ_M2I + tid + WG * u];
        yr[u] = (blockIdx.x == 0) ? a.cq[CQ_Y1 + tid + WG * u] : 0.0;
    }
    cq_stage(xs, nr, kr + 1,
             [&](int q, int i) { return (q < kr) ? p.W[(size_t)q * m + rs + i] : p.bt[rs + i]; });
#pragma unroll
    for (int u = 0; u < CQ_SQ / WG; ++u) {
        const int e = tid + WG * u;
        Mi[e / CQ_MAX][e % CQ_MAX] = mr[u];
    }
    __syncthreads();
    cq_rows_times(xs, Mi, kr);   // rows of (U R2)^{-1} past kr are zero: bt does not enter
    __syncthreads();
    if (blockIdx.x == 0) {
        // the top rows: Y1 (block 0 starts at row n_P; kr <= nr)
#pragma unroll
        for (int u = 0; u < CQ_SQ / WG; ++u) {
            const int e = tid + WG * u, i = e / CQ_MAX, q = e % CQ_MAX;
            if (i < kr && q < kr) xs[i][q] = yr[u];
        }
        __syncthreads();
    }
    {
        const int i = tid % CQ_ROWS, h = tid / CQ_ROWS;
#pragma unroll
        for (int u = 0; u < CQ_MAX / 2; ++u) {
            const int q = h + 2 * u;
            if (q < kr && i < nr) p.V[(size_t)q * m + rs + i] = xs[i][q];
        }
        // V^T rows, coalesced: element e = ii kr + q of the block's rows
        const int di = WG / kr, dq = WG % kr;
        int ii = tid / kr, q = tid % kr;
        for (int e = tid; e < nr * kr; e += WG) {
            p.Vt[(size_t)(rs + ii) * kq + q] = xs[ii][q];
            q += dq;
            ii += di;
            if (q >= kr) {
                q -= kr;
                ++ii;
            }
        }
    }
    // Y^T bt over the block's rows: eight groups of 16 rows, then the groups,
    // each in row order (rows past the panel hold zeros)
    {
        const int q = tid & 31, g = tid >> 5;
        double acc = 0.0;
        if (q < kr)
            for (int r = 0; r < CQ_ROWS / 8; ++r) {
                const int rr = g * (CQ_ROWS / 8) + r;
                acc = fma(xs[rr][q], xs[rr][kr], acc);
            }
        part8[g * CQ_MAX + q] = acc;
    }
    __syncthreads();
    if (tid < CQ_MAX) {
        double acc = 0.0;
        for (int g = 0; g < 8; ++g) acc += part8[g * CQ_MAX + tid];
        a.gpart[(size_t)blockIdx.x * GP_STRIDE + tid] = acc;
    }
}

// CholeskyQR2 panel: bt[n_P + kr : m] -= Y z with z = T^T (Y^T bt) from
// lg_panel_b (which updates the rows n_P .. n_P + kr - 1 itself).
__global__ __launch_bounds__(WG) void lg_cq_bt(LgArgs a) {
    if (!a.ex->cq_ok) return;
    const Prob& p = a.p;
    const int r0 = a.ctl->nP, kr = a.ctl->kr, m = p.m, tid = threadIdx.x;
    double z[CQ_MAX];
#pragma unroll
    for (int t = 0; t < CQ_MAX; ++t) z[t] = (t < kr) ? a.cq[CQ_Z + t] : 0.0;
    for (int row = r0 + kr + (int)blockIdx.x * WG + tid; row < m; row += (int)gridDim.x * WG) {
        double v[CQ_MAX];
#pragma unroll
        for (int t = 0; t < CQ_MAX; ++t) v[t] = (t < kr) ? p.V[(size_t)t * m + row] : 0.0;
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < CQ_MAX; ++t) acc = fma(v[t], z[t], acc);
        p.bt[row] -= acc;
    }
}

// Householder QR of the panel G[n_P:m, 0:kr] with bt[n_P:m] carried as column
// kr (Algorithm 4), spread over the workgroups: each owns `rpw` consecutive
// rows of the panel and keeps them in LDS.  One cross-workgroup exchange per
// column: every workgroup publishes the dots of its part of column t with
// columns t..kr (the first is the squared norm), the owner of the pivot row
// publishes that row, and every workgroup sums the partials in one fixed
// order (so all of them derive bitwise the same reflector).  With x the
// column below the diagonal, x0 its pivot entry and beta the new diagonal,
// the scaled reflector v (v0 = 1) satisfies v^T a_q = (x^T a_q - beta a_q0) /
// (x0 - beta), which is what lets the norm and the dots travel together.
constexpr int PNW = 32;                  // largest number of workgroups of the panel factorisation
constexpr int PANEL_LDS_MAX = 128 * 1024;   // dynamic LDS of one workgroup of the panel factorisation
constexpr int PSLOT = KM + 1;            // published values per workgroup and column

__global__ __launch_bounds__(WG) void lg_panel_mw(LgArgs a, int rpw, int ebase) {
    extern __shared__ double pan[];   // rpw x (kr + 1), row-major
    __shared__ double red[NW][PSLOT];
    __shared__ double dpart[NW][PSLOT];   // per gathering wave: dots of the pivot column with columns t .. kr
    __shared__ double prow[PSLOT];        // pivot row entries of columns t .. kr
    __shared__ double betal[PSLOT];       // new diagonal entries (the same in every workgroup)
    if (a.ex->cq_ok) {   // the CholeskyQR2 kernels factor this panel: their second row pass
        cq_second_pass(a, (lds_double*)pan);
        return;
    }
    const Ctl* ctl = a.ctl;
    const Prob& p = a.p;
    const int r0 = ctl->nP, kr = ctl->kr, m = p.m;
    const int npw = (m - r0 + rpw - 1) / rpw;
    const int w = blockIdx.x;
    const int* gmap = a.ex->gmap;
    if (w >= npw) {
        // workgroups past the panel: accepted candidates' rows above the panel,
        // which are also the new R columns' rows above the panel
        const int row = (w - npw) * WG + threadIdx.x;
        if (row < r0) {
            if (!a.ex->gident) compact_panel_row(p, gmap, kr, row);
            for (int t = 0; t < kr; ++t) p.R[(size_t)p.slot[r0 + t] * p.kc + row] = p.G[(size_t)t * m + row];
        }
        return;
    }
    const int rs = r0 + w * rpw, re = min(m, rs + rpw), nr = re - rs;
    const int ld = kr + 1;
    const int tid = threadIdx.x, lane = tid & 63, wv = wave_index();
    int* err = &a.ex->err;
    u64* DQl = a.pll;                          // [2][PNW][PSLOT] x 2 words, by column parity
    u64* PVl = a.pll + 2 * (2 * PNW * PSLOT);  // [2][PSLOT] x 2 words
    // rows nr .. rpw - 1 are zero: the update below runs over whole row
    // groups without bounds checks and leaves them zero
    for (int e = tid; e < rpw * ld; e += WG) {
        const int i = e / ld, q = e % ld;
        pan[e] = (i >= nr) ? 0.0 : (q < kr) ? p.G[(size_t)gmap[q] * m + rs + i] : p.bt[rs + i];
    }
    __syncthreads();
    // local dots of column 0 with columns 0 .. kr: lanes take columns, waves
    // take every fourth row (later columns' dots come out of the update)
    {
        const int i0 = max(0, r0 - rs);
        for (int c = lane; c < ld; c += 64) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            int i = i0 + wv;
            for (; i + 7 * NW < nr; i += 8 * NW) {
                double xt[8], xq[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    xt[u] = pan[(i + u * NW) * ld];
                    xq[u] = pan[(i + u * NW) * ld + c];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) acc[u & 3] += xt[u] * xq[u];
            }
            for (; i < nr; i += NW) acc[0] += pan[i * ld] * pan[i * ld + c];
            red[wv][c] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        }
    }
    // lanes of the fused update: H row groups of CW lanes, lane (h, cl) takes
    // column t + 1 + cl of rows wv H + h + 4 H k
    const int H = (kr <= 32) ? 2 : 1, CW = 64 / H;
    const int hh = lane / CW, cl = lane % CW;
    for (int t = 0; t < kr; ++t) {
        const int rt = r0 + t, ep = ebase + t, par = t & 1;
        const int i0 = max(0, rt - rs);   // local rows with global index >= rt
        const int nq = kr + 1 - t;        // columns t .. kr
        const bool owner = rt >= rs && rt < re;
        __syncthreads();
        // publish this workgroup's dots (and, from the owner, the pivot row)
        for (int c = tid; c < nq; c += WG) {
            const double d = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
            ll_put(&DQl[2 * ((par * PNW + w) * PSLOT + c)], d, ep);
            if (owner) ll_put(&PVl[2 * (par * PSLOT + c)], pan[(rt - rs) * ld + t + c], ep);
        }
        // gather: wave wv polls the dots of workgroups u = 8 wv .. 8 wv + 7
        // with column t + c (lane c) and adds them in workgroup order; wave 0
        // also takes the pivot row entry.  Each round issues all of a lane's
        // loads before checking any, so a round costs one memory round trip;
        // slots u >= npw are read but never used.
        static_assert(PNW == 8 * NW, "eight workgroups per gathering wave");
        for (int c0 = 0; c0 < nq; c0 += 64) {
            const int c = c0 + lane;
            const int cc = (c < nq) ? c : 0;
            const u64* dq = &DQl[2 * ((par * PNW + 8 * wv) * PSLOT + cc)];
            const u64* pq = &PVl[2 * (par * PSLOT + cc)];
            const u64 e = (u64)(unsigned)ep;
            const int nu = min(8, max(0, npw - 8 * wv));   // workgroups of this wave
            double val[8], pv = 0.0;
            unsigned pend = 0;   // bit j: workgroup 8 wv + j, bit 8: pivot row
            if (c < nq) pend = ((1u << nu) - 1) | ((wv == 0) ? (1u << 8) : 0u);
#pragma unroll
            for (int j = 0; j < 8; ++j) val[j] = 0.0;
            long long it = 0;
            while (true) {
                u64 w0[9], w1[9];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    w0[j] = __hip_atomic_load(dq + 2 * j * PSLOT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    w1[j] = __hip_atomic_load(dq + 2 * j * PSLOT + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                }
                if (wv == 0) {
                    w0[8] = __hip_atomic_load(pq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    w1[8] = __hip_atomic_load(pq + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                } else {
                    w0[8] = w1[8] = 0;
                }
#pragma unroll
                for (int j = 0; j <= 8; ++j) {
                    const bool rdy = ((pend >> j) & 1) && (w0[j] >> 32) == e && (w1[j] >> 32) == e;
                    const double v = __longlong_as_double((long long)((w1[j] << 32) | (w0[j] & 0xffffffffull)));
                    if (j < 8) val[j] = rdy ? v : val[j];
                    else pv = rdy ? v : pv;
                    pend &= rdy ? ~(1u << j) : ~0u;
                }
                if (__all(pend == 0)) break;
                if (++it > SPIN_LIMIT) {
                    if (lane == 0) atomicExch(err, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (c < nq) {
                // val[j] stays 0.0 for the workgroups past npw
                double d = 0.0;
#pragma unroll
                for (int j = 0; j < 8; ++j) d += val[j];
                dpart[wv][c] = d;
                if (wv == 0) prow[c] = pv;
            }
        }
        __syncthreads();
        auto dsum = [&](int q) { return ((dpart[0][q] + dpart[1][q]) + dpart[2][q]) + dpart[3][q]; };
        const double x0 = prow[0];
        const double normx = sqrt(dsum(0));
        double tau = 0.0, beta = x0, scal = 0.0;
        if (normx > 0.0) {
            beta = (x0 >= 0.0) ? -normx : normx;
            tau = (beta - x0) / beta;
            scal = 1.0 / (x0 - beta);
        }
        if (w == 0 && tid == 0) {
            a.ctl->tau[t] = tau;
            a.ctl->beta[t] = beta;
        }
        if (tid == 0) betal[t] = beta;
        // Apply the reflector to columns t+1 .. kr of the local rows >= rt,
        // store the scaled reflector in column t (read by no later step) and
        // accumulate the dots of the updated column t+1 with columns t+1 .. kr
        // over the rows > rt.  Every lane also updates column t+1 of its row
        // itself (same operands as the lane that owns it).  Rows are taken in
        // aligned groups: rows < i0 get vi = 0 and keep their values, rows
        // >= nr are zero.
        const int ncu = nq - 1;
        const bool act = cl < ncu;
        double acc = 0.0;
        if (act) {
            const int c = t + 1 + cl;
            const double sq = tau * (scal * (dsum(1 + cl) - beta * prow[1 + cl]));
            const double sq1 = tau * (scal * (dsum(1) - beta * prow[1]));
            const int rstep = NW * H, grp = 4 * rstep;   // rows per group: 32 (H = 2) or 16
            const int roff = wv * H + hh;
            for (int ib = (i0 / grp) * grp; ib < nr; ib += grp) {
                double xt[4], xt1[4], xq[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = ib + u * rstep + roff;
                    xt[u] = pan[i * ld + t];
                    xt1[u] = pan[i * ld + t + 1];
                    xq[u] = pan[i * ld + c];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = ib + u * rstep + roff;
                    const int gi = rs + i;
                    const double vr = (gi == rt) ? 1.0 : xt[u] * scal;
                    const double vi = (i < i0) ? 0.0 : vr;
                    const double xn = xq[u] - sq * vi;
                    const double pn = xt1[u] - sq1 * vi;
                    pan[i * ld + c] = xn;
                    pan[i * ld + t] = (i < i0) ? xt[u] : vr;
                    acc = fma((gi > rt) ? pn : 0.0, xn, acc);
                }
            }
        }
        if (H == 2) acc += __shfl_xor(acc, 32, 64);
        if (hh == 0 && act) red[wv][cl] = acc;
    }
    __syncthreads();
    for (int e = tid; e < nr * ld; e += WG) {
        const int i = e / ld, q = e % ld;
        if (q < kr) p.G[(size_t)q * m + rs + i] = pan[e];
        else p.bt[rs + i] = pan[e];
    }
    // The reflectors V (column-major) and V^T (row-major) of this workgroup's
    // rows, zero above each pivot (rows above the panel and columns >= kr are
    // never read), and its rows of the new R columns (beta on the diagonal).
    for (int e = tid; e < kr * nr; e += WG) {
        const int t = e / nr, i = e % nr, row = rs + i;
        const double pv = pan[i * ld + t];
        p.V[(size_t)t * m + row] = (row >= r0 + t) ? pv : 0.0;
        if (row <= r0 + t) p.R[(size_t)p.slot[r0 + t] * p.kc + row] = (row < r0 + t) ? pv : betal[t];
    }
    for (int e = tid; e < nr * kr; e += WG) {
        const int i = e / kr, t = e % kr, row = rs + i;
        p.Vt[(size_t)row * p.kq + t] = (row >= r0 + t) ? pan[i * ld + t] : 0.0;
    }
    // Partial V^T V over this workgroup's rows into slot w of gpart (the
    // partial-Gram layout; lg_panel_b adds the npw slots in order): upper 16 x
    // 16 tiles on the matrix cores, V read from LDS with the same zeros as above
    // (the padding rows past nr are zero).
    {
        double* out = a.gpart + (size_t)w * GP_STRIDE;
        const int nt = (kr + 15) / 16;
        const int g = lane >> 4;
        auto vv = [&](int i, int q) {
            const double x = pan[i * ld + min(q, kr - 1)];
            return (q < kr && rs + i >= r0 + q) ? x : 0.0;
        };
        int tile = 0;
        for (int ti = 0; ti < nt; ++ti)
            for (int tj = ti; tj < nt; ++tj, ++tile) {
                if ((tile % NW) != wv) continue;
                d4 acc0 = d4{0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
                const int ca = ti * 16 + (lane & 15), cb = tj * 16 + (lane & 15);
                for (int r = 0; r < rpw; r += 8) {
                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(vv(r + g, ca), vv(r + g, cb), acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(vv(r + 4 + g, ca), vv(r + 4 + g, cb), acc1, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    out[gp_tile(ti, tj) * GP_TILE + (4 * v + (lane >> 4)) * 16 + (lane & 15)] = acc0[v] + acc1[v];
            }
    }
}

// Single-workgroup panel factorisation (used when a row chunk of the panel
// would not fit in LDS).
__global__ __launch_bounds__(WG) void lg_panel_1wg(LgArgs a) {
    __shared__ WgShared s;
    ctl_load(s, a.ctl);
    if (!a.ex->gident)
        for (int row = threadIdx.x; row < a.p.m; row += WG) compact_panel_row(a.p, a.ex->gmap, s.kr, row);
    __syncthreads();
    Wg wg(a.p, a.prm, s);
    wg.panel_qr();
    ctl_store(s, a.ctl);
}

// Explicit reflectors V (zeros above the unit diagonal) in both layouts.
__global__ __launch_bounds__(WG) void lg_panel_v(LgArgs a) {
    const Ctl* ctl = a.ctl;
    const Prob& p = a.p;
    const int r0 = ctl->nP, kr = ctl->kr, m = p.m, kq = p.kq;
    for (int row = blockIdx.x * WG + threadIdx.x; row < m; row += gridDim.x * WG) {
        for (int t = 0; t < kq; ++t) {
            double v = 0.0;
            if (t < kr && row >= r0 + t) v = p.G[(size_t)t * m + row];
            if (t < kr) p.V[(size_t)t * m + row] = v;
            p.Vt[(size_t)row * kq + t] = v;
        }
    }
    // the new columns of R: rows above the panel from the projection, the
    // panel's pivot rows, and the new diagonal
    const int nrow = r0 + kr;
    for (int e = blockIdx.x * WG + threadIdx.x; e < kr * nrow; e += gridDim.x * WG) {
        const int t = e / nrow, i = e % nrow;
        if (i <= r0 + t)
            p.R[(size_t)p.slot[r0 + t] * p.kc + i] = (i < r0 + t) ? p.G[(size_t)t * m + i] : ctl->beta[t];
    }
}

// Compact-WY factor (from V^T V in W), new R columns, feasibility loop on J.
// T and the new diagonal block of R are staged in LDS; the J-loop's triangular
// solves run on one wave (one row per lane).
// T of the compact WY form I - V T V^T of kr reflectors.  Its inverse is
// striu(V^T V) + diag(1 / tau) (the recurrence of the block reflector's T and
// this inverse agree in exact arithmetic), so lane j solves for column j of T
// by itself: T[j][j] = tau_j, T[i][j] = -tau_i sum_{k=i+1..j} (V^T V)[i][k]
// T[k][j], bottom-up, the sums accumulated right-looking as entries become
// known.  Multiplying by tau_i (rather than dividing by 1 / tau_i) keeps a
// zero tau exact.  N >= kr rows are unrolled (register partial sums).
template <int N>
__device__ inline void wy_t_columns(const double (*Wl)[KM + 1], const double* tau, int kr, double (*Tl)[KM + 1],
                                    int j) {
    double acc[N];
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] = 0.0;
    const bool col = j < kr;
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        if (i >= kr) continue;   // uniform
        const double ti = tau[i];
        const double tij = (!col || i > j) ? 0.0 : (i == j) ? ti : -ti * acc[i];
        if (col) Tl[i][j] = tij;
#pragma unroll
        for (int i2 = 0; i2 < i; ++i2) acc[i2] = fma(Wl[i2][i], tij, acc[i2]);
    }
}

// part: nblk partial Gram blocks of V (the panel's workgroups, or 128-row
// blocks), or, when the CholeskyQR2 kernels factored the panel, nblk_cq
// partial vectors V^T bt (the second row pass; T is then lg_cq_b's): this
// kernel then forms z = T^T (V^T bt) for lg_cq_bt and the rows n_P .. n_P +
// kr - 1 of bt = (I - V T^T V^T) bt.
__global__ __launch_bounds__(WG, 1) void lg_panel_b(LgArgs a, const double* part, int nblk, int nblk_cq) {
    __shared__ WgShared s;
    __shared__ double Tl[KM][KM + 1];
    __shared__ double Wl[KM][KM + 1];
    __shared__ double cl[CQ_MAX], zl[CQ_MAX];
    ctl_load(s, a.ctl);
    Wg wg(a.p, a.prm, s);
    const Prob& p = a.p;
    const int kr = s.kr, kq = p.kq, tid = threadIdx.x, m = p.m;
    const int r0 = s.nP;
    const bool cq = a.ex->cq_ok != 0;
    if (cq) {
        // V^T bt: the partial vectors in block order
        if (tid < kr) {
            double c = 0.0;
            for (int b0 = 0; b0 < nblk_cq; b0 += 32) {
                double v[32];
#pragma unroll
                for (int bb = 0; bb < 32; ++bb)
                    v[bb] = (b0 + bb < nblk_cq) ? part[(size_t)(b0 + bb) * GP_STRIDE + tid] : 0.0;
#pragma unroll
                for (int bb = 0; bb < 32; ++bb)
                    if (b0 + bb < nblk_cq) c += v[bb];
            }
            cl[tid] = c;
        }
        // column tid of T and row tid of the top block of V (both from global
        // memory, loaded ahead of the barrier)
        double tc[CQ_MAX], y1[CQ_MAX];
#pragma unroll
        for (int i = 0; i < CQ_MAX; ++i) {
            tc[i] = (tid < kr && i <= tid) ? p.T[(size_t)tid * kq + i] : 0.0;
            y1[i] = (tid < kr && i <= tid) ? a.cq[CQ_Y1 + tid * CQ_MAX + i] : 0.0;
        }
        __syncthreads();
        if (tid < kr) {
            double z = 0.0;
#pragma unroll
            for (int i = 0; i < CQ_MAX; ++i)
                if (i < kr) z = fma(tc[i], cl[i], z);
            zl[tid] = z;
            a.cq[CQ_Z + tid] = z;
        }
        __syncthreads();
        if (tid < kr) {
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < CQ_MAX; ++t)
                if (t < kr) acc = fma(y1[t], zl[t], acc);
            p.bt[r0 + tid] -= acc;
        }
        if (tid == 0) a.ex->ncq += 1;
    } else {
        // T of the compact WY form, from V^T V (summed from the partial blocks)
        gram_upper(part, nblk, kr, [&](int i, int t, double v) { Wl[i][t] = v; });
        __syncthreads();
        if (tid < 64) {
            if (kr <= 32) {
                wy_t_columns<32>(Wl, s.tau, kr, Tl, tid);
            } else {
                // same order of operations, the partial sums kept in Tl itself
                const int j = tid;
                if (j < kr) {
                    for (int i = 0; i < kr; ++i) Tl[i][j] = 0.0;
                    for (int i = kr - 1; i >= 0; --i) {
                        const double tij = (i > j) ? 0.0 : (i == j) ? s.tau[i] : -s.tau[i] * Tl[i][j];
                        Tl[i][j] = tij;
                        for (int i2 = 0; i2 < i; ++i2) Tl[i2][j] = fma(Wl[i2][i], tij, Tl[i2][j]);
                    }
                }
            }
        }
        __syncthreads();
        for (int e = tid; e < kr * kq; e += WG) {
            const int i = e % kq, t = e / kq;
            p.T[(size_t)t * kq + i] = (i < kr) ? Tl[i][t] : 0.0;
        }
    }
    __syncthreads();
    // feasibility loop on J: longest prefix of J whose own LS components are positive
    if (cq) {
        // the new diagonal block of R, as lg_cq_b wrote it into R
        for (int e = tid; e < CQ_SQ; e += WG) Wl[e / CQ_MAX][e % CQ_MAX] = a.cq[CQ_R22 + e];
    } else {
        for (int e = tid; e < kr * kr; e += WG) {
            const int i = e % kr, t = e / kr;
            Wl[i][t] = (i <= t) ? p.R[(size_t)p.slot[r0 + t] * p.kc + r0 + i] : 0.0;
        }
    }
    __syncthreads();
    if (tid < 64) {
        // one wave: row `lane` of R22 scaled by its inverse diagonal entry,
        // strictly upper part, in registers; back substitution with scalar-unit
        // broadcasts, repeated for shorter prefixes while a component is <= 0
        const int lane = tid;
        const bool lk = lane < kr;
        const double rinv = lk ? 1.0 / Wl[lane][lane] : 0.0;
        double rrow[KM];
#pragma unroll
        for (int j = 0; j < KM; ++j) rrow[j] = (lk && j > lane && j < kr) ? Wl[lane][j] * rinv : 0.0;
        // (with cq, this thread itself wrote bt[r0 + lane] above)
        const double bl = lk ? p.bt[r0 + lane] * rinv : 0.0;
        int k = kr;
        while (k > 0 && !a.prm.nojloop) {   // not evaluated in the Theorem 4 regime
            double v = (lane < k) ? bl : 0.0;
            double mn = INFINITY;
#pragma unroll
            for (int j = KM - 1; j >= 0; --j) {
                if (j < k) {
                    const double yj = readlane_d(v, j);
                    mn = fmin(mn, yj);
                    v = fma(-rrow[j], yj, v);
                }
            }
            if (mn > 0.0) break;
            --k;
        }
        if (lane == 0) {
            s.jdrops += kr - k;
            s.k = k;
            s.j1 = s.J[0];
            a.ex->restart = (k == 0);
            if (k == 0) {
                p.excl[s.j1] = 1;
                s.any_excl = 1;
            }
        }
    }
    ctl_store(s, a.ctl);
}

// Commit, pass 1 (all workgroups): snapshot of the appended columns of Q and
// the reset of the exclusions.
__global__ __launch_bounds__(WG) void lg_commit_copy(LgArgs a) {
    const Ctl* ctl = a.ctl;
    const int k = ctl->k;
    if (k == 0) return;
    const Prob& p = a.p;
    const int m = p.m, r0 = ctl->nP;
    const size_t tot = (size_t)m * k;
    for (size_t e = (size_t)blockIdx.x * WG + threadIdx.x; e < tot; e += (size_t)gridDim.x * WG)
        p.Qadd[e] = p.Q[(size_t)r0 * m + e];
    if (ctl->any_excl)
        for (int j = blockIdx.x * WG + threadIdx.x; j < p.n; j += gridDim.x * WG) p.excl[j] = 0;
}

// Commit, pass 2: P grows by J.
__global__ __launch_bounds__(WG) void lg_commit(LgArgs a) {
    __shared__ WgShared s;
    ctl_load(s, a.ctl);
    if (s.k == 0) return;
    const Prob& p = a.p;
    const int r0 = s.nP, k = s.k;
    if (threadIdx.x == 0) {
        for (int t = 0; t < k; ++t) {
            p.P[r0 + t] = s.J[t];
            p.pos[s.J[t]] = r0 + t;
        }
        s.any_excl = 0;
        s.nP = r0 + k;
        s.nPa = r0 + k;
        s.outer += 1;
        a.ex->inner_done = 0;
    }
    ctl_store(s, a.ctl);
}

// One inner iteration's bookkeeping: stop test, step length, new iterate,
// removal set, and the per-column layout of the downdate.  A downdating sweep
// handles at most RQ positions; further removals of the same iteration (their
// x is already 0) are swept by the next call before any new step is taken.
// the inner step's register path: IFC positions per thread (n_P <= 4096), and
// one count per (position slot, wave) in a 64-lane scan
constexpr int IFC = 16, NWI = WG / 64;
static_assert(IFC * NWI == 64, "the removal scan takes one count per lane of a wave");
__device__ void inner_body(LgArgs& a, WgShared& s) {
    ctl_load(s, a.ctl);
    LgExtra* ex = a.ex;
    if (s.k == 0) {
        if (threadIdx.x == 0) ex->inner_done = 1;
        return;
    }
    Wg wg(a.p, a.prm, s);
    const Prob& p = a.p;
    if (ex->pending) {
        wg.collect_removals();
    } else if (s.nP > 0 && s.nP <= WG * IFC) {
        // One inner iteration with the positions in registers: thread t owns
        // positions t + WG u (coalesced).  y and P come in one round trip, x in
        // a second one once the iteration is known to take a step.  The step
        // length, the new iterate and the removal set are those of
        // Wg::inner_step, in the same rounding.
        const int nP = s.nP, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
        double yc[IFC], xc[IFC];
        int jc[IFC];
#pragma unroll
        for (int u = 0; u < IFC; ++u) {
            const int c = min(tid + WG * u, nP - 1);
            yc[u] = p.ybuf[c];
            jc[u] = p.P[c];
        }
        double mn = INFINITY;
#pragma unroll
        for (int u = 0; u < IFC; ++u)
            if (tid + WG * u < nP) mn = fmin(mn, yc[u]);
        mn = wg.vmin(mn);
        if (mn > 0.0) {
            if (tid == 0) ex->inner_done = 1;
            return;
        }
        if (s.inner >= a.prm.max_inner) {
            if (tid == 0) {
                ex->inner_done = 1;
                a.ctl->status = LHDM_STATUS_MAXITER;
            }
            return;
        }
        __syncthreads();
        if (tid == 0) s.inner += 1;
        if (a.prm.signflip && wg.sign_flip()) {
            // y > 0 after the flip (Section 4.2): the inner loop ends, with no downdate
            if (tid == 0) ex->inner_done = 1;
            ctl_store(s, a.ctl);
            return;
        }
#pragma unroll
        for (int u = 0; u < IFC; ++u) xc[u] = p.x[jc[u]];
        double al = INFINITY;
#pragma unroll
        for (int u = 0; u < IFC; ++u)
            if (tid + WG * u < nP && yc[u] <= 0.0) al = fmin(al, step_ratio(xc[u], yc[u]));
        al = wg.vmin(al);
        unsigned fl = 0;   // bit u: position tid + WG u leaves the passive set
        {
#pragma clang fp contract(off)
#pragma unroll
            for (int u = 0; u < IFC; ++u) {
                if (tid + WG * u < nP) {
                    double xn = xc[u] + al * (yc[u] - xc[u]);
                    if (yc[u] <= 0.0 && step_ratio(xc[u], yc[u]) == al) xn = 0.0;
                    if (xn <= 0.0) {
                        xn = 0.0;
                        fl |= 1u << u;
                    }
                    p.x[jc[u]] = xn;
                }
            }
        }
        // rm = the flagged positions in ascending order, which is the order of
        // (u, wave, lane): a count per (u, wave) from the wave's ballot, their
        // exclusive scan by wave 0, then each flagged lane's rank in its ballot
        __shared__ int ucnt[IFC * NWI], ubase[IFC * NWI];
        unsigned long long bm[IFC];
#pragma unroll
        for (int u = 0; u < IFC; ++u) bm[u] = __ballot((fl >> u) & 1u);
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < IFC; ++u) ucnt[u * NWI + wid] = __popcll(bm[u]);
        }
        __syncthreads();
        if (wid == 0) {
            const int v = ucnt[lane];
            int incl = v;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int w = __shfl_up(incl, d, 64);
                if (lane >= d) incl += w;
            }
            ubase[lane] = incl - v;
            if (lane == 63) s.q = incl;
        }
        __syncthreads();
        const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
        for (int u = 0; u < IFC; ++u)
            if ((fl >> u) & 1u) p.rm[ubase[u * NWI + wid] + __popcll(bm[u] & below)] = tid + WG * u;
        __syncthreads();
    } else {
        // the smallest y and, in the same pass, the step length (the smallest
        // ratio x / (x - y) over the positions with y <= 0, which are few)
        double mn = INFINITY, al = INFINITY;
        const int nP = s.nP;
        for (int c0 = threadIdx.x; c0 < nP; c0 += WG * 8) {
            double v[8];   // eight loads in flight per thread
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = (c0 + WG * u < nP) ? p.ybuf[c0 + WG * u] : INFINITY;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                mn = fmin(mn, v[u]);
                if (v[u] <= 0.0) al = fmin(al, step_ratio(p.x[p.P[c0 + WG * u]], v[u]));
            }
        }
        mn = wg.vmin(mn);
        if (mn > 0.0) {
            if (threadIdx.x == 0) ex->inner_done = 1;
            return;
        }
        if (s.inner >= a.prm.max_inner) {
            if (threadIdx.x == 0) {
                ex->inner_done = 1;
                a.ctl->status = LHDM_STATUS_MAXITER;
            }
            return;
        }
        __syncthreads();
        if (threadIdx.x == 0) s.inner += 1;
        if (a.prm.signflip && wg.sign_flip()) {
            // y > 0 after the flip (Section 4.2): the inner loop ends, with no downdate
            if (threadIdx.x == 0) ex->inner_done = 1;
            ctl_store(s, a.ctl);
            return;
        }
        wg.inner_step(true, wg.vmin(al));
    }
    if (threadIdx.x == 0) {
        ex->pending = s.q > RQ;
        if (s.q > RQ) s.q = RQ;
    }
    __syncthreads();
    const int q = s.q, nP = s.nP;
    if (q == 0) {   // nothing to remove (cannot happen after a step: its argmin is removed)
        if (threadIdx.x == 0) {
            ex->first = 0;
            ex->ndown = 0;
            ex->totrot = 0;
            ex->pending = 0;
            ex->inner_done = 0;
        }
        ctl_store(s, a.ctl);
        return;
    }
    if (threadIdx.x == 0) {
        const int first = p.rm[0];
        ex->first = first;
        ex->ndown = nP - q - first;
        // segment t (1..q): kept columns between removal t-1 and removal t carry t rotations
        int off = 0;
        for (int t = 1; t <= q; ++t) {
            const int start_new = p.rm[t - 1] - (t - 1);   // new index of the first kept column after rm[t-1]
            const int end_old = (t < q) ? p.rm[t] : nP;
            ex->seg_start[t] = start_new;
            ex->seg_off[t] = off;
            off += t * (end_old - p.rm[t - 1] - 1);
        }
        ex->totrot = off;
        ex->inner_done = 0;
    }
    __syncthreads();
    for (int op = p.rm[0] + threadIdx.x; op < nP; op += WG) {
        int lo = 0, hi = q;   // number of removed positions < op (binary search)
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (p.rm[mid] < op) lo = mid + 1;
            else hi = mid;
        }
        if (lo < q && p.rm[lo] == op) continue;
        const int L = lo;
        const int c = op - L;
        const int idx = c - ex->first;
        a.ocol[idx] = op;
        a.lcnt[idx] = L;
        a.roff[idx] = ex->seg_off[L] + L * (c - ex->seg_start[L]);
    }
    ctl_store(s, a.ctl);
}
__global__ __launch_bounds__(WG) void lg_inner(LgArgs a, int pub) {
    __shared__ WgShared s;
    inner_body(a, s);
    publish(a, pub);
}

// bt (one more row of Q) through the rotations of a downdate in which every
// new column carries one rotation: rotation e acts on entries first + e and
// first + e + 1, as x_{e+1} = -s_e x_e + c_e y_e (x_e the running entry, y_e =
// bt[first + e + 1]) and bt[first + e] = c_e x_e + s_e y_e.  The recurrence is
// affine in x, so each chunk of 64 rotations is one inclusive scan of the
// maps x -> a x + b across the lanes (six shuffle steps) instead of 64
// dependent steps; the running entry carries from chunk to chunk.
__device__ inline void rotate_bt_unit(const LgArgs& a) {
    // All four waves take chunks at once (CPW each per sweep of 16 chunks): each chunk's
    // map comes from its own scan, one thread composes the chunk maps in order
    // to get every chunk's incoming entry, then each lane writes its output.
    // All loads of a sweep precede its stores (a chunk reads the first entry
    // of the next one).
    constexpr int CPW = 4, NCH = CPW * NW;
    __shared__ double agA[NCH], agB[NCH], xin[NCH + 1];
    const LgExtra* ex = a.ex;
    const int nd = ex->ndown, lane = threadIdx.x & 63, wv = wave_index();
    double* bt = a.p.bt + ex->first;
    double x0 = bt[0];
    for (int r0 = 0; r0 < nd; r0 += 64 * NCH) {
        double cc[CPW], ss[CPW], yy[CPW], A[CPW], B[CPW];
#pragma unroll
        for (int u = 0; u < CPW; ++u) {
            const int q = wv * CPW + u, e0 = r0 + 64 * q;
            const int ne = max(0, min(64, nd - e0));
            double c = 1.0, sn = 0.0, y = 0.0;
            if (lane < ne) {
                const int ro = a.roff[e0 + lane];
                c = a.rotbuf[2 * ro];
                sn = a.rotbuf[2 * ro + 1];
                y = bt[e0 + lane + 1];
            }
            cc[u] = c;
            ss[u] = sn;
            yy[u] = y;
            A[u] = (lane < ne) ? -sn : 1.0;
            B[u] = (lane < ne) ? c * y : 0.0;
        }
        // inclusive scans of the maps x -> A x + B across the lanes
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
#pragma unroll
            for (int u = 0; u < CPW; ++u) {
                const double Ap = __shfl_up(A[u], d, 64), Bp = __shfl_up(B[u], d, 64);
                if (lane >= d) {
                    B[u] = fma(A[u], Bp, B[u]);
                    A[u] = A[u] * Ap;
                }
            }
        }
        if (lane == 63) {
#pragma unroll
            for (int u = 0; u < CPW; ++u) {
                agA[wv * CPW + u] = A[u];   // identity past the chunk: lane 63 holds the whole chunk's map
                agB[wv * CPW + u] = B[u];
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double x = x0;
            for (int q = 0; q < NCH; ++q) {
                xin[q] = x;
                x = fma(agA[q], x, agB[q]);
            }
            xin[NCH] = x;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < CPW; ++u) {
            const int q = wv * CPW + u, e0 = r0 + 64 * q;
            const int ne = max(0, min(64, nd - e0));
            const double xq = xin[q];
            const double xa = fma(A[u], xq, B[u]);
            const double xu = __shfl_up(xa, 1, 64);   // every lane takes part: a source lane must be active
            const double xl = (lane == 0) ? xq : xu;
            if (lane < ne) bt[e0 + lane] = cc[u] * xl + ss[u] * yy[u];
        }
        x0 = xin[NCH];
        __syncthreads();   // xin and the aggregates are rewritten by the next sweep
    }
    if (threadIdx.x == 0) bt[nd] = x0;
}

// The compaction of P and the slots when every passive position fits in the
// registers of the workgroup (CLB per thread) and the removal list in LDS:
// all loads go out before one barrier and the compacted arrays are stored
// after it, with no staging copy (the same result as Wg::compact, which
// takes the other cases).  Returns false when the sizes do not fit.
constexpr int CLB = 16;
constexpr int RM_LDS = 2048;
__device__ inline bool compact_onepass(const Prob& p, WgShared& s) {
    const int q = s.q, nP = s.nP, tid = threadIdx.x;
    if (q == 0) return true;
    if (nP > WG * CLB || q > RM_LDS) return false;
    __shared__ int rms[RM_LDS];
    int pv[CLB], sv[CLB];
#pragma unroll
    for (int u = 0; u < CLB; ++u) {
        const int c = min(tid + WG * u, nP - 1);
        pv[u] = p.P[c];
        sv[u] = p.slot[c];
    }
    for (int t = tid; t < q; t += WG) rms[t] = p.rm[t];
    // every load has returned before any position is overwritten
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    __syncthreads();
#pragma unroll
    for (int u = 0; u < CLB; ++u) {
        const int c = tid + WG * u;
        if (c >= nP) continue;
        int lo = 0, hi = q;   // removals before position c
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (rms[mid] < c) lo = mid + 1;
            else hi = mid;
        }
        const int j = pv[u];
        if (lo < q && rms[lo] == c) {
            p.pos[j] = -1;
            p.slot[nP - q + lo] = sv[u];
        } else {
            const int w = c - lo;
            p.P[w] = j;
            p.slot[w] = sv[u];
            p.pos[j] = w;
        }
    }
    __syncthreads();
    if (tid == 0) s.nP = nP - q;
    __syncthreads();
    return true;
}

// rotbt != 0: also rotate bt (the downdate's columns all carry one rotation;
// the Q rotations then leave bt alone).
__global__ __launch_bounds__(WG) void lg_compact(LgArgs a, int rotbt) {
    __shared__ WgShared s;
    ctl_load(s, a.ctl);
    Wg wg(a.p, a.prm, s);
    if (!compact_onepass(a.p, s)) wg.compact();
    ctl_store(s, a.ctl);
    if (rotbt) rotate_bt_unit(a);
}

// w of the twins -a_j from w of the caller's columns (positivity-trick mode).
__global__ __launch_bounds__(WG) void lg_twin_w(LgArgs a) {
    const Prob& p = a.p;
    const int j = blockIdx.x * WG + threadIdx.x;
    if (j < p.nph) p.w[j + p.nph] = -p.w[j];
}

__global__ __launch_bounds__(WG) void lg_finalize(LgArgs a) {
    __shared__ WgShared s;
    ctl_load(s, a.ctl);
    Wg wg(a.p, a.prm, s);
    wg.finalize();
    if (threadIdx.x == 0 && a.p.info) a.p.info->cq_panels = a.ex->ncq;
}

// --------------------------------------------------------------------------
// X^T D on the FP64 matrix cores.
// X: column-major (ld ldx), rows [0, m), columns [0, ncols).  D: row-major
// m x 16*NT (Dt).  Each workgroup owns 16 columns; its four waves take
// interleaved 32-row steps.  MFMA operand mapping (v_mfma_f64_16x16x4f64):
// A operand lane l = A[l % 16][l / 16], B operand lane l = B[l / 16][l % 16],
// result lane l register v = D[4 v + l / 16][l % 16].  Lane l feeds column
// (l & 15) of the tile and row r0 + 8*(l >> 4) + s of the s-th instruction, on
// both operands, so each lane streams 64 contiguous bytes of its column per step.
// --------------------------------------------------------------------------
enum { MODE_PROJ = 0, MODE_DUAL = 1 };

struct ColmatArgs {
    const double* X;
    long long ldx;
    int m, ncols;
    const double* Dt;
    int ldd;         // row stride of Dt (>= 16 NT)
    int nvec;        // vectors in this launch (<= 16 NT)
    int mode;
    int al16;        // X and ldx allow 16-byte vector loads
    // MODE_PROJ: out[t * ldo + j]
    double* out;
    int ldo;
    // MODE_DUAL
    int v0;          // global index of the first vector of this launch
    int vtot;        // total vectors over all launches
    int kadd;        // vectors 1..kadd are added directions (subtracted)
    int exact;       // 1: u2 recomputed from scratch
    const int* skip; // launch is a no-op when *skip != 0 (may be null)
    Prob p;
    int* recomp;
    int* nrecomp;
};

template <int NT>
__device__ __forceinline__ void colmat_step(const double (&av)[8], const double* __restrict__ Dt, int ldd,
                                            int rowb, int lane, d4 (&acc)[NT]) {
    double bv[NT][8];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int s = 0; s < 8; ++s) bv[t][s] = Dt[(size_t)(rowb + s) * ldd + t * 16 + (lane & 15)];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int s = 0; s < 8; ++s) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[t][s], acc[t], 0, 0, 0);
}

__device__ __forceinline__ void load8(const double* __restrict__ src, bool al16, double (&v)[8]) {
    if (al16) {
        const double2* s2 = reinterpret_cast<const double2*>(src);
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const double2 x = s2[h];
            v[2 * h] = x.x;
            v[2 * h + 1] = x.y;
        }
    } else {
#pragma unroll
        for (int s = 0; s < 8; ++s) v[s] = src[s];
    }
}

template <int NT>
__global__ __launch_bounds__(WG) void lg_colmat_dot(ColmatArgs a) {
    if (a.skip && *a.skip) return;
    __shared__ double part[NW][NT][4][64];
    __shared__ double Ct[16][16 * NT + 1];
    const int lane = threadIdx.x & 63, wv = wave_index();
    const int j0 = blockIdx.x * 16;
    const int kk = lane >> 4;
    // columns past the end repeat the last column (their results are dropped)
    const int col = min(j0 + (lane & 15), a.ncols - 1);
    const double* xc = a.X + (size_t)col * a.ldx;
    const bool al16 = a.al16;
    d4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    const int nfull = a.m / 32;   // full 32-row steps; wave wv takes steps wv, wv + 4, ...
    int st = wv;
    double av[8], an[8];
    if (st < nfull) load8(xc + st * 32 + 8 * kk, al16, av);
    while (st < nfull) {
        const int sn = st + NW;
        if (sn < nfull) load8(xc + sn * 32 + 8 * kk, al16, an);
        colmat_step<NT>(av, a.Dt, a.ldd, st * 32 + 8 * kk, lane, acc);
#pragma unroll
        for (int q = 0; q < 8; ++q) av[q] = an[q];
        st = sn;
    }
    if (wv == (nfull % NW) && nfull * 32 < a.m) {
        // ragged tail: rows [32 nfull, m)
        const int rb = nfull * 32 + 8 * kk;
        double bv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) av[q] = (rb + q < a.m) ? xc[rb + q] : 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                bv[q] = (rb + q < a.m) ? a.Dt[(size_t)(rb + q) * a.ldd + t * 16 + (lane & 15)] : 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) part[wv][t][v][lane] = acc[t][v];
    __syncthreads();
    for (int idx = threadIdx.x; idx < NT * 4 * 64; idx += WG) {
        const int t = idx / 256, v = (idx / 64) % 4, l = idx % 64;
        double sum = part[0][t][v][l];
#pragma unroll
        for (int w = 1; w < NW; ++w) sum += part[w][t][v][l];
        // result layout of v_mfma_f64_16x16x4f64: lane l, register v holds
        // row (column of X) 4*v + l/16 and column (vector) l%16
        Ct[4 * v + (l >> 4)][t * 16 + (l & 15)] = sum;
    }
    __syncthreads();
    if (threadIdx.x >= 16) return;
    const int j = j0 + threadIdx.x;
    if (j >= a.ncols) return;
    const double* c = Ct[threadIdx.x];
    if (a.mode == MODE_PROJ) {
        for (int t = 0; t < a.nvec; ++t) a.out[(size_t)t * a.ldo + j] = c[t];
        return;
    }
    // MODE_DUAL: w_j and the projected-norm update
    const Prob& p = a.p;
    const bool tw = p.nph != p.n;
    int t0 = 0;
    double u2;
    if (a.v0 == 0) {
        p.w[j] = c[0];
        if (tw) p.w[j + p.nph] = -c[0];
        t0 = 1;
        u2 = a.exact ? 0.0 : p.u2[j];
    } else {
        u2 = p.u2[j];
    }
    for (int t = t0; t < a.nvec; ++t) {
        const int gv = a.v0 + t;
        const double d = c[t];
        if (!a.exact && gv <= a.kadd) u2 -= d * d;
        else u2 += d * d;
    }
    if (a.v0 + a.nvec >= a.vtot) {
        u2 = fmax(u2, 0.0);
        if (!a.exact && p.pos[j] < 0 && !twin_passive(p, j) && u2 < RECOMP_FRAC * p.an2[j]) {
            const int slotn = atomicAdd(a.nrecomp, 1);
            a.recomp[slotn] = j;
        }
    }
    p.u2[j] = u2;
    if (tw) p.u2[j + p.nph] = u2;
}

// Column block times vector block on FP64 MFMA 16x16x4, X column-major.
// The vectors are the columns of Dt, stored in the pair layout: element
// (row i, vector t) at ((i / 2) ldd + t) 2 + i % 2, with ldd vectors per row
// and a zero row after an odd last row, so that one 16-byte load gives a
// vector's values on the two rows that a lane feeds to consecutive MFMAs.  A workgroup owns CT
// 16-column tiles of X; its four waves take interleaved trips of PF 8-row
// steps over all CT tiles, so at any time the workgroup reads one contiguous
// block of rows of its columns, and Dt is read once per workgroup.  Lane
// (c = l % 16, g = l / 16) reads 16 bytes of its column per step (64
// contiguous bytes per column per load instruction).  Each wave keeps two
// register sets: the loads of the next trip are in flight while the current
// one is multiplied.  The waves meet once, to add their partial results.
//
// DUAL: vector 0 of the dual update (Dt column 0 = r) goes through the vector
// units and gives w = A^T r; Dt columns 1 .. 16 NT are the added, dropped or
// trailing directions of Q, whose squared dot products update the projected
// norms u2 (added: subtracted; others: added; exact mode: from zero).
// PROJ: Dt columns 0 .. 16 NT - 1; out[t * ldo + j] = X[:, j] . Dt[:, t].
template <int NT, int CT, int PF, bool DUAL, int DEPTH = 2>
__global__ __launch_bounds__(WG) void lg_colmat2(ColmatArgs a) {
    static_assert(DEPTH == 2 || DEPTH == 3, "two or three register sets");
    if (a.skip && *a.skip) return;
    constexpr int VO = DUAL ? 1 : 0;   // Dt column of MFMA vector 0
    constexpr int NCOL = 16 * CT;
    __shared__ double Cs[NW][CT][NT][4][64];   // per wave, column tile, vector tile, register, lane
    __shared__ double Rs[NW][CT][64];
    const int tid = threadIdx.x, lane = tid & 63, wv = wave_index(), g = lane >> 4, cl = lane & 15;
    const int j0 = blockIdx.x * NCOL;
    const double* __restrict__ Dt = a.Dt;
    const int m = a.m, ldd = a.ldd;
    const double* xc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) xc[c] = a.X + (size_t)min(j0 + 16 * c + cl, a.ncols - 1) * a.ldx;
    d4 acc[CT][NT];
    double rd[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        rd[c] = 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[c][t] = d4{0.0, 0.0, 0.0, 0.0};
    }
    struct Buf {
        double2 v[PF][CT];
        double rv[PF][2], bv[PF][2][NT];
    };
    auto ld = [&](int s0, Buf& B, auto guard) {
        constexpr bool G = decltype(guard)::value;
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int row = (s0 + u) * 8 + 2 * g;
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                if (!G) {
                    B.v[u][c] = *reinterpret_cast<const double2*>(xc[c] + row);
                } else {
                    B.v[u][c].x = (row < m) ? xc[c][row] : 0.0;
                    B.v[u][c].y = (row + 1 < m) ? xc[c][row + 1] : 0.0;
                }
            }
            // rows row and row + 1 of the pair layout: one 16-byte load per vector
            const bool ok = !G || row < m;
            const double2* d2 = reinterpret_cast<const double2*>(Dt) + (size_t)(ok ? row >> 1 : 0) * ldd;
            if (DUAL) {
                const double2 x = ok ? d2[0] : double2{0.0, 0.0};
                B.rv[u][0] = x.x;
                B.rv[u][1] = x.y;
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const double2 x = ok ? d2[VO + 16 * t + cl] : double2{0.0, 0.0};
                B.bv[u][0][t] = x.x;
                B.bv[u][1][t] = x.y;
            }
        }
    };
    auto mm = [&](const Buf& B) {
#pragma unroll
        for (int u = 0; u < PF; ++u)
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                if (DUAL) {
                    rd[c] = fma(B.v[u][c].x, B.rv[u][0], rd[c]);
                    rd[c] = fma(B.v[u][c].y, B.rv[u][1], rd[c]);
                }
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    acc[c][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(B.v[u][c].x, B.bv[u][0][t], acc[c][t], 0, 0, 0);
                    acc[c][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(B.v[u][c].y, B.bv[u][1][t], acc[c][t], 0, 0, 0);
                }
            }
    };
    // Full trips unguarded (16-byte loads need an aligned X, checked by the
    // host), then the ragged rows with bounds checks.
    const int nst = (m + 7) / 8, nfull = m / 8, step = NW * PF;
    int s0 = wv * PF;
    // full trips of this wave: s0 + i step for i < nfw.  The prefetch past the
    // last one re-reads the last one (its values are never used), so the loop
    // body has no branch and the loads stay ahead of the products.
    const int nfw = (nfull - s0 >= PF) ? (nfull - s0 - PF) / step + 1 : 0;
    if (nfw > 0 && DEPTH == 2) {
        const int slast = s0 + (nfw - 1) * step;
        Buf B0, B1;
        ld(s0, B0, std::false_type{});
        int i = 0;
        for (; i + 2 <= nfw; i += 2) {
            ld(s0 + step, B1, std::false_type{});
            mm(B0);
            ld(min(s0 + 2 * step, slast), B0, std::false_type{});
            mm(B1);
            s0 += 2 * step;
        }
        if (i < nfw) {
            mm(B0);
            s0 += step;
        }
    } else if (nfw > 0) {
        // three register sets: the loads run two trips ahead of the products
        const int slast = s0 + (nfw - 1) * step;
        Buf B0, B1, B2;
        ld(s0, B0, std::false_type{});
        ld(min(s0 + step, slast), B1, std::false_type{});
        int i = 0;
        for (; i + 3 <= nfw; i += 3) {
            ld(min(s0 + 2 * step, slast), B2, std::false_type{});
            mm(B0);
            ld(min(s0 + 3 * step, slast), B0, std::false_type{});
            mm(B1);
            ld(min(s0 + 4 * step, slast), B1, std::false_type{});
            mm(B2);
            s0 += 3 * step;
        }
        // B0 and B1 hold trips i and i + 1 where they exist
        if (i < nfw) {
            mm(B0);
            s0 += step;
        }
        if (i + 1 < nfw) {
            mm(B1);
            s0 += step;
        }
    }
    for (; s0 < nst; s0 += step) {
        Buf B;
        ld(s0, B, std::true_type{});
        mm(B);
    }
    // partial results: lane l, register v of a tile holds column 4 v + l / 16,
    // vector l % 16
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        if (DUAL) {
            double r = rd[c];
            r += __shfl_xor(r, 16, 64);
            r += __shfl_xor(r, 32, 64);
            Rs[wv][c][lane] = r;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) Cs[wv][c][t][v][lane] = acc[c][t][v];
    }
    __syncthreads();
    if (!DUAL) {
        // element (vector q, column jj): tile jj / 16, register (jj % 16) / 4,
        // lane (jj % 4) * 16 + q % 16, vector tile q / 16
        for (int e = tid; e < a.nvec * NCOL; e += WG) {
            const int q = e / NCOL, jj = e % NCOL, j = j0 + jj;
            if (j >= a.ncols) continue;
            const int c = jj >> 4, v = (jj & 15) >> 2, l = (jj & 3) * 16 + (q & 15), t = q >> 4;
            a.out[(size_t)q * a.ldo + j] =
                ((Cs[0][c][t][v][l] + Cs[1][c][t][v][l]) + Cs[2][c][t][v][l]) + Cs[3][c][t][v][l];
        }
        return;
    }
    if (tid >= NCOL) return;
    // thread tid: column j0 + tid, i.e. tile tid / 16, column 4 v + l / 16 = tid % 16
    const int c = tid >> 4, jc = tid & 15, v = jc >> 2;
    const int j = j0 + tid;
    if (j >= a.ncols) return;
    const double rsum = ((Rs[0][c][jc] + Rs[1][c][jc]) + Rs[2][c][jc]) + Rs[3][c][jc];
    const Prob& p = a.p;
    p.w[j] = rsum;
    if (p.nph != p.n) p.w[j + p.nph] = -rsum;
    double u2 = a.exact ? 0.0 : p.u2[j];
    for (int q = 0; q + 1 < a.nvec; ++q) {
        // vector 1 + q: tile q / 16, lane (jc % 4) * 16 + q % 16, register v
        const int t = q >> 4, l = (jc & 3) * 16 + (q & 15);
        const double d = ((Cs[0][c][t][v][l] + Cs[1][c][t][v][l]) + Cs[2][c][t][v][l]) + Cs[3][c][t][v][l];
        if (!a.exact && q + 1 <= a.kadd) u2 -= d * d;
        else u2 += d * d;
    }
    u2 = fmax(u2, 0.0);
    if (!a.exact && p.pos[j] < 0 && !twin_passive(p, j) && u2 < RECOMP_FRAC * p.an2[j]) {
        const int slotn = atomicAdd(a.nrecomp, 1);
        a.recomp[slotn] = j;
    }
    p.u2[j] = u2;
    if (p.nph != p.n) p.u2[j + p.nph] = u2;
}

// Dual pass with producer and consumer waves, for up to 32 MFMA vectors.
// A workgroup owns 64 columns of A and walks down them in stages of
// DW_ROWS rows.  Four producer waves read a stage with one column per load
// instruction (128 consecutive rows, 1 KB, non-temporal: A is read once and
// must not push the vector block out of L2) and write it to one of two
// padded LDS buffers; four consumer waves take the previous stage from LDS in
// the MFMA operand layout of lg_colmat2 (lane (cl, g): column 16 c + cl, rows
// 2 g and 2 g + 1 of an 8-row group; the 16-byte column padding makes those
// reads conflict-free) together with the vector block rows from L2, and
// accumulate w = A^T r on the vector units and the products with the
// directions on v_mfma_f64_16x16x4f64.  The loads never wait behind the
// products: the two roles are separate waves on each SIMD.  The epilogue is
// that of lg_colmat2 (same partial layout, same order of the four-way sum).
constexpr int DW_ROWS = 128;              // rows of A per stage
constexpr int DW_CB = DW_ROWS + 2;        // padded column length of a stage in LDS (doubles)
constexpr int DW_WG = 512;                // four producer and four consumer waves
typedef double dw_d2v __attribute__((ext_vector_type(2)));

// Workgroup barrier without a memory fence (the stage hand-off waits for its
// own LDS stores; a fence would also wait for the next stage's loads); the
// empty asm statements keep the compiler from moving memory accesses across.
__device__ __forceinline__ void dw_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

template <int NT>
__global__ __launch_bounds__(DW_WG) void lg_dual_ws(ColmatArgs a) {
    static_assert(NT == 1 || NT == 2, "one or two vector tiles");
    if (a.skip && *a.skip) return;
    constexpr int NCOL = 64;
    __shared__ __attribute__((aligned(16))) double st[2 * NCOL * DW_CB];
    const int tid = threadIdx.x, lane = tid & 63, wv = wave_index();
    const int m = a.m, j0 = blockIdx.x * NCOL;
    const int ns = (m + DW_ROWS - 1) / DW_ROWS, nfull = m / DW_ROWS;
    d4 acc[4][NT];
    double rd[4];
    if (wv < 4) {
        // producer wave wv: columns 16 wv .. 16 wv + 15 of the block (clamped
        // to the last column; those results are never written)
        const double* xc[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) xc[i] = a.X + (size_t)min(j0 + 16 * wv + i, a.ncols - 1) * a.ldx + 2 * lane;
        auto load = [&](int s, double2 (&R)[16]) {
            const int row = s * DW_ROWS + 2 * lane;
            if (s < nfull) {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const dw_d2v v = __builtin_nontemporal_load(reinterpret_cast<const dw_d2v*>(xc[i] + s * DW_ROWS));
                    R[i].x = v.x;
                    R[i].y = v.y;
                }
            } else {
                // ragged last stage: rows past m are zero
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    R[i].x = (row < m) ? xc[i][s * DW_ROWS] : 0.0;
                    R[i].y = (row + 1 < m) ? xc[i][s * DW_ROWS + 1] : 0.0;
                }
            }
        };
        auto store = [&](int buf, const double2 (&R)[16]) {
#pragma unroll
            for (int i = 0; i < 16; ++i)
                *reinterpret_cast<double2*>(st + (buf * NCOL + 16 * wv + i) * DW_CB + 2 * lane) = R[i];
            __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): the stage is in LDS
        };
        // stage s + 1 is in flight while stage s is stored; one barrier per stage
        double2 R0[16], R1[16];
        load(0, R0);
        for (int s = 0; s < ns; s += 2) {
            if (s + 1 < ns) load(s + 1, R1);
            store(0, R0);
            dw_barrier();
            if (s + 1 < ns) {
                if (s + 2 < ns) load(s + 2, R0);
                store(1, R1);
                dw_barrier();
            }
        }
    } else {
        // consumer wave q: rows 32 q .. 32 q + 31 of every stage, all 64 columns
        const int q = wv - 4, g = lane >> 4, cl = lane & 15;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            rd[c] = 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[c][t] = d4{0.0, 0.0, 0.0, 0.0};
        }
        // vector block rows of row group G (stage G / 4, group G % 4), two
        // groups ahead of their use; rows past m are clamped (A is zero there)
        auto dload = [&](int G, double2 (&D)[1 + NT]) {
            const int row = min((G >> 2) * DW_ROWS + 32 * q + 8 * (G & 3) + 2 * g, m - 1);
            const double2* d2 = reinterpret_cast<const double2*>(a.Dt) + (size_t)(row >> 1) * a.ldd;
            D[0] = d2[0];
#pragma unroll
            for (int t = 0; t < NT; ++t) D[1 + t] = d2[1 + 16 * t + cl];
            asm volatile("" ::: "memory");   // keep the prefetch where it is issued
        };
        auto xload = [&](int buf, int rg, double2 (&X)[4]) {
            const double* sb = st + (buf * NCOL + cl) * DW_CB + 32 * q + 8 * rg + 2 * g;
#pragma unroll
            for (int c = 0; c < 4; ++c) X[c] = *reinterpret_cast<const double2*>(sb + 16 * c * DW_CB);
        };
        auto mm = [&](const double2 (&X)[4], const double2 (&D)[1 + NT]) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                rd[c] = fma(X[c].x, D[0].x, rd[c]);
                rd[c] = fma(X[c].y, D[0].y, rd[c]);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    acc[c][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(X[c].x, D[1 + t].x, acc[c][t], 0, 0, 0);
                    acc[c][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(X[c].y, D[1 + t].y, acc[c][t], 0, 0, 0);
                }
            }
        };
        double2 D0[1 + NT], D1[1 + NT], D2[1 + NT], D3[1 + NT];
        dload(0, D0);
        dload(1, D1);
        for (int s = 0; s < ns; ++s) {
            dw_barrier();
            const int buf = s & 1, G = 4 * s;
            double2 X0[4], X1[4];
            xload(buf, 0, X0);
            dload(G + 2, D2);
            xload(buf, 1, X1);
            mm(X0, D0);
            dload(G + 3, D3);
            xload(buf, 2, X0);
            mm(X1, D1);
            dload(G + 4, D0);
            xload(buf, 3, X1);
            mm(X0, D2);
            dload(G + 5, D1);
            mm(X1, D3);
        }
    }
    __syncthreads();   // every stage consumed: the stage buffers take the partial results
    double* Cs = st;                              // [consumer][c][t][register][lane]
    double* Rs = st + 4 * 4 * NT * 4 * 64;        // [consumer][c][lane]
    if (wv >= 4) {
        const int q = wv - 4;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double r = rd[c];
            r += __shfl_xor(r, 16, 64);
            r += __shfl_xor(r, 32, 64);
            Rs[(q * 4 + c) * 64 + lane] = r;
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) Cs[(((q * 4 + c) * NT + t) * 4 + v) * 64 + lane] = acc[c][t][v];
        }
    }
    __syncthreads();
    if (tid >= NCOL) return;
    // thread tid: column j0 + tid, i.e. tile tid / 16, column 4 v + l / 16 = tid % 16
    const int c = tid >> 4, jc = tid & 15, v = jc >> 2;
    const int j = j0 + tid;
    if (j >= a.ncols) return;
    const auto part = [&](int qq, int t, int l) { return Cs[(((qq * 4 + c) * NT + t) * 4 + v) * 64 + l]; };
    const auto rpart = [&](int qq) { return Rs[(qq * 4 + c) * 64 + jc]; };
    const double rsum = ((rpart(0) + rpart(1)) + rpart(2)) + rpart(3);
    const Prob& p = a.p;
    p.w[j] = rsum;
    if (p.nph != p.n) p.w[j + p.nph] = -rsum;
    double u2 = a.exact ? 0.0 : p.u2[j];
    for (int qv = 0; qv + 1 < a.nvec; ++qv) {
        // vector 1 + qv: tile qv / 16, lane (jc % 4) * 16 + qv % 16, register v
        const int t = qv >> 4, l = (jc & 3) * 16 + (qv & 15);
        const double d = ((part(0, t, l) + part(1, t, l)) + part(2, t, l)) + part(3, t, l);
        if (!a.exact && qv + 1 <= a.kadd) u2 -= d * d;
        else u2 += d * d;
    }
    u2 = fmax(u2, 0.0);
    if (!a.exact && p.pos[j] < 0 && !twin_passive(p, j) && u2 < RECOMP_FRAC * p.an2[j]) {
        const int slotn = atomicAdd(a.nrecomp, 1);
        a.recomp[slotn] = j;
    }
    p.u2[j] = u2;
    if (p.nph != p.n) p.u2[j + p.nph] = u2;
}

__global__ __launch_bounds__(WG) void lg_gather_dual(LgArgs a, int v0, int pair) {
    const LgExtra* ex = a.ex;
    if (a.ex->restart) return;
    const Prob& p = a.p;
    const int nP = a.ctl->nP, m = p.m;
    const size_t tot = (size_t)(pair ? (m + 1) / 2 * 2 : m) * 64;
    for (size_t e = (size_t)blockIdx.x * WG + threadIdx.x; e < tot; e += (size_t)gridDim.x * WG) {
        int row, t;
        dt_coords(e, pair, row, t);
        const int gv = v0 + t;
        double v = 0.0;
        if (gv < ex->nvec && row < m) {
            if (gv == 0) v = p.r[row];
            else if (ex->exact) v = p.Q[(size_t)(nP + gv - 1) * m + row];
            else if (gv <= ex->kadd) v = p.Qadd[(size_t)(gv - 1) * m + row];
            else v = p.Q[(size_t)(nP + gv - 1 - ex->kadd) * m + row];
        }
        a.Dt[e] = v;
    }
}

// First vector block of the dual update in one launch: the sizes of the
// update (exact mode when the trailing columns are fewer), r = b - A_P x_P
// from the residual partials (added in chunk order) as vector 0, and vectors
// 1 .. 63 (added, dropped or trailing columns of Q).
__global__ __launch_bounds__(WG) void lg_dual_prep(LgArgs a, int pair) {
    LgExtra* ex = a.ex;
    if (ex->restart) return;
    const Ctl* c = a.ctl;
    const Prob& p = a.p;
    const int m = p.m, nP = c->nP, kadd = c->k, ndrop = c->nPa - c->nP;
    const int exact = (m - nP) <= kadd + ndrop;
    const int nvec = 1 + (exact ? (m - nP) : (kadd + ndrop));
    const int gid = blockIdx.x * WG + threadIdx.x, gs = gridDim.x * WG;
    if (gid == 0) {
        ex->exact = exact;
        ex->kadd = kadd;
        ex->nvec = nvec;
        ex->nrecomp = 0;
    }
    for (int row = gid; row < m; row += gs) {
        double acc = 0.0;
        for (int ch = 0; ch < RES_CHUNKS; ++ch) acc += a.rpart[(size_t)ch * m + row];
        const double rv = p.b[row] - acc;
        p.r[row] = rv;
        a.Dt[pair ? (size_t)(row >> 1) * 128 + (row & 1) : (size_t)row * 64] = rv;
    }
    if (pair && (m & 1) && gid == 0) a.Dt[(size_t)(m >> 1) * 128 + 1] = 0.0;   // zero row after an odd last row
    const size_t tot = (size_t)(pair ? (m + 1) / 2 * 2 : m) * 64;
    for (size_t e = gid; e < tot; e += gs) {
        int row, t;
        dt_coords(e, pair, row, t);
        if (t == 0) continue;
        double v = 0.0;
        if (t < nvec && row < m) {
            if (exact) v = p.Q[(size_t)(nP + t - 1) * m + row];
            else if (t <= kadd) v = p.Qadd[(size_t)(t - 1) * m + row];
            else v = p.Q[(size_t)(nP + t - 1 - kadd) * m + row];
        }
        a.Dt[e] = v;
    }
}

// Dt[:, 0] = r, other columns 0 (dual refresh when the solve stops early).
__global__ __launch_bounds__(WG) void lg_gather_r(LgArgs a) {
    const size_t tot = (size_t)a.p.m * 64;
    for (size_t e = (size_t)blockIdx.x * WG + threadIdx.x; e < tot; e += (size_t)gridDim.x * WG)
        a.Dt[e] = ((e % 64) == 0) ? a.p.r[e / 64] : 0.0;
}


// Exact u2 for flagged columns: sum over the trailing columns of Q.
__global__ __launch_bounds__(WG) void lg_recompute(LgArgs a) {
    const LgExtra* ex = a.ex;
    if (ex->restart) return;
    const int cnt = ex->nrecomp;
    const Prob& p = a.p;
    const int lane = threadIdx.x & 63;
    const int nP = a.ctl->nP;
    for (int e = blockIdx.x * NW + wave_index(); e < cnt; e += gridDim.x * NW) {
        const int j = a.recomp[e];
        const double* col = p.A + (size_t)j * p.lda;
        double u2 = 0.0;
        for (int t = nP; t < p.m; ++t) {
            const double* q = p.Q + (size_t)t * p.m;
            double d = 0.0;
            for (int i = lane; i < p.m; i += 64) d += col[i] * q[i];
            d = wave_sum(d);
            u2 += d * d;
        }
        if (lane == 0) {
            p.u2[j] = u2;
            if (p.nph != p.n) p.u2[j + p.nph] = u2;
        }
    }
}

// r = b - A_P x_P in two passes: partial sums over column chunks, then a
// fixed-order reduction.  The first pass also accepts y: unless the inner loop
// stopped at its iteration limit (x then stays the last feasible iterate),
// x_P = y, the sums use y directly and the first row block writes x.
__global__ __launch_bounds__(WG) void lg_residual_part(LgArgs a) {
    const Ctl* c = a.ctl;
    // launched before the host reads the inner decision: runs once the inner
    // loop has ended (and the outer step appended something)
    if (a.ex->restart || !a.ex->inner_done) return;
    const Prob& p = a.p;
    const int nP = c->nP;
    const bool accept = c->status != LHDM_STATUS_MAXITER;
    const int row = blockIdx.x * WG + threadIdx.x;
    const int chunk = blockIdx.y;
    const int per = (nP + RES_CHUNKS - 1) / RES_CHUNKS;
    const int c0 = chunk * per, c1 = min(nP, c0 + per);
    if (accept && blockIdx.x == 0)
        for (int cc = c0 + threadIdx.x; cc < c1; cc += WG) p.x[p.P[cc]] = p.ybuf[cc];
    // the chunk's column indices and coefficients are staged in LDS (RS at a
    // time), so that the column loads do not wait on the index loads; eight
    // columns' loads go out together and the sum keeps the column order
    constexpr int RS = 128, RB = 8;
    __shared__ int js[RS];
    __shared__ double xs[RS];
    double acc = 0.0;
    for (int s0 = c0; s0 < c1; s0 += RS) {
        const int ns = min(RS, c1 - s0);
        __syncthreads();   // the previous stage is consumed
        for (int t = threadIdx.x; t < ns; t += WG) {
            const int j = p.P[s0 + t];
            js[t] = j;
            xs[t] = accept ? p.ybuf[s0 + t] : p.x[j];
        }
        __syncthreads();
        if (row < p.m) {
            for (int cb = 0; cb < ns; cb += RB) {
                double av[RB];
#pragma unroll
                for (int u = 0; u < RB; ++u) {
                    double sg;
                    const double* col = col_ptr(p, js[min(cb + u, ns - 1)], sg);
                    av[u] = sg * col[row];
                }
#pragma unroll
                for (int u = 0; u < RB; ++u)
                    if (cb + u < ns) acc += av[u] * xs[cb + u];
            }
        }
    }
    if (row < p.m) a.rpart[(size_t)chunk * p.m + row] = acc;
}

__global__ __launch_bounds__(WG) void lg_residual_sum(LgArgs a) {
    if (a.ex->restart) return;
    const Prob& p = a.p;
    const int row = blockIdx.x * WG + threadIdx.x;
    if (row >= p.m) return;
    double acc = 0.0;
    for (int ch = 0; ch < RES_CHUNKS; ++ch) acc += a.rpart[(size_t)ch * p.m + row];
    p.r[row] = p.b[row] - acc;
}

// --------------------------------------------------------------------------
// Q[:, nP0:m] <- Q[:, nP0:m] (I - V T V^T) with kr reflectors, 16 rows of Q
// per workgroup.  Pass 1: W = Q_t V on the matrix cores (the four waves split
// the columns of Q_t), W2 = W T.  Pass 2: Q_t -= W2 V^T, computed transposed
// so that each store covers 16 consecutive rows of a column of Q.
// --------------------------------------------------------------------------
// Q[:, n_P:m] <- Q[:, n_P:m] (I - V T V^T) in two passes over the trailing
// columns.  Pass 1: W = Q_t V on FP64 MFMA, tile by tile.  Pass 2 (16 rows
// of Q per workgroup): W = the sum of the tiles' partial products, W2 = W T,
// then Q_t -= W2 V^T, four 16-column tiles in flight per wave.
constexpr int QRB = 128;  // rows per tile of pass 1
constexpr int QCB = 256;  // trailing columns per tile of pass 1
constexpr int QU1 = 16;   // 4-column steps in flight per wave (pass 1)
constexpr int QU2 = 4;    // 16-column tiles in flight per wave (pass 2)

// Pass 1 on a tile of QRB rows x QCB trailing columns: wave w owns rows
// 32 w .. 32 w + 31 of the tile (two 16-row MFMA tiles) and all its columns, so
// together the waves read 1 KB of every column of the tile.  The tile's
// product with V (QRB x kr) goes to its slot of wpart; pass 2 adds the slots.
__global__ __launch_bounds__(WG) void lg_qup1(LgArgs a) {
    const Ctl* ctl = a.ctl;
    const Prob& p = a.p;
    const int kr = ctl->kr, r0 = ctl->nP0, m = p.m, kq = p.kq;
    if (kr == 0) return;
    const int cb = blockIdx.y;
    const int c0 = r0 + cb * QCB, c1 = min(m, c0 + QCB);
    if (c0 >= m) return;
    const int lane = threadIdx.x & 63, wv = wave_index();
    const int ntile = (kr + 15) / 16;
    const int rbase = blockIdx.x * QRB + 32 * wv;
    int rows[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) rows[h] = min(rbase + 16 * h + (lane & 15), m - 1);
    d4 acc[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[h][t] = d4{0.0, 0.0, 0.0, 0.0};
    for (int l0 = c0; l0 < c1; l0 += 4 * QU1) {
        double av[QU1][2], bv[QU1][2];
#pragma unroll
        for (int u = 0; u < QU1; ++u) {
            const int l = l0 + 4 * u + (lane >> 4);
            const bool ok = l < c1;
#pragma unroll
            for (int h = 0; h < 2; ++h) av[u][h] = ok ? p.Q[(size_t)l * m + rows[h]] : 0.0;   // A[M=row][K=l]
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int sc = t * 16 + (lane & 15);
                bv[u][t] = (ok && sc < kr) ? p.Vt[(size_t)l * kq + sc] : 0.0;   // B[K=l][N=s]
            }
        }
#pragma unroll
        for (int u = 0; u < QU1; ++u)
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int t = 0; t < 2; ++t)
                    if (t < ntile) acc[h][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][h], bv[u][t], acc[h][t], 0, 0, 0);
        if (ntile > 2) {
            // panels wider than 32 columns: the remaining tiles, loads reissued
#pragma unroll
            for (int u = 0; u < QU1; ++u) {
                const int l = l0 + 4 * u + (lane >> 4);
#pragma unroll
                for (int t = 2; t < 4; ++t) {
                    const int sc = t * 16 + (lane & 15);
                    const double b = (l < c1 && sc < kr) ? p.Vt[(size_t)l * kq + sc] : 0.0;
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        if (t < ntile) acc[h][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][h], b, acc[h][t], 0, 0, 0);
                }
            }
        }
    }
    // lane l, register v of a tile: row 4 v + l / 16 of the 16-row tile, vector l % 16
    double* wp = a.wpart + (size_t)cb * kq * m;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (t < ntile)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = rbase + 16 * h + 4 * v + (lane >> 4), sc = t * 16 + (lane & 15);
                    if (row < m && sc < kr) wp[(size_t)sc * m + row] = acc[h][t][v];
                }
}

template <int NS4>   // 4-wide steps over the panel columns: 8 (kr <= 32) or 16 (kr <= 64)
__global__ __launch_bounds__(WG) void lg_qup2(LgArgs a) {
    const Ctl* ctl = a.ctl;
    const Prob& p = a.p;
    const int kr = ctl->kr, r0 = ctl->nP0, m = p.m, kq = p.kq;
    if (kr == 0) return;
    __shared__ double Wt[16][KM + 1];
    __shared__ double W2[16][KM + 1];
    const int lane = threadIdx.x & 63, wv = wave_index();
    const int i0 = blockIdx.x * 16;
    const int ncb = (m - r0 + QCB - 1) / QCB;   // column tiles of pass 1
    for (int e = threadIdx.x; e < 16 * kr; e += WG) {
        const int rr = e % 16, sc = e / 16;
        double w = 0.0;
        if (i0 + rr < m)
            for (int cb = 0; cb < ncb; ++cb) w += a.wpart[((size_t)cb * kq + sc) * m + i0 + rr];
        Wt[rr][sc] = w;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * kr; e += WG) {
        const int rr = e / kr, sc = e % kr;
        double sum = 0.0;
        for (int l = 0; l <= sc; ++l) sum += Wt[rr][l] * p.T[(size_t)sc * kq + l];
        W2[rr][sc] = sum;
    }
    __syncthreads();
    const int rr = i0 + (lane & 15);
    for (int c0 = r0 + 16 * wv; c0 < m; c0 += 16 * NW * QU2) {
        double qv[QU2][4], va[QU2][NS4];
#pragma unroll
        for (int u = 0; u < QU2; ++u) {
            const int cb = c0 + 16 * NW * u;
            const int cc = cb + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c2 = cb + 4 * v + (lane >> 4);
                qv[u][v] = (rr < m && c2 < m) ? p.Q[(size_t)c2 * m + rr] : 0.0;
            }
#pragma unroll
            for (int s4 = 0; s4 < NS4; ++s4) {
                const int sc = 4 * s4 + (lane >> 4);
                va[u][s4] = (4 * s4 < kr && sc < kr && cc < m) ? p.V[(size_t)sc * m + cc] : 0.0;   // A[M=col][K=s]
            }
        }
#pragma unroll
        for (int u = 0; u < QU2; ++u) {
            const int cb = c0 + 16 * NW * u;
            d4 o = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s4 = 0; s4 < NS4; ++s4) {
                if (4 * s4 < kr) {
                    const int sc = 4 * s4 + (lane >> 4);
                    const double bw = (sc < kr) ? W2[lane & 15][sc] : 0.0;   // B[K=s][N=row]
                    o = __builtin_amdgcn_mfma_f64_16x16x4f64(va[u][s4], bw, o, 0, 0, 0);
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c2 = cb + 4 * v + (lane >> 4);
                if (rr < m && c2 < m) p.Q[(size_t)c2 * m + rr] = qv[u][v] - o[v];
            }
        }
    }
}

// Pass 2 for panels of 3 to 32 reflectors and an even m, in two kernels.
// lg_qw2 forms W2 = W T once for all rows (W the sum of pass 1's tile
// partials, added in tile order, as in lg_qup2) and stores it by reflector,
// W2[s m + row], in the W scratch.  lg_qup2v then applies Q_t -= W2 V^T on the
// vector units: wave w of workgroup (bx, by) owns rows 512 bx + 128 w + 2 lane
// and + 1, so each load and store of a column is 16 bytes per lane and 1 KB
// per wave; its lanes keep their two rows of W2 in registers and the
// reflector entries of the workgroup's cpw (<= QV_COLS) trailing columns are
// broadcast from LDS (the host picks cpw so that the grid has ~512
// workgroups).  The products are about 7 us of FP64 FMA at n_P = m / 2 against
// ~50 us of HBM time, so the pass is bound by the stream of Q.
constexpr int QV_COLS = 64;   // trailing columns per workgroup of lg_qup2v

__global__ __launch_bounds__(WG) void lg_qw2(LgArgs a) {
    const Ctl* ctl = a.ctl;
    const Prob& p = a.p;
    const int kr = ctl->kr, r0 = ctl->nP0, m = p.m, kq = p.kq;
    if (kr == 0) return;
    __shared__ double Wt[16][KM + 1];
    const int i0 = blockIdx.x * 16;
    const int ncb = (m - r0 + QCB - 1) / QCB;   // column tiles of pass 1
    for (int e = threadIdx.x; e < 16 * kr; e += WG) {
        const int rr = e % 16, sc = e / 16;
        double w = 0.0;
        if (i0 + rr < m) {
            // eight tiles' loads at a time; the sum keeps tile order
            const double* q = a.wpart + (size_t)sc * m + i0 + rr;
            int cb = 0;
            for (; cb + 8 <= ncb; cb += 8) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = q[(size_t)(cb + u) * kq * m];
#pragma unroll
                for (int u = 0; u < 8; ++u) w += v[u];
            }
            for (; cb < ncb; ++cb) w += q[(size_t)cb * kq * m];
        }
        Wt[rr][sc] = w;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * kr; e += WG) {
        const int rr = e % 16, sc = e / 16;
        double sum = 0.0;
        for (int l = 0; l <= sc; ++l) sum += Wt[rr][l] * p.T[(size_t)sc * kq + l];
        if (i0 + rr < m) p.W[(size_t)sc * m + i0 + rr] = sum;
    }
}

__global__ __launch_bounds__(WG) void lg_qup2v(LgArgs a, int cpw) {
    const Ctl* ctl = a.ctl;
    const Prob& p = a.p;
    const int kr = ctl->kr, r0 = ctl->nP0, m = p.m, kq = p.kq;
    if (kr == 0) return;
    const int cbeg = r0 + cpw * blockIdx.y;
    if (cbeg >= m) return;
    const int nc = min(m, cbeg + cpw) - cbeg;
    __shared__ __attribute__((aligned(16))) double vs[QV_COLS][32];   // V[column][s], zero for s >= kr
    for (int e = threadIdx.x; e < QV_COLS * 32; e += WG) {
        const int cc = e >> 5, sc = e & 31;
        vs[cc][sc] = (cc < nc && sc < kr) ? p.Vt[(size_t)(cbeg + cc) * kq + sc] : 0.0;
    }
    const int lane = threadIdx.x & 63, wv = wave_index();
    const int row = blockIdx.x * 512 + 128 * wv + 2 * lane;   // even; row + 1 < m when row < m (m even)
    const bool ok = row < m;
    double w2[32][2];
#pragma unroll
    for (int sc = 0; sc < 32; ++sc) {
        double2 v = double2{0.0, 0.0};
        if (ok && sc < kr) v = *reinterpret_cast<const double2*>(p.W + (size_t)sc * m + row);
        w2[sc][0] = v.x;
        w2[sc][1] = v.y;
    }
    __syncthreads();
    double* qc = p.Q + (size_t)cbeg * m + (ok ? row : 0);
    constexpr int CU = 8;   // columns in flight per lane
    for (int c0 = 0; c0 < nc; c0 += CU) {
        double2 q[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u) q[u] = *reinterpret_cast<const double2*>(qc + (size_t)min(c0 + u, nc - 1) * m);
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            if (c0 + u < nc) {
                const int cc = c0 + u;
                double o0 = 0.0, o1 = 0.0;
#pragma unroll
                for (int sc = 0; sc < 32; sc += 2) {
                    const double2 v = *reinterpret_cast<const double2*>(&vs[cc][sc]);
                    o0 = fma(w2[sc][0], v.x, o0);
                    o1 = fma(w2[sc][1], v.x, o1);
                    o0 = fma(w2[sc + 1][0], v.y, o0);
                    o1 = fma(w2[sc + 1][1], v.y, o1);
                }
                if (ok) *reinterpret_cast<double2*>(qc + (size_t)cc * m) = double2{q[u].x - o0, q[u].y - o1};
            }
        }
    }
}

// --------------------------------------------------------------------------
// R y = bt[0:nP]: workgroup g solves row block nb-1-g after the blocks below
// it have published their part of y (epoch-tagged).  Each wave of the
// workgroup takes every fourth dependency block on its own (no workgroup
// barrier in the loop); the R entries of a dependency block are loaded before
// its part of y is awaited.
// --------------------------------------------------------------------------
// Blocks at least TRSV_CHAIN places from the bottom of the chain wait long
// enough for their four waves to invert the row-scaled diagonal block first;
// their final step is then one product with the inverse instead of a chain of
// 64 dependent steps.  The forward error of either form is bounded by the same
// |U^{-1}| |U| |y| (the inverse itself is formed by substitution).
constexpr int TRSV_CHAIN = 4;

// Inverse of the unit upper triangular 64 x 64 block U (row-scaled, diagonal
// 1, strictly upper part in U[i][j], i < j) into X[i][j], i <= j, by the four
// waves of the workgroup: the 16 x 16 diagonal tiles by back substitution
// (lane c of wave w forms column c of tile w), then the off-diagonal tiles
// from the block identity [A B; 0 C]^{-1} = [A^{-1}, -A^{-1} B C^{-1}; 0,
// C^{-1}] on 16- and then 32-wide blocks, with the products on the FP64
// matrix cores.  Entries of X below the diagonal tiles are not written.
// tw: 2 x 16 x 17 doubles, t2: 32 x 33 doubles of scratch.  Ends with a
// workgroup barrier.
__device__ __forceinline__ void tri_inv64(double (*U)[TB + 1], double (*X)[TB + 1], double (*tw)[16][17],
                                          double (*t2)[33]) {
    const int lane = threadIdx.x & 63, wv = wave_index(), r = lane & 15, g = lane >> 4;
    {
        const int o = 16 * wv, c = r;
        double x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) x[i] = (i == c) ? 1.0 : 0.0;
#pragma unroll
        for (int k = 15; k >= 1; --k) {
            const double xk = x[k];
#pragma unroll
            for (int i = 0; i < k; ++i) x[i] = fma(-U[o + i][o + k], xk, x[i]);
        }
        if (lane < 16) {
#pragma unroll
            for (int i = 0; i < 16; ++i) X[o + i][o + c] = x[i];
        }
    }
    __syncthreads();
    if (wv < 2) {
        // X[i][j] = -X[i][i] U[i][j] X[j][j] for the tile pair (i, j) = (2w, 2w + 1)
        const int oi = 32 * wv, oj = oi + 16;
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(U[oi + r][oj + kk + g], X[oj + kk + g][oj + r], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) tw[wv][4 * v + g][r] = acc[v];
        wave_lds_sync();
        acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(X[oi + r][oi + kk + g], tw[wv][kk + g][r], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) X[oi + 4 * v + g][oj + r] = -acc[v];
    }
    __syncthreads();
    // the top-right 32 x 32 block: t2 = B C^{-1}, then -A^{-1} t2, one 16 x 16
    // output tile (ti, tj) per wave; zero tiles of the triangular factors are skipped
    const int ti = wv >> 1, tj = wv & 1;
    {
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
        for (int kt = 0; kt <= tj; ++kt) {
#pragma unroll
            for (int kk = 0; kk < 16; kk += 4)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(U[16 * ti + r][32 + 16 * kt + kk + g],
                                                           X[32 + 16 * kt + kk + g][32 + 16 * tj + r], acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) t2[16 * ti + 4 * v + g][16 * tj + r] = acc[v];
    }
    __syncthreads();
    {
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
        for (int kt = ti; kt < 2; ++kt) {
#pragma unroll
            for (int kk = 0; kk < 16; kk += 4)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(X[16 * ti + r][16 * kt + kk + g],
                                                           t2[16 * kt + kk + g][16 * tj + r], acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) X[16 * ti + 4 * v + g][32 + 16 * tj + r] = -acc[v];
    }
    __syncthreads();
}

// outer != 0: the solve of an outer step, started before the append is
// committed (n_P is then the step's starting n_P plus the accepted columns).
__global__ __launch_bounds__(WG) void lg_trsv(LgArgs a, int epoch, int outer) {
    const Ctl* ctl = a.ctl;
    if (ctl->k == 0) return;
    const Prob& p = a.p;
    const int nP = outer ? ctl->nP0 + ctl->k : ctl->nP;
    const int nb = (nP + TB - 1) / TB;
    const int g = blockIdx.x;
    if (g >= nb) return;
    const int b = nb - 1 - g;
    const int r0 = b * TB, nr = min(nP, r0 + TB) - r0;
    const int tid = threadIdx.x, lane = tid & 63, wv = wave_index();
    __shared__ double part[NW][TB];
    __shared__ __attribute__((aligned(16))) double ys[NW][TB];
    __shared__ double Rd[TB][TB + 1];
    __shared__ double Xd[TB][TB + 1];
    __shared__ double tw[2][16][17];
    __shared__ double t2[32][33];
    __shared__ double dinv[TB];
    // row `lane` past the diagonal of the finishing matrix (the inverse or the
    // scaled block) and of M: entries (lane, 2 jp) and (lane, 2 jp + 1) at
    // [jp][lane], so that a lane reads its row with conflict-free 16-byte loads
    __shared__ double2 fm[TB / 2][TB];
    __shared__ double2 mq[TB / 2][TB];
    __shared__ int nonfin;
    {
        // diagonal block: four threads per column, one slot lookup each
        const int cc = tid >> 2, rq = (tid & 3) * (TB / 4);
        const double* col = (cc < nr) ? p.R + (size_t)p.slot[r0 + cc] * p.kc + r0 : nullptr;
#pragma unroll
        for (int u = 0; u < TB / 4; ++u) {
            const int rr = rq + u;
            Rd[rr][cc] = (col && rr <= cc) ? col[rr] : 0.0;
        }
    }
    const bool rowok = lane < nr;
    const double btv = rowok ? p.bt[r0 + lane] : 0.0;
    // A full block far enough up the chain is inverted (row-scaled) while it
    // waits, and the block below it (b + 1, the last to arrive) is folded in:
    // with X the inverse, D the diagonal and N = R[block b][block b + 1],
    //   y_b = X D^{-1} (bt_b - sum_{c > b + 1} R[b][c] y_c) - (X D^{-1} N) y_{b+1},
    // so once y_{b+1} arrives each wave adds 16 of its columns times M =
    // X D^{-1} N.  Every wave loads its 16 columns of N here.
    const bool by_inv = g >= TRSV_CHAIN && nr == TB;
    const int c1 = (b + 1) * TB, nc1 = by_inv ? min(nP, c1 + TB) - c1 : 0;
    double nv[16];
    if (by_inv) {
        const int slv = p.slot[c1 + min(16 * wv + (lane & 15), nc1 - 1)];
        const double* rowp = p.R + (size_t)(r0 + lane);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int jj = 16 * wv + k;
            const int sj = __builtin_amdgcn_readlane(slv, max(0, min(k, nc1 - 1 - 16 * wv)));
            const double val = rowp[(size_t)sj * p.kc];
            nv[k] = (jj < nc1) ? val : 0.0;
        }
    }
    if (tid == 0) nonfin = 0;
    __syncthreads();
    if (tid < TB) dinv[tid] = (tid < nr) ? 1.0 / Rd[tid][tid] : 0.0;
    __syncthreads();
    if (by_inv) {
        for (int e = tid; e < TB * TB; e += WG) {
            const int i = e >> 6, j = e & (TB - 1);
            if (j > i) Rd[i][j] *= dinv[i];
        }
        __syncthreads();
        tri_inv64(Rd, Xd, tw, t2);
        bool fin = true;
        for (int e = tid; e < TB * TB / 2; e += WG) {
            const int i = e & (TB - 1), jp = e >> 6, j = 2 * jp;
            const double x0 = (j > i) ? Xd[i][j] : 0.0, x1 = (j + 1 > i) ? Xd[i][j + 1] : 0.0;
            fin = fin && fabs(x0) < INFINITY && fabs(x1) < INFINITY;
            fm[jp][i] = double2{x0, x1};
        }
        if (!fin) nonfin = 1;
        __syncthreads();
    }
    // every entry of the inverse finite, else the chain on the scaled block
    const bool use_inv = by_inv && nonfin == 0;
    double2 mrow[8];   // this wave's 16 columns of row `lane` of M
    if (use_inv) {
        // D^{-1} N into Rd (no longer needed), then M = X (D^{-1} N) on the
        // matrix cores: wave w forms M's column tile w, skipping X's zero tiles
        const double di = dinv[lane];
#pragma unroll
        for (int k = 0; k < 16; ++k) Rd[lane][16 * wv + k] = nv[k] * di;
        __syncthreads();
        const int r = lane & 15, gq = lane >> 4;
        for (int ti = 0; ti < 4; ++ti) {
            d4 acc = d4{0.0, 0.0, 0.0, 0.0};
            for (int kt = ti; kt < 4; ++kt) {
#pragma unroll
                for (int kk = 0; kk < 16; kk += 4)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Xd[16 * ti + r][16 * kt + kk + gq],
                                                               Rd[16 * kt + kk + gq][16 * wv + r], acc, 0, 0, 0);
            }
            double* mdst = reinterpret_cast<double*>(&mq[8 * wv + (r >> 1)][0]) + (r & 1);
#pragma unroll
            for (int v = 0; v < 4; ++v) mdst[2 * (16 * ti + 4 * v + gq)] = acc[v];
        }
        wave_lds_sync();   // the wave reads back only its own column tile
#pragma unroll
        for (int k = 0; k < 8; ++k) mrow[k] = mq[8 * wv + k][lane];
    } else {
        for (int e = tid; e < TB * TB / 2; e += WG) {
            const int i = e & (TB - 1), jp = e >> 6, j = 2 * jp;
            const double sc = by_inv ? 1.0 : dinv[i];   // an inverted block's Rd is already scaled
            fm[jp][i] = double2{(j > i) ? Rd[i][j] * sc : 0.0, (j + 1 > i) ? Rd[i][j + 1] * sc : 0.0};
        }
        __syncthreads();
    }
    // the dependency blocks, every fourth one per wave (block b + 1 too when
    // it is not folded in); the wave that receives block b + 1 finishes a
    // block solved by substitution
    const int fw = (b == nb - 1) ? 0 : ((nb - 2 - b) & (NW - 1));
    const int last = use_inv ? b + 1 : b;
    double acc = 0.0;
    for (int cb = nb - 1 - wv; cb > last; cb -= NW) {
        const int c0 = cb * TB, nc = min(nP, c0 + TB) - c0;
        // the block's slot indices in one vector load, each broadcast from its
        // lane, so the 64 column loads wait on a single round trip; addresses
        // are clamped into the block and the values masked, with no branch
        const int slv = p.slot[c0 + min(lane, nc - 1)];
        const double* rowp = p.R + (size_t)(r0 + min(lane, nr - 1));
        double rv[TB];
#pragma unroll
        for (int j = 0; j < TB; ++j) {
            const int sj = __builtin_amdgcn_readlane(slv, min(j, nc - 1));
            const double val = rowp[(size_t)sj * p.kc];
            rv[j] = (j < nc && rowok) ? val : 0.0;
        }
        if (cb != b + 1) ll_wait_word(&a.yll[2 * (c0 + nc - 1) + 1], epoch, &a.ex->err);
        const double yv = ll_get<true>(&a.yll[2 * (c0 + min(lane, nc - 1))], lane < nc, epoch, &a.ex->err);
        ys[wv][lane] = (lane < nc) ? yv : 0.0;
        wave_lds_sync();
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
        for (int j = 0; j < TB; j += 4) {
            a0 += rv[j] * ys[wv][j];
            a1 += rv[j + 1] * ys[wv][j + 1];
            a2 += rv[j + 2] * ys[wv][j + 2];
            a3 += rv[j + 3] * ys[wv][j + 3];
        }
        acc += (a0 + a1) + (a2 + a3);
        wave_lds_sync();
    }
    part[wv][lane] = acc;
    __syncthreads();
    double v = 0.0;
    if (rowok) v = (btv - (((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane])) * dinv[lane];
    if (use_inv) {
        // X s over this wave's 16 columns (s broadcast from LDS), before y_{b+1}
        ys[wv][lane] = v;
        wave_lds_sync();
        const double2* s2 = reinterpret_cast<const double2*>(ys[wv]) + 8 * wv;
        double q0 = 0.0, q1 = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const double2 f = fm[8 * wv + k][lane], sv = s2[k];
            q0 = fma(f.x, sv.x, q0);
            q1 = fma(f.y, sv.y, q1);
        }
        // then minus M y_{b+1} over the same columns
        const double yv = ll_get<true>(&a.yll[2 * (c1 + 16 * wv + max(0, min(lane & 15, nc1 - 1 - 16 * wv)))],
                                       lane < 16, epoch, &a.ex->err);
        ys[wv][lane] = (16 * wv + lane < nc1 && lane < 16) ? yv : 0.0;
        wave_lds_sync();
        const double2* y2 = reinterpret_cast<const double2*>(ys[wv]);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const double2 yy = y2[k];
            q0 = fma(-mrow[k].x, yy.x, q0);
            q1 = fma(-mrow[k].y, yy.y, q1);
        }
        __syncthreads();   // every wave is past its reads of part
        part[wv][lane] = q0 + q1;
        __syncthreads();
        if (wv != 0) return;
        v += ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
    } else {
        if (wv != fw) return;
        // column-oriented back substitution on the row-scaled block: entry j
        // is final when step j reads it, and is broadcast through the scalar unit
        double rrow[TB];
#pragma unroll
        for (int jp = 0; jp < TB / 2; ++jp) {
            const double2 f = fm[jp][lane];
            rrow[2 * jp] = f.x;
            rrow[2 * jp + 1] = f.y;
        }
#pragma unroll
        for (int j = TB - 1; j >= 0; --j) {
            const double yj = readlane_d(v, j);
            v = fma(-rrow[j], yj, v);
        }
    }
    if (rowok) {
        ll_put(&a.yll[2 * (r0 + lane)], v, epoch);
        p.ybuf[r0 + lane] = v;
    }
}

// --------------------------------------------------------------------------
// Algorithm 5 on R.  Block b (one wave) owns new columns first + 64 b .. +64:
// it applies, in order, the rotations published by every earlier block to its
// columns, then generates its own column by column (bottom-up within a column)
// and publishes them.  A block whose columns carry one rotation each (a single
// removal in this stretch) keeps the 65 rows it touches in registers; any
// other block keeps the at most 64 + RQ rows it touches in an LDS window.
// Block metadata (rotation counts, offsets, old columns) is read one column
// per lane and broadcast by readlane, so no scalar load sits on the chain.
// --------------------------------------------------------------------------
constexpr int GW = GB + RQ;   // rows of a block's LDS window
constexpr int RCH = 16;       // rotations per chunk a unit block publishes while rotating

// Rotation zeroing b in (a, b) on every lane without branching; the scaled
// path is taken (uniformly) only when the lane that matters needs it.
__device__ __forceinline__ void givens_lane(double a, double b, int t, double& c, double& s) {
    const double mx = fmax(fabs(a), fabs(b));
    const double q = fma(a, a, b * b);
    const double y = rsqrt(q);
    c = a * y;
    s = b * y;
    if (b == 0.0) {
        c = 1.0;
        s = 0.0;
    }
    const bool bad = (b != 0.0) && !(mx > 0x1p-480 && mx < 0x1p480);
    if (__builtin_amdgcn_readlane((int)bad, t)) {
        double r;
        givens(a, b, c, s, r);
    }
}

// Algorithm 5 for a single removal, in closed form.  Deleting the column at
// position p leaves, in rows p.., the carried row r (row p) over an upper
// triangular T (rows p + 1.., one column to the left), and the new trailing
// factor R' satisfies R'^T R' = T^T T + r r^T.  The rotation that zeroes T_aa
// against the carried row (rho > 0, c = carried / rho, s = T_aa / rho, as the
// chained path takes it) has a closed form: with v = T^{-T} r, sigma_a = 1 +
// sum_{i<=a} v_i^2 and pi_a = prod_{i<a} (-sign T_ii), the carried entry is
// pi_a T_aa v_a / sqrt(sigma_{a-1}), so
//   c_a = pi_a sign(T_aa) v_a / sqrt(sigma_a),
//   s_a = sign(T_aa) sqrt(sigma_{a-1} / sigma_a).
// The serial part is one forward substitution for v, chained over the blocks
// of 64 new columns (each block waits for the v of the blocks before it); the
// sums and sign products are scans; each column then applies its rotations on
// its own.  The forward substitution is backward stable, so the entry that
// each column's last rotation leaves below its diagonal stays at rounding
// level whatever the conditioning of T.  Values pass between blocks through
// the epoch-tagged words of rotll past the chained path's 4 kc, which a single
// removal never uses.  A block whose rotations are not finite or not of unit
// norm (sigma overflowing, a zero pivot) makes every block leave its columns
// unchanged for the chained path (lg_givens, launched after it with the same
// epoch).  On success ex->cfok = epoch and lg_givens has nothing left to do.
//
// One workgroup of four waves per 64 new columns.  Column j of the block is
// new column idx = 64 b + j; its entries in rows p.. sit contiguously in its
// storage, so every load and store below takes 64 consecutive rows of one
// column (lane = row), and LDS turns them into columns for the lanes that
// carry a column's recurrence.
constexpr int CFW = 16;          // columns of the block per wave in the coalesced passes
constexpr int CF_MAXROT = 4096;  // rotations a workgroup keeps in LDS (longer downdates: lg_givens)
__global__ __launch_bounds__(WG) void lg_cfdown(LgArgs a, int epoch) {
    const LgExtra* ex = a.ex;
    if (ex->inner_done) return;   // launched before the host reads the inner decision
    const int nd = ex->ndown, first = ex->first;
    if (ex->totrot != nd || nd < 1 || nd > CF_MAXROT) return;
    const int b = blockIdx.x, nb = (nd + GB - 1) / GB;
    if (b >= nb) return;
    const Prob& p = a.p;
    const int tid = threadIdx.x, lane = tid & 63, wv = wave_index();
    int* err = &a.ex->err;
    const size_t kc = (size_t)p.kc;
    u64* cf = a.rotll + 4 * kc;   // v at 2 i, c at 2 (kc + i), s at 2 (2 kc + i); block ends past 6 kc
    u64* cfe = cf + 6 * kc;       // block b: sigma at 6 b, pi at 6 b + 2, ok at 6 b + 4
    __shared__ double tl[2][GB][GB + 1];    // tiles [row][column]
    __shared__ double2 rw[CF_MAXROT];       // rotations (c, s) 0 .. the block's last column
    __shared__ double vb[GB];
    __shared__ int okall_s;
    const int kmax = nd - 1 - b * GB;   // the block's last valid column
    // this wave's 16 columns: storage of column 16 wv + jj from row p on
    const int jw = CFW * wv + (lane & (CFW - 1));
    const int slw = p.slot[a.ocol[b * GB + min(jw, kmax)]];
    double* hw[CFW];
#pragma unroll
    for (int jj = 0; jj < CFW; ++jj)
        hw[jj] = p.R + (size_t)__builtin_amdgcn_readlane(slw, jj) * kc + first;
    // wave 0's lane j carries column j: its r (row p) and storage
    const int idc = min(b * GB + lane, nd - 1);
    const bool valid = b * GB + lane < nd;
    double* hc = p.R + (size_t)p.slot[a.ocol[idc]] * kc + first;
    const double r0 = (wv == 0) ? hc[0] : 0.0;
    // the block's diagonal tile T[64 b + k][column j] (rows clamped into storage)
    {
        const int rr = 1 + min(b * GB + lane, nd - 1);
#pragma unroll
        for (int jj = 0; jj < CFW; ++jj) tl[1][lane][CFW * wv + jj] = hw[jj][rr];
    }
    __syncthreads();
    // its diagonal, and the strictly upper part scaled by the row's inverse
    // diagonal entry (zero elsewhere), ahead of the wait for the blocks before
    if (tid < GB) vb[tid] = tl[1][min(tid, kmax)][tid];
    __syncthreads();
    for (int e = tid; e < GB * GB; e += WG) {
        const int k = e >> 6, j = e & (GB - 1);
        tl[1][k][j] = (k < j) ? tl[1][k][j] / vb[k] : 0.0;
    }
    // forward substitution, the blocks before this one: lane k of every wave
    // accumulates T[64 c + k][j] v_{64 c + k} for its 16 columns
    double acc[CFW];
#pragma unroll
    for (int jj = 0; jj < CFW; ++jj) acc[jj] = 0.0;
    if (b > 0) {
        double tv[CFW];
#pragma unroll
        for (int jj = 0; jj < CFW; ++jj) tv[jj] = hw[jj][1 + lane];   // block 0's rows (below every column here)
        for (int c = 0; c < b; ++c) {
            double tn[CFW];
            const int cn = min(c + 1, b - 1);
#pragma unroll
            for (int jj = 0; jj < CFW; ++jj) tn[jj] = hw[jj][1 + cn * GB + lane];
            if (c != b - 1) ll_wait_word(&cf[2 * (c * GB + GB - 1) + 1], epoch, err);
            // v of block c; wave 0 also takes block c - 1's rotations (long
            // published) in the same round trip, for the rotation table
            double vk = 0.0, ck = 0.0, sk = 0.0;
            bool okv = false, okr = wv != 0 || c == 0;
            for (long long it = 0;; ++it) {
                if (!okv) okv = ll_try(&cf[2 * (c * GB + lane)], epoch, vk);
                if (!okr) {
                    const int kp = (c - 1) * GB + lane;
                    okr = ll_try(&cf[2 * (kc + kp)], epoch, ck) && ll_try(&cf[2 * (2 * kc + kp)], epoch, sk);
                }
                if (__all(okv && okr)) break;
                if (it > SPIN_LIMIT) {
                    if (lane == 0) atomicExch(err, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (wv == 0 && c > 0) rw[(c - 1) * GB + lane] = double2{ck, sk};
#pragma unroll
            for (int jj = 0; jj < CFW; ++jj) {
                acc[jj] = fma(tv[jj], vk, acc[jj]);
                tv[jj] = tn[jj];
            }
        }
    }
#pragma unroll
    for (int jj = 0; jj < CFW; ++jj) tl[0][lane][CFW * wv + jj] = acc[jj];
    __syncthreads();
    if (wv == 0) {
        // column j's sum over the rows, then this block's part: forward
        // substitution on the column-scaled diagonal tile, each solved entry
        // broadcast through the scalar unit
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < GB; ++k) s4[k & 3] += tl[0][k][lane];
        double v = valid ? r0 - ((s4[0] + s4[1]) + (s4[2] + s4[3])) : 0.0;
        double tc[GB];
#pragma unroll
        for (int k = 0; k < GB; ++k) tc[k] = tl[1][k][lane];
        const double dg = vb[lane];   // T[idx][idx]
        const double dl = 1.0 / dg;
#pragma unroll
        for (int k = 0; k < GB; ++k) {
            const double vk = readlane_d(v, k);
            v = fma(-tc[k], vk, v);
        }
        const double vv = valid ? v * dl : 0.0;
        if (valid) ll_put(&cf[2 * (b * GB + lane)], vv, epoch);
        // sigma and the sign product across the block (scans), continued from
        // the previous block's end values
        double s0 = 1.0, p0 = 1.0, ok0 = 1.0;
        if (b > 0) {
            s0 = ll_get<true>(&cfe[6 * (b - 1)], true, epoch, err);
            p0 = ll_get<true>(&cfe[6 * (b - 1) + 2], true, epoch, err);
            ok0 = ll_get<true>(&cfe[6 * (b - 1) + 4], true, epoch, err);
            // the previous block's rotations, for the table
            const int kp = (b - 1) * GB + lane;
            const double ck = ll_get<true>(&cf[2 * (kc + kp)], true, epoch, err);
            const double sk = ll_get<true>(&cf[2 * (2 * kc + kp)], true, epoch, err);
            rw[kp] = double2{ck, sk};
        }
        double inc = vv * vv;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            vb[lane] = inc;
            wave_lds_sync();
            if (lane >= d) inc += vb[lane - d];
            wave_lds_sync();
        }
        vb[lane] = inc;
        wave_lds_sync();
        const double exc = (lane > 0) ? vb[lane - 1] : 0.0;
        const double sig = s0 + inc, sigm = s0 + exc;
        const bool pos = dg > 0.0;
        const unsigned long long pm = __ballot(valid && pos);
        const int npos = __popcll(pm & ((1ull << lane) - 1ull));
        const double pia = (npos & 1) ? -p0 : p0;
        const double sg = pos ? 1.0 : -1.0;
        const double rs = 1.0 / sqrt(sig);
        const double cc = pia * sg * vv * rs, ss = sg * sqrt(sigm) * rs;
        const bool good = !valid || (dg != 0.0 && fabs(fma(cc, cc, ss * ss) - 1.0) < 0x1p-40);
        rw[b * GB + lane] = double2{cc, ss};
        if (valid) {
            ll_put(&cf[2 * (kc + b * GB + lane)], cc, epoch);
            ll_put(&cf[2 * (2 * kc + b * GB + lane)], ss, epoch);
            a.rotbuf[2 * a.roff[b * GB + lane]] = cc;
            a.rotbuf[2 * a.roff[b * GB + lane] + 1] = ss;
        }
        const bool allgood = __all(good) && ok0 != 0.0;
        const double send = readlane_d(sig, min(kmax, GB - 1));   // sigma at the block's last column
        if (lane == 0) {
            ll_put(&cfe[6 * b], send, epoch);
            ll_put(&cfe[6 * b + 2], (__popcll(pm) & 1) ? -p0 : p0, epoch);
            ll_put(&cfe[6 * b + 4], allgood ? 1.0 : 0.0, epoch);
        }
        // every block's rotations are known once the last block reports (the
        // blocks are resident together; the wait is bounded): then apply them,
        // or leave the columns to the chained path
        const double okall = ll_get<true>(&cfe[6 * (nb - 1) + 4], true, epoch, err);
        if (lane == 0) okall_s = okall != 0.0;
    }
    __syncthreads();
    if (!okall_s) return;
    if (b == 0 && tid == 0) a.ex->cfok = epoch;
    // Apply the rotations, 64 rows at a time: rotation a meets rows p + a and
    // p + a + 1; column j runs the carried entry down rows 1 .. idx + 1 of its
    // column (lane j of wave 0), and its rows p .. p + idx + 1 are rewritten
    // (the last one to the zero its own rotation made).  All four waves load
    // and store the tiles (coalesced); the next tile's loads are in flight
    // while the current one is rotated.
    const int amax = min(nd - 1, b * GB + GB - 1);
    const int ntile = amax / GB + 1;
    double carry = r0;
    auto load_tile = [&](int t, double (&ld)[CFW]) {
#pragma unroll
        for (int jj = 0; jj < CFW; ++jj) ld[jj] = hw[jj][1 + min(t * GB + lane, nd - 1)];
    };
    auto put_tile = [&](int buf, const double (&ld)[CFW]) {
#pragma unroll
        for (int jj = 0; jj < CFW; ++jj) tl[buf][lane][CFW * wv + jj] = ld[jj];
    };
    // wave 0 rotates its column's 64 rows of tile t, eight at a time: the
    // next eight entries and rotations are read while the current ones run.
    // Table entries past amax (inside the table: amax + 1 rounds up to at most
    // CF_MAXROT) are never written; their steps lie past every column's own
    // rotation, so they only rotate carried entries that are not stored again.
    constexpr int RB = 8;
    auto rotate_tile = [&](int t) {
        const int buf = t & 1;
        const double2* rt = rw + t * GB;
        double cq[RB], cn[RB];
        double2 rq[RB], rn[RB];
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            cq[u] = tl[buf][u][lane];
            rq[u] = rt[u];
        }
#pragma unroll
        for (int q = 0; q < GB / RB; ++q) {
            if (q + 1 < GB / RB) {
#pragma unroll
                for (int u = 0; u < RB; ++u) {
                    cn[u] = tl[buf][RB * (q + 1) + u][lane];
                    rn[u] = rt[RB * (q + 1) + u];
                }
            }
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                // past the column's own rotation the carried entry and the
                // rows are never stored again (the row the own rotation zeroed
                // is stored as 0 by store_tile), so every step runs unmasked
                const double nv = fma(rq[u].x, carry, rq[u].y * cq[u]);
                carry = fma(-rq[u].y, carry, rq[u].x * cq[u]);
                cq[u] = nv;
            }
#pragma unroll
            for (int u = 0; u < RB; ++u) tl[buf][RB * q + u][lane] = cq[u];
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                cq[u] = cn[u];
                rq[u] = rn[u];
            }
        }
    };
    // rows p + 64 t + lane of the wave's columns, written up to each column's idx + 1
    auto store_tile = [&](int t) {
        const int buf = t & 1;
#pragma unroll
        for (int jj = 0; jj < CFW; ++jj) {
            const int j = CFW * wv + jj;
            const int aa = t * GB + lane;
            if (b * GB + j < nd && aa <= b * GB + j + 1) hw[jj][aa] = (aa <= b * GB + j) ? tl[buf][lane][j] : 0.0;
        }
    };
    // two tiles in flight: tile t + 1 waits in registers while tile t is
    // rotated, and tile t + 2's loads go out after tile t's stores
    double ra[CFW], rb[CFW];
    load_tile(0, ra);
    if (ntile > 1) load_tile(1, rb);
    put_tile(0, ra);
    if (ntile > 2) load_tile(2, ra);
    __syncthreads();
    for (int t = 0; t < ntile; t += 2) {
        if (wv == 0) rotate_tile(t);
        __syncthreads();
        store_tile(t);
        if (t + 1 < ntile) put_tile(1, rb);
        if (t + 3 < ntile) load_tile(t + 3, rb);
        __syncthreads();
        if (t + 1 >= ntile) break;
        if (wv == 0) rotate_tile(t + 1);
        __syncthreads();
        store_tile(t + 1);
        if (t + 2 < ntile) put_tile(0, ra);
        if (t + 4 < ntile) load_tile(t + 4, ra);
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void lg_givens(LgArgs a, int epoch) {
    const LgExtra* ex = a.ex;
    if (ex->inner_done) return;   // no inner step (the solver launches it only for one)
    const Prob& p = a.p;
    const int nd = ex->ndown, first = ex->first;
    const int nb = (nd + GB - 1) / GB;
    const int b = blockIdx.x;
    if (b >= nb) return;
    const int lane = threadIdx.x;
    const int idx = b * GB + lane;
    const bool valid = idx < nd;
    int* err = &a.ex->err;
    __shared__ double win[GW][64];
    __shared__ double rcl[RQ], rsl[RQ];
    if (ex->cfok == epoch) return;   // done in closed form by lg_cfdown
    // lanes past the last new column read the last one's storage (never written)
    double* col = p.R + (size_t)p.slot[a.ocol[valid ? idx : nd - 1]] * p.kc;
    // A full own block's rows 1..64 are touched by no earlier block: they are
    // staged in the LDS window while the previous block's rotations stream in,
    // and its row 0 is the previous pass's last row (kept in a register).
    const bool own_full = (b + 1) * GB <= nd;
    double x64 = 0.0;
    bool pre = false;
    for (int bb = 0; bb <= b; ++bb) {
        const bool own = bb == b;
        const int e0 = bb * GB, e1 = min(nd, e0 + GB), ne = e1 - e0;
        const int ml = e0 + min(lane, ne - 1);
        const int lc_l = a.lcnt[ml], ro_l = a.roff[ml], oc_l = a.ocol[ml];
        const int lc_last = __builtin_amdgcn_readlane(lc_l, ne - 1);
        const bool unit = __builtin_amdgcn_readlane(lc_l, 0) == 1 && lc_last == 1 && ne == GB;
        const int off = __builtin_amdgcn_readlane(ro_l, 0);
        const int rlo = first + e0;
        bool fallback = false;   // a unit block whose own rotations need the scaled path
        if (unit) {
            // rotation e of this block acts on rows (rlo + e, rlo + e + 1)
            double x[GB + 1];
            double* cp = col + rlo;   // per-lane base: the 65 accesses take immediate offsets
            if (own && pre) {
                x[0] = x64;
#pragma unroll
                for (int r = 1; r <= GB; ++r) x[r] = win[r - 1][lane];
            } else {
#pragma unroll
                for (int r = 0; r <= GB; ++r) x[r] = cp[r];
            }
            if (!own && bb != b - 1) {
                ll_wait_word(&a.rotll[4 * (off + GB - 1) + 3], epoch, err);
                const double rcv = ll_get<true>(&a.rotll[4 * (off + lane)], true, epoch, err);
                const double rsv = ll_get<true>(&a.rotll[4 * (off + lane) + 2], true, epoch, err);
                // rotation e reaches every lane through LDS (the loads run ahead
                // of the dependent updates)
                rcl[lane] = rcv;
                rsl[lane] = rsv;
                wave_lds_sync();
#pragma unroll
                for (int e = 0; e < GB; ++e) {
                    const double cs = rcl[e], sn = rsl[e];
                    const double x0 = x[e], x1 = x[e + 1];
                    x[e] = cs * x0 + sn * x1;
                    x[e + 1] = -sn * x0 + cs * x1;
                }
                wave_lds_sync();
            } else if (!own) {
                // the previous block is still rotating: take its rotations in
                // the chunks it publishes them in
#pragma unroll
                for (int ch = 0; ch < GB / RCH; ++ch) {
                    double st[RCH];   // own rows 1 + ch RCH .. in flight during this chunk
                    if (own_full) {
#pragma unroll
                        for (int u = 0; u < RCH; ++u) st[u] = cp[GB + 1 + ch * RCH + u];
                    }
                    const int k = ch * RCH + (lane & (RCH - 1));
                    const double rcv = ll_get<true>(&a.rotll[4 * (off + k)], lane < RCH, epoch, err);
                    const double rsv = ll_get<true>(&a.rotll[4 * (off + k) + 2], lane < RCH, epoch, err);
                    if (lane < RCH) {
                        rcl[k] = rcv;
                        rsl[k] = rsv;
                    }
                    wave_lds_sync();
#pragma unroll
                    for (int e = ch * RCH; e < ch * RCH + RCH; ++e) {
                        const double cs = rcl[e], sn = rsl[e];
                        const double x0 = x[e], x1 = x[e + 1];
                        x[e] = cs * x0 + sn * x1;
                        x[e + 1] = -sn * x0 + cs * x1;
                    }
                    if (own_full) {
#pragma unroll
                        for (int u = 0; u < RCH; ++u) win[ch * RCH + u][lane] = st[u];
                    }
                }
                wave_lds_sync();
            } else {
                int bad = -1;   // last step whose chunk passed the check
                // Every lane evaluates a rotation from its own entries; lane t's
                // is used at step t.  All lanes apply it (rows t and t + 1 of the
                // columns left of t are below their diagonal), so the step needs
                // no per-lane branch or mask; the rotation is kept in LDS and the
                // exact zero below lane t's diagonal is stored after the write-
                // back.  The unscaled rotation is taken on speculation: inputs
                // whose squares leave the normal range give a rotation that is
                // not finite or not of unit norm, and the block is then redone by
                // the general path below (scaled rotations) from the unchanged
                // column storage.  Chunks published before the check are
                // recomputed there with the same formulas up to rounding.
#pragma unroll
                for (int t = 0; t < GB; ++t) {
                    const double xa = x[t], xb = x[t + 1];
                    // 1 / sqrt(q) from the hardware estimate and one third-order
                    // correction, folded into c and s directly
                    const double q = fma(xa, xa, xb * xb);
                    const double y0 = __builtin_amdgcn_rsq(q);
                    const double e = fma(-q * y0, y0, 1.0);
                    const double pe = fma(e, 0.375, 0.5);
                    const double ca = ((xb == 0.0) ? fabs(xa) : xa) * y0, sa = xb * y0;
                    const double cl = fma(ca * e, pe, ca), sl = fma(sa * e, pe, sa);
                    const double cs = readlane_d(cl, t), sn = readlane_d(sl, t);
                    rcl[t] = cs;
                    rsl[t] = sn;
                    x[t] = cs * xa + sn * xb;
                    x[t + 1] = -sn * xa + cs * xb;
                    if ((t % RCH) == RCH - 1) {
                        // publish rotations t - RCH + 1 .. t for the next block
                        // once they are checked
                        wave_lds_sync();
                        const int k = t - RCH + 1 + (lane & (RCH - 1));
                        const double ck = rcl[k], sk = rsl[k];
                        const double nk = fma(ck, ck, sk * sk) - 1.0;
                        if (__any(!(fabs(nk) < 0x1p-40))) break;   // leaves the unrolled chain
                        if (lane < RCH) {
                            ll_put(&a.rotll[4 * (off + k)], ck, epoch);
                            ll_put(&a.rotll[4 * (off + k) + 2], sk, epoch);
                        }
                        bad = t;
                    }
                }
                fallback = bad != GB - 1;   // the last checked step is not the last one
                if (!fallback) {
                    wave_lds_sync();
                    a.rotbuf[2 * (off + lane)] = rcl[lane];
                    a.rotbuf[2 * (off + lane) + 1] = rsl[lane];
                }
                wave_lds_sync();
            }
            if (valid && !fallback) {
#pragma unroll
                for (int r = 0; r <= GB; ++r) cp[r] = x[r];
                if (own) cp[lane + 1] = 0.0;   // the entry this lane's rotation zeroed
            }
            x64 = x[GB];
            pre = !own && bb == b - 1 && own_full;
        }
        if (!unit || fallback) {
            // rows rlo .. rhi of this lane's column in the LDS window
            const int rhi = rlo + ne - 1 + lc_last;
            for (int r0 = rlo; r0 <= rhi; r0 += 8) {
                // eight loads in flight before their LDS writes
                double tmp[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) tmp[u] = (r0 + u <= rhi) ? col[r0 + u] : 0.0;
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (r0 + u <= rhi) win[r0 + u - rlo][lane] = tmp[u];
            }
            wave_lds_sync();
            if (!own) {
                const int kend = __builtin_amdgcn_readlane(ro_l, ne - 1) + lc_last;   // rotations [off, kend)
                if (bb != b - 1 && kend > off) ll_wait_word(&a.rotll[4 * (kend - 1) + 3], epoch, err);
                int kc0 = INT_MIN / 2;
                double rcv = 1.0, rsv = 0.0;
                for (int e = 0; e < ne; ++e) {
                    const int L = __builtin_amdgcn_readlane(lc_l, e), op = __builtin_amdgcn_readlane(oc_l, e);
                    const int ko = __builtin_amdgcn_readlane(ro_l, e);
                    if (L == 0) continue;
                    double run = win[op - rlo][lane];
                    for (int gg = 0; gg < L; ++gg) {
                        const int k = ko + gg;
                        if (k >= kc0 + 64) {
                            kc0 = k;
                            const int kk = min(k + lane, kend - 1);
                            rcv = ll_get<true>(&a.rotll[4 * kk], k + lane < kend, epoch, err);
                            rsv = ll_get<true>(&a.rotll[4 * kk + 2], k + lane < kend, epoch, err);
                        }
                        const double cs = readlane_d(rcv, k - kc0), sn = readlane_d(rsv, k - kc0);
                        const int i = op - gg;
                        const double v0 = win[i - 1 - rlo][lane];
                        win[i - rlo][lane] = -sn * v0 + cs * run;
                        run = cs * v0 + sn * run;
                    }
                    win[op - L - rlo][lane] = run;
                }
            } else {
                for (int e = 0; e < ne; ++e) {
                    const int L = __builtin_amdgcn_readlane(lc_l, e), op = __builtin_amdgcn_readlane(oc_l, e);
                    const int ko = __builtin_amdgcn_readlane(ro_l, e);
                    if (L == 0) continue;
                    if (lane == e) {
                        // bottom-up: zero rows op, op - 1, ..., op - L + 1 of this column
                        double run = win[op - rlo][lane];
                        for (int gg = 0; gg < L; ++gg) {
                            const int i = op - gg;
                            const double v0 = win[i - 1 - rlo][lane];
                            double cs, sn, rr;
                            givens_fast(v0, run, cs, sn, rr);
                            win[i - rlo][lane] = 0.0;
                            run = cs * v0 + sn * run;
                            rcl[gg] = cs;
                            rsl[gg] = sn;
                            ll_put(&a.rotll[4 * (ko + gg)], cs, epoch);
                            ll_put(&a.rotll[4 * (ko + gg) + 2], sn, epoch);
                            a.rotbuf[2 * (ko + gg)] = cs;
                            a.rotbuf[2 * (ko + gg) + 1] = sn;
                        }
                        win[op - L - rlo][lane] = run;
                    }
                    wave_lds_sync();
                    if (lane > e && valid) {
                        double run = win[op - rlo][lane];
                        for (int gg = 0; gg < L; ++gg) {
                            const double cs = rcl[gg], sn = rsl[gg];
                            const int i = op - gg;
                            const double v0 = win[i - 1 - rlo][lane];
                            win[i - rlo][lane] = -sn * v0 + cs * run;
                            run = cs * v0 + sn * run;
                        }
                        win[op - L - rlo][lane] = run;
                    }
                    wave_lds_sync();
                }
            }
            wave_lds_sync();
            if (valid)
                for (int r = rlo; r <= rhi; ++r) col[r] = win[r - rlo][lane];
        }
    }
}

// The downdate's rotations applied to the columns of Q and to bt (bt is
// handled as one more row of Q).  One lane per row; a workgroup holds 64 rows
// and 1 + QNL waves.  The loader waves stream the rows' entries in the touched
// columns of Q (blocks of QLB columns, loader l takes blocks l, l + QNL, ...)
// into an LDS ring of QW columns; the rotating wave takes the new columns in
// chunks of QC, waits until the loaders have delivered every column its chunk
// touches, rotates in the ring (the running entry of a stretch of single
// rotations stays in a register) and writes back the columns no later
// rotation touches.  Ring columns are reused only below the lowest column the
// rotating wave still needs; every wait is bounded.
constexpr int QC = 64;        // new columns per chunk
constexpr int QW = 256;       // ring columns (a chunk touches at most QC + RQ); a power of two
constexpr int QNL = 3;        // loader waves
constexpr int QLB = 64;       // columns per loader block

// skipbt != 0: bt is rotated elsewhere (lg_compact); its lane works on scratch.
__global__ __launch_bounds__(64 * (1 + QNL)) void lg_qrot(LgArgs a, int skipbt) {
    __shared__ double win[QW][64];
    __shared__ int lprog[QNL];   // blocks completed by each loader
    __shared__ int consumed;     // lowest column the rotating wave still needs
    __shared__ double2 rcs[QC];  // the chunk's rotations (c, s), read by broadcast
    const LgExtra* ex = a.ex;
    const Prob& p = a.p;
    const int m = p.m, nd = ex->ndown, first = ex->first;
    if (nd <= 0) return;
    const int lane = threadIdx.x & 63, wv = wave_index();
    const int row = blockIdx.x * 64 + lane;
    // rows past bt read and write a slot of the residual scratch (rewritten
    // before its next use), so no access below needs a lane mask
    const bool isbt = row == m && !skipbt;
    double* base = (row < m) ? p.Q + row : isbt ? p.bt : a.rpart + lane;
    const size_t stride = (row < m) ? (size_t)m : isbt ? 1 : 0;
    const int* lcnt = a.lcnt;
    const double* rot = a.rotbuf;
    int* err = &a.ex->err;
    const int rend = first + nd - 1 + lcnt[nd - 1];   // highest column touched
    if (threadIdx.x < QNL) lprog[threadIdx.x] = 0;
    if (threadIdx.x == 0) consumed = first;
    __syncthreads();
    if (wv > 0) {
        // loader wave l = wv - 1
        const int l = wv - 1;
        int done = 0;
        for (int k = l; first + k * QLB <= rend; k += QNL) {
            const int cb = first + k * QLB;
            long long it = 0;
            while (cb + QLB - 1 - __hip_atomic_load(&consumed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= QW) {
                if (++it > SPIN_LIMIT) {
                    if (lane == 0) atomicExch(err, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            double v[QLB];
#pragma unroll
            for (int u = 0; u < QLB; ++u) v[u] = (cb + u <= rend) ? base[(size_t)(cb + u) * stride] : 0.0;
#pragma unroll
            for (int u = 0; u < QLB; ++u)
                if (cb + u <= rend) win[(cb + u) & (QW - 1)][lane] = v[u];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
            ++done;
            if (lane == 0) __hip_atomic_store(&lprog[l], done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        return;
    }
    const int nch = (nd + QC - 1) / QC;
    const int totrot = ex->totrot;
    // rotations of a chunk whose columns carry one rotation each: lane u holds
    // the rotation of column e0 + u (loaded one chunk ahead)
    double rc_pf, rs_pf;
    {
        const int ro = a.roff[0] + lane;
        rc_pf = (lane < min(nd, QC) && ro < totrot) ? rot[2 * ro] : 1.0;
        rs_pf = (lane < min(nd, QC) && ro < totrot) ? rot[2 * ro + 1] : 0.0;
    }
    for (int ch = 0; ch < nch; ++ch) {
        const int e0 = ch * QC, e1 = min(nd, e0 + QC);
        const int need_hi = first + e1 - 1 + lcnt[e1 - 1];
        const double rc_cur = rc_pf, rs_cur = rs_pf;
        if (ch + 1 < nch) {
            const int en = min(nd, e1 + QC) - 1;
            const int ro = a.roff[e1] + lane;
            rc_pf = (e1 + lane <= en && ro < totrot) ? rot[2 * ro] : 1.0;
            rs_pf = (e1 + lane <= en && ro < totrot) ? rot[2 * ro + 1] : 0.0;
        }
        // wait until every block up to the one holding column need_hi is in the ring
        {
            const int kmax = (need_hi - first) / QLB;
            long long it = 0;
            while (true) {
                bool ok = true;
#pragma unroll
                for (int l = 0; l < QNL; ++l) {
                    if (kmax >= l) {
                        const int need_blocks = (kmax - l) / QNL + 1;
                        ok = ok && __hip_atomic_load(&lprog[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >=
                                       need_blocks;
                    }
                }
                if (ok) break;
                if (++it > SPIN_LIMIT) {
                    if (lane == 0) atomicExch(err, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        }
        if (lcnt[e0] == 1 && lcnt[e1 - 1] == 1) {
            // column e rotates rows (first + e, first + e + 1) with rotation roff[e]
            const int s0 = (first + e0) & (QW - 1);
            double x = win[s0][lane];
            double* q = base + (size_t)(first + e0) * stride;
            if (e1 - e0 == QC) {
                // whole chunk: rotations and ring entries read sixteen at a time
                // ahead of the dependent updates
                rcs[lane] = double2{rc_cur, rs_cur};
                wave_lds_sync();
#pragma unroll
                for (int g0 = 0; g0 < QC; g0 += 16) {
                    double yv[16];
                    double2 r2[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        yv[u] = win[(s0 + g0 + u + 1) & (QW - 1)][lane];
                        r2[u] = rcs[g0 + u];
                    }
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        const double cs = r2[u].x, sn = r2[u].y;
                        *q = cs * x + sn * yv[u];
                        q += stride;
                        x = -sn * x + cs * yv[u];
                    }
                }
                wave_lds_sync();
            } else {
#pragma unroll
                for (int u = 0; u < QC; ++u) {
                    if (e0 + u < e1) {
                        const double cs = readlane_d(rc_cur, u), sn = readlane_d(rs_cur, u);
                        const double y = win[(s0 + u + 1) & (QW - 1)][lane];
                        *q = cs * x + sn * y;
                        q += stride;
                        x = -sn * x + cs * y;
                    }
                }
            }
            win[(first + e1) & (QW - 1)][lane] = x;
        } else {
            for (int e = e0; e < e1; ++e) {
                // bottom-up: rotation gg acts on rows (op - gg - 1, op - gg)
                const int L = lcnt[e], off = a.roff[e], op = a.ocol[e];
                double r = win[op & (QW - 1)][lane];
                for (int gg = 0; gg < L; ++gg) {
                    const int i = op - gg;
                    const double cs = rot[2 * (off + gg)], sn = rot[2 * (off + gg) + 1];
                    const double v0 = win[(i - 1) & (QW - 1)][lane];
                    win[i & (QW - 1)][lane] = -sn * v0 + cs * r;
                    r = cs * v0 + sn * r;
                }
                win[(op - L) & (QW - 1)][lane] = r;
            }
            for (int rr = first + e0; rr < first + e1; ++rr) base[(size_t)rr * stride] = win[rr & (QW - 1)][lane];
        }
        // columns below first + e1 are final: their ring slots may be reused
        wave_lds_sync();
        if (lane == 0) __hip_atomic_store(&consumed, first + e1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    for (int rr = first + nd; rr <= rend; ++rr) base[(size_t)rr * stride] = win[rr & (QW - 1)][lane];
}

// --------------------------------------------------------------------------
// host driver
// --------------------------------------------------------------------------
struct LargeLayout {
    size_t slot, ybuf, Vt, Dt, rot, ocol, lcnt, roff, flt, flg, recomp, rpart, gpart, selv, seli, candw, candi, ctl,
        ex, misc,
        ppart, wfall, wpart, cq, total;
};

static LargeLayout large_layout(int m, int n, int kmax) {
    LargeLayout L;
    const size_t kc = (size_t)(m < n ? m : n);
    const size_t kq = (size_t)panel_cols(kmax);
    size_t o = 0;
    auto put = [&](size_t& off, size_t bytes) {
        off = o;
        o += pad256(bytes);
    };
    // hand-off buffers first: fixed offsets for a given kc
    put(L.flt, sizeof(u64) * 2 * kc);
    put(L.flg, sizeof(u64) * 4 * kc * RQ);
    put(L.ppart, sizeof(u64) * 2 * (2 * PNW + 2) * PSLOT);
    put(L.slot, slot_bytes(m, n, kmax));
    put(L.ybuf, sizeof(double) * kc);
    put(L.Vt, sizeof(double) * (size_t)m * kq);
    put(L.Dt, sizeof(double) * (size_t)(m + 1) * 64);
    put(L.rot, sizeof(double) * 2 * kc * RQ);
    put(L.ocol, sizeof(int) * kc);
    put(L.lcnt, sizeof(int) * kc);
    put(L.roff, sizeof(int) * kc);
    put(L.recomp, sizeof(int) * (size_t)n);
    put(L.rpart, sizeof(double) * (size_t)RES_CHUNKS * m);
    put(L.gpart, sizeof(double) * (size_t)std::max((m + GRAM_ROWS - 1) / GRAM_ROWS, PNW) * GP_STRIDE);
    put(L.selv, sizeof(double) * 3 * 64);
    put(L.seli, sizeof(int) * 64);
    put(L.candw, sizeof(double) * CAND_CAP);
    put(L.candi, sizeof(int) * CAND_CAP);
    put(L.ctl, sizeof(Ctl));
    put(L.ex, sizeof(LgExtra));
    put(L.misc, 256);
    put(L.wfall, sizeof(double) * (size_t)n);
    put(L.wpart, sizeof(double) * (size_t)((m + QCB - 1) / QCB) * kq * m);
    put(L.cq, sizeof(double) * CQ_DOUBLES);
    L.total = o;
    return L;
}

static size_t large_workspace_bytes(int m, int n, int kmax) { return large_layout(m, n, kmax).total; }

static int colmat_launch(hipStream_t st, ColmatArgs ca) {
    ca.al16 = ((((uintptr_t)ca.X) & 15) == 0) && ((ca.ldx & 1) == 0);
    const int grid = (ca.ncols + 15) / 16;
    if (grid == 0 || ca.nvec <= 0) return 0;
    const int nt = (ca.nvec + 15) / 16;
    if (nt <= 1) hipLaunchKernelGGL(lg_colmat_dot<1>, dim3(grid), dim3(WG), 0, st, ca);
    else if (nt == 2) hipLaunchKernelGGL(lg_colmat_dot<2>, dim3(grid), dim3(WG), 0, st, ca);
    else if (nt == 3) hipLaunchKernelGGL(lg_colmat_dot<3>, dim3(grid), dim3(WG), 0, st, ca);
    else hipLaunchKernelGGL(lg_colmat_dot<4>, dim3(grid), dim3(WG), 0, st, ca);
    HIPCHK(hipGetLastError());
    return 0;
}

// The pipelined column-block kernel applies when X allows 16-byte loads and
// the vector block fits 48 MFMA vectors (one launch for the whole dual
// update); its vectors are in the pair layout.  Otherwise colmat_launch
// (row-major vectors) is taken.
static bool colmat2_fits(const ColmatArgs& ca) {
    const bool al16 = ((((uintptr_t)ca.X) & 15) == 0) && ((ca.ldx & 1) == 0);
    if (!al16 || ca.ncols <= 0 || ca.nvec <= 0) return false;
    if (ca.mode == MODE_DUAL) return ca.v0 == 0 && ca.nvec == ca.vtot && ca.nvec <= 49;
    return ca.nvec <= 48;
}
// ev0 / ev1 (dual pass only, may be null): events the launch itself records at
// the kernel's start and end.
static void colmat2_launch(hipStream_t st, ColmatArgs ca, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
    ca.al16 = 1;
    if (ca.mode == MODE_DUAL) {
        // up to 32 directions: producer/consumer kernel; 33 to 48: the products
        // outweigh the stream and the single-role kernel keeps the MFMAs busier
        const dim3 g((ca.ncols + 63) / 64);
        if (ca.nvec <= 17) hipExtLaunchKernelGGL((lg_dual_ws<1>), g, dim3(DW_WG), 0, st, ev0, ev1, 0, ca);
        else if (ca.nvec <= 33) hipExtLaunchKernelGGL((lg_dual_ws<2>), g, dim3(DW_WG), 0, st, ev0, ev1, 0, ca);
        else hipExtLaunchKernelGGL((lg_colmat2<3, 4, 2, true, 3>), g, dim3(WG), 0, st, ev0, ev1, 0, ca);
        return;
    }
    const dim3 g((ca.ncols + 15) / 16);
    if (ca.nvec <= 16) hipLaunchKernelGGL((lg_colmat2<1, 1, 2, false>), g, dim3(WG), 0, st, ca);
    else if (ca.nvec <= 32) hipLaunchKernelGGL((lg_colmat2<2, 1, 2, false>), g, dim3(WG), 0, st, ca);
    else hipLaunchKernelGGL((lg_colmat2<3, 1, 2, false>), g, dim3(WG), 0, st, ca);
}

// The instance's state and the engine's buffers carved from a workspace laid
// out by large_layout (the caller's A, b and outputs are set by the caller).
static void large_bind(LgArgs& a, const LargeLayout& L, char* base, int m, int n, const DevParams& prm) {
    Prob& p = a.p;
    carve_slot(p, base + L.slot, m, n, prm.kmax);
    p.ybuf = (double*)(base + L.ybuf);
    p.Vt = (double*)(base + L.Vt);
    a.prm = prm;
    a.ctl = (Ctl*)(base + L.ctl);
    a.ex = (LgExtra*)(base + L.ex);
    a.Dt = (double*)(base + L.Dt);
    a.rotbuf = (double*)(base + L.rot);
    a.ocol = (int*)(base + L.ocol);
    a.lcnt = (int*)(base + L.lcnt);
    a.roff = (int*)(base + L.roff);
    a.yll = (u64*)(base + L.flt);
    a.rotll = (u64*)(base + L.flg);
    a.recomp = (int*)(base + L.recomp);
    a.rpart = (double*)(base + L.rpart);
    a.wpart = (double*)(base + L.wpart);
    a.gpart = (double*)(base + L.gpart);
    a.selv = (double*)(base + L.selv);
    a.seli = (int*)(base + L.seli);
    a.candw = (double*)(base + L.candw);
    a.candi = (int*)(base + L.candi);
    a.pll = (u64*)(base + L.ppart);
    a.cq = (double*)(base + L.cq);
    a.hmir = nullptr;
}

static int large_solve(hipStream_t st, int m, int n, const double* A, long long lda, const double* b,
                       const DevParams& prm, double* x, double* w, int* passive, lhdm_info* info, void* ws,
                       size_t ws_bytes) {
    const LargeLayout L = large_layout(m, n, prm.kmax);
    if (ws == nullptr) {
        int rc = cached_workspace(L.total, &ws);
        if (rc) return rc;
        ws_bytes = L.total;
    }
    if (ws_bytes < L.total || ((uintptr_t)ws & 255)) return LHDM_EWORKSPACE;
    if (L.ex - L.ctl != CTL_SPAN) return LHDM_EINVAL;   // Mirror assumes this spacing
    char* base = (char*)ws;
    LgArgs a;
    Prob& p = a.p;
    large_bind(a, L, base, m, n, prm);
    if (prm.twin) p.nph = n / 2;   // n counts the columns of [A, -A]
    p.A = A;
    p.lda = lda;
    p.b = b;
    p.x = x;
    p.w = w ? w : (double*)(base + L.wfall);
    p.passive = passive;
    p.info = info;
    unsigned long long* anmax_bits = (unsigned long long*)(base + L.misc);
    int* bad = (int*)(base + L.misc + 8);

    // The hand-off buffers are matched by epoch.  They are cleared at the start of
    // every solve and the epochs restart from 1, so no word left in the
    // workspace by an earlier call (of any entry point) can carry a live epoch.
    // Epochs stay below 2^30 within one solve (at most a few per outer and inner
    // step, bounded by max_outer and max_inner).
    HIPCHK(hipMemsetAsync(base + L.flt, 0, L.slot - L.flt, st));
    int ep_t = 0, ep_g = 0, ep_p = 0;
    // Host mirror in fine-grained (coherent) pinned memory: written by the
    // kernels that end with a host decision, polled here through `seq`.
    static thread_local Mirror* mir = nullptr;
    static thread_local int pubseq = 0;
    if (!mir) {
        HIPCHK(hipHostMalloc((void**)&mir, sizeof(Mirror),
                             hipHostMallocPortable | hipHostMallocMapped | hipHostMallocCoherent));
        __atomic_store_n(&mir->seq, -1, __ATOMIC_RELEASE);
    }
    HIPCHK(hipHostGetDevicePointer((void**)&a.hmir, mir, 0));

    // whole-stream synchronisation (start and end of the solve)
    // the loop runs on `cs` and forks the triangular solve onto `os`; at each
    // join the roles swap, so that the next kernel follows the solve on its own
    // stream and only waits on the other chain, which is usually done by then
    hipStream_t cs = st, os = nullptr;
    auto read_ctl = [&]() -> int {
        HIPCHK(hipMemcpyAsync(mir, a.ctl, offsetof(Mirror, seq), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        kprof_drain();
        const LgExtra* hx = reinterpret_cast<const LgExtra*>(mir->ex_head);
        if (hx->err) return LHDM_EHIP;
        return 0;
    };
    // Wait for the mirror published with sequence number `want`.  The stream
    // is queried now and then, so that a failed or drained stream ends the wait.
    auto next_pub = [&]() {
        pubseq = (pubseq + 1) & 0x3fffffff;
        return pubseq;
    };
    auto wait_pub = [&](int want) -> int {
        for (unsigned it = 1;; ++it) {
            if (__atomic_load_n(&mir->seq, __ATOMIC_ACQUIRE) == want) break;
            if ((it & 1023u) == 0) {
                const hipError_t e = hipStreamQuery(cs);
                if (e == hipSuccess && __atomic_load_n(&mir->seq, __ATOMIC_ACQUIRE) == want) break;
                if (e != hipErrorNotReady) return LHDM_EHIP;
            }
            __builtin_ia32_pause();
        }
        kprof_drain_if_half();
        const LgExtra* hx = reinterpret_cast<const LgExtra*>(mir->ex_head);
        return hx->err ? LHDM_EHIP : 0;
    };
    auto ex_h = [&]() { return reinterpret_cast<const LgExtra*>(mir->ex_head); };

    HIPCHK(hipMemsetAsync(base + L.misc, 0, 256, st));
    HIPCHK(hipMemsetAsync(a.ex, 0, sizeof(LgExtra), st));
    hipLaunchKernelGGL(lg_init_cols, dim3((p.nph + NW - 1) / NW), dim3(WG), 0, st, a, anmax_bits, bad);
    hipLaunchKernelGGL(lg_fill_identity, dim3(1024), dim3(WG), 0, st, p.Q, m);
    hipLaunchKernelGGL(lg_init_ctl, dim3(1), dim3(WG), 0, st, a, (const unsigned long long*)anmax_bits,
                       (const int*)bad);
    HIPCHK(hipGetLastError());
    int rc = read_ctl();
    if (rc) return rc;

    // side stream (default priority) and fork/join events, per host thread and device
    static thread_local int side_dev = -1;
    static thread_local hipStream_t side = nullptr;
    static thread_local hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    {
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        if (side_dev != dev) {
            HIPCHK(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
            HIPCHK(hipEventCreate(&ev_fork));
            HIPCHK(hipEventCreate(&ev_join));
            side_dev = dev;
        }
    }
    os = side;
    const int ggrid = 256;
    const int tgrid = (p.kc + TB - 1) / TB;
    const int rgrid = (m + WG - 1) / WG;
    bool stop = mir->ctl.status != LHDM_STATUS_OK;
    while (!stop) {
        if (ep_t > (1 << 30) || ep_g > (1 << 30) || ep_p > (1 << 22)) {
            // every earlier launch is ordered before this point on cs
            HIPCHK(hipMemsetAsync(base + L.flt, 0, L.slot - L.flt, cs));
            ep_t = ep_g = ep_p = 0;
        }
        hipLaunchKernelGGL(lg_sel_part, dim3(NSEL), dim3(WG), 0, cs, a, a.selv, a.seli);
        if (!prm.lh && prm.kmax > 1)
            hipLaunchKernelGGL(lg_sel_cand, dim3(NSEL), dim3(WG), 0, cs, a, (const double*)a.selv, (const int*)a.seli);
        const int ps = next_pub();
        hipLaunchKernelGGL(lg_sel_main, dim3(1), dim3(WG), 0, cs, a, (const double*)a.selv, (const int*)a.seli, ps);
        HIPCHK(hipGetLastError());
        // candidate projection G = Q^T A_J.  When the pipelined kernel can take
        // all kq panel columns it goes out before the selection is read: the
        // gather and the projection read J and its size on the device and skip
        // when the selection ended the solve (columns past ncol come out zero).
        ColmatArgs ca{};
        ca.X = p.Q;
        ca.ldx = m;
        ca.m = m;
        ca.ncols = m;
        ca.Dt = a.Dt;
        ca.ldd = 64;
        ca.mode = MODE_PROJ;
        ca.out = p.G;
        ca.ldo = m;
        ca.p = p;
        ca.nvec = p.kq;
        const bool early = colmat2_fits(ca);
        if (early) {
            ca.skip = &a.ctl->done;
            hipLaunchKernelGGL(lg_gather_cand, dim3(ggrid), dim3(WG), 0, cs, a, 1);
            colmat2_launch(cs, ca);
            HIPCHK(hipGetLastError());
        }
        if ((rc = wait_pub(ps))) return rc;
        if (mir->ctl.done) break;
        if (!early) {
            ca.nvec = mir->ctl.ncol;
            const bool pair = colmat2_fits(ca);
            hipLaunchKernelGGL(lg_gather_cand, dim3(ggrid), dim3(WG), 0, cs, a, (int)pair);
            if (pair) colmat2_launch(cs, ca);
            else if ((rc = colmat_launch(cs, ca))) return rc;
            HIPCHK(hipGetLastError());
        }
        const int gblk = (m + GRAM_ROWS - 1) / GRAM_ROWS;
        if (mir->ctl.ncol > 1) {
            hipLaunchKernelGGL(lg_gram_part, dim3(gblk), dim3(WG), 0, cs, a, 0, a.gpart);
        }
        int pblk = 0;   // partial Gram blocks of V read by lg_panel_b
        const int mp = m - mir->ctl.nP;
        const int cqb = (mp + CQ_ROWS - 1) / CQ_ROWS;   // row blocks of the CholeskyQR2 passes
        bool cq_try = false;
        {
            int rpw = std::max(64, (mp + PNW - 1) / PNW);
            rpw = ((rpw + 63) / 64) * 64;
            const int npw = (mp + rpw - 1) / rpw;
            const size_t lds = sizeof(double) * (size_t)rpw * (mir->ctl.ncol + 1);
            // CholeskyQR2 when the block may have 2 .. CQ_MAX columns; lg_greedy
            // decides (ex->cq_ok) and lg_panel_mw stands by for the rest
            cq_try = !prm.panel_hh && mir->ctl.ncol > 1 && mir->ctl.ncol <= CQ_MAX && lds <= (size_t)PANEL_LDS_MAX;
            hipLaunchKernelGGL(lg_greedy, dim3(1), dim3(WG), 0, cs, a, (const double*)a.gpart, (int)cq_try);
            if (cq_try) {
                hipLaunchKernelGGL(lg_cq_p1, dim3(cqb + (mir->ctl.nP + WG - 1) / WG), dim3(WG), 0, cs, a);
                hipLaunchKernelGGL(lg_cq_b, dim3(1), dim3(WG), 0, cs, a);
            }
            // the attribute is per device: set it once on each device a thread uses
            static thread_local unsigned long long attr_devs = 0;
            int cur_dev = 0;
            HIPCHK(hipGetDevice(&cur_dev));
            const unsigned long long bit = cur_dev < 64 ? (1ull << cur_dev) : 0ull;
            if (!(attr_devs & bit) || bit == 0) {
                HIPCHK(hipFuncSetAttribute((const void*)lg_panel_mw, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           PANEL_LDS_MAX));
                attr_devs |= bit;
            }
            ++ep_p;
            if (lds <= (size_t)PANEL_LDS_MAX) {
                // also writes V, V^T, the new R columns and the partial V^T V;
                // after a CholeskyQR2 factorisation only the second row pass
                const int gmw = npw + (mir->ctl.nP + WG - 1) / WG;
                hipLaunchKernelGGL(lg_panel_mw, dim3(cq_try ? std::max(gmw, cqb) : gmw), dim3(WG),
                                   cq_try ? std::max(lds, CQ_P2_LDS) : lds, cs, a, rpw, ep_p * 256);
                pblk = npw;
            } else {
                hipLaunchKernelGGL(lg_panel_1wg, dim3(1), dim3(WG), 0, cs, a);
                hipLaunchKernelGGL(lg_panel_v, dim3(64), dim3(WG), 0, cs, a);
                hipLaunchKernelGGL(lg_gram_part, dim3(gblk), dim3(WG), 0, cs, a, 1, a.gpart);
                pblk = (m - mir->ctl.nP + GRAM_ROWS - 1) / GRAM_ROWS;   // the blocks of rows >= n_P
            }
        }
        // the fork and join events are the launches' own end events
        // (hipExtLaunchKernelGGL), so no marker goes onto either stream
        hipExtLaunchKernelGGL(lg_panel_b, dim3(1), dim3(WG), 0, cs, nullptr, ev_fork, 0, a, (const double*)a.gpart,
                              pblk, cqb);
        // the triangular solve needs R, bt and the accepted count only: it runs
        // beside the Q update and the commit, on two streams.  The longer of
        // the two branches follows lg_panel_b on its stream and the other one
        // waits for the fork event: the Q update while the trailing part of Q
        // is wide, the solve (a chain over n_P / 64 row blocks) once n_P passes
        // about two thirds of m, where the two cross on a 4096-row instance.
        const bool solve_direct = 3 * mir->ctl.nP > 2 * m;
        hipStream_t qs = solve_direct ? os : cs, ts = solve_direct ? cs : os;
        HIPCHK(hipStreamWaitEvent(os, ev_fork, 0));
        ++ep_t;
        hipLaunchKernelGGL(lg_trsv, dim3(tgrid), dim3(WG), 0, ts, a, ep_t, 1);
        HIPCHK(hipGetLastError());
        if (cq_try) hipLaunchKernelGGL(lg_cq_bt, dim3((mp + WG - 1) / WG), dim3(WG), 0, qs, a);
        hipLaunchKernelGGL(lg_qup1, dim3((m + QRB - 1) / QRB, (m - mir->ctl.nP + QCB - 1) / QCB), dim3(WG), 0, qs, a);
        // one or two reflectors (plain LH): the single-kernel pass 2 is cheaper
        // than forming W2 in a launch of its own
        if (mir->ctl.ncol <= 32 && mir->ctl.ncol > 2 && (m & 1) == 0) {
            const int mp = m - mir->ctl.nP, gx = (m + 511) / 512;
            const int cpw = std::min(QV_COLS, std::max(8, (mp * gx / 512) / 8 * 8));
            hipLaunchKernelGGL(lg_qw2, dim3((m + 15) / 16), dim3(WG), 0, qs, a);
            hipLaunchKernelGGL(lg_qup2v, dim3(gx, (mp + cpw - 1) / cpw), dim3(WG), 0, qs, a, cpw);
        } else if (mir->ctl.ncol <= 32) {
            hipLaunchKernelGGL(lg_qup2<8>, dim3((m + 15) / 16), dim3(WG), 0, qs, a);
        } else {
            hipLaunchKernelGGL(lg_qup2<16>, dim3((m + 15) / 16), dim3(WG), 0, qs, a);
        }
        hipLaunchKernelGGL(lg_commit_copy, dim3(256), dim3(WG), 0, qs, a);
        hipExtLaunchKernelGGL(lg_commit, dim3(1), dim3(WG), 0, qs, nullptr, ev_join, 0, a);
        HIPCHK(hipGetLastError());
        // the loop continues on the solve's stream once the other branch is in
        HIPCHK(hipStreamWaitEvent(ts, ev_join, 0));
        if (!solve_direct) std::swap(cs, os);
        bool restart = false;
        while (true) {
            const int pi = next_pub();
            hipLaunchKernelGGL(lg_inner, dim3(1), dim3(WG), 0, cs, a, pi);
            // both continuations go out before the decision is read, each
            // checking it on the device: the downdate of an inner step (in
            // closed form for one removal), and x = y with the residual
            // partials when the inner loop ends
            ++ep_g;
            hipLaunchKernelGGL(lg_cfdown, dim3((p.kc + GB - 1) / GB), dim3(WG), 0, cs, a, ep_g);
            hipLaunchKernelGGL(lg_residual_part, dim3(rgrid, RES_CHUNKS), dim3(WG), 0, cs, a);
            HIPCHK(hipGetLastError());
            if ((rc = wait_pub(pi))) return rc;
            if (ex_h()->restart) {
                restart = true;
                break;
            }
            if (ex_h()->inner_done) {
                if (mir->ctl.status == LHDM_STATUS_MAXITER) stop = true;
                break;
            }
            // the chained rotations, for a removal the closed form declined
            // (launched once the inner step is known to go on, so the outer
            // steps do not pay for it; it returns at once after lg_cfdown)
            hipLaunchKernelGGL(lg_givens, dim3((p.kc + GB - 1) / GB), dim3(64), 0, cs, a, ep_g);
            if (ex_h()->totrot == ex_h()->ndown) {
                // one rotation per column: bt is rotated with the compaction, and
                // the Q rotations run on the other stream beside the triangular
                // solve, which is the longer of the two and so follows the
                // compaction directly (no event wait on its path)
                hipExtLaunchKernelGGL(lg_compact, dim3(1), dim3(WG), 0, cs, nullptr, ev_fork, 0, a, 1);
                HIPCHK(hipStreamWaitEvent(os, ev_fork, 0));
                ++ep_t;
                hipLaunchKernelGGL(lg_trsv, dim3(tgrid), dim3(WG), 0, cs, a, ep_t, 0);
                HIPCHK(hipGetLastError());
                hipExtLaunchKernelGGL(lg_qrot, dim3((m + 1 + 63) / 64), dim3(64 * (1 + QNL)), 0, os, nullptr, ev_join,
                                      0, a, 1);
                HIPCHK(hipGetLastError());
                HIPCHK(hipStreamWaitEvent(cs, ev_join, 0));
            } else {
                hipLaunchKernelGGL(lg_qrot, dim3((m + 1 + 63) / 64), dim3(64 * (1 + QNL)), 0, cs, a, 0);
                hipLaunchKernelGGL(lg_compact, dim3(1), dim3(WG), 0, cs, a, 0);
                ++ep_t;
                hipLaunchKernelGGL(lg_trsv, dim3(tgrid), dim3(WG), 0, cs, a, ep_t, 0);
                HIPCHK(hipGetLastError());
            }
        }
        if (restart) continue;
        // x = y and r's partials are already queued (they ran once the inner loop ended)
        if (stop) {
            hipLaunchKernelGGL(lg_residual_sum, dim3(rgrid), dim3(WG), 0, cs, a);
            HIPCHK(hipGetLastError());
            break;
        }
        HIPCHK(hipGetLastError());
        // dual w = A^T r fused with the projected-norm update
        const int nP = mir->ctl.nP, kadd = mir->ctl.k, ndrop = mir->ctl.nPa - mir->ctl.nP;
        const int exact = (m - nP) <= kadd + ndrop;
        const int nvec = 1 + (exact ? (m - nP) : (kadd + ndrop));
        for (int v0 = 0; v0 < nvec; v0 += 64) {
            ColmatArgs ca{};
            ca.X = A;
            ca.ldx = lda;
            ca.m = m;
            ca.ncols = p.nph;   // the caller's columns (their twins are written beside them)
            ca.Dt = a.Dt;
            ca.ldd = 64;
            ca.mode = MODE_DUAL;
            ca.nvec = std::min(64, nvec - v0);
            ca.v0 = v0;
            ca.vtot = nvec;
            ca.kadd = kadd;
            ca.exact = exact;
            ca.p = p;
            ca.recomp = a.recomp;
            ca.nrecomp = &a.ex->nrecomp;
            // algorithmic bytes: A once, the vector block, w written, u2 read and written
            const double bytes = 8.0 * ((double)m * p.nph + (double)m * 64 + 3.0 * n);
            const bool pair = colmat2_fits(ca);
            // the first block also forms r and the sizes of the update
            if (v0 == 0) hipLaunchKernelGGL(lg_dual_prep, dim3(ggrid), dim3(WG), 0, cs, a, (int)pair);
            else hipLaunchKernelGGL(lg_gather_dual, dim3(ggrid), dim3(WG), 0, cs, a, v0, (int)pair);
            if (pair) {
                // the launch records its own start and stop events
                const int ev = kprof_slot();
                colmat2_launch(cs, ca, kprof_event(ev), kprof_event(ev < 0 ? -1 : ev + 1));
                HIPCHK(hipGetLastError());
                kprof_commit(ev, bytes);
            } else {
                const int ev = kprof_begin(cs);
                if ((rc = colmat_launch(cs, ca))) return rc;
                HIPCHK(hipGetLastError());
                kprof_end(cs, ev, bytes);
            }
        }
        hipLaunchKernelGGL(lg_recompute, dim3(64), dim3(WG), 0, cs, a);
        HIPCHK(hipGetLastError());
    }
    if (stop && mir->ctl.status == LHDM_STATUS_MAXITER) {
        // x is the last feasible iterate: refresh w for it
        hipLaunchKernelGGL(lg_gather_r, dim3(ggrid), dim3(WG), 0, cs, a);
        ColmatArgs ca{};
        ca.X = A;
        ca.ldx = lda;
        ca.m = m;
        ca.ncols = p.nph;
        ca.Dt = a.Dt;
        ca.ldd = 64;
        ca.mode = MODE_PROJ;
        ca.out = p.w;
        ca.ldo = n;
        ca.nvec = 1;
        ca.p = p;
        if ((rc = colmat_launch(cs, ca))) return rc;
        if (p.nph != n) hipLaunchKernelGGL(lg_twin_w, dim3((p.nph + WG - 1) / WG), dim3(WG), 0, cs, a);
    }
    hipLaunchKernelGGL(lg_finalize, dim3(1), dim3(WG), 0, cs, a);
    if (cs != st) {
        // the caller's stream takes over from the one the loop ended on
        HIPCHK(hipEventRecord(ev_join, cs));
        HIPCHK(hipStreamWaitEvent(st, ev_join, 0));
    }
    HIPCHK(hipGetLastError());
    if ((rc = read_ctl())) return rc;
    return 0;
}

}  // namespace lhdm
