// Test-only entry points (declared in lhdm_testing.h): single solver steps on
// caller-given state.  They run the solvers' own device code; only the set-up
// and the read-back here are specific to the tests.
#pragma once

#include <vector>

#include "lhdm_testing.h"
#include "lhdm_large.hpp"

namespace lhdm {

constexpr int TRSV_TEST_MAX = 8192;   // largest n of the triangular-solve test entry

// One-workgroup engine: the removal set is read from x (x <= 0 marks a
// removed position) and deleted in one sweep, compaction included.
__global__ __launch_bounds__(WG) void wg_test_downdate_kernel(Prob p, DevParams prm, int nP) {
    __shared__ WgLds lds;
    WgShared& s = lds.sh;
    Wg wg(p, prm, s, (lds_double*)lds.x);
    if (threadIdx.x == 0) {
        s.nP = nP;
        s.q = 0;
    }
    __syncthreads();
    wg.collect_removals();
    wg.downdate();
}

struct DeviceBuffer {
    void* ptr = nullptr;
    ~DeviceBuffer() {
        if (ptr) (void)hipFree(ptr);
    }
};

static int test_downdate(hipStream_t st, int engine, int m, int nP, const double* Q, const double* R,
                         const double* bt, int q, const int* rm, double* Qo, double* Ro, double* bto, int* Po,
                         int* sweeps) {
    if (m < 1 || nP < 1 || q < 1 || q > nP || !Q || !R || !bt || !rm || !Qo || !Ro || !bto) return LHDM_EINVAL;
    if (engine != 1 && engine != 2) return LHDM_EINVAL;
    for (int t = 0; t < q; ++t)
        if (rm[t] < 0 || rm[t] >= nP || (t > 0 && rm[t] <= rm[t - 1])) return LHDM_EINVAL;
    if (nP > m || (engine == 1 && m > MMAX_WG)) return LHDM_EUNSUPPORTED;
    DevParams prm{};
    prm.tau1 = 0.6;
    prm.tau2 = 0.15;
    prm.delta = 0.9;
    prm.kkt_tol = 1e-9;
    prm.kmax = 2;
    prm.max_outer = 1 << 30;
    prm.max_inner = 1 << 30;
    prm.lh = 0;
    const int n = nP;   // position c holds column c
    // host copies of the integer state: P = pos = slot = identity, x marks the removals
    std::vector<int> ident(nP);
    std::vector<double> xs(nP, 1.0);
    for (int c = 0; c < nP; ++c) ident[c] = c;
    for (int t = 0; t < q; ++t) xs[rm[t]] = 0.0;
    DeviceBuffer buf;
    Prob* pp = nullptr;
    LgArgs a;
    size_t base_total = 0;
    if (engine == 2) {
        const LargeLayout L = large_layout(m, n, prm.kmax);
        base_total = L.total + pad256(sizeof(double) * n) + pad256(sizeof(Mirror));
        HIPCHK(hipMalloc(&buf.ptr, base_total));
        char* base = (char*)buf.ptr;
        large_bind(a, L, base, m, n, prm);
        a.p.x = (double*)(base + L.total);
        a.p.w = (double*)(base + L.wfall);
        a.hmir = (Mirror*)(base + L.total + pad256(sizeof(double) * n));
        HIPCHK(hipMemsetAsync(base + L.flt, 0, L.slot - L.flt, st));
        pp = &a.p;
    } else {
        base_total = slot_bytes(m, n, prm.kmax) + pad256(sizeof(double) * n);
        HIPCHK(hipMalloc(&buf.ptr, base_total));
        carve_slot(a.p, (char*)buf.ptr, m, n, prm.kmax);
        a.p.x = (double*)((char*)buf.ptr + slot_bytes(m, n, prm.kmax));
        a.p.ybuf = nullptr;
        a.p.Vt = nullptr;
        pp = &a.p;
    }
    Prob& p = *pp;
    p.A = nullptr;
    p.b = nullptr;
    p.lda = m;
    p.passive = nullptr;
    p.info = nullptr;
    // kc = min(m, nP) = nP: R's leading dimension is nP, as the caller's
    HIPCHK(hipMemcpyAsync(p.Q, Q, sizeof(double) * (size_t)m * m, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(p.R, R, sizeof(double) * (size_t)nP * nP, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(p.bt, bt, sizeof(double) * (size_t)m, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(p.P, ident.data(), sizeof(int) * nP, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(p.pos, ident.data(), sizeof(int) * nP, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(p.slot, ident.data(), sizeof(int) * nP, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(p.x, xs.data(), sizeof(double) * nP, hipMemcpyHostToDevice, st));
    int nsweep = 0;
    if (engine == 1) {
        hipLaunchKernelGGL(wg_test_downdate_kernel, dim3(1), dim3(WG), 0, st, p, prm, nP);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        nsweep = 1;
    } else {
        // control block: nP positions, one accepted column (an inner step follows
        // an append), the removal set pending (read from x by the next inner call)
        Ctl c{};
        c.nP = nP;
        c.nP0 = nP;
        c.nPa = nP;
        c.k = 1;
        c.kr = 1;
        c.status = LHDM_STATUS_OK;
        LgExtra ex{};
        ex.pending = 1;
        HIPCHK(hipMemcpyAsync(a.ctl, &c, sizeof(Ctl), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(a.ex, &ex, sizeof(LgExtra), hipMemcpyHostToDevice, st));
        int left = q, ep_g = 0, pub = 0;
        while (left > 0) {
            hipLaunchKernelGGL(lg_inner, dim3(1), dim3(WG), 0, st, a, ++pub);
            ++ep_g;
            hipLaunchKernelGGL(lg_cfdown, dim3((p.kc + GB - 1) / GB), dim3(WG), 0, st, a, ep_g);
            hipLaunchKernelGGL(lg_givens, dim3((p.kc + GB - 1) / GB), dim3(64), 0, st, a, ep_g);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(&c, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(&ex, a.ex, sizeof(LgExtra), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (ex.err || ex.inner_done || c.q < 1 || c.q > left) return LHDM_EHIP;
            if (ex.totrot == ex.ndown) {
                hipLaunchKernelGGL(lg_compact, dim3(1), dim3(WG), 0, st, a, 1);
                hipLaunchKernelGGL(lg_qrot, dim3((m + 1 + 63) / 64), dim3(64 * (1 + QNL)), 0, st, a, 1);
            } else {
                hipLaunchKernelGGL(lg_qrot, dim3((m + 1 + 63) / 64), dim3(64 * (1 + QNL)), 0, st, a, 0);
                hipLaunchKernelGGL(lg_compact, dim3(1), dim3(WG), 0, st, a, 0);
            }
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(&ex, a.ex, sizeof(LgExtra), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (ex.err) return LHDM_EHIP;
            left -= c.q;
            ++nsweep;
            if ((left > 0) != (ex.pending != 0)) return LHDM_EHIP;
        }
    }
    // read back: the kept columns of R through their slots, Q and bt
    const int nk = nP - q;
    std::vector<double> Rh((size_t)nP * nP), Rk((size_t)nk * nk, 0.0);
    std::vector<int> sl(nP), Ph(nP);
    HIPCHK(hipMemcpyAsync(Rh.data(), p.R, sizeof(double) * Rh.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(sl.data(), p.slot, sizeof(int) * nP, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(Ph.data(), p.P, sizeof(int) * nP, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int cc = 0; cc < nk; ++cc)
        for (int i = 0; i <= cc; ++i) Rk[(size_t)cc * nk + i] = Rh[(size_t)sl[cc] * nP + i];
    if (nk > 0) HIPCHK(hipMemcpyAsync(Ro, Rk.data(), sizeof(double) * Rk.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(Qo, p.Q, sizeof(double) * (size_t)m * m, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(bto, p.bt, sizeof(double) * (size_t)m, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    if (Po)
        for (int cc = 0; cc < nk; ++cc) Po[cc] = Ph[cc];
    if (sweeps) *sweeps = nsweep;
    return 0;
}

// The one-wave factorisations of the CholeskyQR2 panel on caller matrices
// (column-major n x n in, column-major n x n out).
__global__ __launch_bounds__(WG, 1) void test_cq_factors_kernel(int n, const double* G, const double* W, double* R,
                                                                double* Ri, double* U, double* Li, double* L,
                                                                double* Ui, double* sg, double* sg2, double* sin2) {
    __shared__ double G_[CQ_MAX][CQ_MAX + 1], W_[CQ_MAX][CQ_MAX + 1], R_[CQ_MAX][CQ_MAX + 1],
        Ri_[CQ_MAX][CQ_MAX + 1], U_[CQ_MAX][CQ_MAX + 1], Li_[CQ_MAX][CQ_MAX + 1], L_[CQ_MAX][CQ_MAX + 1],
        Ui_[CQ_MAX][CQ_MAX + 1];
    __shared__ double sg_[CQ_MAX], sg2_[CQ_MAX], rowbuf_[64];
    const int tid = threadIdx.x;
    for (int e = tid; e < CQ_SQ; e += WG) {
        const int i = e / CQ_MAX, j = e % CQ_MAX;
        const bool in = i < n && j < n;
        G_[i][j] = in ? G[(size_t)j * n + i] : 0.0;
        W_[i][j] = in ? W[(size_t)j * n + i] : 0.0;
    }
    __syncthreads();
    if (wave_index() == 0) {
        const double q = chol_inv_wave((CqRow*)G_, n, (CqRow*)R_, (CqRow*)Ri_, (lds_double*)rowbuf_);
        if (tid == 0) *sin2 = q;
        lu_rows_wave((CqRow*)W_, n, (CqRow*)U_, (CqRow*)Li_, (lds_double*)sg_);
    } else if (wave_index() == 1) {   // the column elimination, as the solver runs it beside the row one
        lu_inv_wave((CqRow*)W_, n, (CqRow*)L_, (CqRow*)Ui_, (lds_double*)sg2_);
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += WG) {
        const int j = e / n, i = e % n;
        R[e] = R_[i][j];
        Ri[e] = Ri_[i][j];
        U[e] = U_[i][j];
        Li[e] = Li_[i][j];
        L[e] = L_[i][j];
        Ui[e] = Ui_[i][j];
    }
    if (tid < n) {
        sg[tid] = sg_[tid];
        sg2[tid] = sg2_[tid];
    }
}

static int test_cq_factors(hipStream_t st, int n, const double* G, const double* W, double* R, double* Ri, double* U,
                           double* Li, double* L, double* Ui, double* sg, double* sg2, double* sin2) {
    if (n < 1 || n > CQ_MAX || !G || !W || !R || !Ri || !U || !Li || !L || !Ui || !sg || !sg2 || !sin2)
        return LHDM_EINVAL;
    double* d = nullptr;
    HIPCHK(hipMalloc(&d, sizeof(double)));
    hipLaunchKernelGGL(test_cq_factors_kernel, dim3(1), dim3(WG), 0, st, n, G, W, R, Ri, U, Li, L, Ui, sg, sg2,
                       d);
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipMemcpyAsync(sin2, d, sizeof(double), hipMemcpyDeviceToHost, st);
    const hipError_t e3 = hipStreamSynchronize(st);
    const hipError_t e4 = hipFree(d);
    HIPCHK(e1);
    HIPCHK(e2);
    HIPCHK(e3);
    HIPCHK(e4);
    return 0;
}

// The whole-device engine's chained triangular solve on a caller's n x n R
// (slots = positions, R's leading dimension n) and right-hand side.
static int test_trsv(hipStream_t st, int n, const double* R, const double* bt, double* y, int* inv_blocks) {
    if (n < 1 || !R || !bt || !y) return LHDM_EINVAL;
    if (n > TRSV_TEST_MAX) return LHDM_EUNSUPPORTED;
    DevParams prm{};
    prm.tau1 = 0.6;
    prm.tau2 = 0.15;
    prm.delta = 0.9;
    prm.kkt_tol = 1e-9;
    prm.kmax = 2;
    prm.max_outer = 1 << 30;
    prm.max_inner = 1 << 30;
    const int m = n;   // kc = n: R's leading dimension is the caller's
    std::vector<int> ident(n);
    for (int c = 0; c < n; ++c) ident[c] = c;
    const LargeLayout L = large_layout(m, n, prm.kmax);
    DeviceBuffer buf;
    HIPCHK(hipMalloc(&buf.ptr, L.total));
    char* base = (char*)buf.ptr;
    LgArgs a;
    large_bind(a, L, base, m, n, prm);
    Prob& p = a.p;
    HIPCHK(hipMemsetAsync(base + L.flt, 0, L.slot - L.flt, st));
    HIPCHK(hipMemcpyAsync(p.R, R, sizeof(double) * (size_t)n * n, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(p.bt, bt, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(p.slot, ident.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
    Ctl c{};
    c.nP = n;
    c.nP0 = n;
    c.nPa = n;
    c.k = 1;   // the solve runs after an accepted column
    c.kr = 1;
    c.status = LHDM_STATUS_OK;
    LgExtra ex{};
    HIPCHK(hipMemcpyAsync(a.ctl, &c, sizeof(Ctl), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(a.ex, &ex, sizeof(LgExtra), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(lg_trsv, dim3((n + TB - 1) / TB), dim3(WG), 0, st, a, 1, 0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&ex, a.ex, sizeof(LgExtra), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(y, p.ybuf, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    if (ex.err) return LHDM_EHIP;
    if (inv_blocks) {
        // full 64-row blocks at least TRSV_CHAIN places from the bottom
        const int nb = (n + TB - 1) / TB, full = n / TB;
        int cnt = 0;
        for (int g = TRSV_CHAIN; g < nb; ++g)
            if (nb - 1 - g < full) ++cnt;
        *inv_blocks = cnt;
    }
    return 0;
}

}  // namespace lhdm

extern "C" int lhdm_test_trsv(void* stream, int32_t n, const double* R, const double* bt, double* y,
                              int32_t* inv_blocks) {
    return lhdm::test_trsv((hipStream_t)stream, n, R, bt, y, inv_blocks);
}

extern "C" int lhdm_test_cq_factors(void* stream, int32_t n, const double* G, const double* W, double* R, double* Ri,
                                    double* U, double* Li, double* L, double* Ui, double* sg, double* sg2,
                                    double* sin2) {
    return lhdm::test_cq_factors((hipStream_t)stream, n, G, W, R, Ri, U, Li, L, Ui, sg, sg2, sin2);
}

extern "C" int lhdm_test_downdate(void* stream, int32_t engine, int32_t m, int32_t nP, const double* Q,
                                  const double* R, const double* bt, int32_t q, const int32_t* rm, double* Q_out,
                                  double* R_out, double* bt_out, int32_t* P_out, int32_t* sweeps) {
    return lhdm::test_downdate((hipStream_t)stream, engine, m, nP, Q, R, bt, q, rm, Q_out, R_out, bt_out, P_out,
                               sweeps);
}
