// Adjoint of the NNLS solution map through its final passive set.
//
// On the returned passive set P the solution is the least-squares solution of
// the subproblem of Section 2.1, x_P = (A_P^T A_P)^{-1} A_P^T b, x_Z = 0.  For an
// upstream gradient g = dL/dx, with A_P = Q R (Householder, recomputed here):
//     R^T z = g_P,  R lambda = z          (lambda = (A_P^T A_P)^{-1} g_P)
//     grad_b = A_P lambda
//     grad_A[:, P] = r lambda^T - (A_P lambda) x_P^T,  r = b - A_P x_P
//     grad_A[:, Z] = 0.
// One workgroup handles one instance; grad_A is written column by column with
// coalesced stores (it is the dominant HBM traffic of this kernel).
#pragma once

#include <vector>

#include "lhdm_device.hpp"
#include "lhdm_host.hpp"

namespace lhdm {

struct BwdIn {
    const double* A;
    const double* b;
    const double* x;
    const int* passive;
    const double* g;
    double* gA;
    double* gb;
    int m, n;
    size_t ws_off;   // byte offset of this instance's scratch
};

constexpr int BWD_MREG = 512;   // instances up to this m keep the reflector in LDS and columns in registers

struct BwdShared {
    double rd[NW];
    double z[YMAX];
    double c[YMAX];
    double vl[BWD_MREG];   // reflector of the current step (rows below the pivot)
    double tau;
    int nP;
};

__global__ __launch_bounds__(WG) void backward_kernel(const BwdIn* __restrict__ ins, char* wsbase) {
    __shared__ BwdShared s;
    const BwdIn in = ins[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wid = wave_index();
    const int m = in.m, n = in.n;
    const int kc = m < n ? m : n;
    double* F = (double*)(wsbase + in.ws_off);        // m x kc: A_P, then its QR
    double* Al = F + (size_t)m * kc;                   // m
    double* r = Al + m;                                // m
    auto wsum = [&](double v) {
        v = wave_sum(v);
        __syncthreads();
        if (lane == 0) s.rd[wid] = v;
        __syncthreads();
        double t = s.rd[0];
        for (int i = 1; i < NW; ++i) t += s.rd[i];
        return t;
    };
    if (tid == 0) {
        int k = 0;
        while (k < kc && in.passive[k] >= 0) ++k;
        s.nP = k;
    }
    __syncthreads();
    const int nP = s.nP;
    // gather A_P and g_P
    for (int c = 0; c < nP; ++c) {
        const double* a = in.A + (size_t)in.passive[c] * m;
        for (int i = tid; i < m; i += WG) F[(size_t)c * m + i] = a[i];
    }
    for (int c = tid; c < nP; c += WG) s.c[c] = in.g[in.passive[c]];
    __syncthreads();
    // Householder QR of F (m x nP), R in the upper triangle
    for (int t = 0; t < nP && m <= BWD_MREG; ++t) {
        // the reflector stays in LDS (only R is used afterwards); each wave
        // takes four columns at a time, their rows held in registers, so their
        // loads go out together and no store waits in between
        constexpr int RM = BWD_MREG / 64, CB = 4;
        const double* v = F + (size_t)t * m;
        double part = 0.0;
        for (int i = t + tid; i < m; i += WG) {
            const double vi = v[i];
            s.vl[i] = vi;
            part += vi * vi;
        }
        const double nrm = sqrt(wsum(part));
        const double x0 = s.vl[t];
        double tau = 0.0, beta = x0, scal = 0.0;
        if (nrm > 0.0) {
            beta = (x0 >= 0.0) ? -nrm : nrm;
            tau = (beta - x0) / beta;
            scal = 1.0 / (x0 - beta);
        }
        for (int i = t + 1 + tid; i < m; i += WG) s.vl[i] *= scal;
        __syncthreads();
        const int r0 = t + 1;
        for (int cb = t + 1 + wid * CB; cb < nP; cb += NW * CB) {
            double fv[CB][RM], d[CB], ft[CB];
#pragma unroll
            for (int u = 0; u < CB; ++u) {
                const double* f = F + (size_t)min(cb + u, nP - 1) * m;
                ft[u] = f[t];
                d[u] = (lane == 0) ? ft[u] : 0.0;
#pragma unroll
                for (int k = 0; k < RM; ++k) {
                    const int i = r0 + lane + 64 * k;
                    fv[u][k] = (i < m) ? f[i] : 0.0;
                }
            }
#pragma unroll
            for (int k = 0; k < RM; ++k) {
                const int i = r0 + lane + 64 * k;
                if (i < m) {
                    const double vi = s.vl[i];
#pragma unroll
                    for (int u = 0; u < CB; ++u) d[u] += vi * fv[u][k];
                }
            }
#pragma unroll
            for (int u = 0; u < CB; ++u) d[u] = wave_sum(d[u]) * tau;
#pragma unroll
            for (int u = 0; u < CB; ++u) {
                if (cb + u < nP) {
                    double* f = F + (size_t)(cb + u) * m;
                    if (lane == 0) f[t] = ft[u] - d[u];
#pragma unroll
                    for (int k = 0; k < RM; ++k) {
                        const int i = r0 + lane + 64 * k;
                        if (i < m) f[i] = fv[u][k] - d[u] * s.vl[i];
                    }
                }
            }
        }
        __syncthreads();
        if (tid == 0) F[(size_t)t * m + t] = beta;
        __syncthreads();
    }
    for (int t = 0; t < nP && m > BWD_MREG; ++t) {
        double* v = F + (size_t)t * m;
        double part = 0.0;
        for (int i = t + tid; i < m; i += WG) part += v[i] * v[i];
        const double nrm = sqrt(wsum(part));
        const double x0 = v[t];
        double tau = 0.0, beta = x0, scal = 0.0;
        if (nrm > 0.0) {
            beta = (x0 >= 0.0) ? -nrm : nrm;
            tau = (beta - x0) / beta;
            scal = 1.0 / (x0 - beta);
        }
        __syncthreads();
        for (int i = t + 1 + tid; i < m; i += WG) v[i] *= scal;
        __syncthreads();
        // apply to the remaining columns: one wave per column
        for (int c = t + 1 + wid; c < nP; c += NW) {
            double* f = F + (size_t)c * m;
            double d = (lane == 0) ? f[t] : 0.0;
            for (int i = t + 1 + lane; i < m; i += 64) d += v[i] * f[i];
            d = wave_sum(d) * tau;
            if (lane == 0) f[t] -= d;
            for (int i = t + 1 + lane; i < m; i += 64) f[i] -= d * v[i];
        }
        __syncthreads();
        if (tid == 0) v[t] = beta;
        __syncthreads();
    }
    // R^T z = g_P (forward substitution, column-oriented on R^T)
    for (int i = 0; i < nP; ++i) {
        const double zi = s.c[i] / F[(size_t)i * m + i];
        __syncthreads();
        if (tid == 0) s.z[i] = zi;
        for (int l = i + 1 + tid; l < nP; l += WG) s.c[l] -= F[(size_t)l * m + i] * zi;
        __syncthreads();
    }
    // R lambda = z (back substitution); lambda into s.c
    for (int i = tid; i < nP; i += WG) s.c[i] = s.z[i];
    for (int j = nP - 1; j >= 0; --j) {
        __syncthreads();
        const double lj = s.c[j] / F[(size_t)j * m + j];
        __syncthreads();
        if (tid == 0) s.z[j] = lj;
        for (int i = tid; i < j; i += WG) s.c[i] -= lj * F[(size_t)j * m + i];
    }
    __syncthreads();
    // lambda now in s.z; Al = A_P lambda and r = b - A_P x_P
    for (int i = tid; i < m; i += WG) {
        double al = 0.0, rr = in.b[i];
        for (int c = 0; c < nP; ++c) {
            const int j = in.passive[c];
            const double a = in.A[(size_t)j * m + i];
            al += a * s.z[c];
            rr -= a * in.x[j];
        }
        Al[i] = al;
        r[i] = rr;
        in.gb[i] = al;
    }
    __syncthreads();
    // grad_A: zero on Z, rank-two form on P
    for (int j = 0; j < n; ++j) {
        double* out = in.gA + (size_t)j * m;
        for (int i = tid; i < m; i += WG) out[i] = 0.0;
    }
    __syncthreads();
    for (int c = 0; c < nP; ++c) {
        const int j = in.passive[c];
        const double lc = s.z[c], xj = in.x[j];
        double* out = in.gA + (size_t)j * m;
        for (int i = tid; i < m; i += WG) out[i] = r[i] * lc - Al[i] * xj;
    }
}

static size_t bwd_scratch_bytes(int m, int n) {
    const size_t kc = (size_t)(m < n ? m : n);
    return pad256(sizeof(double) * ((size_t)m * kc + 2 * (size_t)m));
}

static size_t backward_workspace_bytes(int batch, const int* m, const int* n) {
    if (batch < 1 || !m || !n) return 0;
    size_t tot = pad256(sizeof(BwdIn) * (size_t)batch);
    for (int i = 0; i < batch; ++i) tot += bwd_scratch_bytes(m[i], n[i]);
    return tot;
}

static int backward_run(hipStream_t st, int batch, const int* m, const int* n, const int64_t* a_off,
                        const double* A_pool, const int64_t* b_off, const double* b_pool, const int64_t* x_off,
                        const double* x_pool, const int* passive_pool, const double* gx_pool, double* gA_pool,
                        double* gb_pool, void* ws, size_t ws_bytes) {
    if (batch < 1 || !m || !n || !a_off || !b_off || !x_off || !A_pool || !b_pool || !x_pool || !passive_pool ||
        !gx_pool || !gA_pool || !gb_pool)
        return LHDM_EINVAL;
    for (int i = 0; i < batch; ++i) {
        if (m[i] < 1 || n[i] < 1) return LHDM_EINVAL;
        if ((m[i] < n[i] ? m[i] : n[i]) > YMAX) return LHDM_EUNSUPPORTED;
    }
    const size_t need = backward_workspace_bytes(batch, m, n);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255)) return LHDM_EWORKSPACE;
    std::vector<BwdIn> ins(batch);
    size_t off = pad256(sizeof(BwdIn) * (size_t)batch);
    for (int i = 0; i < batch; ++i) {
        BwdIn& b = ins[i];
        b.A = A_pool + a_off[i];
        b.b = b_pool + b_off[i];
        b.x = x_pool + x_off[i];
        b.passive = passive_pool + x_off[i];
        b.g = gx_pool + x_off[i];
        b.gA = gA_pool + a_off[i];
        b.gb = gb_pool + b_off[i];
        b.m = m[i];
        b.n = n[i];
        b.ws_off = off;
        off += bwd_scratch_bytes(m[i], n[i]);
    }
    hipError_t e = hipMemcpyAsync(ws, ins.data(), sizeof(BwdIn) * batch, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(backward_kernel, dim3(batch), dim3(WG), 0, st, (const BwdIn*)ws, (char*)ws);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_last_hip_error((int)e);
        return LHDM_EHIP;
    }
    return 0;
}

}  // namespace lhdm
