// C ABI of the gfx950 LH / LHDM library (declarations and contracts in lhdm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "lhdm.h"
#include "lhdm_host.hpp"
#include "lhdm_device.hpp"
#include "lhdm_wg.hpp"
#include "lhdm_large.hpp"
#include "lhdm_backward.hpp"
#include "lhdm_testing.hpp"
#include "lhdm_tuning.hpp"

namespace lhdm {

// ---------------------------------------------------------------------------
// kernels of the workgroup engine
// ---------------------------------------------------------------------------
struct ProbIn {
    const double* A;
    long long lda;
    const double* b;
    double* x;
    double* w;
    int* passive;
    lhdm_info* info;
    int m, n;
};

// Persistent batched solve ("fused" engine): each workgroup owns one workspace
// slot and takes instances from the queue `order` (largest first; NULL: the
// given order) until it is exhausted.  An instance without a w buffer
// (in.w == NULL) keeps its dual in its slot at byte offset w_off.  OCC is the
// number of workgroups per compute unit the kernel is compiled for (its
// register budget: 512 or 256 per lane).
template <int OCC>
__global__ __launch_bounds__(WG, OCC) void wg_solve_kernel(const ProbIn* __restrict__ ins, int nprob,
                                                      const int* __restrict__ order, int* counter,
                                                      char* slots, size_t slot_stride, DevParams prm,
                                                      size_t w_off) {
    __shared__ WgLds lds;
    WgShared& sh = lds.sh;
    int& sidx = lds.sidx;
    char* base = slots + (size_t)blockIdx.x * slot_stride;
    while (true) {
        if (threadIdx.x == 0) sidx = atomicAdd(counter, 1);
        __syncthreads();
        const int idx = sidx;
        __syncthreads();
        if (idx >= nprob) break;
        const ProbIn in = ins[order ? order[idx] : idx];
        Prob p;
        p.A = in.A;
        p.lda = in.lda;
        p.b = in.b;
        p.x = in.x;
        p.w = in.w ? in.w : (double*)(base + w_off);
        p.passive = in.passive;
        p.info = in.info;
        carve_slot(p, base, in.m, in.n, prm.kmax);
        if (prm.twin) p.nph = in.n / 2;   // in.n counts the columns of [A, -A]
        // iteration limits <= 0 select 3 n of this instance
        DevParams q = prm;
        if (q.max_outer <= 0) q.max_outer = 3 * in.n;
        if (q.max_inner <= 0) q.max_inner = 3 * in.n;
        Wg wg(p, q, sh, (lds_double*)lds.x);
        wg.run();
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// phased batched engine: one kernel per stage of the outer step over every
// instance (Wg::stage_*), the rounds captured as a HIP graph.  Each instance
// keeps its whole state between launches: its control block in `ctl`, its
// workspace slice (slot_bytes of its own m, n), then its least-squares
// solution y (kc doubles); its dual goes to in.w, which must be given.
// ---------------------------------------------------------------------------
constexpr int PH_INIT = -1;

__device__ __forceinline__ void ph_prob(Prob& p, const ProbIn& in, char* base, const DevParams& prm) {
    p.A = in.A;
    p.lda = in.lda;
    p.b = in.b;
    p.x = in.x;
    p.passive = in.passive;
    p.info = in.info;
    carve_slot(p, base, in.m, in.n, prm.kmax);
    p.ybuf = (double*)(base + slot_bytes(in.m, in.n, prm.kmax));
    p.w = in.w;
    if (prm.twin) p.nph = in.n / 2;
}

__host__ __device__ inline size_t ph_slot_bytes(int m, int n, int kmax) {
    const int kc = m < n ? m : n;
    return slot_bytes(m, n, kmax) + pad256(sizeof(double) * kc);
}

// One workgroup per instance (blockIdx.x through `order`); instances not in
// stage PH return at once.
template <int PH>
__global__ __launch_bounds__(WG, 2) void ph_kernel(const ProbIn* __restrict__ ins,
                                                   const int* __restrict__ order,
                                                   const size_t* __restrict__ soff, Ctl* __restrict__ ctl,
                                                   char* slots, DevParams prm) {
    __shared__ WgLds lds;
    const int idx = order[blockIdx.x];
    Ctl* c = ctl + idx;
    if (PH != PH_INIT && c->stage != PH) return;
    const ProbIn in = ins[idx];
    Prob p;
    ph_prob(p, in, slots + soff[idx], prm);
    DevParams q = prm;
    if (q.max_outer <= 0) q.max_outer = 3 * in.n;
    if (q.max_inner <= 0) q.max_inner = 3 * in.n;
    Wg wg(p, q, lds.sh, (lds_double*)lds.x);
    if (PH == PH_INIT) {
        wg.start();
    } else {
        ctl_load(lds.sh, c);
        if (PH == ST_APPEND) wg.stage_append();
        else if (PH == ST_INNER) wg.stage_inner();
        else wg.stage_accept();
    }
    if (lds.sh.stage == ST_DONE) wg.finalize();
    ctl_store(lds.sh, c);
}

// Number of instances not finished, into live[0] (one workgroup).
__global__ __launch_bounds__(WG) void ph_count_kernel(const Ctl* __restrict__ ctl, int nprob, int* live) {
    __shared__ int part[NW];
    int cnt = 0;
    for (int i = threadIdx.x; i < nprob; i += WG) cnt += (ctl[i].stage != ST_DONE) ? 1 : 0;
    cnt = wave_sum_int(cnt);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < NW; ++w) t += part[w];
        live[0] = t;
    }
}

// Instances cut off by the round limit end with the iteration-limit status.
__global__ __launch_bounds__(WG) void ph_cutoff_kernel(const ProbIn* __restrict__ ins,
                                                       const int* __restrict__ order,
                                                       const size_t* __restrict__ soff, Ctl* __restrict__ ctl,
                                                       char* slots, DevParams prm) {
    __shared__ WgLds lds;
    const int idx = order[blockIdx.x];
    Ctl* c = ctl + idx;
    if (c->stage == ST_DONE) return;
    const ProbIn in = ins[idx];
    Prob p;
    ph_prob(p, in, slots + soff[idx], prm);
    Wg wg(p, prm, lds.sh, (lds_double*)lds.x);
    ctl_load(lds.sh, c);
    if (threadIdx.x == 0) {
        lds.sh.status = LHDM_STATUS_MAXITER;
        lds.sh.stage = ST_DONE;
    }
    __syncthreads();
    wg.refresh_dual();
    wg.finalize();
    ctl_store(lds.sh, c);
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
static bool params_ok(const lhdm_params* p) {
    if (!p) return false;
    if (!(p->tau1 > 0.0 && p->tau1 <= 1.0)) return false;
    if (!(p->tau2 > 0.0 && p->tau2 <= 1.0)) return false;
    if (!(p->delta > 0.0 && p->delta <= 1.0)) return false;
    if (!(p->kkt_tol >= 0.0)) return false;
    if (p->kmax < 1 || p->kmax > KM) return false;
    if ((p->flags & LHDM_FLAG_NO_JLOOP) &&
        !(p->tau1 == 1.0 && p->tau2 <= 0.5 && (p->kmax <= 1 || p->delta <= p->tau2 / (p->kmax - 1))))
        return false;
    return true;
}

static DevParams dev_params(const lhdm_params* p, int n, int lh) {
    DevParams d{};
    d.tau1 = p->tau1;
    d.tau2 = p->tau2;
    d.delta = p->delta;
    d.kkt_tol = p->kkt_tol;
    d.kmax = lh ? 1 : p->kmax;
    d.max_outer = p->max_outer > 0 ? p->max_outer : 3 * n;
    d.max_inner = p->max_inner > 0 ? p->max_inner : 3 * n;
    d.lh = lh;
    d.nojloop = (p->flags & LHDM_FLAG_NO_JLOOP) ? 1 : 0;
    d.panel_hh = (p->flags & LHDM_FLAG_PANEL_HOUSEHOLDER) ? 1 : 0;
    return d;
}

// Layout of the workgroup-engine workspace:
// [ProbIn x batch | order x batch | counter | slots x nslot]
struct WgLayout {
    size_t off_in, off_order, off_counter, off_slots, slot_stride, total;
    int nslot;
};

// Batched engines: the fused persistent kernel compiled for one or for two
// workgroups per compute unit, or the phased kernels.
enum { BE_FUSED1 = 0, BE_FUSED2 = 1, BE_PHASED = 2 };

static int device_cus() {
    // compute units of the current device (queried per call: a process may use several devices)
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return cus;
}

static int wg_slots_for(int batch, int eng = BE_FUSED1) {
    int occ = 0;
    const hipError_t e = (eng == BE_FUSED2)
                             ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, wg_solve_kernel<2>, WG, 0)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, wg_solve_kernel<1>, WG, 0);
    if (e != hipSuccess || occ < 1) occ = 1;
    return std::max(1, std::min(batch, device_cus() * occ));
}

static WgLayout wg_layout(int batch, int mmax, int nmax, int kmax, int eng = BE_FUSED1) {
    WgLayout L;
    L.nslot = wg_slots_for(batch, eng);
    size_t o = 0;
    L.off_in = o;
    o += pad256(sizeof(ProbIn) * (size_t)batch);
    L.off_order = o;
    o += pad256(sizeof(int) * (size_t)batch);
    L.off_counter = o;
    o += 256;
    L.off_slots = o;
    L.slot_stride = slot_bytes(mmax, nmax, kmax);
    o += L.slot_stride * (size_t)L.nslot;
    L.total = o;
    return L;
}

// largest instances first (longest-processing-time order)
static std::vector<int> lpt_order(const std::vector<int>& mm, const std::vector<int>& nn) {
    std::vector<int> order(mm.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (long long)mm[a] * nn[a] > (long long)mm[b] * nn[b];
    });
    return order;
}

static int run_wg_engine(hipStream_t st, const std::vector<ProbIn>& ins, const std::vector<int>& mm,
                         const std::vector<int>& nn, const DevParams& prm, void* ws, size_t ws_bytes,
                         int eng = BE_FUSED1) {
    const int batch = (int)ins.size();
    const int mmax = *std::max_element(mm.begin(), mm.end());
    const int nmax = *std::max_element(nn.begin(), nn.end());
    WgLayout L = wg_layout(batch, mmax, nmax, prm.kmax, eng);
    if (ws == nullptr) {
        int rc = cached_workspace(L.total, &ws);
        if (rc) return rc;
    } else if (ws_bytes < L.total || ((uintptr_t)ws & 255)) {
        return LHDM_EWORKSPACE;
    }
    char* base = (char*)ws;
    const std::vector<int> order = lpt_order(mm, nn);
    HIPCHK(hipMemcpyAsync(base + L.off_in, ins.data(), sizeof(ProbIn) * batch, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(base + L.off_order, order.data(), sizeof(int) * batch, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(base + L.off_counter, 0, sizeof(int), st));
    if (eng == BE_FUSED2)
        hipLaunchKernelGGL(wg_solve_kernel<2>, dim3(L.nslot), dim3(WG), 0, st, (const ProbIn*)(base + L.off_in),
                           batch, (const int*)(base + L.off_order), (int*)(base + L.off_counter),
                           base + L.off_slots, L.slot_stride, prm, (size_t)0);
    else
        hipLaunchKernelGGL(wg_solve_kernel<1>, dim3(L.nslot), dim3(WG), 0, st, (const ProbIn*)(base + L.off_in),
                           batch, (const int*)(base + L.off_order), (int*)(base + L.off_counter),
                           base + L.off_slots, L.slot_stride, prm, (size_t)0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return 0;
}

// Layout of the phased engine's workspace:
// [ProbIn x batch | order x batch | slot offsets x batch | Ctl x batch | live count | slots]
// with one slot (ph_slot_bytes of its own size) per instance.
struct PhLayout {
    size_t off_in, off_order, off_soff, off_ctl, off_live, off_slots, total;
};

static PhLayout ph_layout(int batch, const int* m, const int* n, int kmax, std::vector<size_t>* soff) {
    PhLayout L;
    size_t o = 0;
    L.off_in = o;
    o += pad256(sizeof(ProbIn) * (size_t)batch);
    L.off_order = o;
    o += pad256(sizeof(int) * (size_t)batch);
    L.off_soff = o;
    o += pad256(sizeof(size_t) * (size_t)batch);
    L.off_ctl = o;
    o += pad256(sizeof(Ctl) * (size_t)batch);
    L.off_live = o;
    o += 256;
    L.off_slots = o;
    size_t so = 0;
    for (int i = 0; i < batch; ++i) {
        if (soff) soff->push_back(so);
        so += ph_slot_bytes(m[i], n[i], kmax);
    }
    L.total = o + so;
    return L;
}

// Rounds (one APPEND, INNER and ACCEPT launch each) per graph replay.
constexpr int PH_ROUNDS_PER_GRAPH = 4;

// A stream per device for graph capture (capture needs a stream other than the
// legacy default one; the graph is then launched on the caller's stream).
static int capture_stream(hipStream_t* out) {
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return LHDM_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(mu);
    if (!streams[dev]) HIPCHK(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking));
    *out = streams[dev];
    return 0;
}

static int run_phased(hipStream_t st, const std::vector<ProbIn>& ins, const std::vector<int>& mm,
                      const std::vector<int>& nn, const DevParams& prm, void* ws, size_t ws_bytes) {
    const int batch = (int)ins.size();
    std::vector<size_t> soff;
    const PhLayout L = ph_layout(batch, mm.data(), nn.data(), prm.kmax, &soff);
    if (ws == nullptr) {
        int rc = cached_workspace(L.total, &ws);
        if (rc) return rc;
    } else if (ws_bytes < L.total || ((uintptr_t)ws & 255)) {
        return LHDM_EWORKSPACE;
    }
    char* base = (char*)ws;
    const std::vector<int> order = lpt_order(mm, nn);
    HIPCHK(hipMemcpyAsync(base + L.off_in, ins.data(), sizeof(ProbIn) * batch, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(base + L.off_order, order.data(), sizeof(int) * batch, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(base + L.off_soff, soff.data(), sizeof(size_t) * batch, hipMemcpyHostToDevice, st));
    const ProbIn* d_in = (const ProbIn*)(base + L.off_in);
    const int* d_order = (const int*)(base + L.off_order);
    const size_t* d_soff = (const size_t*)(base + L.off_soff);
    Ctl* d_ctl = (Ctl*)(base + L.off_ctl);
    int* d_live = (int*)(base + L.off_live);
    char* slots = base + L.off_slots;
    hipLaunchKernelGGL(ph_kernel<PH_INIT>, dim3(batch), dim3(WG), 0, st, d_in, d_order, d_soff, d_ctl, slots, prm);
    HIPCHK(hipGetLastError());
    // the rounds, captured once per call
    hipStream_t cs;
    int rc = capture_stream(&cs);
    if (rc) return rc;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    for (int r = 0; r < PH_ROUNDS_PER_GRAPH; ++r) {
        hipLaunchKernelGGL(ph_kernel<ST_APPEND>, dim3(batch), dim3(WG), 0, cs, d_in, d_order, d_soff, d_ctl, slots,
                           prm);
        hipLaunchKernelGGL(ph_kernel<ST_INNER>, dim3(batch), dim3(WG), 0, cs, d_in, d_order, d_soff, d_ctl, slots,
                           prm);
        hipLaunchKernelGGL(ph_kernel<ST_ACCEPT>, dim3(batch), dim3(WG), 0, cs, d_in, d_order, d_soff, d_ctl, slots,
                           prm);
    }
    hipLaunchKernelGGL(ph_count_kernel, dim3(1), dim3(WG), 0, cs, (const Ctl*)d_ctl, batch, d_live);
    HIPCHK(hipStreamEndCapture(cs, &graph));
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        hipGraphDestroy(graph);
        set_last_hip_error((int)ie);
        return LHDM_EHIP;
    }
    // every round advances each unfinished instance by one outer step or one
    // exclusion; the limit below is far above what the iteration limits allow
    int nmax = 1;
    for (int v : nn) nmax = std::max(nmax, v);
    const long long outer_cap = prm.max_outer > 0 ? prm.max_outer : 3LL * nmax;
    const long long max_graphs = (4 * outer_cap + 16) / PH_ROUNDS_PER_GRAPH + 1;
    int live = batch;
    int err = 0;
    for (long long g = 0; g < max_graphs && live > 0; ++g) {
        hipError_t e = hipGraphLaunch(exec, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&live, d_live, sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            set_last_hip_error((int)e);
            err = LHDM_EHIP;
            break;
        }
    }
    hipGraphExecDestroy(exec);
    hipGraphDestroy(graph);
    if (err) return err;
    if (live > 0) {
        hipLaunchKernelGGL(ph_cutoff_kernel, dim3(batch), dim3(WG), 0, st, d_in, d_order, d_soff, d_ctl, slots,
                           prm);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(st));
    return 0;
}

static bool use_wg_engine(int m, int n) {
    // a single workgroup streams A once per outer step: fine while A is small
    return m <= MMAX_WG && (long long)m * n <= (1LL << 18);
}

static bool pick_wg(int m, int n, int flags) {
    if (flags & LHDM_FLAG_ENGINE_DEVICE) return false;
    if (flags & LHDM_FLAG_ENGINE_WORKGROUP) return true;
    return use_wg_engine(m, n);
}

static int solve_one(void* stream, int32_t m, int32_t n, const double* A, int64_t lda, const double* b,
                     const DevParams& prm, int flags, double* x, double* w, int32_t* passive, lhdm_info* info,
                     void* ws, size_t ws_bytes) {
    if (m < 1 || n < 1 || lda < m || !A || !b || !x) return LHDM_EINVAL;
    if ((flags & LHDM_FLAG_ENGINE_WORKGROUP) && (flags & LHDM_FLAG_ENGINE_DEVICE)) return LHDM_EINVAL;
    if ((flags & LHDM_FLAG_ENGINE_WORKGROUP) && m > MMAX_WG) return LHDM_EUNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    if (!pick_wg(m, n, flags)) {
        return large_solve(st, m, n, A, lda, b, prm, x, w, passive, info, ws, ws_bytes);
    }
    // w is required by the engine; use the workspace tail when the caller passes NULL
    std::vector<ProbIn> ins(1);
    ins[0].A = A;
    ins[0].lda = lda;
    ins[0].b = b;
    ins[0].x = x;
    ins[0].w = w;
    ins[0].passive = passive;
    ins[0].info = info;
    ins[0].m = m;
    ins[0].n = n;
    WgLayout L = wg_layout(1, m, n, prm.kmax);
    const size_t extra = pad256(sizeof(double) * (size_t)n);
    if (ws == nullptr) {
        int rc = cached_workspace(L.total + extra, &ws);
        if (rc) return rc;
        ws_bytes = L.total + extra;
    }
    if (ws_bytes < L.total + extra || ((uintptr_t)ws & 255)) return LHDM_EWORKSPACE;
    if (!w) ins[0].w = (double*)((char*)ws + L.total);
    std::vector<int> mm{m}, nn{n};
    return run_wg_engine(st, ins, mm, nn, prm, ws, L.total);
}

// ---------------------------------------------------------------------------
// allocation-free batched solve (lhdm_solve_batched_noalloc)
// ---------------------------------------------------------------------------
// Every buffer of the call beyond the caller's inputs and outputs lives in this
// fixed array: the batch's size and offset arrays, the instance descriptors,
// the queue counter and the workgroups' slots (each slot also holds its
// instance's dual).  Each device the library runs on holds its own copy until
// the process ends.  Host code never passes `scratch` itself to a kernel or a
// copy: in host code the name is a host-side stand-in, not the device address;
// noalloc_scratch() returns the address on the current device.
static __device__ __align__(256) char scratch[LHDM_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;

// Device address of `scratch` on the current device, looked up once per device
// (with that device current) and kept.
static int noalloc_scratch(char** out) {
    static std::mutex mu;
    static char* ptrs[NOALLOC_MAX_DEVICES] = {};
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return LHDM_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(mu);
    if (!ptrs[dev]) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return LHDM_EHIP;
        ptrs[dev] = (char*)ptr;
    }
    *out = ptrs[dev];
    return 0;
}

// Layout of the scratch for one call: [m | n | a_off | b_off | x_off | ProbIn
// x batch | counter | slots].  A slot is the instance state of slot_bytes()
// followed by the dual (nmax doubles).
struct NoallocLayout {
    size_t off_m, off_n, off_a, off_b, off_x, off_in, off_counter, off_slots, slot_stride, w_off, head;
};

static NoallocLayout noalloc_layout(int batch, int mmax, int nmax, int kmax) {
    NoallocLayout L;
    size_t o = 0;
    L.off_m = o;
    o += pad256(sizeof(int32_t) * (size_t)batch);
    L.off_n = o;
    o += pad256(sizeof(int32_t) * (size_t)batch);
    L.off_a = o;
    o += pad256(sizeof(int64_t) * (size_t)batch);
    L.off_b = o;
    o += pad256(sizeof(int64_t) * (size_t)batch);
    L.off_x = o;
    o += pad256(sizeof(int64_t) * (size_t)batch);
    L.off_in = o;
    o += pad256(sizeof(ProbIn) * (size_t)batch);
    L.off_counter = o;
    o += 256;
    L.off_slots = o;
    L.head = o;
    L.w_off = slot_bytes(mmax, nmax, kmax);
    L.slot_stride = L.w_off + pad256(sizeof(double) * (size_t)nmax);
    return L;
}

// Instance descriptors from the size and offset arrays (one thread each); the
// queue counter starts at 0 (a kernel store: no memset node on the stream).
__global__ __launch_bounds__(WG) void noalloc_describe(int batch, const int32_t* m, const int32_t* n,
                                                        const int64_t* ao, const double* Ap, const int64_t* bo,
                                                        const double* bp, const int64_t* xo, double* xp,
                                                        int32_t* pp, lhdm_info* infos, ProbIn* out, int* counter) {
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i == 0) *counter = 0;
    if (i >= batch) return;
    ProbIn in;
    in.A = Ap + ao[i];
    in.lda = m[i];
    in.b = bp + bo[i];
    in.x = xp + xo[i];
    in.w = nullptr;   // the dual stays in the slot
    in.passive = pp ? pp + xo[i] : nullptr;
    in.info = infos ? infos + i : nullptr;
    in.m = m[i];
    in.n = n[i];
    out[i] = in;
}

static int solve_batched_noalloc(hipStream_t st, int batch, const int32_t* m, const int32_t* n,
                                 const int64_t* a_off, const double* A_pool, const int64_t* b_off,
                                 const double* b_pool, const int64_t* x_off, double* x_pool, int32_t* passive_pool,
                                 const lhdm_params* p, int use_lh, lhdm_info* infos) {
    if (batch < 1 || !m || !n || !a_off || !b_off || !x_off || !A_pool || !b_pool || !x_pool) return LHDM_EINVAL;
    if (!params_ok(p)) return LHDM_EINVAL;
    int mmax = 1, nmax = 1;
    for (int i = 0; i < batch; ++i) {
        if (m[i] < 1 || n[i] < 1) return LHDM_EINVAL;
        if (m[i] > MMAX_WG) return LHDM_EUNSUPPORTED;
        mmax = std::max(mmax, (int)m[i]);
        nmax = std::max(nmax, (int)n[i]);
    }
    const int kmax = use_lh ? 1 : p->kmax;
    const NoallocLayout L = noalloc_layout(batch, mmax, nmax, kmax);
    // the bookkeeping and at least one slot must fit the fixed scratch
    if (L.head > (size_t)LHDM_NOALLOC_SCRATCH_BYTES ||
        L.slot_stride > (size_t)LHDM_NOALLOC_SCRATCH_BYTES - L.head)
        return LHDM_EUNSUPPORTED;
    char* base = nullptr;
    int rc = noalloc_scratch(&base);
    if (rc) return rc;
    const int fit = (int)std::min<size_t>((size_t)INT_MAX, ((size_t)LHDM_NOALLOC_SCRATCH_BYTES - L.head) / L.slot_stride);
    const int nslot = std::max(1, std::min(wg_slots_for(batch), fit));
    HIPCHK(hipMemcpyAsync(base + L.off_m, m, sizeof(int32_t) * batch, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(base + L.off_n, n, sizeof(int32_t) * batch, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(base + L.off_a, a_off, sizeof(int64_t) * batch, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(base + L.off_b, b_off, sizeof(int64_t) * batch, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(base + L.off_x, x_off, sizeof(int64_t) * batch, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(noalloc_describe, dim3((batch + WG - 1) / WG), dim3(WG), 0, st, batch,
                       (const int32_t*)(base + L.off_m), (const int32_t*)(base + L.off_n),
                       (const int64_t*)(base + L.off_a), A_pool, (const int64_t*)(base + L.off_b), b_pool,
                       (const int64_t*)(base + L.off_x), x_pool, passive_pool, infos, (ProbIn*)(base + L.off_in),
                       (int*)(base + L.off_counter));
    HIPCHK(hipGetLastError());
    DevParams prm = dev_params(p, nmax, use_lh ? 1 : 0);
    prm.max_outer = p->max_outer > 0 ? p->max_outer : 0;   // <= 0: 3 n per instance
    prm.max_inner = p->max_inner > 0 ? p->max_inner : 0;
    hipLaunchKernelGGL(wg_solve_kernel<1>, dim3(nslot), dim3(WG), 0, st, (const ProbIn*)(base + L.off_in), batch,
                       (const int*)nullptr, (int*)(base + L.off_counter), base + L.off_slots, L.slot_stride, prm,
                       L.w_off);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return 0;
}

// x = z[:n] - z[n:] (the signed solution of the positivity trick).
__global__ __launch_bounds__(WG) void signed_combine(const double* __restrict__ z, double* __restrict__ x, int n) {
    const int j = blockIdx.x * WG + threadIdx.x;
    if (j < n) x[j] = z[j] - z[j + n];
}

// The NNLS form of the squared-l1 regularised problem (Section 3.3): M =
// [1^T, 1^T; lam A, -lam A] ((m + 1) x 2n, column-major, ld m + 1) and
// rhs = [0; lam b].
__global__ __launch_bounds__(WG) void l1_assemble(const double* __restrict__ A, long long lda,
                                                   const double* __restrict__ b, double lam, int m, int n,
                                                   double* __restrict__ M, double* __restrict__ rhs) {
    const long long ld = m + 1, tot = ld * 2 * (long long)n;
    for (long long e = (long long)blockIdx.x * WG + threadIdx.x; e < tot; e += (long long)gridDim.x * WG) {
        const int j = (int)(e / ld), i = (int)(e % ld);
        double v = 1.0;
        if (i > 0) {
            const double a = A[(size_t)(j < n ? j : j - n) * lda + (i - 1)];
            v = (j < n) ? lam * a : -(lam * a);
        }
        M[e] = v;
    }
    for (int i = blockIdx.x * WG + threadIdx.x; i <= m; i += gridDim.x * WG) rhs[i] = (i == 0) ? 0.0 : lam * b[i - 1];
}

struct L1Layout {
    size_t M, rhs, z, solver, total;
};

static L1Layout l1_layout(int m, int n, const lhdm_params* p) {
    L1Layout L;
    lhdm_params q = *p;
    if (q.kmax < 1) q.kmax = 1;
    size_t o = 0;
    L.M = o;
    o += pad256(sizeof(double) * (size_t)(m + 1) * 2 * n);
    L.rhs = o;
    o += pad256(sizeof(double) * (size_t)(m + 1));
    L.z = o;
    o += pad256(sizeof(double) * 2 * (size_t)n);
    L.solver = o;
    o += lhdm_workspace_bytes(m + 1, 2 * n, &q);
    L.total = o;
    return L;
}

static size_t signed_workspace(int m, int n, const lhdm_params* p, size_t* solver_bytes) {
    const size_t zb = pad256(sizeof(double) * 2 * (size_t)n);
    lhdm_params q = *p;
    if (q.kmax < 1) q.kmax = 1;
    const size_t sb = lhdm_workspace_bytes(m, 2 * n, &q);
    if (solver_bytes) *solver_bytes = sb;
    return sb + zb;
}

}  // namespace lhdm

using namespace lhdm;

extern "C" {

void lhdm_default_params(lhdm_params* p) {
    if (!p) return;
    p->tau1 = 0.6;
    p->tau2 = 0.15;
    p->delta = 0.9;
    p->kkt_tol = 1e-9;
    p->kmax = 32;
    p->max_outer = 0;
    p->max_inner = 0;
    p->flags = 0;
}

size_t lhdm_workspace_bytes(int32_t m, int32_t n, const lhdm_params* p) {
    if (m < 1 || n < 1) return 0;
    const int kmax = p ? p->kmax : 32;
    if (pick_wg(m, n, p ? p->flags : 0) && m <= MMAX_WG) {
        WgLayout L = wg_layout(1, m, n, kmax < 1 ? 1 : kmax);
        return L.total + pad256(sizeof(double) * (size_t)n);
    }
    return large_workspace_bytes(m, n, kmax < 1 ? 1 : kmax);
}

int lhdm_solve(void* stream, int32_t m, int32_t n, const double* A, int64_t lda, const double* b,
               const lhdm_params* p, double* x, double* w, int32_t* passive, lhdm_info* info, void* ws,
               size_t ws_bytes) {
    lhdm_params def;
    if (!p) {
        lhdm_default_params(&def);
        p = &def;
    }
    if (!params_ok(p)) return LHDM_EINVAL;
    return solve_one(stream, m, n, A, lda, b, dev_params(p, n, 0), p->flags, x, w, passive, info, ws, ws_bytes);
}

size_t lhdm_signed_workspace_bytes(int32_t m, int32_t n, const lhdm_params* p) {
    lhdm_params def;
    if (!p) {
        lhdm_default_params(&def);
        p = &def;
    }
    if (m < 1 || n < 1 || n > INT_MAX / 2) return 0;
    return signed_workspace(m, n, p, nullptr);
}

int lhdm_solve_signed(void* stream, int32_t m, int32_t n, const double* A, int64_t lda, const double* b,
                      const lhdm_params* p, int32_t sign_flip, double* x, double* z, int32_t* passive,
                      lhdm_info* info, void* ws, size_t ws_bytes) {
    lhdm_params def;
    if (!p) {
        lhdm_default_params(&def);
        p = &def;
    }
    if (!params_ok(p)) return LHDM_EINVAL;
    if (m < 1 || n < 1 || n > INT_MAX / 2 || lda < m || !A || !b || !x) return LHDM_EINVAL;
    size_t solver_bytes = 0;
    const size_t need = signed_workspace(m, n, p, &solver_bytes);
    if (ws == nullptr) {
        int rc = cached_workspace(need, &ws);
        if (rc) return rc;
        ws_bytes = need;
    }
    if (ws_bytes < need || ((uintptr_t)ws & 255)) return LHDM_EWORKSPACE;
    double* zb = z ? z : (double*)((char*)ws + solver_bytes);
    DevParams prm = dev_params(p, 2 * n, 0);
    prm.twin = 1;
    prm.signflip = sign_flip ? 1 : 0;
    int rc = solve_one(stream, m, 2 * n, A, lda, b, prm, p->flags, zb, nullptr, passive, info, ws, solver_bytes);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(signed_combine, dim3((n + WG - 1) / WG), dim3(WG), 0, st, (const double*)zb, x, n);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return 0;
}

size_t lhdm_l1_workspace_bytes(int32_t m, int32_t n, const lhdm_params* p) {
    lhdm_params def;
    if (!p) {
        lhdm_default_params(&def);
        p = &def;
    }
    if (m < 1 || n < 1 || n > INT_MAX / 2 || m == INT_MAX) return 0;
    return l1_layout(m, n, p).total;
}

int lhdm_solve_l1(void* stream, int32_t m, int32_t n, const double* A, int64_t lda, const double* b, double lambda,
                  const lhdm_params* p, double* x, double* z, int32_t* passive, lhdm_info* info, void* ws,
                  size_t ws_bytes) {
    lhdm_params def;
    if (!p) {
        lhdm_default_params(&def);
        p = &def;
    }
    if (!params_ok(p)) return LHDM_EINVAL;
    if (m < 1 || n < 1 || n > INT_MAX / 2 || m == INT_MAX || lda < m || !A || !b || !x) return LHDM_EINVAL;
    if (!(lambda > 0.0) || !(lambda < INFINITY)) return LHDM_EINVAL;
    const L1Layout L = l1_layout(m, n, p);
    if (ws == nullptr) {
        int rc = cached_workspace(L.total, &ws);
        if (rc) return rc;
        ws_bytes = L.total;
    }
    if (ws_bytes < L.total || ((uintptr_t)ws & 255)) return LHDM_EWORKSPACE;
    char* base = (char*)ws;
    double* M = (double*)(base + L.M);
    double* rhs = (double*)(base + L.rhs);
    double* zb = z ? z : (double*)(base + L.z);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(l1_assemble, dim3(1024), dim3(WG), 0, st, A, (long long)lda, b, lambda, m, n, M, rhs);
    HIPCHK(hipGetLastError());
    const int lh = p->kmax == 1;
    int rc = solve_one(stream, m + 1, 2 * n, M, m + 1, rhs, dev_params(p, 2 * n, lh), p->flags, zb, nullptr,
                       passive, info, base + L.solver, L.total - L.solver);
    if (rc) return rc;
    hipLaunchKernelGGL(signed_combine, dim3((n + WG - 1) / WG), dim3(WG), 0, st, (const double*)zb, x, n);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return 0;
}

int lh_solve(void* stream, int32_t m, int32_t n, const double* A, int64_t lda, const double* b, double kkt_tol,
             int32_t max_outer, double* x, double* w, int32_t* passive, lhdm_info* info, void* ws,
             size_t ws_bytes) {
    lhdm_params p;
    lhdm_default_params(&p);
    p.kkt_tol = kkt_tol;
    p.max_outer = max_outer;
    p.kmax = 1;
    if (!(kkt_tol >= 0.0)) return LHDM_EINVAL;
    return solve_one(stream, m, n, A, lda, b, dev_params(&p, n, 1), 0, x, w, passive, info, ws, ws_bytes);
}

}  // extern "C"

namespace lhdm {

// The batched engine: forced by a flag, else the tuning table's first row whose
// bounds hold for (instances per compute unit, largest m).
static int batch_engine(int batch, const int32_t* m, const int32_t* n, int flags) {
    if (flags & LHDM_FLAG_BATCH_PHASED) return BE_PHASED;
    if (flags & LHDM_FLAG_BATCH_FUSED2) return BE_FUSED2;
    if (flags & LHDM_FLAG_BATCH_FUSED) return BE_FUSED1;
    int mmax = 1;
    for (int i = 0; i < batch; ++i) mmax = std::max(mmax, (int)m[i]);
    (void)n;
    const double per_cu = (double)batch / device_cus();
    for (const TuneRow& r : kTuneRows)
        if (per_cu <= r.per_cu_hi && mmax <= r.m_hi) return r.engine;
    return BE_FUSED1;
}

}  // namespace lhdm

extern "C" {

size_t lhdm_batched_workspace_bytes(int32_t batch, const int32_t* m, const int32_t* n, const lhdm_params* p) {
    if (batch < 1 || !m || !n) return 0;
    int mmax = 1, nmax = 1;
    size_t wextra = 0;
    for (int i = 0; i < batch; ++i) {
        mmax = std::max(mmax, (int)m[i]);
        nmax = std::max(nmax, (int)n[i]);
        wextra += (size_t)std::max(0, (int)n[i]);
    }
    const int kmax = p ? std::max(1, (int)p->kmax) : 32;
    const int eng = batch_engine(batch, m, n, p ? p->flags : 0);
    if (eng == BE_PHASED) return ph_layout(batch, m, n, kmax, nullptr).total + pad256(sizeof(double) * wextra);
    WgLayout L = wg_layout(batch, mmax, nmax, kmax, eng);
    return L.total + pad256(sizeof(double) * wextra);
}

int lhdm_solve_batched(void* stream, int32_t batch, const int32_t* m, const int32_t* n, const int64_t* a_off,
                       const double* A_pool, const int64_t* b_off, const double* b_pool, const int64_t* x_off,
                       double* x_pool, int32_t* passive_pool, const lhdm_params* p, int32_t use_lh,
                       lhdm_info* infos, void* ws, size_t ws_bytes) {
    lhdm_params def;
    if (!p) {
        lhdm_default_params(&def);
        p = &def;
    }
    if (batch < 1 || !m || !n || !a_off || !b_off || !x_off || !A_pool || !b_pool || !x_pool) return LHDM_EINVAL;
    if (!params_ok(p)) return LHDM_EINVAL;
    std::vector<int> mm(batch), nn(batch);
    int nmax = 1;
    for (int i = 0; i < batch; ++i) {
        if (m[i] < 1 || n[i] < 1) return LHDM_EINVAL;
        if (m[i] > MMAX_WG) return LHDM_EUNSUPPORTED;
        mm[i] = m[i];
        nn[i] = n[i];
        nmax = std::max(nmax, (int)n[i]);
    }
    const size_t need = lhdm_batched_workspace_bytes(batch, m, n, p);
    if (ws == nullptr) {
        int rc = cached_workspace(need, &ws);
        if (rc) return rc;
        ws_bytes = need;
    }
    if (ws_bytes < need || ((uintptr_t)ws & 255)) return LHDM_EWORKSPACE;
    const int kmax = use_lh ? 1 : p->kmax;
    const int eng = batch_engine(batch, m, n, p->flags);
    // the workspace size above was computed with p->kmax; use_lh only shrinks the slots
    const size_t lay = (eng == BE_PHASED) ? ph_layout(batch, m, n, kmax, nullptr).total
                                          : wg_layout(batch, *std::max_element(mm.begin(), mm.end()), nmax, kmax,
                                                      eng).total;
    double* wpool = (double*)((char*)ws + lay);
    std::vector<ProbIn> ins(batch);
    size_t wo = 0;
    for (int i = 0; i < batch; ++i) {
        ins[i].A = A_pool + a_off[i];
        ins[i].lda = m[i];
        ins[i].b = b_pool + b_off[i];
        ins[i].x = x_pool + x_off[i];
        ins[i].w = wpool + wo;
        wo += n[i];
        ins[i].passive = passive_pool ? passive_pool + x_off[i] : nullptr;
        ins[i].info = infos ? infos + i : nullptr;
        ins[i].m = m[i];
        ins[i].n = n[i];
    }
    DevParams prm = dev_params(p, nmax, use_lh ? 1 : 0);
    // non-positive limits are resolved per instance (3 n_i) by the kernel
    prm.max_outer = p->max_outer > 0 ? p->max_outer : 0;
    prm.max_inner = p->max_inner > 0 ? p->max_inner : 0;
    if (eng == BE_PHASED) return run_phased((hipStream_t)stream, ins, mm, nn, prm, ws, lay);
    return run_wg_engine((hipStream_t)stream, ins, mm, nn, prm, ws, lay, eng);
}

int lhdm_solve_batched_noalloc(void* stream, int32_t batch, const int32_t* m, const int32_t* n,
                               const int64_t* a_off, const double* A_pool, const int64_t* b_off,
                               const double* b_pool, const int64_t* x_off, double* x_pool, int32_t* passive_pool,
                               const lhdm_params* p, int32_t use_lh, lhdm_info* infos) {
    lhdm_params def;
    if (!p) {
        lhdm_default_params(&def);
        p = &def;
    }
    return solve_batched_noalloc((hipStream_t)stream, batch, m, n, a_off, A_pool, b_off, b_pool, x_off, x_pool,
                                 passive_pool, p, use_lh, infos);
}

size_t lhdm_backward_workspace_bytes(int32_t batch, const int32_t* m, const int32_t* n) {
    return backward_workspace_bytes(batch, m, n);
}

int lhdm_backward(void* stream, int32_t batch, const int32_t* m, const int32_t* n, const int64_t* a_off,
                  const double* A_pool, const int64_t* b_off, const double* b_pool, const int64_t* x_off,
                  const double* x_pool, const int32_t* passive_pool, const double* grad_x_pool,
                  double* grad_A_pool, double* grad_b_pool, void* ws, size_t ws_bytes) {
    if (ws == nullptr && batch > 0 && m && n) {
        ws_bytes = backward_workspace_bytes(batch, m, n);
        int rc = cached_workspace(ws_bytes, &ws);
        if (rc) return rc;
    }
    return backward_run((hipStream_t)stream, batch, m, n, a_off, A_pool, b_off, b_pool, x_off, x_pool,
                        passive_pool, grad_x_pool, grad_A_pool, grad_b_pool, ws, ws_bytes);
}

const char* lhdm_status_string(int code) {
    switch (code) {
        case LHDM_STATUS_OK: return "ok: KKT conditions hold at the requested tolerance";
        case LHDM_STATUS_MAXITER: return "iteration limit reached";
        case LHDM_STATUS_NONFINITE: return "non-finite input";
        case LHDM_STATUS_RANK: return "no numerically independent column with positive dual left";
        case LHDM_EINVAL: return "invalid argument";
        case LHDM_EWORKSPACE: return "workspace too small or misaligned";
        case LHDM_EHIP: return "HIP runtime error";
        case LHDM_EUNSUPPORTED: return "size not supported by this build";
        default: return "unknown code";
    }
}

int lhdm_last_hip_error(void) { return g_last_hip; }

void lhdm_profile_enable(int on) {
    KernelProfile& k = kprof();
    k.on = on != 0;
    k.ms = 0.0;
    k.launches = 0;
    k.bytes = 0.0;
    k.pending.clear();
    k.next = 0;
}

int lhdm_profile_read(double* total_ms, int64_t* launches, double* bytes) {
    KernelProfile& k = kprof();
    if (total_ms) *total_ms = k.ms;
    if (launches) *launches = k.launches;
    if (bytes) *bytes = k.bytes;
    return 0;
}

void lhdm_release(void) { release_workspaces(); }

}  // extern "C"
