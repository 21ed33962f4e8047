// C-ABI entry points (include/cjt.h) and the execution sequence
// (Sec. 4, "Execution"):
//   forward: recurrence rows -> Hahn blocks (DCT-I + DST-I per block and term)
//            -> T_N^{-1} (diagonally scaled DCT-I)                    (eqs. CJT, PNASY)
//   inverse: f = T_{2N}^T [c; 0], g = w .* f -> transposed Hahn blocks
//            -> recurrence columns -> times 1/A_n                      (eq. CJTT)
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "cjt_internal.h"
#include "plan.h"

struct cjt_plan_s {
    cjt::Plan p;
};

namespace cjt {

// ------------------------------------------------------------------ errors

static thread_local std::string t_err;

void set_error(const std::string& msg) { t_err = msg; }

cjt_status fail(cjt_status st, const std::string& msg)
{
    t_err = msg;
    return st;
}

// ------------------------------------------------------------------ kernel timing

namespace {

struct ProfRec {
    const char* name;
    hipEvent_t a, b;
    double flops, bytes;
};

std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_ev_pool;

hipEvent_t ev_get()
{
    if (!g_ev_pool.empty()) {
        hipEvent_t e = g_ev_pool.back();
        g_ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

}  // namespace

ProfScope::ProfScope(const char* name, double flops, double bytes, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on || !name) return;
    ProfRec r{};
    r.name = name;
    r.flops = flops;
    r.bytes = bytes;
    r.a = ev_get();
    r.b = ev_get();
    if (!r.a || !r.b) return;
    if (hipEventRecord(r.a, s) != hipSuccess) return;
    st = s;
    slot = (int)g_prof.size();
    g_prof.push_back(r);
    on = true;
}

ProfScope::~ProfScope()
{
    if (!on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (slot >= 0 && slot < (int)g_prof.size()) {
        if (hipEventRecord(g_prof[slot].b, st) != hipSuccess) g_prof[slot].name = nullptr;
    }
}

// ------------------------------------------------------------------ workspace (one per stream)

namespace {

struct Workspace {
    void* dev = nullptr;
    size_t bytes = 0;
    hipStream_t aux = nullptr;    // second stream for the recurrence kernels (default priority)
    hipEvent_t fork = nullptr, join = nullptr;
    ExecDesc* d_desc = nullptr;
    size_t desc_cap = 0;
    ExecDesc* h_desc = nullptr;   // pinned staging
    hipEvent_t copied = nullptr;  // staging buffer free once this completes
    bool pending = false;
};

std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

size_t ws_limit()
{
    static size_t lim = [] {
        const char* e = getenv("CJT_WORKSPACE_MB");
        size_t mb = e ? (size_t)atoll(e) : (size_t)4096;
        if (mb < 64) mb = 64;
        return mb << 20;
    }();
    return lim;
}

cjt_status ws_reserve(Workspace& w, size_t bytes, size_t ndesc, hipStream_t st)
{
    if (w.pending) {
        CJT_HIP_TRY(hipEventSynchronize(w.copied));
        w.pending = false;
    }
    if (bytes > w.bytes) {
        CJT_HIP_TRY(hipStreamSynchronize(st));
        if (w.dev) CJT_HIP_TRY(hipFree(w.dev));
        w.dev = nullptr;
        w.bytes = 0;
        if (hipMalloc(&w.dev, bytes) != hipSuccess) return fail(CJT_ENOMEM, "workspace allocation failed");
        w.bytes = bytes;
    }
    if (ndesc > w.desc_cap) {
        CJT_HIP_TRY(hipStreamSynchronize(st));
        if (w.d_desc) CJT_HIP_TRY(hipFree(w.d_desc));
        if (w.h_desc) CJT_HIP_TRY(hipHostFree(w.h_desc));
        w.d_desc = nullptr;
        w.h_desc = nullptr;
        w.desc_cap = 0;
        size_t cap = std::max<size_t>(ndesc, 64);
        if (hipMalloc(&w.d_desc, cap * sizeof(ExecDesc)) != hipSuccess) return fail(CJT_ENOMEM, "descriptor buffer");
        if (hipHostMalloc((void**)&w.h_desc, cap * sizeof(ExecDesc), hipHostMallocDefault) != hipSuccess)
            return fail(CJT_ENOMEM, "descriptor staging buffer");
        w.desc_cap = cap;
    }
    if (!w.copied) CJT_HIP_TRY(hipEventCreateWithFlags(&w.copied, hipEventDisableTiming));
    if (!w.aux) CJT_HIP_TRY(hipStreamCreateWithFlags(&w.aux, hipStreamNonBlocking));
    if (!w.fork) CJT_HIP_TRY(hipEventCreateWithFlags(&w.fork, hipEventDisableTiming));
    if (!w.join) CJT_HIP_TRY(hipEventCreateWithFlags(&w.join, hipEventDisableTiming));
    return CJT_OK;
}

// Zero a vector without hipMemset (kept free of memset nodes for graph capture).
__global__ void k_zero_out(const ExecDesc* __restrict__ descs)
{
    const ExecDesc& d = descs[blockIdx.y];
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n <= d.N) d.out[n] = 0.0;
}

struct Inst {
    const Plan* P;
    const double* in;
    double* out;
};

// Per-instance workspace needs (bytes), split by use: p, p2 and part live for
// the whole call (all instances at once), tmp only for the instance's chunk.
struct Need {
    size_t p, p2, part, tmp;
};

Need need_of(const Plan& P, bool inverse, bool fp32)
{
    const Part& pt = inverse ? P.inv : P.fwd;
    const int64_t L = inverse ? 2 * P.N : P.N;
    Need n;
    n.p = sizeof(double) * (size_t)(inverse ? 2 * P.N + 1 : P.N + 1);
    n.p2 = inverse ? 0 : sizeof(double) * (size_t)(P.N + 1);
    n.part = inverse ? sizeof(double) * (size_t)std::max<int64_t>(1, P.part_total_i) : 0;
    const int64_t jobs = (int64_t)pt.nblk * pt.M;
    n.tmp = (size_t)std::max<int64_t>(jobs, 1) * fft_job_bytes(L, fp32);
    // the boundary DCTs (FP64) may need an intermediate as well
    n.tmp = std::max(n.tmp, fft_job_bytes(L, false));
    return n;
}

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// Timing labels of an engine launch; the work is split between the column and
// row passes in proportion to their FFT stages (half each) for two-pass
// lengths, and all to the single pass otherwise.
void label(EngineArgs& ea, const char* n1, const char* n2, double flops, double bytes)
{
    ea.name1 = n1;
    ea.name2 = n2;
    ea.flops1 = 0.5 * flops;
    ea.flops2 = 0.5 * flops;
    ea.bytes1 = 0.5 * bytes;
    ea.bytes2 = 0.5 * bytes;
}

// Algorithmic work of one transform's kernels (see cjt_profile_enable).
struct Work {
    double rec_flops = 0, asy_flops = 0, bnd_flops = 0;
    double rec_bytes = 0, asy_bytes = 0, bnd_bytes = 0;
};

Work work_of(const Plan& P, bool inverse)
{
    Work w;
    const Part& pt = inverse ? P.inv : P.fwd;
    const std::vector<RecTask>& tasks = inverse ? P.tasks_i : P.tasks_f;
    for (const RecTask& t : tasks) w.rec_flops += (double)t.np * (double)t.cut * (t.mode == 0 ? 6.0 : 10.0);
    const double N = (double)P.N, Lr = inverse ? 4.0 * N : 2.0 * N;  // real FFT length
    const double fft = 2.5 * Lr * log2(Lr);
    for (int k = 0; k < pt.nblk; ++k) {
        const double wk = (double)(pt.win_hi[k] - pt.win_lo[k] + 1), dk = (double)(pt.deg_hi[k] - pt.deg_lo[k]);
        w.asy_flops += pt.M * (fft + 4.0 * wk + 2.0 * dk);
    }
    w.bnd_flops = fft + Lr / 2;
    const double gN = inverse ? 2.0 * N + 1 : N + 1;  // grid points
    // recurrence: coefficients in, point values out (forward) / g in, y out (inverse)
    w.rec_bytes = 8.0 * (inverse ? gN + (N + 1) : (N + 1) + gN);
    // Hahn blocks: coefficients and diagonals in (C_{n,m}, u_m, v_m), values out
    w.asy_bytes = pt.nblk ? 8.0 * (gN + (N + 1)) + 8.0 * pt.M * (N + 1) + 16.0 * pt.M * gN : 0.0;
    w.bnd_bytes = 8.0 * ((N + 1) + gN) + (inverse ? 8.0 * gN : 0.0);
    return w;
}

cjt_status execute(bool inverse, const std::vector<Inst>& insts, hipStream_t st)
{
    if (insts.empty()) return CJT_OK;
    int dev = 0;
    CJT_HIP_TRY(hipGetDevice(&dev));
    const bool fp32 = (insts[0].P->flags & CJT_FP32_BULK) != 0;
    for (auto& x : insts) {
        if (((x.P->flags & CJT_FP32_BULK) != 0) != fp32)
            return fail(CJT_EINVAL, "all plans of a batch must share the precision flag");
        if (x.P->device != dev) return fail(CJT_EINVAL, "plan belongs to another device");
    }
    // group by degree (one FFT length per launch), keeping the caller's order inside a group
    std::vector<size_t> order(insts.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return insts[a].P->N < insts[b].P->N; });

    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace& ws = g_ws[{dev, st}];

    // chunks: runs of equal N whose FFT intermediates fit the limit
    struct Chunk {
        size_t first, count;
        size_t tmp_bytes;
    };
    std::vector<Chunk> chunks;
    size_t max_tmp = 0, persist = 0;
    for (size_t i = 0; i < order.size();) {
        const int64_t N = insts[order[i]].P->N;
        Chunk c{i, 0, 0};
        while (i < order.size() && insts[order[i]].P->N == N) {
            Need nd = need_of(*insts[order[i]].P, inverse, fp32);
            if (c.count > 0 && c.tmp_bytes + a256(nd.tmp) > ws_limit()) break;
            c.tmp_bytes += a256(nd.tmp);
            persist += a256(nd.p) + a256(nd.p2) + a256(nd.part);
            ++c.count;
            ++i;
        }
        max_tmp = std::max(max_tmp, c.tmp_bytes);
        chunks.push_back(c);
    }
    cjt_status s = ws_reserve(ws, persist + max_tmp, insts.size(), st);
    if (s != CJT_OK) return s;

    // descriptors for every instance, in chunk order, copied once
    {
        char* base = (char*)ws.dev;
        size_t poff = 0;                 // persistent region [0, persist)
        for (const Chunk& c : chunks) {
            size_t toff = persist;       // chunk region [persist, persist + max_tmp)
            for (size_t q = 0; q < c.count; ++q) {
                const size_t idx = c.first + q;
                const Inst& x = insts[order[idx]];
                const Plan& P = *x.P;
                const Part& pt = inverse ? P.inv : P.fwd;
                Need nd = need_of(P, inverse, fp32);
                ExecDesc d{};
                d.N = P.N;
                d.G = inverse ? 2 * P.N : P.N;
                d.alpha = P.alpha;
                d.beta = P.beta;
                d.M = pt.M;
                d.nblk = pt.nblk;
                for (int k = 0; k < pt.nblk; ++k) {
                    d.deg_lo[k] = pt.deg_lo[k];
                    d.deg_hi[k] = pt.deg_hi[k];
                    d.win_lo[k] = pt.win_lo[k];
                    d.win_hi[k] = pt.win_hi[k];
                }
                d.C = P.C;
                d.uv = inverse ? P.uv_i : P.uv_f;
                d.w = P.w;
                d.s = P.s;
                d.tasks = inverse ? P.d_tasks_i : P.d_tasks_f;
                d.ntasks = (int32_t)(inverse ? P.tasks_i.size() : P.tasks_f.size());
                d.rec0 = inverse ? P.i0 : P.f0;
                d.recp = inverse ? P.ip : P.fp;
                d.recm = inverse ? P.im : P.fm;
                d.in = x.in;
                d.out = x.out;
                d.p = (double*)(base + poff);
                poff += a256(nd.p);
                d.p2 = nd.p2 ? (double*)(base + poff) : nullptr;
                poff += a256(nd.p2);
                d.part = nd.part ? (double*)(base + poff) : nullptr;
                poff += a256(nd.part);
                d.tmp = nd.tmp ? (void*)(base + toff) : nullptr;
                toff += a256(nd.tmp);
                ws.h_desc[idx] = d;
            }
        }
    }
    CJT_HIP_TRY(hipMemcpyAsync(ws.d_desc, ws.h_desc, sizeof(ExecDesc) * insts.size(), hipMemcpyHostToDevice, st));
    CJT_HIP_TRY(hipEventRecord(ws.copied, st));
    ws.pending = true;

    // whole-call arguments for the recurrence kernels (any mix of N)
    EngineArgs all{};
    all.d_desc = ws.d_desc;
    all.count = (int)insts.size();
    all.stream = ws.aux;
    int64_t maxN = 0;
    Work wall;
    for (const Inst& x : insts) {
        const Plan& P = *x.P;
        all.max_tasks = std::max(all.max_tasks, (int)(inverse ? P.tasks_i.size() : P.tasks_f.size()));
        maxN = std::max(maxN, P.N);
        Work w = work_of(P, inverse);
        wall.rec_flops += w.rec_flops;
        wall.rec_bytes += w.rec_bytes;
    }
    auto chunk_args = [&](const Chunk& c, Work* wk) {
        EngineArgs ea{};
        ea.d_desc = ws.d_desc + c.first;
        ea.count = (int)c.count;
        ea.stream = st;
        for (size_t q = 0; q < c.count; ++q) {
            const Plan& P = *insts[order[c.first + q]].P;
            const Part& pt = inverse ? P.inv : P.fwd;
            ea.max_jobs = std::max(ea.max_jobs, pt.nblk * pt.M);
            if (pt.nblk > 0) ea.max_m = std::max(ea.max_m, pt.M);
            Work x = work_of(P, inverse);
            wk->asy_flops += x.asy_flops;
            wk->bnd_flops += x.bnd_flops;
            wk->asy_bytes += x.asy_bytes;
            wk->bnd_bytes += x.bnd_bytes;
        }
        return ea;
    };

    if (!inverse) {
        // recurrence part on the auxiliary stream, Hahn blocks on the caller's, then the final DCT-I
        CJT_HIP_TRY(hipEventRecord(ws.fork, st));
        CJT_HIP_TRY(hipStreamWaitEvent(ws.aux, ws.fork, 0));
        {
            ProfScope ps("rec_forward", wall.rec_flops, wall.rec_bytes, ws.aux);
            if ((s = launch_rec_fwd(all)) != CJT_OK) return s;
        }
        CJT_HIP_TRY(hipEventRecord(ws.join, ws.aux));
        for (const Chunk& c : chunks) {
            Work wk;
            EngineArgs ea = chunk_args(c, &wk);
            const int64_t N = insts[order[c.first]].P->N;
            if (ea.max_jobs > 0) {
                if ((s = fft_geometry(N, fp32, st, &ea.geom)) != CJT_OK) return s;
                label(ea, fp32 ? "hahn_fwd_cols_fp32" : "hahn_fwd_cols", fp32 ? "hahn_fwd_rows_fp32" : "hahn_fwd_rows",
                      wk.asy_flops, wk.asy_bytes);
                if ((s = launch_rdft(ea, Src::FwdAsy, Sink::FwdAsy, fp32)) != CJT_OK) return s;
            }
        }
        CJT_HIP_TRY(hipStreamWaitEvent(st, ws.join, 0));
        for (const Chunk& c : chunks) {
            Work wk;
            EngineArgs ea = chunk_args(c, &wk);
            const int64_t N = insts[order[c.first]].P->N;
            if ((s = fft_geometry(N, false, st, &ea.geom)) != CJT_OK) return s;
            label(ea, "dct1_final_cols", "dct1_final_rows", wk.bnd_flops, wk.bnd_bytes);
            if ((s = launch_rdft(ea, Src::FwdFinal, Sink::FwdFinal, false)) != CJT_OK) return s;
        }
    } else {
        for (const Chunk& c : chunks) {
            Work wk;
            EngineArgs ea = chunk_args(c, &wk);
            const int64_t N = insts[order[c.first]].P->N;
            if ((s = fft_geometry(2 * N, false, st, &ea.geom)) != CJT_OK) return s;
            label(ea, "dct1_initial_cols", "dct1_initial_rows", wk.bnd_flops, wk.bnd_bytes);
            if ((s = launch_rdft(ea, Src::InvInit, Sink::InvInit, false)) != CJT_OK) return s;
        }
        CJT_HIP_TRY(hipEventRecord(ws.fork, st));
        CJT_HIP_TRY(hipStreamWaitEvent(ws.aux, ws.fork, 0));
        {
            ProfScope ps("rec_inverse", wall.rec_flops, wall.rec_bytes, ws.aux);
            if ((s = launch_rec_inv(all)) != CJT_OK) return s;
        }
        CJT_HIP_TRY(hipEventRecord(ws.join, ws.aux));
        for (const Chunk& c : chunks) {
            Work wk;
            EngineArgs ea = chunk_args(c, &wk);
            const int64_t N = insts[order[c.first]].P->N;
            if (ea.max_jobs > 0) {
                if ((s = fft_geometry(2 * N, fp32, st, &ea.geom)) != CJT_OK) return s;
                label(ea, fp32 ? "hahn_inv_cols_fp32" : "hahn_inv_cols", fp32 ? "hahn_inv_rows_fp32" : "hahn_inv_rows",
                      wk.asy_flops, wk.asy_bytes);
                if ((s = launch_rdft(ea, Src::InvAsy, Sink::InvAsy, fp32)) != CJT_OK) return s;
            } else {
                dim3 grid((unsigned)((N + 1 + 255) / 256), (unsigned)c.count);
                hipLaunchKernelGGL(k_zero_out, grid, dim3(256), 0, st, ea.d_desc);
                CJT_HIP_TRY(hipGetLastError());
            }
        }
        CJT_HIP_TRY(hipStreamWaitEvent(st, ws.join, 0));
        all.stream = st;
        ProfScope ps("rec_inverse_reduce", 0.0, 16.0 * (double)(maxN + 1) * all.count, st);
        if ((s = launch_rec_inv_reduce(all, maxN)) != CJT_OK) return s;
    }
    return CJT_OK;
}

void fill_part_info(const Part& p, cjt_partition_info* o)
{
    memset(o, 0, sizeof(*o));
    o->grid = p.G;
    o->M = p.M;
    o->nblocks = p.nblk;
    o->n_M = p.n_M;
    o->alpha_N = p.alpha_N;
    o->K = p.K;
    o->theta_bar = (int32_t)p.theta_bar;
    for (int k = 0; k < p.nblk; ++k) {
        o->deg_lo[k] = p.deg_lo[k];
        o->deg_hi[k] = p.deg_hi[k];
        o->win_lo[k] = p.win_lo[k];
        o->win_hi[k] = p.win_hi[k];
    }
    o->rec_entries = p.rec_entries;
}

cjt_status check_args(int64_t N, double alpha, double beta, int M, unsigned flags)
{
    if (N < 1) return fail(CJT_EINVAL, "N must be >= 1");
    if (N > kMaxN) return fail(CJT_EUNSUPPORTED, "N above 2^21 is not supported");
    if (!isfinite(alpha) || !isfinite(beta) || !(alpha > -0.5 && alpha <= 0.5) || !(beta > -0.5 && beta <= 0.5))
        return fail(CJT_EDOMAIN, "alpha and beta must lie in (-1/2, 1/2]");
    if (M != 0 && (M < 2 || M > kMaxM)) return fail(CJT_EDOMAIN, "M must be 0 (auto) or in [2, 30]");
    if (flags & ~(unsigned)CJT_FP32_BULK) return fail(CJT_EINVAL, "unknown flag");
    return CJT_OK;
}

void describe(const Plan& P, cjt_plan_info* out)
{
    memset(out, 0, sizeof(*out));
    out->N = P.N;
    out->alpha = P.alpha;
    out->beta = P.beta;
    out->M = std::max(P.fwd.M, P.inv.M);
    out->flags = P.flags;
    out->eps = 2.220446049250313080847263336181640625e-16;
    fill_part_info(P.fwd, &out->fwd);
    fill_part_info(P.inv, &out->inv);
    out->fft_len_fwd = P.N;
    out->fft_len_inv = 2 * P.N;
    out->fft_count_fwd = (int64_t)P.fwd.nblk * P.fwd.M;
    out->fft_count_inv = (int64_t)P.inv.nblk * P.inv.M;
    out->device_bytes = P.arena_bytes;
}

void plan_host(Plan* P, int64_t N, double alpha, double beta, int M, unsigned flags)
{
    P->N = N;
    P->alpha = alpha;
    P->beta = beta;
    P->flags = flags;
    choose_partitions(N, alpha, beta, M, &P->fwd, &P->inv);
    build_tasks(P->fwd, kRecWidthFwd, &P->tasks_f, &P->part_total_f);
    build_tasks(P->inv, kRecWidthInv, &P->tasks_i, &P->part_total_i);
}

}  // namespace

}  // namespace cjt

using namespace cjt;

extern "C" {

const char* cjt_strerror(cjt_status s)
{
    switch (s) {
        case CJT_OK: return "success";
        case CJT_EINVAL: return "invalid argument";
        case CJT_EDOMAIN: return "parameter outside the method's domain";
        case CJT_ENOMEM: return "out of memory";
        case CJT_EDEVICE: return "HIP runtime error";
        case CJT_EBUSY: return "resource busy";
        case CJT_EUNSUPPORTED: return "not supported by this build";
    }
    return "unknown status";
}

const char* cjt_last_error(void) { return t_err.c_str(); }

int cjt_version(void) { return 100; }

cjt_status cjt_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return CJT_OK;
}

cjt_status cjt_profile_collect(cjt_kernel_stat* out, int max, int* n_out)
{
    if (!n_out || (max > 0 && !out)) return fail(CJT_EINVAL, "null argument");
    CJT_HIP_TRY(hipDeviceSynchronize());
    std::lock_guard<std::mutex> lk(g_prof_mu);
    std::vector<cjt_kernel_stat> agg;
    cjt_status st = CJT_OK;
    for (ProfRec& r : g_prof) {
        g_ev_pool.push_back(r.a);
        g_ev_pool.push_back(r.b);
        if (!r.name) continue;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) st = fail(CJT_EDEVICE, "event timing failed");
        size_t i = 0;
        for (; i < agg.size(); ++i)
            if (strncmp(agg[i].name, r.name, sizeof(agg[i].name)) == 0) break;
        if (i == agg.size()) {
            cjt_kernel_stat k{};
            strncpy(k.name, r.name, sizeof(k.name) - 1);
            agg.push_back(k);
        }
        agg[i].launches += 1;
        agg[i].total_ms += ms;
        agg[i].flops += r.flops;
        agg[i].bytes += r.bytes;
    }
    g_prof.clear();
    int n = (int)std::min<size_t>(agg.size(), (size_t)std::max(max, 0));
    for (int i = 0; i < n; ++i) out[i] = agg[i];
    *n_out = n;
    return st;
}

cjt_status cjt_plan_describe(int64_t N, double alpha, double beta, int M, unsigned flags, cjt_plan_info* out)
{
    if (!out) return fail(CJT_EINVAL, "null output");
    cjt_status s = check_args(N, alpha, beta, M, flags);
    if (s != CJT_OK) return s;
    Plan P;
    plan_host(&P, N, alpha, beta, M, flags);
    describe(P, out);
    // estimate of the device arena
    const int64_t nf = N + 1, ni = 2 * N + 1;
    const int Mx = out->M;
    out->device_bytes = sizeof(double) * (size_t)Mx * nf + 16 * (size_t)P.fwd.M * nf + 16 * (size_t)P.inv.M * ni +
                        8 * (size_t)ni * 2 + 8 * (size_t)nf + 32 * 6 * (size_t)nf +
                        sizeof(RecTask) * (P.tasks_f.size() + P.tasks_i.size());
    return CJT_OK;
}

cjt_status cjt_plan(cjt_plan_t* out, int64_t N, double alpha, double beta, int M, unsigned flags, void* stream)
{
    if (!out) return fail(CJT_EINVAL, "null output");
    *out = nullptr;
    cjt_status s = check_args(N, alpha, beta, M, flags);
    if (s != CJT_OK) return s;
    cjt_plan_s* h = new (std::nothrow) cjt_plan_s;
    if (!h) return fail(CJT_ENOMEM, "host allocation failed");
    plan_host(&h->p, N, alpha, beta, M, flags);
    if (hipGetDevice(&h->p.device) != hipSuccess) {
        delete h;
        return fail(CJT_EDEVICE, "no HIP device");
    }
    s = build_plan_device(&h->p, (hipStream_t)stream);
    if (s != CJT_OK) {
        if (h->p.arena) (void)hipFree(h->p.arena);
        delete h;
        return s;
    }
    *out = h;
    return CJT_OK;
}

cjt_status cjt_plan_destroy(cjt_plan_t plan)
{
    if (!plan) return CJT_OK;
    if (plan->p.arena) {
        CJT_HIP_TRY(hipDeviceSynchronize());
        CJT_HIP_TRY(hipFree(plan->p.arena));
    }
    delete plan;
    return CJT_OK;
}

cjt_status cjt_plan_query(cjt_plan_t plan, cjt_plan_info* out)
{
    if (!plan || !out) return fail(CJT_EINVAL, "null argument");
    describe(plan->p, out);
    return CJT_OK;
}

static cjt_status single(bool inverse, cjt_plan_t plan, const double* d_in, double* d_out, void* stream)
{
    if (!plan || !d_in || !d_out) return fail(CJT_EINVAL, "null argument");
    if ((const void*)d_in == (const void*)d_out) return fail(CJT_EINVAL, "in-place transforms are not supported");
    std::vector<Inst> v = {Inst{&plan->p, d_in, d_out}};
    return execute(inverse, v, (hipStream_t)stream);
}

cjt_status cjt_forward(cjt_plan_t plan, const double* d_in, double* d_out, void* stream)
{
    return single(false, plan, d_in, d_out, stream);
}

cjt_status cjt_inverse(cjt_plan_t plan, const double* d_in, double* d_out, void* stream)
{
    return single(true, plan, d_in, d_out, stream);
}

static cjt_status batched(bool inverse, const cjt_plan_t* plans, int64_t count, const int64_t* offsets,
                          const double* d_in, double* d_out, void* stream)
{
    if (count < 0 || (count > 0 && (!plans || !offsets || !d_in || !d_out)))
        return fail(CJT_EINVAL, "null argument");
    if (count == 0) return CJT_OK;
    if ((const void*)d_in == (const void*)d_out) return fail(CJT_EINVAL, "in-place transforms are not supported");
    std::vector<Inst> v;
    v.reserve((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        if (!plans[i]) return fail(CJT_EINVAL, "null plan in batch");
        if (offsets[i] < 0 || offsets[i + 1] - offsets[i] != plans[i]->p.N + 1)
            return fail(CJT_EINVAL, "offsets do not match the plans' N + 1");
        v.push_back(Inst{&plans[i]->p, d_in + offsets[i], d_out + offsets[i]});
    }
    return execute(inverse, v, (hipStream_t)stream);
}

cjt_status cjt_forward_batched(const cjt_plan_t* plans, int64_t count, const int64_t* offsets, const double* d_in,
                               double* d_out, void* stream)
{
    return batched(false, plans, count, offsets, d_in, d_out, stream);
}

cjt_status cjt_inverse_batched(const cjt_plan_t* plans, int64_t count, const int64_t* offsets, const double* d_in,
                               double* d_out, void* stream)
{
    return batched(true, plans, count, offsets, d_in, d_out, stream);
}

}  // extern "C"
