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
#include "exec.h"
#include "plan.h"


// A persistent batch: the launch program, its descriptors and work items
// resident on the device, and its own workspace; executing it only launches
// kernels, so it can be captured into a HIP graph.
struct cjt_batch_s {
    int device = 0;
    bool inverse = false;
    cjt::Built b;
    void* ws = nullptr;
    char* meta = nullptr;  // descriptors, then items
    size_t dbytes = 0;
    hipStream_t aux = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
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
    char* d_meta = nullptr;       // descriptors and work items on the device
    char* h_meta = nullptr;       // pinned staging of the same
    size_t meta_cap = 0;
    hipEvent_t copied = nullptr;  // staging buffer free once this completes
    double* mid = nullptr;        // Jacobi-to-Jacobi: Chebyshev coefficients between the two halves
    size_t mid_cap = 0;           // doubles
    double* shift = nullptr;      // CJT_SHIFT forward: input moved to the core's parameters
    size_t shift_cap = 0;         // doubles
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

cjt_status ws_reserve(Workspace& w, size_t bytes, size_t meta, hipStream_t st)
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
    if (meta > w.meta_cap) {
        CJT_HIP_TRY(hipStreamSynchronize(st));
        if (w.d_meta) CJT_HIP_TRY(hipFree(w.d_meta));
        if (w.h_meta) CJT_HIP_TRY(hipHostFree(w.h_meta));
        w.d_meta = nullptr;
        w.h_meta = nullptr;
        w.meta_cap = 0;
        const size_t cap = std::max<size_t>(meta + meta / 2, 1 << 16);
        if (hipMalloc((void**)&w.d_meta, cap) != hipSuccess) return fail(CJT_ENOMEM, "descriptor buffer");
        if (hipHostMalloc((void**)&w.h_meta, cap, hipHostMallocDefault) != hipSuccess)
            return fail(CJT_ENOMEM, "descriptor staging buffer");
        w.meta_cap = cap;
    }
    if (!w.copied) CJT_HIP_TRY(hipEventCreateWithFlags(&w.copied, hipEventDisableTiming));
    if (!w.aux) CJT_HIP_TRY(hipStreamCreateWithFlags(&w.aux, hipStreamNonBlocking));
    if (!w.fork) CJT_HIP_TRY(hipEventCreateWithFlags(&w.fork, hipEventDisableTiming));
    if (!w.join) CJT_HIP_TRY(hipEventCreateWithFlags(&w.join, hipEventDisableTiming));
    return CJT_OK;
}

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

cjt_status check_batch(const std::vector<const Plan*>& plans)
{
    int dev = 0;
    CJT_HIP_TRY(hipGetDevice(&dev));
    const bool fp32 = (plans[0]->flags & CJT_FP32_BULK) != 0;
    for (const Plan* P : plans) {
        if (((P->flags & CJT_FP32_BULK) != 0) != fp32)
            return fail(CJT_EINVAL, "all plans of a batch must share the precision flag");
        if (P->device != dev) return fail(CJT_EINVAL, "plan belongs to another device");
    }
    return CJT_OK;
}

cjt_status execute_core(bool inverse, const std::vector<const Plan*>& plans, const std::vector<int64_t>& io_off,
                        const double* in, double* out, hipStream_t st)
{
    if (plans.empty()) return CJT_OK;
    cjt_status s = check_batch(plans);
    if (s != CJT_OK) return s;
    int dev = 0;
    CJT_HIP_TRY(hipGetDevice(&dev));
    Built b;
    if ((s = build_program(plans, io_off, inverse, ws_limit(), false, st, &b)) != CJT_OK) return s;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace& ws = g_ws[{dev, st}];
    const size_t dbytes = a256(sizeof(ExecDesc) * b.pr.descs.size());
    const size_t ibytes = sizeof(Item) * b.pr.items.size();
    if ((s = ws_reserve(ws, std::max<size_t>(b.ws_bytes, 256), dbytes + ibytes, st)) != CJT_OK) return s;
    bind_workspace(b, ws.dev);
    for (ExecDesc& d : b.pr.descs) {
        d.in = in + d.io_off;
        d.out = out + d.io_off;
    }
    memcpy(ws.h_meta, b.pr.descs.data(), sizeof(ExecDesc) * b.pr.descs.size());
    if (ibytes) memcpy(ws.h_meta + dbytes, b.pr.items.data(), ibytes);
    CJT_HIP_TRY(hipMemcpyAsync(ws.d_meta, ws.h_meta, dbytes + ibytes, hipMemcpyHostToDevice, st));
    CJT_HIP_TRY(hipEventRecord(ws.copied, st));
    ws.pending = true;
    return run_program(b.pr, (const ExecDesc*)ws.d_meta, (const Item*)(ws.d_meta + dbytes), st, ws.aux, ws.fork,
                       ws.join, in, out);
}

// The transform with plans that shift their parameters (CJT_SHIFT): the
// forward moves the input's coefficients to the core's parameters in a
// per-stream buffer first; the inverse moves the core's output to the
// caller's parameters in place afterwards.  Instances are contiguous from
// io_off[0] (offsets of the batched calls).
cjt_status execute(bool inverse, const std::vector<const Plan*>& plans, const std::vector<int64_t>& io_off,
                   const double* in, double* out, hipStream_t st)
{
    bool any = false;
    for (const Plan* P : plans) any = any || P->sh_a != 0 || P->sh_b != 0;
    if (!any) return execute_core(inverse, plans, io_off, in, out, st);
    cjt_status s = CJT_OK;
    if (inverse) {
        if ((s = execute_core(true, plans, io_off, in, out, st)) != CJT_OK) return s;
        for (size_t i = 0; i < plans.size(); ++i)
            if ((s = apply_shift(*plans[i], out + io_off[i], false, st)) != CJT_OK) return s;
        return CJT_OK;
    }
    const int64_t lo = io_off.front(), hi = io_off.back() + plans.back()->N + 1;
    int dev = 0;
    CJT_HIP_TRY(hipGetDevice(&dev));
    double* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        Workspace& ws = g_ws[{dev, st}];
        if ((size_t)hi > ws.shift_cap) {
            CJT_HIP_TRY(hipStreamSynchronize(st));
            if (ws.shift) CJT_HIP_TRY(hipFree(ws.shift));
            ws.shift = nullptr;
            ws.shift_cap = 0;
            if (hipMalloc((void**)&ws.shift, sizeof(double) * (size_t)hi) != hipSuccess)
                return fail(CJT_ENOMEM, "shift buffer allocation failed");
            ws.shift_cap = (size_t)hi;
        }
        base = ws.shift;
    }
    CJT_HIP_TRY(hipMemcpyAsync(base + lo, in + lo, sizeof(double) * (size_t)(hi - lo), hipMemcpyDeviceToDevice, st));
    for (size_t i = 0; i < plans.size(); ++i)
        if ((s = apply_shift(*plans[i], base + io_off[i], true, st)) != CJT_OK) return s;
    return execute_core(false, plans, io_off, base, out, st);
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

void describe(const Plan& P, cjt_plan_info* out)
{
    memset(out, 0, sizeof(*out));
    out->N = P.N;
    out->alpha = P.alpha + P.sh_a;  // the caller's parameters
    out->beta = P.beta + P.sh_b;
    out->shift_alpha = P.sh_a;
    out->shift_beta = P.sh_b;
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
    FftGeom g;
    geometry_shape(P.N, &g, P.lg1_f);
    out->fft_log2_cols_fwd = g.single ? 0 : g.logL1;
    geometry_shape(2 * P.N, &g, P.lg1_i);
    out->fft_log2_cols_inv = g.single ? 0 : g.logL1;
}

}  // namespace

cjt_status check_args(int64_t N, double alpha, double beta, int M, unsigned flags)
{
    if (N < 1) return fail(CJT_EINVAL, "N must be >= 1");
    if (N > kMaxN) return fail(CJT_EUNSUPPORTED, "N above 2^21 is not supported");
    if (flags & CJT_SHIFT) {
        if (!isfinite(alpha) || !isfinite(beta) || !(alpha > -1.0 && alpha <= kMaxShiftParam) ||
            !(beta > -1.0 && beta <= kMaxShiftParam))
            return fail(CJT_EDOMAIN, "with CJT_SHIFT, alpha and beta must lie in (-1, 5/2]");
    } else if (!isfinite(alpha) || !isfinite(beta) || !(alpha > -0.5 && alpha <= 0.5) ||
               !(beta > -0.5 && beta <= 0.5)) {
        return fail(CJT_EDOMAIN, "alpha and beta must lie in (-1/2, 1/2]");
    }
    if (M != 0 && (M < 2 || M > kMaxM)) return fail(CJT_EDOMAIN, "M must be 0 (auto) or in [2, 30]");
    if (flags & ~(unsigned)(CJT_FP32_BULK | CJT_BATCH_INVARIANT | CJT_SHIFT)) return fail(CJT_EINVAL, "unknown flag");
    return CJT_OK;
}

void plan_host(Plan* P, int64_t N, double alpha, double beta, int M, unsigned flags)
{
    if (flags & CJT_SHIFT) {  // the core at the base parameters
        shift_split(alpha, &P->sh_a, &alpha);
        shift_split(beta, &P->sh_b, &beta);
    }
    P->N = N;
    P->alpha = alpha;
    P->beta = beta;
    P->flags = flags;
    choose_partitions(N, alpha, beta, M, &P->fwd, &P->inv);
    build_tasks(P->fwd, kRecWidthFwd, &P->tasks_f, &P->part_total_f);
    build_tasks(P->inv, kRecWidthInv, &P->tasks_i, &P->part_total_i);
    plan_layout(P);
}

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
        case CJT_ECANCELED: return "request cancelled";
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
    s = build_plan_device(&h->p, (hipStream_t)stream, nullptr, nullptr);
    if (s != CJT_OK) {
        delete h;
        return s;
    }
    *out = h;
    return CJT_OK;
}

cjt_status cjt_plan_destroy(cjt_plan_t plan)
{
    if (!plan) return CJT_OK;
    if (plan->p.arena && plan->p.own_arena) {
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
    return execute(inverse, {&plan->p}, {0}, d_in, d_out, (hipStream_t)stream);
}

cjt_status cjt_forward(cjt_plan_t plan, const double* d_in, double* d_out, void* stream)
{
    return single(false, plan, d_in, d_out, stream);
}

cjt_status cjt_inverse(cjt_plan_t plan, const double* d_in, double* d_out, void* stream)
{
    return single(true, plan, d_in, d_out, stream);
}

static cjt_status gather(const cjt_plan_t* plans, int64_t count, const int64_t* offsets, std::vector<const Plan*>* v,
                         std::vector<int64_t>* off)
{
    v->reserve((size_t)count);
    off->reserve((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        if (!plans[i]) return fail(CJT_EINVAL, "null plan in batch");
        if (offsets[i] < 0 || offsets[i + 1] - offsets[i] != plans[i]->p.N + 1)
            return fail(CJT_EINVAL, "offsets do not match the plans' N + 1");
        v->push_back(&plans[i]->p);
        off->push_back(offsets[i]);
    }
    return CJT_OK;
}

static cjt_status batched(bool inverse, const cjt_plan_t* plans, int64_t count, const int64_t* offsets,
                          const double* d_in, double* d_out, void* stream)
{
    if (count < 0 || (count > 0 && (!plans || !offsets || !d_in || !d_out)))
        return fail(CJT_EINVAL, "null argument");
    if (count == 0) return CJT_OK;
    if ((const void*)d_in == (const void*)d_out) return fail(CJT_EINVAL, "in-place transforms are not supported");
    std::vector<const Plan*> v;
    std::vector<int64_t> off;
    cjt_status s = gather(plans, count, offsets, &v, &off);
    if (s != CJT_OK) return s;
    return execute(inverse, v, off, d_in, d_out, (hipStream_t)stream);
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

// Forward with `from`, inverse with `to`, through the stream's buffer of
// Chebyshev coefficients (total doubles).
static cjt_status compose(const std::vector<const Plan*>& from, const std::vector<const Plan*>& to,
                          const std::vector<int64_t>& off, int64_t total, const double* in, double* out,
                          hipStream_t st)
{
    if ((from[0]->flags & CJT_FP32_BULK) != (to[0]->flags & CJT_FP32_BULK))
        return fail(CJT_EINVAL, "source and target plans must share the precision flag");
    for (size_t i = 0; i < from.size(); ++i)
        if (from[i]->N != to[i]->N) return fail(CJT_EINVAL, "source and target plans differ in N");
    int dev = 0;
    CJT_HIP_TRY(hipGetDevice(&dev));
    double* mid = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        Workspace& ws = g_ws[{dev, st}];
        if ((size_t)total > ws.mid_cap) {
            CJT_HIP_TRY(hipStreamSynchronize(st));
            if (ws.mid) CJT_HIP_TRY(hipFree(ws.mid));
            ws.mid = nullptr;
            ws.mid_cap = 0;
            if (hipMalloc((void**)&ws.mid, sizeof(double) * (size_t)total) != hipSuccess)
                return fail(CJT_ENOMEM, "Chebyshev buffer allocation failed");
            ws.mid_cap = (size_t)total;
        }
        mid = ws.mid;
    }
    cjt_status s = execute(false, from, off, in, mid, st);
    if (s != CJT_OK) return s;
    return execute(true, to, off, mid, out, st);
}

cjt_status cjt_jacobi_to_jacobi(cjt_plan_t from, cjt_plan_t to, const double* d_in, double* d_out, void* stream)
{
    if (!from || !to || !d_in || !d_out) return fail(CJT_EINVAL, "null argument");
    if ((const void*)d_in == (const void*)d_out) return fail(CJT_EINVAL, "in-place transforms are not supported");
    return compose({&from->p}, {&to->p}, {0}, from->p.N + 1, d_in, d_out, (hipStream_t)stream);
}

cjt_status cjt_jacobi_to_jacobi_batched(const cjt_plan_t* from, const cjt_plan_t* to, int64_t count,
                                        const int64_t* offsets, const double* d_in, double* d_out, void* stream)
{
    if (count < 0 || (count > 0 && (!from || !to || !offsets || !d_in || !d_out)))
        return fail(CJT_EINVAL, "null argument");
    if (count == 0) return CJT_OK;
    if ((const void*)d_in == (const void*)d_out) return fail(CJT_EINVAL, "in-place transforms are not supported");
    std::vector<const Plan*> vf, vt;
    std::vector<int64_t> off, off2;
    cjt_status s = gather(from, count, offsets, &vf, &off);
    if (s != CJT_OK) return s;
    if ((s = gather(to, count, offsets, &vt, &off2)) != CJT_OK) return s;
    return compose(vf, vt, off, offsets[count], d_in, d_out, (hipStream_t)stream);
}

static void batch_free(cjt_batch_s* b)
{
    if (b->ws) (void)hipFree(b->ws);
    if (b->meta) (void)hipFree(b->meta);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    if (b->aux) (void)hipStreamDestroy(b->aux);
    delete b;
}

cjt_status cjt_batch_create(cjt_batch_t* out, const cjt_plan_t* plans, int64_t count, const int64_t* offsets,
                            unsigned flags, void* stream)
{
    if (!out) return fail(CJT_EINVAL, "null output");
    *out = nullptr;
    if (count <= 0 || !plans || !offsets) return fail(CJT_EINVAL, "empty batch or null argument");
    if (flags != CJT_DIR_FWD && flags != CJT_DIR_INV) return fail(CJT_EINVAL, "flags must be CJT_DIR_FWD or CJT_DIR_INV");
    std::vector<const Plan*> v;
    std::vector<int64_t> off;
    cjt_status s = gather(plans, count, offsets, &v, &off);
    if (s != CJT_OK) return s;
    if ((s = check_batch(v)) != CJT_OK) return s;
    for (const Plan* P : v)
        if (P->sh_a != 0 || P->sh_b != 0)
            return fail(CJT_EUNSUPPORTED, "persistent batches take plans without parameter shifts");
    hipStream_t st = (hipStream_t)stream;
    cjt_batch_s* b = new (std::nothrow) cjt_batch_s;
    if (!b) return fail(CJT_ENOMEM, "host allocation failed");
    b->inverse = flags == CJT_DIR_INV;
    do {
        if (hipGetDevice(&b->device) != hipSuccess) { s = fail(CJT_EDEVICE, "no HIP device"); break; }
        // the whole batch's FFT intermediates at once: no chunking
        if ((s = build_program(v, off, b->inverse, SIZE_MAX, true, st, &b->b)) != CJT_OK) break;
        if (hipMalloc(&b->ws, std::max<size_t>(b->b.ws_bytes, 256)) != hipSuccess) {
            s = fail(CJT_ENOMEM, "batch workspace allocation failed");
            break;
        }
        bind_workspace(b->b, b->ws);
        b->dbytes = a256(sizeof(ExecDesc) * b->b.pr.descs.size());
        const size_t ibytes = sizeof(Item) * b->b.pr.items.size();
        if (hipMalloc((void**)&b->meta, b->dbytes + ibytes + 1) != hipSuccess) {
            s = fail(CJT_ENOMEM, "batch descriptor allocation failed");
            break;
        }
        if (hipMemcpy(b->meta, b->b.pr.descs.data(), sizeof(ExecDesc) * b->b.pr.descs.size(), hipMemcpyHostToDevice) !=
                hipSuccess ||
            (ibytes && hipMemcpy(b->meta + b->dbytes, b->b.pr.items.data(), ibytes, hipMemcpyHostToDevice) != hipSuccess)) {
            s = fail(CJT_EDEVICE, "batch upload failed");
            break;
        }
        if (hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess) {
            s = fail(CJT_EDEVICE, "batch stream setup failed");
            break;
        }
    } while (0);
    if (s != CJT_OK) {
        batch_free(b);
        return s;
    }
    *out = b;
    return CJT_OK;
}

cjt_status cjt_batch_execute(cjt_batch_t batch, const double* d_in, double* d_out, void* stream)
{
    if (!batch || !d_in || !d_out) return fail(CJT_EINVAL, "null argument");
    if ((const void*)d_in == (const void*)d_out) return fail(CJT_EINVAL, "in-place transforms are not supported");
    int dev = 0;
    CJT_HIP_TRY(hipGetDevice(&dev));
    if (dev != batch->device) return fail(CJT_EINVAL, "batch belongs to another device");
    return run_program(batch->b.pr, (const ExecDesc*)batch->meta, (const Item*)(batch->meta + batch->dbytes),
                       (hipStream_t)stream, batch->aux, batch->fork, batch->join, d_in, d_out);
}

cjt_status cjt_batch_query(cjt_batch_t batch, cjt_batch_info* out)
{
    if (!batch || !out) return fail(CJT_EINVAL, "null argument");
    memset(out, 0, sizeof(*out));
    out->count = (int64_t)batch->b.pr.descs.size();
    out->launches = (int64_t)batch->b.pr.launches.size();
    out->items = (int64_t)batch->b.pr.items.size();
    out->workspace_bytes = batch->b.ws_bytes;
    out->inverse = batch->inverse ? 1 : 0;
    return CJT_OK;
}

cjt_status cjt_batch_destroy(cjt_batch_t batch)
{
    if (!batch) return CJT_OK;
    CJT_HIP_TRY(hipDeviceSynchronize());
    batch_free(batch);
    return CJT_OK;
}

cjt_status cjt_autotune(int64_t N, unsigned flags, int64_t batch, int reps, void* stream, cjt_tune_entry* out,
                        int* n_out)
{
    if (!out || !n_out) return fail(CJT_EINVAL, "null output");
    *n_out = 0;
    if (reps < 1 || reps > 1000) return fail(CJT_EINVAL, "reps must be in [1, 1000]");
    if (batch < 1 || batch > 4096) return fail(CJT_EINVAL, "batch must be in [1, 4096]");
    const unsigned prec = flags & CJT_FP32_BULK;
    if (flags & ~(unsigned)CJT_FP32_BULK) return fail(CJT_EINVAL, "flags must be CJT_FP64 or CJT_FP32_BULK");
    const double a = 0.1, b = 0.1;
    cjt_status s = check_args(N, a, b, 0, prec);
    if (s != CJT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    CJT_HIP_TRY(hipGetDevice(&dev));
    // synthetic input c_n = 1/(n+1) and an output buffer
    const size_t n1 = (size_t)N + 1, total = n1 * (size_t)batch;
    std::vector<double> host(total);
    for (size_t i = 0; i < total; ++i) host[i] = 1.0 / (double)(i % n1 + 1);
    double* buf = nullptr;
    if (hipMalloc((void**)&buf, sizeof(double) * 2 * total) != hipSuccess)
        return fail(CJT_ENOMEM, "autotune buffers");
    double* d_in = buf;
    double* d_out = buf + total;
    std::vector<int64_t> offs((size_t)batch);
    for (int64_t i = 0; i < batch; ++i) offs[(size_t)i] = i * (int64_t)n1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    s = CJT_OK;
    if (hipMemcpy(d_in, host.data(), sizeof(double) * host.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        s = fail(CJT_EDEVICE, "autotune set-up");
    for (int inv = 0; inv < 2 && s == CJT_OK; ++inv) {
        const int64_t L = inv ? 2 * N : N;
        FftGeom g;
        geometry_shape(L, &g, -1);
        if (g.single) continue;
        const int64_t F = fft_power_length(L);
        const int lg = g.bluestein ? g.logP : g.logL;
        int lo = 0, hi = 0;
        split_range(lg, &lo, &hi);
        const bool chirp = g.bluestein != 0;
        cjt_tune_entry e{};
        e.fft_len = F;
        e.inverse = inv;
        e.chirp = chirp ? 1 : 0;
        e.fp32 = prec ? 1 : 0;
        e.log2_cols_default = tuned_split(F, prec != 0, chirp, inv != 0);
        if (e.log2_cols_default < 0) e.log2_cols_default = lg / 2;
        double best = 1e300;
        for (int lg1 = lo; lg1 <= hi && s == CJT_OK; ++lg1) {
            set_tuned_split(F, prec != 0, chirp, inv != 0, lg1);
            Plan P;
            plan_host(&P, N, a, b, 0, prec);
            P.device = dev;
            if ((s = build_plan_device(&P, st, nullptr, nullptr)) != CJT_OK) break;
            float ms = 0.0f;
            const std::vector<const Plan*> plans((size_t)batch, &P);
            if ((s = execute(inv != 0, plans, offs, d_in, d_out, st)) == CJT_OK &&
                hipEventRecord(e0, st) == hipSuccess) {
                for (int r = 0; r < reps && s == CJT_OK; ++r) s = execute(inv != 0, plans, offs, d_in, d_out, st);
                if (s == CJT_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    s = fail(CJT_EDEVICE, "autotune timing");
            }
            (void)hipStreamSynchronize(st);
            if (P.arena && P.own_arena) (void)hipFree(P.arena);
            if (s != CJT_OK) break;
            const double t = (double)ms / reps;
            e.candidates += 1;
            if (lg1 == e.log2_cols_default) e.ms_default = t;
            if (t < best) {
                best = t;
                e.log2_cols_best = lg1;
                e.ms_best = t;
            }
        }
        set_tuned_split(F, prec != 0, chirp, inv != 0, s == CJT_OK ? e.log2_cols_best : -1);
        if (s == CJT_OK && *n_out < 2) out[(*n_out)++] = e;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    return s;
}

}  // extern "C"
