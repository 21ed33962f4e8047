// Launch program of a transform call (Sec. 4, "Execution"):
//   forward: recurrence rows (auxiliary stream)  ||  Hahn blocks (DCT-I + DST-I
//            per block and term)  ->  T_N^{-1} (diagonally scaled DCT-I)      (eqs. CJT, PNASY)
//   inverse: f = T_{2N}^T [c; 0], g = w .* f  ->  recurrence columns (auxiliary
//            stream)  ||  transposed Hahn blocks  ->  sum, times 1/A_n       (eq. CJTT)
// Each step is one launch (or a few, by kernel shape) over a flat list of work
// items covering every instance of the call, whatever their degrees.
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "exec.h"

namespace cjt {

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// Calls with at most this many instances run the Hahn jobs of short lengths
// one workgroup each (latency); larger calls loop over the jobs inside one
// workgroup per instance (no intermediate traffic).
constexpr size_t kJobParallelMax = 64;

// Algorithmic work of one transform's kernels (the counting of cjt_profile_enable).
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

// Sets in/out of every descriptor from the call's base pointers.
__global__ void k_patch(ExecDesc* __restrict__ descs, int count, const double* in, double* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    descs[i].in = in + descs[i].io_off;
    descs[i].out = out + descs[i].io_off;
}

}  // namespace

cjt_status build_program(const std::vector<const Plan*>& plans, const std::vector<int64_t>& io_off, bool inverse,
                         size_t tmp_limit, bool with_patch, hipStream_t, Built* out)
{
    Built& b = *out;
    b = Built{};
    Program& pr = b.pr;
    const size_t n = plans.size();
    if (n == 0) return CJT_OK;
    const bool fp32 = (plans[0]->flags & CJT_FP32_BULK) != 0;

    // descriptors
    std::vector<const RecTask*> tasks(n);
    std::vector<double> asy_f(n), asy_b(n), bnd_f(n), bnd_b(n);
    double rec_f = 0, rec_b = 0, red_b = 0;
    pr.descs.resize(n);
    for (size_t i = 0; i < n; ++i) {
        const Plan& P = *plans[i];
        const Part& pt = inverse ? P.inv : P.fwd;
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
        d.io_off = io_off[i];
        d.geo = inverse ? P.geo_i : P.geo_f;
        d.geob = fp32 ? (inverse ? P.geob_i : P.geob_f) : d.geo;
        pr.descs[i] = d;
        tasks[i] = inverse ? P.tasks_i.data() : P.tasks_f.data();
        const Work w = work_of(P, inverse);
        asy_f[i] = w.asy_flops;
        asy_b[i] = w.asy_bytes;
        bnd_f[i] = w.bnd_flops;
        bnd_b[i] = w.bnd_bytes;
        rec_f += w.rec_flops;
        rec_b += w.rec_bytes;
        red_b += 16.0 * (double)(P.N + 1);
    }
    // recurrence segment length: from the whole call, or per instance for
    // plans that ask for results independent of the rest of the call
    {
        std::vector<int> all(n);
        for (size_t i = 0; i < n; ++i) all[i] = (int)i;
        const int32_t S = rec_segment_length(pr, tasks, all);
        for (size_t i = 0; i < n; ++i)
            pr.descs[i].rec_seg =
                (plans[i]->flags & CJT_BATCH_INVARIANT) ? rec_segment_length(pr, tasks, std::vector<int>{(int)i}) : S;
    }
    // few instances: spread the Hahn jobs of single-workgroup lengths over workgroups
    const bool job_parallel = n <= kJobParallelMax;

    // workspace: persistent p, p2, part, seg for all instances, then one
    // region of FFT intermediates reused by consecutive chunks of instances
    b.offs.resize(n);
    size_t off = 0;
    std::vector<size_t> tmp_need(n);
    for (size_t i = 0; i < n; ++i) {
        const ExecDesc& d = pr.descs[i];
        const Plan& P = *plans[i];
        DescOffsets& o = b.offs[i];
        o.p = off;
        off += a256(sizeof(double) * (size_t)(d.G + 1));
        o.p2 = SIZE_MAX;
        if (!inverse) {
            o.p2 = off;
            off += a256(sizeof(double) * (size_t)(d.N + 1));
        }
        o.part = SIZE_MAX;
        if (inverse) {
            o.part = off;
            off += a256(sizeof(double) * (size_t)std::max<int64_t>(1, P.part_total_i));
        }
        const int64_t segd = rec_seg_doubles(d, tasks[i]);
        o.seg = SIZE_MAX;
        if (segd > 0) {
            o.seg = off;
            off += a256(sizeof(double) * (size_t)segd);
        }
        const int64_t jobs = (int64_t)d.nblk * d.M;
        size_t t = fft_tmp_bytes(d.geob, jobs, fp32, job_parallel);   // Hahn blocks
        t = std::max(t, fft_tmp_bytes(d.geo, 1, false, job_parallel));  // boundary transform (FP64)
        tmp_need[i] = a256(t);
    }
    const size_t persist = off;
    std::vector<std::vector<int>> chunks;
    size_t max_chunk = 0;
    {
        size_t cur = 0;
        chunks.emplace_back();
        for (size_t i = 0; i < n; ++i) {
            if (!chunks.back().empty() && cur + tmp_need[i] > tmp_limit) {
                chunks.emplace_back();
                cur = 0;
            }
            b.offs[i].tmp = tmp_need[i] ? persist + cur : SIZE_MAX;
            cur += tmp_need[i];
            chunks.back().push_back((int)i);
            max_chunk = std::max(max_chunk, cur);
        }
    }
    b.ws_bytes = persist + max_chunk;

    // launches
    if (with_patch) {
        Launch L;
        L.kind = Kind::Patch;
        L.nth = 64;
        L.nitems = (int64_t)n;
        pr.launches.push_back(L);
    }
    auto mark = [&](Kind k) {
        Launch L;
        L.kind = k;
        pr.launches.push_back(L);
    };
    cjt_status s = CJT_OK;
    if (!inverse) {
        mark(Kind::Fork);
        add_rec_fwd(pr, tasks, 1, rec_f, rec_b);
        for (auto& c : chunks)
            if ((s = add_fft(pr, c, Src::FwdAsy, Sink::FwdAsy, fp32, 0, fp32 ? "hahn_fwd_cols_fp32" : "hahn_fwd_cols",
                             fp32 ? "hahn_fwd_rows_fp32" : "hahn_fwd_rows", asy_f, asy_b, job_parallel)) != CJT_OK)
                return s;
        mark(Kind::Join);
        for (auto& c : chunks)
            if ((s = add_fft(pr, c, Src::FwdFinal, Sink::FwdFinal, false, 0, "dct1_final_cols", "dct1_final_rows",
                             bnd_f, bnd_b)) != CJT_OK)
                return s;
    } else {
        for (auto& c : chunks)
            if ((s = add_fft(pr, c, Src::InvInit, Sink::InvInit, false, 0, "dct1_initial_cols", "dct1_initial_rows",
                             bnd_f, bnd_b)) != CJT_OK)
                return s;
        mark(Kind::Fork);
        add_rec_inv(pr, tasks, 1, rec_f, rec_b);
        for (auto& c : chunks)
            if ((s = add_fft(pr, c, Src::InvAsy, Sink::InvAsy, fp32, 0, fp32 ? "hahn_inv_cols_fp32" : "hahn_inv_cols",
                             fp32 ? "hahn_inv_rows_fp32" : "hahn_inv_rows", asy_f, asy_b, job_parallel)) != CJT_OK)
                return s;
        mark(Kind::Join);
        add_rec_inv_reduce(pr, 0, red_b);
    }
    // every launch that keeps intermediates must find them: a missing buffer
    // is an error here rather than a null pointer on the device
    for (const Launch& L : pr.launches) {
        switch (L.kind) {
        case Kind::FftPass1: case Kind::FftPass1Terms: case Kind::FftPass2: case Kind::JobRowReduce: case Kind::BsCol1: case Kind::BsRowConv:
        case Kind::BsCol2Inv: case Kind::BsUntangle: case Kind::FftJobs: case Kind::BsJobs: case Kind::JobReduce:
            for (int64_t q = 0; q < L.nitems; ++q)
                if (b.offs[pr.items[L.item_off + q].desc].tmp == SIZE_MAX)
                    return fail(CJT_EINVAL, "internal: FFT intermediates missing for a two-pass or job-parallel launch");
            break;
        case Kind::RecFwdSeg: case Kind::RecFwdCombine: case Kind::RecInvMaps: case Kind::RecInvInit:
            for (int64_t q = 0; q < L.nitems; ++q)
                if (b.offs[pr.items[L.item_off + q].desc].seg == SIZE_MAX)
                    return fail(CJT_EINVAL, "internal: segment records missing for a split recurrence");
            break;
        default: break;
        }
    }
    return CJT_OK;
}

void bind_workspace(Built& b, void* base)
{
    char* c = (char*)base;
    for (size_t i = 0; i < b.pr.descs.size(); ++i) {
        ExecDesc& d = b.pr.descs[i];
        const DescOffsets& o = b.offs[i];
        d.p = (double*)(c + o.p);
        d.p2 = o.p2 != SIZE_MAX ? (double*)(c + o.p2) : nullptr;
        d.part = o.part != SIZE_MAX ? (double*)(c + o.part) : nullptr;
        d.tmp = o.tmp != SIZE_MAX ? (void*)(c + o.tmp) : nullptr;
        d.seg = o.seg != SIZE_MAX ? (double*)(c + o.seg) : nullptr;
    }
}

cjt_status run_program(const Program& pr, const ExecDesc* d_desc, const Item* d_items, hipStream_t st,
                       hipStream_t aux, hipEvent_t fork, hipEvent_t join, const double* in_base, double* out_base)
{
    cjt_status s = CJT_OK;
    for (const Launch& L : pr.launches) {
        hipStream_t ls = L.stream ? aux : st;
        const Item* it = d_items + L.item_off;
        switch (L.kind) {
        case Kind::Fork:
            CJT_HIP_TRY(hipEventRecord(fork, st));
            CJT_HIP_TRY(hipStreamWaitEvent(aux, fork, 0));
            break;
        case Kind::Join:
            CJT_HIP_TRY(hipEventRecord(join, aux));
            CJT_HIP_TRY(hipStreamWaitEvent(st, join, 0));
            break;
        case Kind::Patch:
            hipLaunchKernelGGL(k_patch, dim3((unsigned)((L.nitems + 63) / 64)), dim3(64), 0, ls,
                               const_cast<ExecDesc*>(d_desc), (int)L.nitems, in_base, out_base);
            CJT_HIP_TRY(hipGetLastError());
            break;
        case Kind::FftSingle:
        case Kind::FftPass1:
        case Kind::FftPass1Terms:
        case Kind::FftPass2:
        case Kind::JobRowReduce:
        case Kind::BsSingle:
        case Kind::BsCol1:
        case Kind::BsRowConv:
        case Kind::BsCol2Inv:
        case Kind::BsUntangle:
        case Kind::FftJobs:
        case Kind::BsJobs:
        case Kind::JobReduce:
            if ((s = launch_fft(L, d_desc, it, ls)) != CJT_OK) return s;
            break;
        default:
            if ((s = launch_rec(L, d_desc, it, ls)) != CJT_OK) return s;
            break;
        }
    }
    return CJT_OK;
}

}  // namespace cjt
