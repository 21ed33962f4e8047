// Transform server: a stream of independent requests (any degree, direction
// and parameters) served by continuous batching over the batched transform,
// with plans kept resident inside a fixed device budget.  The paper's
// plan/execute split (Sec. 4) is what makes this pay: a plan is made once per
// (N, alpha, beta, precision) and reused by every request with that key.
//
// Threads: the caller's (submit / wait / query), a batcher that forms and
// launches calls, and a completer that waits for each call's event and
// stamps the latency of its requests.  Device memory: one allocation of the
// whole budget, split into the execution workspace, one descriptor buffer per
// call in flight, and a first-fit heap for plan arenas and plan-build scratch.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cjt_internal.h"
#include "exec.h"
#include "plan.h"

namespace cjt {
namespace {

using Clock = std::chrono::steady_clock;

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over byte offsets [0, size); blocks 256-byte aligned,
// neighbours merged on release.
class Heap {
  public:
    void init(size_t bytes)
    {
        free_.clear();
        used_ = 0;
        if (bytes) free_[0] = bytes;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = a256(std::max<size_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, o = it->first + bytes;
            free_.erase(it);
            if (rest) free_[o] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = a256(std::max<size_t>(bytes, 1));
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }

  private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

struct Key {
    int64_t N;
    uint64_t a, b;
    unsigned prec;
    bool operator==(const Key& o) const { return N == o.N && a == o.a && b == o.b && prec == o.prec; }
};

struct KeyHash {
    size_t operator()(const Key& k) const
    {
        uint64_t h = (uint64_t)k.N * 0x9E3779B97F4A7C15ull;
        h ^= k.a + 0x7F4A7C159E3779B9ull + (h << 6) + (h >> 2);
        h ^= k.b + 0x94D049BB133111EBull + (h << 6) + (h >> 2);
        h ^= (uint64_t)k.prec + (h << 6) + (h >> 2);
        return (size_t)h;
    }
};

uint64_t bits_of(double x)
{
    uint64_t u;
    memcpy(&u, &x, sizeof(u));
    return u;
}

// A resident plan.  refs counts the requests of calls being formed or in
// flight that use it; only the batcher raises it, the completer lowers it
// after the call's event completed, so refs == 0 means the arena is idle.
struct Entry {
    Key key{};
    Plan P;
    size_t off = 0;
    std::atomic<int> refs{0};
    std::list<Entry*>::iterator lru;
};

struct Request {
    int64_t ticket;
    unsigned flags;  // direction | precision
    int64_t N;
    double alpha, beta;
    const double* in;
    double* out;
    Clock::time_point arrival;
    Entry* plan;
    bool made_plan;  // its plan was made for it (a cache miss)
};

struct Result {
    bool done = false;
    cjt_status status = CJT_OK;
    double latency_us = 0.0;
};

struct Call {
    int slot = 0;
    cjt_status status = CJT_OK;  // launch status
    std::vector<Request> reqs;
};

constexpr unsigned kDirs = CJT_DIR_FWD | CJT_DIR_INV;

}  // namespace
}  // namespace cjt

using namespace cjt;

struct cjt_server_s {
    int dev = 0;
    cjt_server_config cfg{};
    char* pool = nullptr;  // the whole budget
    size_t ws_bytes = 0;   // [0, ws_bytes): execution workspace
    size_t meta_off = 0, meta_cap = 0;  // descriptor buffer of slot i at meta_off + i * meta_cap
    size_t heap_off = 0;   // plan heap from here to the end
    std::vector<char*> h_meta;          // pinned staging, one per slot
    std::vector<hipEvent_t> done_ev;    // completion event, one per slot
    hipStream_t st = nullptr, aux = nullptr, pst = nullptr;  // calls, recurrences, plan builds
    hipEvent_t fork = nullptr, join = nullptr;

    // batcher thread only
    Heap heap;
    std::unordered_map<Key, std::unique_ptr<Entry>, KeyHash> plans;
    std::list<Entry*> lru;  // front: most recently used

    // shared, under mu
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request> queue;
    std::unordered_map<int64_t, Result> results;
    std::list<Call> calls;  // in flight, launch order
    std::vector<int> free_slots;
    int64_t next_ticket = 0;
    int64_t pending = 0;      // submitted, not completed / failed / cancelled
    int64_t completions = 0;  // calls completed
    bool paused = false, stop = false, batcher_done = false;
    // statistics (under mu)
    int64_t submitted = 0, completed = 0, failed = 0, cancelled = 0, batches = 0, batched_reqs = 0;
    int64_t hits = 0, misses = 0, evictions = 0, stalls = 0, resident = 0;
    size_t plan_bytes = 0, peak = 0;
    std::vector<double> lat;

    std::thread batcher, completer;
};

namespace {

size_t fixed_bytes(const cjt_server_s* S) { return S->heap_off; }

void note_usage(cjt_server_s* S)
{
    std::lock_guard<std::mutex> lk(S->mu);
    S->peak = std::max(S->peak, fixed_bytes(S) + S->heap.used());
}

void evict(cjt_server_s* S, Entry* e)
{
    S->heap.release(e->off, e->P.arena_bytes);
    S->lru.erase(e->lru);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->plan_bytes -= a256(e->P.arena_bytes);
        S->resident -= 1;
        S->evictions += 1;
    }
    const Key k = e->key;  // e is destroyed by the erase
    S->plans.erase(k);
}

// Heap allocation, evicting idle plans (least recently used first) until it fits.
bool alloc_evicting(cjt_server_s* S, size_t bytes, size_t* off)
{
    while (!S->heap.alloc(bytes, off)) {
        Entry* victim = nullptr;
        for (auto it = S->lru.rbegin(); it != S->lru.rend(); ++it)
            if ((*it)->refs.load() == 0) {
                victim = *it;
                break;
            }
        if (!victim) return false;
        evict(S, victim);
    }
    note_usage(S);
    return true;
}

// Resident plan for r, made if absent (*made set).  CJT_EBUSY: it does not
// fit now because every other plan in the heap is in use.
cjt_status get_plan(cjt_server_s* S, const Request& r, Entry** out, bool* made)
{
    *made = false;
    const unsigned prec = r.flags & CJT_FP32_BULK;
    const Key k{r.N, bits_of(r.alpha), bits_of(r.beta), prec};
    auto it = S->plans.find(k);
    if (it != S->plans.end()) {
        Entry* e = it->second.get();
        S->lru.splice(S->lru.begin(), S->lru, e->lru);
        *out = e;
        return CJT_OK;
    }
    std::unique_ptr<Entry> E(new (std::nothrow) Entry);
    if (!E) return fail(CJT_ENOMEM, "host allocation failed");
    E->key = k;
    plan_host(&E->P, r.N, r.alpha, r.beta, S->cfg.M, prec | CJT_BATCH_INVARIANT);
    E->P.device = S->dev;
    size_t ao = 0, so = 0;
    if (!alloc_evicting(S, E->P.arena_bytes, &ao)) return CJT_EBUSY;
    if (!alloc_evicting(S, std::max<size_t>(E->P.scratch_bytes, 256), &so)) {
        S->heap.release(ao, E->P.arena_bytes);
        return CJT_EBUSY;
    }
    cjt_status s = build_plan_device(&E->P, S->pst, S->pool + S->heap_off + ao, S->pool + S->heap_off + so);
    S->heap.release(so, std::max<size_t>(E->P.scratch_bytes, 256));
    if (s != CJT_OK) {
        S->heap.release(ao, E->P.arena_bytes);
        return s;
    }
    E->off = ao;
    Entry* e = E.get();
    S->lru.push_front(e);
    e->lru = S->lru.begin();
    S->plans.emplace(k, std::move(E));
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->resident += 1;
        S->plan_bytes += a256(e->P.arena_bytes);
    }
    *out = e;
    *made = true;
    return CJT_OK;
}

// Uploads the program's descriptors and items through the slot's staging
// buffer and launches it on the server stream, then records the slot event.
cjt_status launch_call(cjt_server_s* S, Built& b, const std::vector<Request>& reqs, int slot)
{
    bind_workspace(b, S->pool);
    for (size_t i = 0; i < reqs.size(); ++i) {
        b.pr.descs[i].in = reqs[i].in;
        b.pr.descs[i].out = reqs[i].out;
    }
    const size_t dbytes = a256(sizeof(ExecDesc) * b.pr.descs.size());
    const size_t ibytes = sizeof(Item) * b.pr.items.size();
    char* h = S->h_meta[slot];
    char* d = S->pool + S->meta_off + (size_t)slot * S->meta_cap;
    memcpy(h, b.pr.descs.data(), sizeof(ExecDesc) * b.pr.descs.size());
    if (ibytes) memcpy(h + dbytes, b.pr.items.data(), ibytes);
    CJT_HIP_TRY(hipMemcpyAsync(d, h, dbytes + ibytes, hipMemcpyHostToDevice, S->st));
    cjt_status s = run_program(b.pr, (const ExecDesc*)d, (const Item*)(d + dbytes), S->st, S->aux, S->fork, S->join,
                               nullptr, nullptr);
    if (hipEventRecord(S->done_ev[slot], S->st) != hipSuccess && s == CJT_OK)
        s = fail(CJT_EDEVICE, "event record failed");
    return s;
}

// Turns the candidate requests (one direction and precision, queue order)
// into one call.  Requests that must wait for memory go to `back` (in order),
// requests that cannot run at all to `failed`.
void form_call(cjt_server_s* S, std::vector<Request>& cand, bool others_in_flight, Call* call,
               std::vector<Request>* back, std::vector<std::pair<Request, cjt_status>>* failed)
{
    std::vector<Request> take;
    for (size_t k = 0; k < cand.size(); ++k) {
        Request& r = cand[k];
        Entry* e = nullptr;
        bool made = false;
        cjt_status s = get_plan(S, r, &e, &made);
        if (made) r.made_plan = true;
        if (s == CJT_EBUSY) {
            if (others_in_flight || !take.empty()) {
                back->assign(cand.begin() + (ptrdiff_t)k, cand.end());
                break;
            }
            s = fail(CJT_ENOMEM, "plan does not fit in the server budget");
        }
        if (s != CJT_OK) {
            failed->push_back({r, s});
            continue;
        }
        e->refs.fetch_add(1);
        r.plan = e;
        take.push_back(r);
    }
    const bool inverse = (cand.front().flags & CJT_DIR_INV) != 0;
    while (!take.empty()) {
        std::vector<const Plan*> pl;
        for (const Request& r : take) pl.push_back(&r.plan->P);
        std::vector<int64_t> zero(take.size(), 0);
        Built b;
        cjt_status s = build_program(pl, zero, inverse, S->ws_bytes / 2, false, S->st, &b);
        const size_t meta = a256(sizeof(ExecDesc) * b.pr.descs.size()) + sizeof(Item) * b.pr.items.size();
        if (s == CJT_OK && b.ws_bytes <= S->ws_bytes && meta <= S->meta_cap) {
            call->status = launch_call(S, b, take, call->slot);
            call->reqs = std::move(take);
            return;
        }
        if (s == CJT_OK && take.size() > 1) {
            // too large for the workspace or descriptor buffer: run a leading
            // part that fits by the measured ratio, the rest goes back
            const double over = std::max((double)b.ws_bytes / (double)S->ws_bytes, (double)meta / (double)S->meta_cap);
            size_t h = (size_t)(0.9 * (double)take.size() / over);
            h = std::min(std::max<size_t>(h, 1), take.size() - 1);
            std::vector<Request> rest(take.begin() + (ptrdiff_t)h, take.end());
            for (Request& r : rest) r.plan->refs.fetch_sub(1);
            back->insert(back->begin(), rest.begin(), rest.end());
            take.resize(h);
            continue;
        }
        if (s == CJT_OK) s = fail(CJT_ENOMEM, "request does not fit in the server workspace");
        for (Request& r : take) {
            r.plan->refs.fetch_sub(1);
            failed->push_back({r, s});
        }
        take.clear();
    }
}

void finish(cjt_server_s* S, const Request& r, cjt_status s, Clock::time_point t)
{
    Result& R = S->results[r.ticket];
    R.done = true;
    R.status = s;
    R.latency_us = std::chrono::duration<double, std::micro>(t - r.arrival).count();
    if (s == CJT_OK) {
        S->completed += 1;
        S->lat.push_back(R.latency_us);
    } else if (s == CJT_ECANCELED) {
        S->cancelled += 1;
    } else {
        S->failed += 1;
    }
    S->pending -= 1;
}

void batcher_main(cjt_server_s* S)
{
    (void)hipSetDevice(S->dev);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv.wait(lk, [&] {
            return (S->stop && S->queue.empty()) || (!S->paused && !S->queue.empty() && !S->free_slots.empty());
        });
        if (S->queue.empty()) break;
        const unsigned grp = S->queue.front().flags;
        std::vector<Request> cand;
        for (auto it = S->queue.begin(); it != S->queue.end() && (int)cand.size() < S->cfg.max_batch;) {
            if (it->flags == grp) {
                cand.push_back(*it);
                it = S->queue.erase(it);
            } else {
                ++it;
            }
        }
        Call call;
        call.slot = S->free_slots.back();
        S->free_slots.pop_back();
        const bool others = !S->calls.empty();
        const int64_t c0 = S->completions;
        lk.unlock();
        std::vector<Request> back;
        std::vector<std::pair<Request, cjt_status>> failed;
        form_call(S, cand, others, &call, &back, &failed);
        lk.lock();
        const Clock::time_point now = Clock::now();
        for (auto& f : failed) finish(S, f.first, f.second, now);
        S->queue.insert(S->queue.begin(), back.begin(), back.end());
        if (!call.reqs.empty()) {
            S->batches += 1;
            S->batched_reqs += (int64_t)call.reqs.size();
            for (const Request& r : call.reqs) (r.made_plan ? S->misses : S->hits) += 1;
            S->calls.push_back(std::move(call));
        } else {
            S->free_slots.push_back(call.slot);
        }
        S->cv.notify_all();
        if (call.reqs.empty() && !back.empty() && others) {  // admission stall: wait for memory held by running calls
            S->stalls += 1;
            S->cv.wait(lk, [&] { return S->completions != c0; });
        }
    }
    S->batcher_done = true;
    S->cv.notify_all();
}

void completer_main(cjt_server_s* S)
{
    (void)hipSetDevice(S->dev);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv.wait(lk, [&] { return !S->calls.empty() || S->batcher_done; });
        if (S->calls.empty()) break;
        const int slot = S->calls.front().slot;
        lk.unlock();
        const hipError_t e = hipEventSynchronize(S->done_ev[slot]);
        const Clock::time_point t = Clock::now();
        lk.lock();
        Call c = std::move(S->calls.front());
        S->calls.pop_front();
        const cjt_status st = c.status != CJT_OK ? c.status : (e == hipSuccess ? CJT_OK : CJT_EDEVICE);
        for (const Request& r : c.reqs) {
            finish(S, r, st, t);
            r.plan->refs.fetch_sub(1);
        }
        S->free_slots.push_back(slot);
        S->completions += 1;
        S->cv.notify_all();
    }
}

cjt_status submit_at(cjt_server_s* S, unsigned flags, int64_t N, double alpha, double beta, const double* d_in,
                     double* d_out, Clock::time_point arrival, int64_t* ticket)
{
    const unsigned dir = flags & kDirs;
    if ((dir != CJT_DIR_FWD && dir != CJT_DIR_INV) || (flags & ~(kDirs | CJT_FP32_BULK)))
        return fail(CJT_EINVAL, "flags must be CJT_DIR_FWD or CJT_DIR_INV, optionally with CJT_FP32_BULK");
    cjt_status s = check_args(N, alpha, beta, S->cfg.M, flags & CJT_FP32_BULK);
    if (s != CJT_OK) return s;
    if (!d_in || !d_out) return fail(CJT_EINVAL, "null buffer");
    if ((const void*)d_in == (const void*)d_out) return fail(CJT_EINVAL, "in-place transforms are not supported");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(CJT_EBUSY, "server is shutting down");
    const int64_t t = S->next_ticket++;
    S->queue.push_back(Request{t, flags, N, alpha, beta, d_in, d_out, arrival, nullptr, false});
    S->results.emplace(t, Result{});
    S->pending += 1;
    S->submitted += 1;
    S->cv.notify_all();
    *ticket = t;
    return CJT_OK;
}

void release(cjt_server_s* S)
{
    if (S->st) (void)hipStreamSynchronize(S->st);
    if (S->aux) (void)hipStreamSynchronize(S->aux);
    if (S->pst) (void)hipStreamSynchronize(S->pst);
    S->plans.clear();
    S->lru.clear();
    for (hipEvent_t e : S->done_ev)
        if (e) (void)hipEventDestroy(e);
    for (char* h : S->h_meta)
        if (h) (void)hipHostFree(h);
    if (S->fork) (void)hipEventDestroy(S->fork);
    if (S->join) (void)hipEventDestroy(S->join);
    if (S->st) (void)hipStreamDestroy(S->st);
    if (S->aux) (void)hipStreamDestroy(S->aux);
    if (S->pst) (void)hipStreamDestroy(S->pst);
    if (S->pool) (void)hipFree(S->pool);
    delete S;
}

}  // namespace

extern "C" {

cjt_status cjt_server_create(cjt_server_t* out, const cjt_server_config* cfg)
{
    if (!out || !cfg) return fail(CJT_EINVAL, "null argument");
    *out = nullptr;
    cjt_server_config c = *cfg;
    if (c.max_batch == 0) c.max_batch = 256;
    if (c.max_inflight == 0) c.max_inflight = 2;
    if (c.max_batch < 1 || c.max_inflight < 1 || c.max_inflight > 16)
        return fail(CJT_EINVAL, "max_batch >= 1 and 1 <= max_inflight <= 16");
    if (c.M != 0 && (c.M < 2 || c.M > kMaxM)) return fail(CJT_EDOMAIN, "M must be 0 (auto) or in [2, 30]");
    if (c.workspace_bytes == 0) c.workspace_bytes = c.hbm_budget / 4;
    const size_t ws = a256(c.workspace_bytes);
    const size_t meta_cap = a256(std::max<size_t>((size_t)16 << 20, (size_t)c.max_batch * (256u << 10)));
    const size_t fixed = ws + meta_cap * (size_t)c.max_inflight;
    if (c.hbm_budget < fixed + ((size_t)1 << 20))
        return fail(CJT_EINVAL, "budget too small for the workspace and descriptor buffers");
    cjt_server_s* S = new (std::nothrow) cjt_server_s;
    if (!S) return fail(CJT_ENOMEM, "host allocation failed");
    S->cfg = c;
    S->paused = c.start_paused != 0;
    S->ws_bytes = ws;
    S->meta_off = ws;
    S->meta_cap = meta_cap;
    S->heap_off = fixed;
    S->peak = fixed;
    S->heap.init(c.hbm_budget - fixed);
    cjt_status s = CJT_OK;
    do {
        if (hipGetDevice(&S->dev) != hipSuccess) {
            s = fail(CJT_EDEVICE, "no HIP device");
            break;
        }
        if (hipMalloc((void**)&S->pool, c.hbm_budget) != hipSuccess) {
            S->pool = nullptr;
            s = fail(CJT_ENOMEM, "budget allocation failed");
            break;
        }
        if (hipStreamCreateWithFlags(&S->st, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&S->aux, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&S->pst, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&S->fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&S->join, hipEventDisableTiming) != hipSuccess) {
            s = fail(CJT_EDEVICE, "stream or event creation failed");
            break;
        }
        S->h_meta.assign((size_t)c.max_inflight, nullptr);
        S->done_ev.assign((size_t)c.max_inflight, nullptr);
        for (int i = 0; i < c.max_inflight && s == CJT_OK; ++i) {
            if (hipHostMalloc((void**)&S->h_meta[i], meta_cap, hipHostMallocDefault) != hipSuccess)
                s = fail(CJT_ENOMEM, "pinned staging allocation failed");
            else if (hipEventCreateWithFlags(&S->done_ev[i], hipEventDisableTiming) != hipSuccess)
                s = fail(CJT_EDEVICE, "event creation failed");
            S->free_slots.push_back(c.max_inflight - 1 - i);
        }
    } while (0);
    if (s != CJT_OK) {
        release(S);
        return s;
    }
    S->batcher = std::thread(batcher_main, S);
    S->completer = std::thread(completer_main, S);
    *out = S;
    return CJT_OK;
}

cjt_status cjt_server_submit(cjt_server_t s, unsigned flags, int64_t N, double alpha, double beta,
                             const double* d_in, double* d_out, int64_t* ticket)
{
    if (!s || !ticket) return fail(CJT_EINVAL, "null argument");
    *ticket = -1;
    return submit_at(s, flags, N, alpha, beta, d_in, d_out, Clock::now(), ticket);
}

cjt_status cjt_server_replay(cjt_server_t s, int64_t count, const unsigned* flags, const int64_t* N,
                             const double* alpha, const double* beta, const double* const* d_in,
                             double* const* d_out, const double* arrival_us, int64_t* tickets)
{
    if (!s || count < 0 || (count > 0 && (!flags || !N || !alpha || !beta || !d_in || !d_out || !arrival_us ||
                                          !tickets)))
        return fail(CJT_EINVAL, "null argument");
    for (int64_t i = 1; i < count; ++i)
        if (!(arrival_us[i] >= arrival_us[i - 1])) return fail(CJT_EINVAL, "arrival times must not decrease");
    const Clock::time_point t0 = Clock::now();
    for (int64_t i = 0; i < count; ++i) {
        const Clock::time_point at =
            t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double, std::micro>(arrival_us[i]));
        while (Clock::now() < at) {
            if (at - Clock::now() > std::chrono::microseconds(200)) std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
        tickets[i] = -1;
        if (submit_at(s, flags[i], N[i], alpha[i], beta[i], d_in[i], d_out[i], at, &tickets[i]) != CJT_OK) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->submitted += 1;
            s->failed += 1;
        }
    }
    return CJT_OK;
}

cjt_status cjt_server_wait(cjt_server_t s, int64_t ticket, cjt_status* result, double* latency_us)
{
    if (!s) return fail(CJT_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->results.find(ticket);
    if (it == s->results.end()) return fail(CJT_EINVAL, "unknown ticket");
    s->cv.wait(lk, [&] { return s->results[ticket].done; });
    const Result R = s->results[ticket];
    s->results.erase(ticket);
    if (result) *result = R.status;
    if (latency_us) *latency_us = R.latency_us;
    return CJT_OK;
}

cjt_status cjt_server_cancel(cjt_server_t s, int64_t ticket)
{
    if (!s) return fail(CJT_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it)
        if (it->ticket == ticket) {
            const Request r = *it;
            s->queue.erase(it);
            finish(s, r, CJT_ECANCELED, Clock::now());
            s->cv.notify_all();
            return CJT_OK;
        }
    if (s->results.count(ticket)) return fail(CJT_EBUSY, "request already taken into a call");
    return fail(CJT_EINVAL, "unknown ticket");
}

cjt_status cjt_server_pause(cjt_server_t s, int paused)
{
    if (!s) return fail(CJT_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    s->paused = paused != 0;
    s->cv.notify_all();
    return CJT_OK;
}

cjt_status cjt_server_drain(cjt_server_t s)
{
    if (!s) return fail(CJT_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [&] { return s->pending == 0 || (s->paused && !s->queue.empty()); });
    if (s->pending != 0) return fail(CJT_EBUSY, "server is paused with requests queued");
    return CJT_OK;
}

cjt_status cjt_server_query(cjt_server_t s, cjt_server_stats* out, int reset)
{
    if (!s || !out) return fail(CJT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->failed = s->failed;
    out->cancelled = s->cancelled;
    out->batches = s->batches;
    out->mean_batch = s->batches ? (double)s->batched_reqs / (double)s->batches : 0.0;
    out->plan_hits = s->hits;
    out->plan_misses = s->misses;
    out->plan_evictions = s->evictions;
    out->admission_stalls = s->stalls;
    out->plans_resident = s->resident;
    out->plan_bytes = s->plan_bytes;
    out->budget_bytes = s->cfg.hbm_budget;
    out->peak_used_bytes = s->peak;
    out->lat_count = (int64_t)s->lat.size();
    if (!s->lat.empty()) {
        std::vector<double> v = s->lat;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            const size_t i = (size_t)std::min<double>((double)v.size() - 1, floor(q * (double)(v.size() - 1) + 0.5));
            return v[i];
        };
        out->lat_p50_us = pct(0.50);
        out->lat_p99_us = pct(0.99);
        double sum = 0.0;
        for (double x : v) sum += x;
        out->lat_mean_us = sum / (double)v.size();
        out->lat_max_us = v.back();
    }
    if (reset) {
        s->lat.clear();
        s->submitted = s->completed = s->failed = s->cancelled = 0;
        s->batches = s->batched_reqs = 0;
        s->hits = s->misses = s->evictions = s->stalls = 0;
        s->peak = fixed_bytes(s) + s->plan_bytes;
    }
    return CJT_OK;
}

cjt_status cjt_server_destroy(cjt_server_t s)
{
    if (!s) return CJT_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->paused = false;
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->batcher.joinable()) s->batcher.join();
    if (s->completer.joinable()) s->completer.join();
    release(s);
    return CJT_OK;
}

}  // extern "C"
