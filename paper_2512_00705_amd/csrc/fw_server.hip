// Walk server: continuous batching of walk requests against a resident graph.
//
// A server thread runs ticks.  A tick is one batched launch per (logic kind, weighting)
// over the walkers of every admitted request; each walker advances at most `tick_steps`
// steps and is then suspended (its progress kept in a per-walker counter, its current and
// previous vertex in its own path row).  Between ticks the thread retires finished
// requests (results copied to host memory, device block freed) and admits waiting ones in
// arrival order while their device block fits the HBM budget.  A request that arrives
// while others run therefore joins at the next tick and shares every later launch with
// them.  The results of the requests that finished in a tick are copied out while the
// next tick runs (a copy stream beside the launch stream; the finished requests' blocks
// are no longer touched by later launches and are freed once copied).  Walker i of a
// request draws from the request's seed with Philox counter
// (i, step, draw, tag), so its result is the same alone, in any mix and for any tick
// length.
#include <stdarg.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fw_host.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kAlign = 256;

size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit suballocator over one device allocation of `cap` bytes (offsets only).
class Arena {
  public:
    void reset(size_t cap)
    {
        free_.clear();
        if (cap) free_[0] = cap;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = round_up(bytes);
        if (bytes == 0) {  // empty request: no block
            *off = 0;
            return true;
        }
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = round_up(bytes);
        if (bytes == 0) return;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

  private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0, peak_ = 0;
};

struct Request {
    uint64_t id = 0;
    fw_logic logic{};
    int64_t n = 0;
    int32_t L = 0;
    uint64_t seed = 0;
    std::vector<int32_t> starts;  // host copy until admitted
    size_t off = 0, bytes = 0;    // device block: starts | lengths | prog | paths
    size_t o_starts = 0, o_len = 0, o_prog = 0, o_paths = 0;
    int32_t slot = -1;
    Clock::time_point t_submit, t_done;
    std::vector<int32_t> paths, lengths;
    int state = 0;  // 0 waiting, 1 admitted, 2 finished
};

size_t request_bytes(int64_t n, int32_t L)
{
    const size_t v = round_up(sizeof(int32_t) * (size_t)n);
    return 3 * v + round_up(sizeof(int32_t) * (size_t)n * ((size_t)L + 1));
}

}  // namespace

// one batched launch per (logic kind, weighting)
constexpr int kGroups = 2 * fw::kNumKinds;

struct fw_server {
    fw_graph *g = nullptr;
    fw_plan plan{};
    int32_t strategy = FW_AUTO;
    int32_t tick_steps = 16;
    int32_t max_pending = 0;
    int32_t max_active = 0;
    size_t budget = 0;
    char *arena_base = nullptr;
    Arena arena;
    hipStream_t stream = nullptr;              // launches, uploads, the done counters
    hipStream_t cstream = nullptr;             // result copies, beside the next tick
    hipEvent_t ev_tick = nullptr;              // a tick's launches and done-counter copy are complete
    int32_t *d_done = nullptr;                 // finished walkers per slot
    fw::QueryDev *d_table = nullptr;           // kGroups groups x max_active entries
    fw::QueryDev *h_table = nullptr;           // pinned staging of the same
    unsigned long long *d_queue = nullptr;     // one walker counter per group
    unsigned long long *d_stats = nullptr;     // FW_NSTATS counters
    int32_t *h_done = nullptr;                 // pinned copy of d_done after each tick
    std::vector<int32_t> free_slots;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> waiting;
    std::vector<Request *> active;             // touched by the server thread only
    std::vector<Request *> done_tick;          // finished in the last tick, results not yet copied (server thread)
    std::deque<uint64_t> finished;
    std::unordered_map<uint64_t, Request *> reqs;
    uint64_t next_id = 1;
    bool stop = false;
    int err = FW_OK;
    std::string err_msg;
    uint64_t ticks = 0, n_admitted = 0, n_finished = 0;
    std::thread th;
};

namespace {

int server_fail(fw_server *s, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    std::lock_guard<std::mutex> lk(s->mu);
    s->err = code;
    s->err_msg = buf;
    s->cv_done.notify_all();
    return code;
}

#define SRV_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return server_fail(s, FW_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Take waiting requests in arrival order while their blocks fit the budget and a slot
// is free.  Caller holds mu; no HIP call here.
void pick(fw_server *s, std::vector<Request *> &out)
{
    while (!s->waiting.empty() && !s->free_slots.empty()) {
        Request *r = s->waiting.front();
        size_t off = 0;
        if (!s->arena.alloc(r->bytes, &off)) break;
        s->waiting.pop_front();
        r->off = off;
        r->slot = s->free_slots.back();
        s->free_slots.pop_back();
        const size_t v = round_up(sizeof(int32_t) * (size_t)r->n);
        r->o_starts = off;
        r->o_len = off + v;
        r->o_prog = off + 2 * v;
        r->o_paths = off + 3 * v;
        out.push_back(r);
    }
}

// Upload the picked requests' starts, clear their progress and done counters.
int admit(fw_server *s, std::vector<Request *> &picked)
{
    for (Request *r : picked) {
        if (r->n > 0)
            SRV_TRY(hipMemcpyAsync(s->arena_base + r->o_starts, r->starts.data(), sizeof(int32_t) * (size_t)r->n,
                                   hipMemcpyHostToDevice, s->stream));
        SRV_TRY(fw::launch_fill_i32((int32_t *)(s->arena_base + r->o_prog), r->n, 0, s->stream));
        SRV_TRY(fw::launch_fill_i32(s->d_done + r->slot, 1, 0, s->stream));
        r->state = 1;
        s->active.push_back(r);
    }
    if (!picked.empty()) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->n_admitted += picked.size();
    }
    return FW_OK;
}

// One tick: a batched launch per group of admitted requests, then the done counters' copy
// and an event (nothing waits here; tick_wait does).
int tick(fw_server *s)
{
    for (int grp = 0; grp < kGroups; ++grp) {
        const int kind = 1 + grp / 2;  // FW_NODE2VEC, FW_METAPATH, FW_SECOND_PR
        const bool weighted_logic = (grp & 1) != 0;
        fw::QueryDev *tab = s->h_table + (size_t)grp * s->max_active;
        int32_t nq = 0;
        int64_t total = 0;
        const fw_logic *lg0 = nullptr;
        for (Request *r : s->active) {
            if (r->logic.kind != kind || (r->logic.weighted != 0) != weighted_logic) continue;
            fw::QueryDev &d = tab[nq++];
            fw::host::fill_query(&r->logic, d);
            d.first = total;
            d.n = r->n;
            d.starts = (const int32_t *)(s->arena_base + r->o_starts);
            d.paths = (int32_t *)(s->arena_base + r->o_paths);
            d.lengths = (int32_t *)(s->arena_base + r->o_len);
            d.prog = (int32_t *)(s->arena_base + r->o_prog);
            d.done = s->d_done + r->slot;
            d.L = r->L;
            d.key0 = (uint32_t)r->seed;
            d.key1 = (uint32_t)(r->seed >> 32);
            total += r->n;
            lg0 = &r->logic;
        }
        if (total == 0) continue;
        fw::QueryDev *dtab = s->d_table + (size_t)grp * s->max_active;
        SRV_TRY(hipMemcpyAsync(dtab, tab, sizeof(fw::QueryDev) * (size_t)nq, hipMemcpyHostToDevice, s->stream));
        fw::WalkArgs a;
        fw::host::fill_args(s->g, lg0, a);
        fw::host::plan_args(&s->plan, s->strategy, a);
        a.n = total;
        a.queue = s->d_queue + grp;
        a.err = (int *)(s->g->scratch + 1);
        a.stats = s->d_stats;
        a.queries = dtab;
        a.nq = nq;
        a.tick_steps = s->tick_steps;
        const bool weighted = weighted_logic && s->g->h;
        const int grid = s->plan.grid > 0 ? s->plan.grid : fw::walk_grid(kind, weighted, true, a.lds_cap, total);
        SRV_TRY(fw::launch_zero(s->d_queue + grp, 1, s->stream));
        SRV_TRY(fw::launch_walk(a, kind, weighted, true, grid, s->stream));
    }
    SRV_TRY(hipMemcpyAsync(s->h_done, s->d_done, sizeof(int32_t) * (size_t)s->max_active, hipMemcpyDeviceToHost,
                           s->stream));
    SRV_TRY(hipEventRecord(s->ev_tick, s->stream));
    return FW_OK;
}

// Wait for the tick, then move the requests whose walkers all finished from `active` to
// `done_tick` (their results are copied out by retire, beside the next tick).
int tick_wait(fw_server *s)
{
    SRV_TRY(hipEventSynchronize(s->ev_tick));
    s->ticks++;
    std::vector<Request *> still;
    for (Request *r : s->active) {
        if (s->h_done[(size_t)r->slot] < r->n) still.push_back(r);
        else s->done_tick.push_back(r);
    }
    s->active.swap(still);
    return FW_OK;
}

// Copy out and release the requests of `done_tick`.
int retire(fw_server *s)
{
    if (s->done_tick.empty()) return FW_OK;
    for (Request *r : s->done_tick) {
        r->paths.resize((size_t)r->n * ((size_t)r->L + 1));
        r->lengths.resize((size_t)r->n);
        if (r->n > 0) {
            SRV_TRY(hipMemcpyAsync(r->paths.data(), s->arena_base + r->o_paths, sizeof(int32_t) * r->paths.size(),
                                   hipMemcpyDeviceToHost, s->cstream));
            SRV_TRY(hipMemcpyAsync(r->lengths.data(), s->arena_base + r->o_len, sizeof(int32_t) * r->lengths.size(),
                                   hipMemcpyDeviceToHost, s->cstream));
        }
    }
    SRV_TRY(hipStreamSynchronize(s->cstream));
    std::lock_guard<std::mutex> lk(s->mu);
    const auto now = Clock::now();
    for (Request *r : s->done_tick) {
        s->arena.release(r->off, r->bytes);
        s->free_slots.push_back(r->slot);
        r->slot = -1;
        r->state = 2;
        r->t_done = now;
        std::vector<int32_t>().swap(r->starts);
        s->finished.push_back(r->id);
        s->n_finished++;
    }
    s->done_tick.clear();
    s->cv_done.notify_all();
    return FW_OK;
}

void serve(fw_server *s)
{
    if (hipSetDevice(s->g->device) != hipSuccess) {
        server_fail(s, FW_E_DEVICE, "server thread: hipSetDevice failed");
        return;
    }
    for (;;) {
        std::vector<Request *> picked;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->stop || s->err != FW_OK) break;
            pick(s, picked);
            if (s->active.empty() && picked.empty() && s->done_tick.empty()) {
                s->cv_work.wait(lk, [s] { return s->stop || !s->waiting.empty(); });
                continue;
            }
        }
        if (admit(s, picked) != FW_OK) break;
        const bool launched = !s->active.empty();
        if (launched && tick(s) != FW_OK) break;
        // the last tick's finished requests are copied out while this one runs
        if (retire(s) != FW_OK) break;
        if (launched && tick_wait(s) != FW_OK) break;
    }
}

void server_free(fw_server *s)
{
    if (!s) return;
    for (auto &kv : s->reqs) delete kv.second;
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->cstream) (void)hipStreamDestroy(s->cstream);
    if (s->ev_tick) (void)hipEventDestroy(s->ev_tick);
    if (s->h_done) (void)hipHostFree(s->h_done);
    (void)hipFree(s->arena_base);
    (void)hipFree(s->d_done);
    (void)hipFree(s->d_table);
    (void)hipFree(s->d_queue);
    (void)hipFree(s->d_stats);
    if (s->h_table) (void)hipHostFree(s->h_table);
    delete s;
}

}  // namespace

extern "C" {

int fw_server_create(fw_graph *g, const fw_plan *plan, int32_t strategy, uint64_t hbm_budget, int32_t tick_steps,
                     int32_t max_active, int32_t max_pending, fw_server **out)
{
    using fw::host::fail;
    if (!g || !plan || !out) return fail(FW_E_INVALID, "fw_server_create: null argument");
    int rc = fw::host::check_plan(plan);
    if (rc != FW_OK) return rc;
    if (plan->hub_deg > 0 && plan->hub_lanes != 64)
        return fail(FW_E_INVALID, "fw_server_create: hub lanes (hub_lanes > 64) apply to fw_walk launches only");
    if (!fw::valid_strategy(strategy))
        return fail(FW_E_INVALID, "fw_server_create: bad strategy %d", strategy);
    if (tick_steps < 1) return fail(FW_E_INVALID, "fw_server_create: tick_steps must be >= 1");
    if (max_active < 1 || max_active > (1 << 20)) return fail(FW_E_INVALID, "fw_server_create: max_active in [1, 2^20]");
    if (max_pending < 1) return fail(FW_E_INVALID, "fw_server_create: max_pending must be >= 1");
    if (hbm_budget < kAlign) return fail(FW_E_INVALID, "fw_server_create: budget too small");
    if (g->h && strategy != FW_RVS_ONLY && !g->prepped)
        return fail(FW_E_STATE, "fw_server_create: call fw_graph_preprocess first");
    HIP_TRY(hipSetDevice(g->device));
    fw_server *s = new fw_server();
    s->g = g;
    s->plan = *plan;
    s->strategy = strategy;
    s->tick_steps = tick_steps;
    s->max_active = max_active;
    s->max_pending = max_pending;
    s->budget = (size_t)hbm_budget;
    for (int32_t i = max_active - 1; i >= 0; --i) s->free_slots.push_back(i);
    if (hipMalloc((void **)&s->arena_base, s->budget) != hipSuccess ||
        hipMalloc((void **)&s->d_done, sizeof(int32_t) * (size_t)max_active) != hipSuccess ||
        hipMalloc((void **)&s->d_table, sizeof(fw::QueryDev) * kGroups * (size_t)max_active) != hipSuccess ||
        hipMalloc((void **)&s->d_queue, kGroups * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void **)&s->d_stats, FW_NSTATS * sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc((void **)&s->h_table, sizeof(fw::QueryDev) * kGroups * (size_t)max_active, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void **)&s->h_done, sizeof(int32_t) * (size_t)max_active, hipHostMallocDefault) != hipSuccess) {
        server_free(s);
        return fail(FW_E_NOMEM, "fw_server_create: allocation failed");
    }
    s->arena.reset(s->budget);
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->cstream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s->ev_tick, hipEventDisableTiming) != hipSuccess ||
        hipMemset(s->d_stats, 0, FW_NSTATS * sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(s->d_done, 0, sizeof(int32_t) * (size_t)max_active) != hipSuccess) {
        server_free(s);
        return fail(FW_E_DEVICE, "fw_server_create: stream or memset failed");
    }
    s->th = std::thread(serve, s);
    *out = s;
    return fw::host::ok();
}

int fw_server_submit(fw_server *s, const fw_logic *logic, const int32_t *starts, int64_t n, int32_t L, uint64_t seed,
                     uint64_t *req_id)
{
    using fw::host::fail;
    if (!s || !logic || !req_id || (n > 0 && !starts)) return fail(FW_E_INVALID, "fw_server_submit: null argument");
    int rc = fw::host::check_logic(s->g, logic);
    if (rc != FW_OK) return rc;
    if ((rc = fw::host::check_bound(s->g, &s->plan, logic)) != FW_OK) return rc;
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(FW_E_INVALID, "fw_server_submit: n must be in [0, 2^31)");
    if (L < 0 || L >= (1 << 20)) return fail(FW_E_INVALID, "fw_server_submit: L must be in [0, 2^20)");
    const size_t bytes = request_bytes(n, L);
    if (bytes > s->budget) return fail(FW_E_INVALID, "fw_server_submit: request needs %zu bytes, budget %zu", bytes, s->budget);
    // starts are host memory: checked here, so a served request never trips the graph's
    // device error flag, which the server does not read
    for (int64_t i = 0; i < n; ++i)
        if (starts[i] < 0 || (int64_t)starts[i] >= s->g->nv)
            return fail(FW_E_INVALID, "fw_server_submit: start %lld (vertex %d) outside [0, %lld)", (long long)i,
                        starts[i], (long long)s->g->nv);
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->err != FW_OK) return fail(s->err, "server stopped: %s", s->err_msg.c_str());
    if ((int64_t)s->waiting.size() >= s->max_pending) return fail(FW_E_BUSY, "fw_server_submit: %d requests already waiting", s->max_pending);
    Request *r = new Request();
    r->id = s->next_id++;
    r->logic = *logic;
    r->n = n;
    r->L = L;
    r->seed = seed;
    r->bytes = bytes;
    r->starts.assign(starts, starts + n);
    r->t_submit = Clock::now();
    s->reqs[r->id] = r;
    s->waiting.push_back(r);
    *req_id = r->id;
    s->cv_work.notify_one();
    return fw::host::ok();
}

int fw_server_next_done(fw_server *s, int32_t timeout_ms, uint64_t *req_id)
{
    using fw::host::fail;
    if (!s || !req_id) return fail(FW_E_INVALID, "fw_server_next_done: null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    *req_id = 0;
    s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms),
                        [s] { return !s->finished.empty() || s->err != FW_OK; });
    if (s->err != FW_OK) return fail(s->err, "server stopped: %s", s->err_msg.c_str());
    if (!s->finished.empty()) {
        *req_id = s->finished.front();
        s->finished.pop_front();
    }
    return fw::host::ok();
}

int fw_server_result(fw_server *s, uint64_t req_id, int32_t *paths, int32_t *lengths, double *latency_s)
{
    using fw::host::fail;
    if (!s) return fail(FW_E_INVALID, "fw_server_result: null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) return fail(FW_E_INVALID, "fw_server_result: unknown request %llu", (unsigned long long)req_id);
    Request *r = it->second;
    if (r->state != 2) return fail(FW_E_STATE, "fw_server_result: request %llu not finished", (unsigned long long)req_id);
    if (paths && !r->paths.empty()) memcpy(paths, r->paths.data(), sizeof(int32_t) * r->paths.size());
    if (lengths && !r->lengths.empty()) memcpy(lengths, r->lengths.data(), sizeof(int32_t) * r->lengths.size());
    if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    s->reqs.erase(it);
    delete r;
    return fw::host::ok();
}

int fw_server_stats(fw_server *s, uint64_t *out)
{
    using fw::host::fail;
    if (!s || !out) return fail(FW_E_INVALID, "fw_server_stats: null argument");
    unsigned long long dev[FW_NSTATS];
    HIP_TRY(hipMemcpy(dev, s->d_stats, sizeof(dev), hipMemcpyDeviceToHost));
    std::lock_guard<std::mutex> lk(s->mu);
    out[0] = s->waiting.size();
    out[1] = s->n_admitted - s->n_finished;
    out[2] = s->n_finished;
    out[3] = s->ticks;
    out[4] = dev[0];
    out[5] = s->arena.used();
    out[6] = s->arena.peak();
    out[7] = dev[7];
    return fw::host::ok();
}

int fw_server_destroy(fw_server *s)
{
    if (!s) return fw::host::ok();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    (void)hipStreamSynchronize(s->stream);
    (void)hipStreamSynchronize(s->cstream);
    server_free(s);
    return fw::host::ok();
}

}  // extern "C"
