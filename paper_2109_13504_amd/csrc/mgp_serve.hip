// mgp_serve.hip -- the resample server: admission by HBM budget, continuous
// micro-batching over several HIP streams, completion tracking.
//
// One scheduler thread owns the device work. Each pass it
//   1. reaps finished micro-batches (event query), records completion times,
//      returns their workspaces to the pool;
//   2. admits queued requests in arrival order while their outputs and
//      workspace fit the pool (first fit, 256-byte granules);
//   3. dispatches admitted requests as a micro-batch (the batched kernels:
//      segmented reduction, per-request finalize, accept loop with fused
//      gather) on a stream that has no batch in flight.
// Requests that arrive while batches run are admitted and dispatched on the
// other streams at once, so their work overlaps on the device.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mgp.h"
#include "mgp_batch_internal.h"
#include "mgp_device.h"
#include "mgp_internal.h"

namespace mgp {
namespace {

constexpr uint64_t kGranule = 256;

uint64_t round_up(uint64_t x) { return (x + kGranule - 1) / kGranule * kGranule; }

// First-fit allocator over [0, size) (host-side bookkeeping of the pool).
class Pool {
public:
    void reset(uint64_t size)
    {
        size_ = size;
        free_.clear();
        if (size) free_[0] = size;
        used_ = peak_ = 0;
    }
    bool alloc(uint64_t bytes, uint64_t* off)
    {
        bytes = round_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const uint64_t start = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[start + bytes] = rest;
            *off = start;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes)
    {
        bytes = round_up(bytes);
        if (!bytes) return;
        auto next = free_.lower_bound(off);
        uint64_t start = off, len = bytes;
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && off + bytes == next->first) {
            len += next->second;
            free_.erase(next);
        }
        free_[start] = len;
        used_ -= bytes;
    }
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }

private:
    uint64_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;  // offset -> length, coalesced
};

struct Req {
    mgp_request in{};
    int state = MGP_REQ_QUEUED;
    int32_t status = 0;
    uint32_t B = 0;
    uint64_t out_off = 0, out_bytes = 0;  // ancestors + gathered states (kept until release)
    uint64_t ws_off = 0, ws_bytes = 0;    // mirror + offsets (freed at completion)
    bool has_out = false, has_ws = false;
    uint64_t anc_bytes = 0;
    double t_submit = 0, t_admit = 0, t_dispatch = 0, t_done = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    double sim_done_at = 0;
    bool sim_fail = false;
    std::vector<uint64_t> tickets;
    // device tables and their pinned staging copies
    char* dmem = nullptr;
    FilterDev* d_fd = nullptr;
    RTile* d_rt = nullptr;
    LTile* d_lt = nullptr;
    Partial* d_parts = nullptr;
    mgp_stats* d_stats = nullptr;
    uint32_t* d_q = nullptr;     // queue counters [kMaxXcd + 1]
    uint32_t* d_qoff = nullptr;  // queue offsets [kMaxXcd + 1]
    size_t lt_offset = 0;        // start of the loop tiles in the upload region
    char* hmem = nullptr;
    FilterDev* h_fd = nullptr;
    RTile* h_rt = nullptr;
    LTile* h_lt = nullptr;
    mgp_stats* h_stats = nullptr;
    uint32_t* h_qoff = nullptr;
};

}  // namespace
}  // namespace mgp

using namespace mgp;

struct mgp_server {
    mgp_server_config cfg{};
    int variant = kMegopolis;
    LoopShape shape{64, 4, 1};
    uint32_t b_max = kDefaultBMax;
    uint32_t n_w = 32;
    int nxcd = 1;
    int device = 0;  // the device current at create; the scheduler thread binds it
    int64_t max_particles = 1 << 24;
    uint32_t max_n = 1u << 22;
    uint32_t cap_f = 0, cap_rt = 0, cap_lt = 0;
    char* pool_base = nullptr;  // device pool (or a fake base when simulating)
    Pool pool;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv;       // wakes the scheduler
    std::condition_variable done_cv;  // wakes waiters
    std::unordered_map<uint64_t, Req> reqs;
    std::deque<uint64_t> queue;     // submitted, not admitted
    std::deque<uint64_t> admitted;  // admitted, not dispatched
    uint64_t next_ticket = 1;
    bool stopping = false;
    std::thread worker;
    std::chrono::steady_clock::time_point t0;
    mgp_server_stats st{};
    int64_t batches_running = 0;
    int last_error = 0;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

uint64_t mirror_bytes(uint32_t n) { return round_up(4ull * (2ull * n + kMirrorPad)); }

void footprint(const mgp_server* s, const mgp_request& r, Req& q)
{
    q.anc_bytes = round_up(4ull * (uint64_t)r.n);
    q.out_bytes = q.anc_bytes + ((r.states_dev && s->cfg.d > 0) ? round_up(4ull * (uint64_t)r.n * s->cfg.d) : 0);
    q.ws_bytes = s->variant == kMegopolis ? mirror_bytes((uint32_t)r.n) + round_up(4ull * s->b_max) : 0;
}

bool try_admit(mgp_server* s, Req& q)
{
    uint64_t o = 0, w = 0;
    if (!s->pool.alloc(q.out_bytes, &o)) return false;
    if (q.ws_bytes && !s->pool.alloc(q.ws_bytes, &w)) {
        s->pool.release(o, q.out_bytes);
        return false;
    }
    q.out_off = o;
    q.has_out = true;
    q.ws_off = w;
    q.has_ws = q.ws_bytes > 0;
    q.t_admit = s->now();
    return true;
}

void release_ws(mgp_server* s, Req& q)
{
    if (q.has_ws) s->pool.release(q.ws_off, q.ws_bytes);
    q.has_ws = false;
}

void release_out(mgp_server* s, Req& q)
{
    if (q.has_out) s->pool.release(q.out_off, q.out_bytes);
    q.has_out = false;
}

// Builds the slot's tables for the requests and enqueues the batch. Called
// without the lock; the requests are RUNNING, so nobody else touches them.
int launch_batch(mgp_server* s, Slot& sl, const std::vector<Req*>& rs)
{
    const uint32_t count = (uint32_t)rs.size();
    std::vector<uint32_t> ns(count);
    std::vector<double> cost(count);
    uint32_t need_rt = 0;
    for (uint32_t f = 0; f < count; ++f) need_rt += reduce_blocks((uint32_t)rs[f]->in.n);
    if (count > s->cap_f || need_rt > s->cap_rt) return fail(MGP_ERANGE, "micro-batch exceeds the slot tables");
    uint32_t nrt = 0;
    for (uint32_t f = 0; f < count; ++f) {
        const Req& q = *rs[f];
        const uint32_t n = (uint32_t)q.in.n;
        FilterDev& F = sl.h_fd[f];
        memset(&F, 0, sizeof F);
        char* out = s->pool_base + q.out_off;
        F.w = q.in.w_dev;
        F.anc = reinterpret_cast<int32_t*>(out);
        const bool gather = q.in.states_dev && s->cfg.d > 0;
        F.states = gather ? q.in.states_dev : nullptr;
        F.out = gather ? reinterpret_cast<float*>(out + q.anc_bytes) : nullptr;
        F.stats_user = nullptr;
        if (s->variant == kMegopolis) {
            char* ws = s->pool_base + q.ws_off;
            F.mirror = reinterpret_cast<float*>(ws);
            F.offsets = reinterpret_cast<uint32_t*>(ws + mirror_bytes(n));
        }
        F.eps = q.in.epsilon;
        F.n = n;
        F.B_user = q.in.B;
        F.b_max = s->b_max;
        F.key0 = (uint32_t)q.in.seed;
        F.key1 = (uint32_t)(q.in.seed >> 32);
        F.stream_id = q.in.stream_id;
        F.nparts = reduce_blocks(n);
        F.chunk = reduce_chunk(n, F.nparts);
        F.part_base = nrt;
        F.n_w = s->n_w;
        F.n_part = (uint32_t)(((uint64_t)n + s->n_w - 1u) / s->n_w);
        F.vec = (((uintptr_t)q.in.w_dev & 15u) == 0 && (s->variant != kMegopolis || n % 4u == 0)) ? 1u : 0u;
        F.rows4 = (s->cfg.d % 4 == 0 && ((uintptr_t)q.in.states_dev & 15u) == 0) ? 1u : 0u;
        for (uint32_t c = 0; c < F.nparts; ++c) sl.h_rt[nrt + c] = RTile{f, c};
        nrt += F.nparts;
        ns[f] = n;
        cost[f] = (double)n;  // B is found on the device during the run
    }
    std::vector<LTile> table;
    build_tile_table(ns, cost, s->shape, s->nxcd, table, sl.h_qoff);
    if (table.empty()) table.push_back(LTile{kNoFilter, 0});
    if (table.size() > s->cap_lt) return fail(MGP_ERANGE, "micro-batch exceeds the slot tables");
    memcpy(sl.h_lt, table.data(), table.size() * sizeof(LTile));
    hipStream_t st = sl.stream;
    // one upload: the qoff, filter and tile tables share one layout on both sides
    const size_t upload = sl.lt_offset + table.size() * sizeof(LTile);
    if (hipMemcpyAsync(sl.dmem, sl.hmem, upload, hipMemcpyHostToDevice, st) != hipSuccess)
        return fail(MGP_EHIP, "uploading micro-batch tables failed");
    const uint32_t grid = (uint32_t)table.size();
    int rc = enqueue_batch(s->variant, s->shape, sl.d_fd, count, sl.d_rt, nrt, sl.d_parts, sl.d_stats, sl.d_lt, grid,
                           sl.d_qoff, sl.d_q, (uint32_t)s->nxcd, (uint32_t)s->cfg.d, st);
    if (rc) return rc;
    if (hipMemcpyAsync(sl.h_stats, sl.d_stats, count * sizeof(mgp_stats), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipEventRecord(sl.done, st) != hipSuccess)
        return fail(MGP_EHIP, "recording micro-batch completion failed");
    return MGP_OK;
}

bool slot_finished(mgp_server* s, Slot& sl)
{
    if (!sl.busy) return false;
    if (s->cfg.simulate) return s->now() >= sl.sim_done_at;
    return hipEventQuery(sl.done) != hipErrorNotReady;
}

// Completes a finished slot's requests (lock held).
void reap(mgp_server* s, Slot& sl)
{
    const double t = s->now();
    const bool dev_ok = s->cfg.simulate ? !sl.sim_fail : (hipEventQuery(sl.done) == hipSuccess);
    for (size_t f = 0; f < sl.tickets.size(); ++f) {
        auto it = s->reqs.find(sl.tickets[f]);
        if (it == s->reqs.end()) continue;
        Req& q = it->second;
        q.t_done = t;
        release_ws(s, q);
        if (!dev_ok) {
            q.state = MGP_REQ_FAILED;
            release_out(s, q);
            ++s->st.failed;
        } else {
            q.state = MGP_REQ_DONE;
            if (s->cfg.simulate) {
                q.status = MGP_OK;
                q.B = q.in.B ? q.in.B : 1u;
            } else {
                q.status = sl.h_stats[f].status;
                q.B = sl.h_stats[f].B;
            }
            ++s->st.completed;
        }
        --s->st.in_flight;
    }
    sl.tickets.clear();
    sl.busy = false;
    --s->batches_running;
    s->done_cv.notify_all();
}

void scheduler(mgp_server* s)
{
    // the current device is per thread: bind the one the pool and streams
    // were allocated on before any launch, copy or event query
    std::unique_lock<std::mutex> lk(s->mu);
    if (!s->cfg.simulate && hipSetDevice(s->device) != hipSuccess) s->last_error = MGP_EHIP;
    int64_t batch_counter = 0;
    for (;;) {
        bool any_busy = false;
        for (Slot& sl : s->slots) {
            if (slot_finished(s, sl)) reap(s, sl);
            any_busy = any_busy || sl.busy;
        }
        // admission, in arrival order
        while (!s->queue.empty()) {
            auto it = s->reqs.find(s->queue.front());
            if (it == s->reqs.end() || it->second.state != MGP_REQ_QUEUED) {
                s->queue.pop_front();
                continue;
            }
            if (!try_admit(s, it->second)) break;
            s->admitted.push_back(s->queue.front());
            s->queue.pop_front();
            ++s->st.admitted;
            ++s->st.in_flight;
        }
        // dispatch micro-batches onto idle streams
        for (size_t k = 0; k < s->slots.size() && !s->admitted.empty(); ++k) {
            Slot& sl = s->slots[k];
            if (sl.busy) continue;
            std::vector<Req*> rs;
            int64_t parts = 0;
            while (!s->admitted.empty() && (int)rs.size() < s->cfg.max_batch) {
                Req& q = s->reqs[s->admitted.front()];
                if (!rs.empty() && parts + q.in.n > s->max_particles) break;
                parts += q.in.n;
                q.state = MGP_REQ_RUNNING;
                q.t_dispatch = s->now();
                rs.push_back(&q);
                sl.tickets.push_back(s->admitted.front());
                s->admitted.pop_front();
            }
            sl.busy = true;
            ++s->batches_running;
            ++s->st.micro_batches;
            s->st.max_concurrent_batches = std::max(s->st.max_concurrent_batches, s->batches_running);
            ++batch_counter;
            if (s->cfg.simulate) {
                sl.sim_done_at = s->now() + 1e-6 * (s->cfg.sim_us_fixed + 1e-3 * s->cfg.sim_ns_per_particle * parts);
                sl.sim_fail = s->cfg.sim_fail_every > 0 && batch_counter % s->cfg.sim_fail_every == 0;
            } else {
                lk.unlock();
                const int rc = launch_batch(s, sl, rs);
                lk.lock();
                if (rc) {
                    // nothing usable was enqueued: fail the batch's requests
                    s->last_error = rc;
                    (void)hipStreamSynchronize(sl.stream);
                    sl.sim_fail = true;
                    for (uint64_t t : sl.tickets) {
                        Req& q = s->reqs[t];
                        q.state = MGP_REQ_FAILED;
                        q.t_done = s->now();
                        release_ws(s, q);
                        release_out(s, q);
                        ++s->st.failed;
                        --s->st.in_flight;
                    }
                    sl.tickets.clear();
                    sl.busy = false;
                    --s->batches_running;
                    s->done_cv.notify_all();
                }
            }
            any_busy = any_busy || sl.busy;
        }
        if (s->stopping) {
            // no new admissions: requests still queued are cancelled
            for (uint64_t t : s->queue) {
                auto it = s->reqs.find(t);
                if (it != s->reqs.end() && it->second.state == MGP_REQ_QUEUED) {
                    it->second.state = MGP_REQ_CANCELLED;
                    it->second.t_done = s->now();
                    ++s->st.cancelled;
                }
            }
            s->queue.clear();
            s->done_cv.notify_all();
        }
        if (s->stopping && s->admitted.empty() && !any_busy) break;
        if (any_busy) {
            // poll the device closely while batches run, without holding the lock
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            s->cv.wait_for(lk, std::chrono::milliseconds(50));
        }
    }
}

// A slot's tables: the uploaded part [qoff | filters | reduce tiles | loop
// tiles] has the same layout on the host (pinned) and the device, so one
// copy of its used prefix uploads a micro-batch.
struct SlotLayout {
    size_t qoff, fd, rt, lt, upload_end;  // upload region
    size_t parts, stats, qcount, dev_end; // device-only region
    size_t h_stats, host_end;             // host-only region
};

SlotLayout slot_layout(const mgp_server* s)
{
    SlotLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return o;
    };
    L.qoff = take(sizeof(uint32_t) * (kMaxXcd + 1));
    L.fd = take(sizeof(FilterDev) * s->cap_f);
    L.rt = take(sizeof(RTile) * s->cap_rt);
    L.lt = take(sizeof(LTile) * s->cap_lt);
    L.upload_end = off;
    L.parts = take(sizeof(Partial) * s->cap_rt);
    L.stats = take(sizeof(mgp_stats) * s->cap_f);
    L.qcount = take(sizeof(uint32_t) * (kMaxXcd + 1));
    L.dev_end = off;
    off = L.upload_end;
    L.h_stats = take(sizeof(mgp_stats) * s->cap_f);
    L.host_end = off;
    return L;
}

int alloc_slot(mgp_server* s, Slot& sl)
{
    const SlotLayout L = slot_layout(s);
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
        return fail(MGP_EHIP, "creating a server stream failed");
    if (hipMalloc(&sl.dmem, L.dev_end) != hipSuccess) return fail(MGP_ENOMEM, "server tables: hipMalloc failed");
    if (hipHostMalloc(reinterpret_cast<void**>(&sl.hmem), L.host_end) != hipSuccess)
        return fail(MGP_ENOMEM, "server staging: hipHostMalloc failed");
    sl.d_fd = reinterpret_cast<FilterDev*>(sl.dmem + L.fd);
    sl.d_rt = reinterpret_cast<RTile*>(sl.dmem + L.rt);
    sl.d_lt = reinterpret_cast<LTile*>(sl.dmem + L.lt);
    sl.d_parts = reinterpret_cast<Partial*>(sl.dmem + L.parts);
    sl.d_stats = reinterpret_cast<mgp_stats*>(sl.dmem + L.stats);
    sl.d_q = reinterpret_cast<uint32_t*>(sl.dmem + L.qcount);
    sl.d_qoff = reinterpret_cast<uint32_t*>(sl.dmem + L.qoff);
    sl.h_fd = reinterpret_cast<FilterDev*>(sl.hmem + L.fd);
    sl.h_rt = reinterpret_cast<RTile*>(sl.hmem + L.rt);
    sl.h_lt = reinterpret_cast<LTile*>(sl.hmem + L.lt);
    sl.h_stats = reinterpret_cast<mgp_stats*>(sl.hmem + L.h_stats);
    sl.h_qoff = reinterpret_cast<uint32_t*>(sl.hmem + L.qoff);
    sl.lt_offset = L.lt;
    return MGP_OK;
}

void free_server(mgp_server* s)
{
    // best-effort teardown
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.dmem) (void)hipFree(sl.dmem);
        if (sl.hmem) (void)hipHostFree(sl.hmem);
    }
    if (!s->cfg.simulate && s->pool_base) (void)hipFree(s->pool_base);
    delete s;
}

int validate_request(const mgp_server* s, const mgp_request* r)
{
    if (!r) return fail(MGP_EINVAL, "request is NULL");
    if (!r->w_dev) return fail(MGP_EINVAL, "request weights are NULL");
    if (r->n < 1 || (uint32_t)r->n > s->max_n) return fail(MGP_ERANGE, "request n = %d out of [1, %u]", r->n, s->max_n);
    if (r->reserved) return fail(MGP_EINVAL, "request.reserved must be 0");
    if (r->B == 0 && (!(r->epsilon > 0.0) || !(r->epsilon <= 1.0)))
        return fail(MGP_EINVAL, "epsilon must be in (0, 1] when B is 0");
    if (r->B > s->b_max) return fail(MGP_ERANGE, "B = %u above b_max = %u", r->B, s->b_max);
    return MGP_OK;
}

void fill_result(const mgp_server* s, const Req& q, mgp_request_result* r)
{
    r->state = q.state;
    r->status = q.status;
    r->B = q.B;
    r->n = q.in.n;
    const bool ready = q.state == MGP_REQ_DONE && q.has_out;
    r->ancestors_dev = ready ? reinterpret_cast<const int32_t*>(s->pool_base + q.out_off) : nullptr;
    r->out_states_dev = (ready && q.out_bytes > q.anc_bytes)
                            ? reinterpret_cast<const float*>(s->pool_base + q.out_off + q.anc_bytes)
                            : nullptr;
    r->t_submit = q.t_submit;
    r->t_admit = q.t_admit;
    r->t_dispatch = q.t_dispatch;
    r->t_done = q.t_done;
}

}  // namespace

extern "C" {

int mgp_server_create(const mgp_server_config* cfg, mgp_server** out)
{
    clear_error();
    if (!cfg || !out) return fail(MGP_EINVAL, "NULL argument");
    *out = nullptr;
    if (cfg->variant < MGP_METROPOLIS || cfg->variant > MGP_MEGOPOLIS) return fail(MGP_EINVAL, "unknown variant");
    if (cfg->d < 0 || cfg->streams < 1 || cfg->max_batch < 1 || cfg->hbm_budget == 0 || cfg->reserved)
        return fail(MGP_EINVAL, "need d >= 0, streams >= 1, max_batch >= 1, hbm_budget > 0, reserved = 0");
    const uint32_t pb = cfg->partition_bytes ? cfg->partition_bytes : 128u;
    if (pb < 4u || pb % 4u) return fail(MGP_EINVAL, "partition_bytes must be a positive multiple of 4");
    mgp_server* s = new mgp_server();
    s->cfg = *cfg;
    s->variant = cfg->variant;
    s->b_max = cfg->b_max ? cfg->b_max : kDefaultBMax;
    s->n_w = pb / 4u;
    s->max_particles = cfg->max_batch_particles > 0 ? cfg->max_batch_particles : (int64_t)1 << 24;
    s->max_n = cfg->max_n > 0 ? (uint32_t)cfg->max_n : (1u << 22);
    if (s->max_n > kMirrorMaxN || s->b_max > kBMaxLimit) {
        delete s;
        return fail(MGP_ERANGE, "max_n or b_max too large");
    }
    s->max_particles = std::max<int64_t>(s->max_particles, s->max_n);
    s->shape = s->variant == kMegopolis ? LoopShape{64, 4, 1} : LoopShape{256, 1, 1};
    const uint32_t tile = (uint32_t)(s->shape.bt * s->shape.ppt);
    s->cap_f = (uint32_t)cfg->max_batch;
    s->cap_rt = (uint32_t)(s->max_particles / kReduceChunk + 2 * (int64_t)cfg->max_batch + 1);
    s->t0 = std::chrono::steady_clock::now();
    s->slots.resize(cfg->streams);
    if (cfg->simulate) {
        s->nxcd = 1;
        s->pool_base = reinterpret_cast<char*>((uintptr_t)1 << 40);  // fake addresses, never dereferenced
    } else {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            delete s;
            return fail(MGP_EHIP, "no HIP device");
        }
        s->device = dev;
        s->nxcd = (cus >= 64 && cus % kMaxXcd == 0) ? kMaxXcd : 1;
        if (hipMalloc(&s->pool_base, cfg->hbm_budget) != hipSuccess) {
            s->pool_base = nullptr;
            free_server(s);
            return fail(MGP_ENOMEM, "could not allocate the %llu-byte pool", (unsigned long long)cfg->hbm_budget);
        }
    }
    s->cap_lt = (uint32_t)(s->nxcd * (s->max_particles / tile + 2 * (int64_t)cfg->max_batch + 1));
    if (!cfg->simulate) {
        for (Slot& sl : s->slots) {
            int rc = alloc_slot(s, sl);
            if (rc) {
                free_server(s);
                return rc;
            }
        }
    }
    s->pool.reset(cfg->hbm_budget);
    s->st.pool_bytes = cfg->hbm_budget;
    s->worker = std::thread(scheduler, s);
    *out = s;
    return MGP_OK;
}

int mgp_server_submit(mgp_server* s, const mgp_request* r, uint64_t* ticket)
{
    clear_error();
    if (!s || !ticket) return fail(MGP_EINVAL, "NULL argument");
    int rc = validate_request(s, r);
    if (rc) return rc;
    Req q;
    q.in = *r;
    footprint(s, *r, q);
    if (q.out_bytes + q.ws_bytes > s->pool.size())
        return fail(MGP_ENOMEM, "request needs %llu bytes, the pool has %llu",
                    (unsigned long long)(q.out_bytes + q.ws_bytes), (unsigned long long)s->pool.size());
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) return fail(MGP_EBUSY, "server is stopping");
        q.t_submit = s->now();
        *ticket = s->next_ticket++;
        s->reqs.emplace(*ticket, q);
        s->queue.push_back(*ticket);
        ++s->st.submitted;
    }
    s->cv.notify_one();
    return MGP_OK;
}

int mgp_server_poll(mgp_server* s, uint64_t ticket, mgp_request_result* r)
{
    clear_error();
    if (!s || !r) return fail(MGP_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(MGP_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    fill_result(s, it->second, r);
    return MGP_OK;
}

int mgp_server_wait(mgp_server* s, uint64_t ticket, double timeout_ms, mgp_request_result* r)
{
    clear_error();
    if (!s || !r) return fail(MGP_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto finished = [&]() {
        auto it = s->reqs.find(ticket);
        return it == s->reqs.end() || it->second.state >= MGP_REQ_DONE;
    };
    if (timeout_ms < 0)
        s->done_cv.wait(lk, finished);
    else if (!s->done_cv.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), finished))
        return fail(MGP_EBUSY, "request %llu not finished", (unsigned long long)ticket);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(MGP_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    fill_result(s, it->second, r);
    return MGP_OK;
}

int mgp_server_copy_outputs(mgp_server* s, uint64_t ticket, int32_t* anc, float* out, void* stream)
{
    clear_error();
    if (!s || !anc) return fail(MGP_EINVAL, "NULL argument");
    if (s->cfg.simulate) return fail(MGP_EINVAL, "a simulated server has no outputs");
    const char* src_anc = nullptr;
    const char* src_out = nullptr;
    size_t anc_bytes = 0, out_bytes = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return fail(MGP_EINVAL, "unknown ticket");
        const Req& q = it->second;
        if (q.state != MGP_REQ_DONE || !q.has_out) return fail(MGP_EBUSY, "request has no outputs (not done)");
        src_anc = s->pool_base + q.out_off;
        anc_bytes = 4ull * (uint64_t)q.in.n;
        if (q.out_bytes > q.anc_bytes) {
            src_out = src_anc + q.anc_bytes;
            out_bytes = 4ull * (uint64_t)q.in.n * (uint64_t)s->cfg.d;
        }
    }
    // the outputs stay allocated until release, which the caller orders
    // after this copy
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(anc, src_anc, anc_bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(MGP_EHIP, "copying ancestors failed");
    if (out && src_out && hipMemcpyAsync(out, src_out, out_bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(MGP_EHIP, "copying gathered states failed");
    return MGP_OK;
}

int mgp_server_cancel(mgp_server* s, uint64_t ticket)
{
    clear_error();
    if (!s) return fail(MGP_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(MGP_EINVAL, "unknown ticket");
    if (it->second.state != MGP_REQ_QUEUED) return fail(MGP_EBUSY, "request already admitted");
    it->second.state = MGP_REQ_CANCELLED;
    it->second.t_done = s->now();
    ++s->st.cancelled;
    s->done_cv.notify_all();
    return MGP_OK;
}

int mgp_server_release(mgp_server* s, uint64_t ticket)
{
    clear_error();
    if (!s) return fail(MGP_EINVAL, "NULL argument");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return fail(MGP_EINVAL, "unknown ticket");
        if (it->second.state < MGP_REQ_DONE) return fail(MGP_EBUSY, "request not finished");
        release_out(s, it->second);
        s->reqs.erase(it);
        ++s->st.released;
    }
    s->cv.notify_one();  // freed memory may admit queued requests
    return MGP_OK;
}

int mgp_server_get_stats(mgp_server* s, mgp_server_stats* out)
{
    clear_error();
    if (!s || !out) return fail(MGP_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->queued = (int64_t)s->queue.size();
    out->pool_in_use = s->pool.used();
    out->pool_peak = s->pool.peak();
    return MGP_OK;
}

int mgp_server_destroy(mgp_server* s)
{
    clear_error();
    if (!s) return MGP_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    free_server(s);
    return MGP_OK;
}

}  // extern "C"
