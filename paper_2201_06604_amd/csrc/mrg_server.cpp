// mrg_server.cpp -- the serving engine: sessions with device-resident streams,
// arrival-order positions, memory admission against a caller-owned output
// pool, continuous batching into persistent launches on several HIP streams,
// per-request completion flags in host-visible memory, and an open-loop
// replay driver.  One scheduler thread does all device work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mrg355.h"
#include "mrg_internal.h"
#include "mrg_math.h"

using namespace mrg355;

mrg_status mrg355_fail(mrg_status st, const char* fmt, ...);  // mrg_api.cpp

namespace {

uint64_t steady_ns() {
    return static_cast<uint64_t>(std::chrono::duration_cast<std::chrono::nanoseconds>(
                                     std::chrono::steady_clock::now().time_since_epoch())
                                     .count());
}

size_t round256(size_t n) { return (n + 255) / 256 * 256; }

// A served request is cut into about this many tiles per 64-stream block (at
// least 96 units each), so that a long request runs on many waves at once;
// the lane workspaces are sized for it.
constexpr uint32_t kServeSplit = 64;

// First-fit allocator over [0, total) in 256-byte granules; neighbours merge
// on release.
struct Pool {
    std::map<size_t, size_t> free_;  // offset -> bytes
    size_t total = 0, in_use = 0, peak = 0;

    void init(size_t bytes) {
        total = bytes / 256 * 256;
        free_.clear();
        if (total) free_[0] = total;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = round256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            in_use += bytes;
            peak = std::max(peak, in_use);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = round256(bytes);
        in_use -= bytes;
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
};

enum TState { kPending = 0, kInFlight = 1, kDone = 2 };

struct Ticket {
    uint32_t session;
    uint64_t n;
    mrg_dist dist;
    mrg_dtype dtype;
    double param;
    uint64_t t_arrival, offset, t_done;
    size_t bytes, pool_off;
    int state;
    hipEvent_t ev;  // plain mode
};

struct Lane {
    hipStream_t stream = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    BatchSlot* slots_host = nullptr;  // pinned, host-coherent
    BatchSlot* slots_dev = nullptr;   // the same memory as the device sees it
    char* staging = nullptr;          // pinned copy source of the plan tables
    hipEvent_t done_ev = nullptr;
    bool busy = false;
    bool single = false;              // the lane runs one request as a plain launch
    std::vector<uint64_t> tickets;
    size_t remaining = 0;
    mrg_batch_plan* plan = nullptr;
};

size_t esz_of(mrg_dtype dt) { return dt == MRG_F64 ? 8 : 4; }

// Defaults of the optional configuration fields.
uint32_t cfg_streams(const mrg_server_cfg& c) { return c.streams_per_session ? c.streams_per_session : 64; }
uint32_t cfg_lanes(const mrg_server_cfg& c) { return c.mode == 0 ? (c.lanes ? c.lanes : 4) : 0; }
uint32_t cfg_max_batch(const mrg_server_cfg& c) { return c.max_batch ? c.max_batch : 256; }

// The device workspace a server carves from the caller's buffer: the session
// stream records, then one batch workspace per lane (sized for max_batch
// requests, each cut into at most kServeSplit chunks of ceil(S/64) stream
// blocks), each part 256-byte aligned.
struct WsLayout {
    size_t streams_bytes, lane_bytes, total;
};

WsLayout ws_layout(const mrg_server_cfg& c) {
    const uint32_t S = cfg_streams(c), mb = cfg_max_batch(c);
    WsLayout w{};
    w.streams_bytes = round256(static_cast<size_t>(S) * c.n_sessions * sizeof(mrg_stream));
    const size_t max_tiles = static_cast<size_t>(mb) * ((S + 63) / 64) * kServeSplit;
    w.lane_bytes = 256 + round256(mb * sizeof(BatchSlot)) + round256(mb * sizeof(BatchReq)) +
                   round256(max_tiles * sizeof(BatchTile)) + 1024;
    w.total = w.streams_bytes + static_cast<size_t>(cfg_lanes(c)) * w.lane_bytes;
    return w;
}

// Checks shared by mrg_server_workspace_size and mrg_server_create.
mrg_status check_cfg(const mrg_server_cfg& c) {
    if (c.n_sessions == 0) return mrg355_fail(MRG_E_INVALID_ARG, "no sessions");
    if (c.mode > 1) return mrg355_fail(MRG_E_INVALID_ARG, "mode must be 0 or 1");
    if (c.lanes > 64) return mrg355_fail(MRG_E_INVALID_ARG, "at most 64 lanes");
    if (c.max_batch > 65536) return mrg355_fail(MRG_E_INVALID_ARG, "max_batch above 65536");
    const uint32_t S = cfg_streams(c);
    if (S > 65536) return mrg355_fail(MRG_E_INVALID_ARG, "streams_per_session above 65536");
    if (static_cast<uint64_t>(S) * c.n_sessions > (1ull << 31)) return mrg355_fail(MRG_E_INVALID_ARG, "too many streams");
    return MRG_OK;
}

}  // namespace

struct mrg_server {
    mrg_server_cfg cfg{};
    uint32_t S = 64;
    int device = 0;
    uint32_t* streams_dev = nullptr;  // in the caller's workspace
    std::vector<uint64_t> sess_off;
    Pool pool;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, Ticket> tickets;
    std::deque<uint64_t> completions;
    bool collect = false;
    std::vector<Lane> lanes;
    hipStream_t plain_stream = nullptr;
    std::deque<uint64_t> plain_inflight;
    std::vector<hipEvent_t> free_events;
    uint64_t next_id = 1;
    mrg_server_stats st{};
    uint64_t in_flight = 0;
    std::thread th;
    std::atomic<bool> stop{false};
    mrg_status error = MRG_OK;

    void loop();
    bool launch_batch(Lane& L);
    bool launch_plain();
    bool poll_lanes();
    bool poll_plain();
    void complete(uint64_t id, Ticket& t);
    void note_lanes_busy() {
        uint64_t busy = 0;
        for (const Lane& L : lanes) busy += L.busy ? 1 : 0;
        st.max_lanes_busy = std::max(st.max_lanes_busy, busy);
    }
    void fail_hip(hipError_t e, const char* what) {
        if (error == MRG_OK) {
            mrg355_fail(MRG_E_HIP, "server %s: %s", what, hipGetErrorString(e));
            error = MRG_E_HIP;
        }
    }
};

// ------------------------------------------------------------ scheduler
void mrg_server::complete(uint64_t id, Ticket& t) {
    t.state = kDone;
    t.t_done = steady_ns();
    ++st.completed;
    st.samples_completed += t.n;
    in_flight -= 1;
    if (collect) completions.push_back(id);
}

bool mrg_server::poll_lanes() {
    bool progress = false;
    for (Lane& L : lanes) {
        if (!L.busy) continue;
        if (L.single) {  // one plain launch: its event is the completion
            hipError_t e = hipEventQuery(L.done_ev);
            if (e == hipSuccess) {
                auto it = tickets.find(L.tickets[0]);
                if (it != tickets.end() && it->second.state == kInFlight) complete(L.tickets[0], it->second);
                L.busy = L.single = false;
                L.remaining = 0;
                L.tickets.clear();
                progress = true;
            } else if (e != hipErrorNotReady) {
                fail_hip(e, "plain completion");
            }
            continue;
        }
        for (size_t i = 0; i < L.tickets.size() && L.remaining; ++i) {
            auto it = tickets.find(L.tickets[i]);
            if (it == tickets.end() || it->second.state != kInFlight) continue;
            const volatile uint32_t* done = &L.slots_host[i].done;
            if (*done) {
                complete(L.tickets[i], it->second);
                --L.remaining;
                progress = true;
            }
        }
        if (L.remaining == 0) {
            hipError_t e = hipEventQuery(L.done_ev);
            if (e == hipSuccess) {
                L.busy = false;
                mrg_batch_plan_destroy(L.plan);
                L.plan = nullptr;
                L.tickets.clear();
                progress = true;
            } else if (e != hipErrorNotReady) {
                fail_hip(e, "batch completion");
            }
        }
    }
    return progress;
}

bool mrg_server::poll_plain() {
    bool progress = false;
    while (!plain_inflight.empty()) {
        const uint64_t id = plain_inflight.front();
        Ticket& t = tickets.at(id);
        hipError_t e = hipEventQuery(t.ev);
        if (e == hipErrorNotReady) break;
        if (e != hipSuccess) {
            fail_hip(e, "plain completion");
            break;
        }
        free_events.push_back(t.ev);
        t.ev = nullptr;
        complete(id, t);
        plain_inflight.pop_front();
        progress = true;
    }
    return progress;
}

// Admit pending requests in order while their outputs fit the pool, plan them
// as one persistent launch and enqueue it on the lane.
bool mrg_server::launch_batch(Lane& L) {
    std::vector<uint64_t> ids;
    std::vector<PlanReq> reqs;
    while (!pending.empty() && ids.size() < cfg.max_batch) {
        Ticket& t = tickets.at(pending.front());
        size_t off = 0;
        if (!pool.alloc(t.bytes, &off)) break;  // in order: wait for memory
        t.pool_off = off;
        mrg_request q{};
        q.streams = reinterpret_cast<mrg_stream*>(streams_dev + static_cast<size_t>(t.session) * S * 18);
        q.n_streams = S;
        q.n = t.n;
        q.dist = t.dist;
        q.dtype = t.dtype;
        q.param = t.param;
        q.out = static_cast<char*>(cfg.pool) + off;
        reqs.push_back(PlanReq{q, t.offset, 1, kServeSplit});
        ids.push_back(pending.front());
        pending.pop_front();
    }
    if (ids.empty()) return false;
    if (ids.size() == 1) {  // nothing to batch with: one plain launch, no plan upload
        GenLaunch G{};
        G.streams = reinterpret_cast<uint32_t*>(reqs[0].q.streams);
        G.out = reqs[0].q.out;
        G.S = reqs[0].q.n_streams;
        G.q = reqs[0].q.n / G.S;
        G.r = static_cast<uint32_t>(reqs[0].q.n % G.S);
        G.dist = static_cast<int>(reqs[0].q.dist);
        G.dtype = static_cast<int>(reqs[0].q.dtype);
        G.param = reqs[0].q.dist == MRG_EXPONENTIAL ? 1.0 / reqs[0].q.param : 1.0;
        G.offset = reqs[0].offset;
        G.no_writeback = 1;
        plan_generate(G);
        hipError_t e = launch_generate(G, L.stream);
        if (e == hipSuccess) e = hipEventRecord(L.done_ev, L.stream);
        if (e != hipSuccess) {
            fail_hip(e, "single launch");
            return false;
        }
        L.single = true;
        L.tickets = ids;
        L.remaining = 1;
        L.busy = true;
        tickets.at(ids[0]).state = kInFlight;
        in_flight += 1;
        st.max_in_flight = std::max<uint64_t>(st.max_in_flight, in_flight);
        ++st.launches;
        note_lanes_busy();
        return true;
    }
    mrg_batch_plan* plan = nullptr;
    for (uint32_t tu = cfg.tile_units;; tu *= 2) {  // coarser tiles until the plan fits the lane
        if (plan_internal(reqs, tu, &plan)) {
            error = MRG_E_INVALID_ARG;
            return false;
        }
        if (plan_bytes(plan) <= L.ws_bytes || tu >= (1u << 30)) break;
        mrg_batch_plan_destroy(plan);
        plan = nullptr;
    }
    const size_t toff = plan_table_offset(plan);
    plan_pack_tables(plan, L.staging);
    std::memset(L.slots_host, 0, ids.size() * sizeof(BatchSlot));
    hipError_t e = hipMemcpyAsync(static_cast<char*>(L.ws) + toff, L.staging, plan_bytes(plan) - toff,
                                  hipMemcpyHostToDevice, L.stream);
    if (e != hipSuccess) {
        fail_hip(e, "table upload");
        return false;
    }
    if (plan_launch(plan, L.ws, L.slots_dev, L.stream)) {
        error = MRG_E_HIP;
        return false;
    }
    e = hipEventRecord(L.done_ev, L.stream);
    if (e != hipSuccess) {
        fail_hip(e, "event record");
        return false;
    }
    L.plan = plan;
    L.tickets = ids;
    L.remaining = ids.size();
    L.busy = true;
    for (uint64_t id : ids) tickets.at(id).state = kInFlight;
    in_flight += ids.size();
    st.max_in_flight = std::max<uint64_t>(st.max_in_flight, in_flight);
    ++st.launches;
    note_lanes_busy();
    return true;
}

// Baseline: the pending head, when its output fits, as one plain launch.
bool mrg_server::launch_plain() {
    if (pending.empty() || free_events.empty()) return false;
    Ticket& t = tickets.at(pending.front());
    size_t off = 0;
    if (!pool.alloc(t.bytes, &off)) return false;
    t.pool_off = off;
    GenLaunch G{};
    G.streams = streams_dev + static_cast<size_t>(t.session) * S * 18;
    G.out = static_cast<char*>(cfg.pool) + off;
    G.S = S;
    G.q = t.n / S;
    G.r = static_cast<uint32_t>(t.n % S);
    G.dist = static_cast<int>(t.dist);
    G.dtype = static_cast<int>(t.dtype);
    G.param = t.dist == MRG_EXPONENTIAL ? 1.0 / t.param : 1.0;
    G.offset = t.offset;
    G.no_writeback = 1;
    plan_generate(G);
    hipError_t e = launch_generate(G, plain_stream);
    if (e == hipSuccess) {
        t.ev = free_events.back();
        free_events.pop_back();
        e = hipEventRecord(t.ev, plain_stream);
    }
    if (e != hipSuccess) {
        fail_hip(e, "plain launch");
        return false;
    }
    t.state = kInFlight;
    plain_inflight.push_back(pending.front());
    pending.pop_front();
    ++in_flight;
    st.max_in_flight = std::max<uint64_t>(st.max_in_flight, in_flight);
    ++st.launches;
    return true;
}

// After any activity the scheduler keeps polling (yielding its core) for
// this long before it sleeps on the condition variable: a request that
// arrives within the window is picked up without a thread wake-up.
constexpr uint64_t kSpinWindowNs = 2000000;

void mrg_server::loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    uint64_t last_active = steady_ns();
    while (!stop.load()) {
        bool progress = cfg.mode == 0 ? poll_lanes() : poll_plain();
        if (error == MRG_OK) {
            if (cfg.mode == 0) {
                for (Lane& L : lanes)
                    if (!L.busy && !pending.empty() && launch_batch(L)) progress = true;
            } else {
                while (launch_plain()) progress = true;
            }
        }
        st.pool_in_use = pool.in_use;
        st.pool_peak = pool.peak;
        if (progress) {
            cv.notify_all();
            last_active = steady_ns();
            continue;
        }
        if (in_flight || !pending.empty() || steady_ns() - last_active < kSpinWindowNs) {
            lk.unlock();  // something on the device or recently active: look again soon
            std::this_thread::yield();
            lk.lock();
        } else {
            cv.wait_for(lk, std::chrono::microseconds(50));
        }
    }
}

// ------------------------------------------------------------------ ABI
extern "C" {

uint64_t mrg_now_ns(void) { return steady_ns(); }

static void destroy_resources(mrg_server* s) {
    for (Lane& L : s->lanes) {
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        if (L.plan) mrg_batch_plan_destroy(L.plan);
        if (L.slots_host) (void)hipHostFree(L.slots_host);
        if (L.staging) (void)hipHostFree(L.staging);
        if (L.done_ev) (void)hipEventDestroy(L.done_ev);
        if (L.stream) (void)hipStreamDestroy(L.stream);
    }
    if (s->plain_stream) {
        (void)hipStreamSynchronize(s->plain_stream);
        (void)hipStreamDestroy(s->plain_stream);
    }
    for (auto& kv : s->tickets)
        if (kv.second.ev) (void)hipEventDestroy(kv.second.ev);
    for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
}

mrg_status mrg_server_workspace_size(const mrg_server_cfg* cfg, size_t* bytes) {
    if (!cfg || !bytes) return mrg355_fail(MRG_E_INVALID_ARG, "NULL cfg or bytes");
    if (mrg_status st = check_cfg(*cfg)) return st;
    *bytes = ws_layout(*cfg).total;
    return MRG_OK;
}

mrg_status mrg_server_create(const mrg_server_cfg* cfg, mrg_server** out) {
    if (!cfg || !out) return mrg355_fail(MRG_E_INVALID_ARG, "NULL cfg or server");
    if (mrg_status st = check_cfg(*cfg)) return st;
    if (!cfg->pool || cfg->pool_bytes < 256) return mrg355_fail(MRG_E_INVALID_ARG, "no output pool");
    if (reinterpret_cast<uintptr_t>(cfg->pool) % 256) return mrg355_fail(MRG_E_INVALID_ARG, "pool must be 256-byte aligned");
    const WsLayout W = ws_layout(*cfg);
    if (!cfg->workspace) return mrg355_fail(MRG_E_INVALID_ARG, "no device workspace");
    if (reinterpret_cast<uintptr_t>(cfg->workspace) % 256)
        return mrg355_fail(MRG_E_INVALID_ARG, "workspace must be 256-byte aligned");
    if (cfg->workspace_bytes < W.total)
        return mrg355_fail(MRG_E_NOMEM, "workspace holds %zu bytes, the server needs %zu", cfg->workspace_bytes,
                           W.total);
    {
        const uintptr_t p0 = reinterpret_cast<uintptr_t>(cfg->pool), p1 = p0 + cfg->pool_bytes;
        const uintptr_t w0 = reinterpret_cast<uintptr_t>(cfg->workspace), w1 = w0 + W.total;
        if (p0 < w1 && w0 < p1) return mrg355_fail(MRG_E_INVALID_ARG, "pool and workspace overlap");
    }
    mrg_creator cr;
    if (mrg_status st = mrg_creator_init(MRG_GEN_MRG32K3A, &cr, cfg->seed)) return st;

    mrg_server* s = new (std::nothrow) mrg_server();
    if (!s) return mrg355_fail(MRG_E_NOMEM, "server allocation failed");
    s->cfg = *cfg;
    s->cfg.streams_per_session = cfg_streams(*cfg);
    s->cfg.lanes = cfg_lanes(*cfg);
    s->cfg.max_batch = cfg_max_batch(*cfg);
    if (!s->cfg.tile_units) s->cfg.tile_units = 2048;
    const uint32_t S = s->cfg.streams_per_session;
    s->S = S;
    s->sess_off.assign(cfg->n_sessions, 0);
    s->pool.init(cfg->pool_bytes);
    hipError_t e = hipGetDevice(&s->device);

    // session streams: session i = streams i*S .. i*S+S-1 of one creator, at
    // the start of the caller's workspace
    char* ws = static_cast<char*>(cfg->workspace);
    s->streams_dev = reinterpret_cast<uint32_t*>(ws);
    const uint64_t n_streams = static_cast<uint64_t>(S) * cfg->n_sessions;
    if (e == hipSuccess) e = launch_create(kGen32k3a, s->streams_dev, n_streams, cr.s, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();

    // lanes: a batch workspace each (device, from the caller's buffer), and
    // the completion flags and table staging in pinned host memory, which
    // the library allocates here once
    s->lanes.resize(s->cfg.lanes);
    for (size_t i = 0; i < s->lanes.size(); ++i) {
        Lane& L = s->lanes[i];
        if (e != hipSuccess) break;
        L.ws = ws + W.streams_bytes + i * W.lane_bytes;
        L.ws_bytes = W.lane_bytes;
        e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void**>(&L.slots_host), s->cfg.max_batch * sizeof(BatchSlot),
                              hipHostMallocMapped | hipHostMallocCoherent);
        if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&L.slots_dev), L.slots_host, 0);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void**>(&L.staging), W.lane_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done_ev, hipEventDisableTiming);
    }
    if (e == hipSuccess && s->cfg.mode == 1) {
        e = hipStreamCreateWithFlags(&s->plain_stream, hipStreamNonBlocking);
        for (int i = 0; i < 4096 && e == hipSuccess; ++i) {
            hipEvent_t ev = nullptr;
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) s->free_events.push_back(ev);
        }
    }
    if (e != hipSuccess) {
        mrg_status st = mrg355_fail(MRG_E_HIP, "server setup: %s", hipGetErrorString(e));
        destroy_resources(s);
        delete s;
        return st;
    }
    s->th = std::thread([s] { s->loop(); });
    *out = s;
    return MRG_OK;
}

void mrg_server_destroy(mrg_server* s) {
    if (!s) return;
    s->stop.store(true);
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    destroy_resources(s);
    delete s;
}

mrg_status mrg_server_submit(mrg_server* s, uint32_t session, uint64_t n, mrg_dist dist, mrg_dtype dtype,
                             double param, uint64_t t_arrival_ns, uint64_t* ticket, uint64_t* offset_out) {
    if (!s || !ticket) return mrg355_fail(MRG_E_INVALID_ARG, "NULL server or ticket");
    if (session >= s->cfg.n_sessions) return mrg355_fail(MRG_E_INVALID_ARG, "no session %u", session);
    if (n == 0) return mrg355_fail(MRG_E_INVALID_ARG, "n must be at least 1");
    if (dist != MRG_UNIFORM && dist != MRG_NORMAL && dist != MRG_EXPONENTIAL && dist != MRG_RAW)
        return mrg355_fail(MRG_E_INVALID_ARG, "unknown distribution");
    if (dtype != MRG_F64 && dtype != MRG_F32 && dtype != MRG_U32)
        return mrg355_fail(MRG_E_INVALID_ARG, "unknown dtype");
    if ((dist == MRG_RAW) != (dtype == MRG_U32))
        return mrg355_fail(MRG_E_INVALID_ARG, "MRG_RAW pairs with MRG_U32 only");
    if (dist == MRG_EXPONENTIAL && !(std::isfinite(param) && param > 0.0))
        return mrg355_fail(MRG_E_INVALID_ARG, "exponential rate must be finite and > 0");
    const size_t bytes = static_cast<size_t>(n) * esz_of(dtype);
    if (n > (SIZE_MAX / 8) || round256(bytes) > s->pool.total) {
        std::lock_guard<std::mutex> g(s->mu);
        ++s->st.rejected;
        return mrg355_fail(MRG_E_NOMEM, "output of %zu bytes exceeds the pool", bytes);
    }
    std::lock_guard<std::mutex> g(s->mu);
    if (s->error) return mrg355_fail(s->error, "server stopped after an error");
    const uint64_t per = (n + s->S - 1) / s->S;
    const uint64_t steps = dist == MRG_NORMAL ? (per + 1) / 2 * 2 : per;
    Ticket t{};
    t.session = session;
    t.n = n;
    t.dist = dist;
    t.dtype = dtype;
    t.param = param;
    t.t_arrival = t_arrival_ns;
    t.offset = s->sess_off[session];
    t.bytes = bytes;
    t.state = kPending;
    s->sess_off[session] += steps;
    const uint64_t id = s->next_id++;
    s->tickets.emplace(id, t);
    s->pending.push_back(id);
    ++s->st.submitted;
    *ticket = id;
    if (offset_out) *offset_out = t.offset;
    s->cv.notify_all();
    return MRG_OK;
}

mrg_status mrg_server_poll(mrg_server* s, uint64_t ticket, int* done, void** dev_out, uint64_t* t_done_ns) {
    if (!s || !done) return mrg355_fail(MRG_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return mrg355_fail(MRG_E_INVALID_ARG, "unknown ticket");
    if (s->error) return mrg355_fail(s->error, "server stopped after an error");
    *done = it->second.state == kDone;
    if (!*done) return MRG_E_BUSY;
    if (dev_out) *dev_out = static_cast<char*>(s->cfg.pool) + it->second.pool_off;
    if (t_done_ns) *t_done_ns = it->second.t_done;
    return MRG_OK;
}

mrg_status mrg_server_release(mrg_server* s, uint64_t ticket) {
    if (!s) return mrg355_fail(MRG_E_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return mrg355_fail(MRG_E_INVALID_ARG, "unknown ticket");
    if (it->second.state != kDone) return mrg355_fail(MRG_E_INVALID_ARG, "request not complete");
    s->pool.release(it->second.pool_off, it->second.bytes);
    s->tickets.erase(it);
    ++s->st.released;
    s->cv.notify_all();
    return MRG_OK;
}

mrg_status mrg_server_stats_get(mrg_server* s, mrg_server_stats* out) {
    if (!s || !out) return mrg355_fail(MRG_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->st;
    out->pool_in_use = s->pool.in_use;
    out->pool_peak = s->pool.peak;
    return MRG_OK;
}

mrg_status mrg_server_drive(mrg_server* s, size_t n, const uint64_t* t_arrival_ns, const uint32_t* session,
                            const uint64_t* n_draws, mrg_dist dist, mrg_dtype dtype, double param,
                            uint64_t* latency_ns, uint64_t* span_ns) {
    if (!s || (n && (!t_arrival_ns || !session || !n_draws || !latency_ns)))
        return mrg355_fail(MRG_E_INVALID_ARG, "NULL argument");
    for (size_t i = 0; i < n; ++i) {
        if (session[i] >= s->cfg.n_sessions) return mrg355_fail(MRG_E_INVALID_ARG, "request %zu: bad session", i);
        if (i && t_arrival_ns[i] < t_arrival_ns[i - 1])
            return mrg355_fail(MRG_E_INVALID_ARG, "arrival times must not decrease");
    }
    std::unordered_map<uint64_t, size_t> index;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->collect = true;
        s->completions.clear();
    }
    const uint64_t t0 = steady_ns();
    uint64_t last = t0;
    size_t next = 0, finished = 0;
    mrg_status status = MRG_OK;
    while (finished < n && status == MRG_OK) {
        const uint64_t now = steady_ns();
        while (next < n && t0 + t_arrival_ns[next] <= now) {
            uint64_t id = 0;
            status = mrg_server_submit(s, session[next], n_draws[next], dist, dtype, param, t0 + t_arrival_ns[next],
                                       &id, nullptr);
            if (status) break;
            index[id] = next++;
        }
        if (status) break;
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->error) {
            status = mrg355_fail(s->error, "server stopped after an error");
            break;
        }
        while (!s->completions.empty()) {
            const uint64_t id = s->completions.front();
            s->completions.pop_front();
            auto ix = index.find(id);
            if (ix == index.end()) continue;  // submitted by someone else: theirs to release
            Ticket& t = s->tickets.at(id);
            latency_ns[ix->second] = t.t_done - t.t_arrival;
            last = std::max(last, t.t_done);
            s->pool.release(t.pool_off, t.bytes);
            s->tickets.erase(id);
            ++s->st.released;
            ++finished;
        }
        if (finished < n) {
            // Sleep (woken early by completions) while the next arrival is far
            // off; within 300 us of it, poll, so that requests are submitted
            // on time rather than a timer slack late.
            const uint64_t now2 = steady_ns();
            const uint64_t wake = next < n ? t0 + t_arrival_ns[next] : now2 + 200000;
            if (wake > now2 + 300000) {
                s->cv.wait_for(lk, std::chrono::nanoseconds(std::min<uint64_t>(wake - now2 - 300000, 200000)));
            } else {
                lk.unlock();
                std::this_thread::yield();
            }
        }
    }
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->collect = false;
    }
    if (span_ns) *span_ns = last - t0;
    return status;
}

}  // extern "C"
