// Continuous-batching server: reach_server_start / reach_submit / reach_poll.
//
// A persistent serving kernel keeps its waves resident; each wave claims the
// next ring sequence number from a device counter and waits for the host to
// publish a query there.  A host service thread admits submitted queries in
// submission order as soon as a slot and enough bytes of the caller's device
// pool are free (first fit), writes their boxes into the slot's pinned staging
// and publishes them into the ring (pinned, coherent host memory) at once; the
// wave that runs a query stages its box into the query's pool block and runs
// from there, and writes the result straight into pinned host result buffers.
// New queries thus start while earlier ones are still running on the GPU.
//
// While the persistent grid runs, the host issues no device work at all (no
// copies, no events): HIP gives work queued on another stream no promise of
// progress when the runtime maps that stream onto the hardware queue that
// holds the never-ending kernel (streams share a few hardware queues), so
// every step of serving is a host-memory exchange with the kernel.
//
// Client calls never wait on the service thread: reach_submit appends to an
// inbox and reach_poll / reach_cancel read an outbox, each under its own short
// lock; everything else (slots, pool, ring, streams) belongs to the service
// thread alone.  A query's latency runs from its arrival (the submit call, or
// the caller's arrival stamp with reach_submit_at) to the moment its box is in
// the caller's arrays.
//
// serve.mode = 1 replaces the persistent kernel by one kernel launch per
// admitted query (round-robin over 8 streams): the baseline the persistent
// path is measured against, with the same admission and accounting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/reach.h"
#include "kernels.hpp"

using namespace reach;

extern "C" int64_t reach_get_option(const reach_ctx* ctx, const char* key);

namespace {

using Clock = std::chrono::steady_clock;

double now_us() {
    return std::chrono::duration<double, std::micro>(Clock::now().time_since_epoch()).count();
}

struct Waiting {
    uint64_t ticket;
    reach_query q;        // host pointers of the caller (r_lo / r_hi written at completion)
    std::vector<double> lo, hi;
    double u_lo = 0, u_hi = 0;
    double t_arrive;
};

struct Running {
    bool used = false;
    bool published = false;    // visible to the kernel (mode 0) or launched (mode 1)
    bool cancel_req = false;   // reach_cancel arrived while it was admitted
    uint64_t ticket = 0;
    uint64_t seq = 0;          // ring sequence (mode 0)
    size_t pool_off = 0, pool_len = 0;
    int64_t n = 0;
    double* r_lo = nullptr;    // caller's result arrays
    double* r_hi = nullptr;
    double t_arrive = 0;
    hipEvent_t ev = nullptr;   // mode 1: completion event
    QDesc d{};
};

// first-fit allocator over [0, bytes)
struct Pool {
    std::map<size_t, size_t> free_;   // offset -> length
    void init(size_t bytes) { free_.clear(); if (bytes) free_[0] = bytes; }
    bool alloc(size_t len, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= len) {
                *off = it->first;
                size_t rest = it->second - len, o = it->first + len;
                free_.erase(it);
                if (rest) free_[o] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t len) {
        auto it = free_.emplace(off, len).first;
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

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// pinned staging per slot: inputs x_lo, x_hi, u_lo, u_hi (2 * 512 + 2 doubles,
// rounded up) and results r_lo at +0, r_hi at +512
constexpr size_t kInDoubles = 1040;
constexpr size_t kOutDoubles = 1024;

struct Done {
    uint64_t ticket;
    reach_status st;
    double lat_us;     // < 0: not counted (cancelled, timed out)
};

}  // namespace

namespace reach_srv {

struct Server {
    int device = 0;
    int mode = 0;
    hipStream_t kstream = nullptr;
    std::vector<hipStream_t> lstreams;   // mode 1: launch streams (inputs copied on them)
    char* pool = nullptr;
    size_t pool_bytes = 0;
    int32_t slots = 0;                 // concurrent queries
    int32_t ring_n = 0;                // ring entries
    ServeSlot* ring = nullptr;         // pinned host
    unsigned int* stop = nullptr;      // pinned host
    unsigned int* slot_words = nullptr;  // pinned host, mode 1: [slot] {flags, cancel}
    unsigned long long* dctl = nullptr;  // device: claim, status, watermark, grid quit
    double* stage_in = nullptr;        // pinned host, slots x kInDoubles
    double* stage_out = nullptr;       // pinned host, slots x kOutDoubles
    bool own_kstream = false;
    double last_probe_us = 0;
    double last_progress_us = 0;
    double drain_limit_us = 60.0e6;
    int64_t grid = 0;
    int64_t idle_cycles = 0;

    // inbox: client threads -> service thread
    std::mutex in_mu;
    std::condition_variable in_cv;
    std::deque<Waiting> incoming;
    std::vector<uint64_t> cancels;
    bool draining = false;
    bool quit = false;
    uint64_t next_ticket = 0;

    // outbox: service thread -> client threads
    std::mutex out_mu;
    std::unordered_map<uint64_t, reach_status> finished;
    std::unordered_set<uint64_t> known;   // submitted and not yet reported done
    std::vector<double> lat;

    // service thread only
    std::thread th;
    Pool alloc;
    std::deque<Waiting> waiting;
    std::vector<Running> run;
    std::vector<int32_t> free_slots;
    std::unordered_map<uint64_t, int32_t> slot_of;   // admitted ticket -> slot
    std::vector<uint64_t> ring_busy;   // per ring entry: sequence+1 occupying it, 0 = free
    uint64_t next_seq = 0;
    std::vector<Done> done_now;
};

}  // namespace reach_srv

using reach_srv::Server;

// The context struct is defined in runtime.cpp; the server pointer lives in
// a side table so the two translation units stay independent.
namespace {
std::mutex g_srv_mu;
std::unordered_map<const reach_ctx*, Server*> g_srv;

Server* srv_of(const reach_ctx* c) {
    std::lock_guard<std::mutex> g(g_srv_mu);
    auto it = g_srv.find(c);
    return it == g_srv.end() ? nullptr : it->second;
}

reach_status flags_to_status(unsigned f) {
    if (f & (unsigned)STATUS_CANCELLED) return REACH_E_CANCELLED;
    if (f & 1u) return REACH_E_NONFINITE;
    if (f & 2u) return REACH_E_ORDER;
    return REACH_OK;
}

// Release slot k and its resources (service thread).
void release(Server* S, int32_t k) {
    Running& r = S->run[k];
    S->alloc.release(r.pool_off, r.pool_len);
    if (S->mode == 0) {
        ServeSlot* sl = &S->ring[r.seq % S->ring_n];
        __atomic_store_n(&sl->seq, (unsigned long long)0, __ATOMIC_RELEASE);
        S->ring_busy[r.seq % S->ring_n] = 0;
    }
    S->slot_of.erase(r.ticket);
    r.used = false;
    r.published = false;
    r.cancel_req = false;
    S->free_slots.push_back(k);
}

// Complete the query in slot k with the kernel's status bits: copy its box to
// the caller (the two sides may have run in different waves, so lower <= upper
// is checked here) and queue its outcome for the outbox.
void finish(Server* S, int32_t k, unsigned flags) {
    Running& r = S->run[k];
    reach_status st;
    double lat = -1.0;
    if (flags & (unsigned)STATUS_CANCELLED) {
        st = REACH_E_CANCELLED;
    } else {
        const int64_t n = r.n;
        const double* lo = S->stage_out + (size_t)k * kOutDoubles;
        const double* hi = lo + 512;
        std::memcpy(r.r_lo, lo, sizeof(double) * n);
        std::memcpy(r.r_hi, hi, sizeof(double) * n);
        for (int64_t j = 0; j < n; ++j)
            if (lo[j] > hi[j]) flags |= 2u;
        st = flags_to_status(flags);
        lat = now_us() - r.t_arrive;
    }
    S->done_now.push_back({r.ticket, st, lat});
    release(S, k);
}

void flush_done(Server* S) {
    if (S->done_now.empty()) return;
    std::lock_guard<std::mutex> g(S->out_mu);
    for (const Done& d : S->done_now) {
        S->finished[d.ticket] = d.st;
        if (d.lat_us >= 0.0) S->lat.push_back(d.lat_us);
    }
    S->done_now.clear();
}

void launch_kernel(Server* S, uint64_t start_seq) {
    // claim counter (two work items per sequence) and watermark restart at
    // the next sequence to publish; the grid quit word is cleared
    unsigned long long init[4] = {2 * start_seq, 0, start_seq, 0};
    hipMemcpy(S->dctl, init, sizeof init, hipMemcpyHostToDevice);
    *(volatile unsigned int*)S->stop = 0u;
    launch_server(S->ring, S->ring_n, S->dctl, (volatile unsigned int*)S->stop,
                  (unsigned int*)(S->dctl + 1), S->idle_cycles, S->grid, S->kstream);
}

void publish(Server* S, int32_t k) {
    Running& r = S->run[k];
    ServeSlot* sl = &S->ring[r.seq % S->ring_n];
    sl->d = r.d;
    sl->d.cancel = &sl->cancel;
    sl->flags[0] = sl->flags[1] = 0;
    __atomic_store_n(&sl->cancel, r.cancel_req ? 1u : 0u, __ATOMIC_RELAXED);
    __atomic_store_n(&sl->done[0], (unsigned long long)0, __ATOMIC_RELAXED);
    __atomic_store_n(&sl->done[1], (unsigned long long)0, __ATOMIC_RELAXED);
    __atomic_store_n(&sl->seq, (unsigned long long)(r.seq + 1), __ATOMIC_RELEASE);
    r.published = true;
}

// Mode 0: the serving grid leaves as a whole after its idle limit.  Before new
// work is published, every admitted query that has not finished moves to a
// fresh sequence number (those already published are published again there)
// and a new grid starts at the first of them.
void revive_kernel(Server* S) {
    if (hipStreamQuery(S->kstream) != hipSuccess) return;   // still running
    const uint64_t start = S->next_seq;
    std::vector<int32_t> moved;
    for (int32_t k = 0; k < S->slots; ++k) {
        Running& r = S->run[k];
        if (!r.used) continue;
        if (r.published) {
            ServeSlot* old = &S->ring[r.seq % S->ring_n];
            __atomic_store_n(&old->seq, (unsigned long long)0, __ATOMIC_RELEASE);
        }
        S->ring_busy[r.seq % S->ring_n] = 0;
        moved.push_back(k);
    }
    std::sort(moved.begin(), moved.end(),
              [&](int32_t x, int32_t y) { return S->run[x].seq < S->run[y].seq; });
    for (int32_t k : moved) {
        Running& r = S->run[k];
        r.seq = S->next_seq++;
        S->ring_busy[r.seq % S->ring_n] = r.seq + 1;
        if (r.published) publish(S, k);
    }
    launch_kernel(S, start);
}

// Requests to cancel: a waiting query is dropped, an admitted one is stopped
// through its cancel word (the kernel reads it every kCancelEvery steps) or,
// if not yet published, completed without running.
void take_cancels(Server* S, const std::vector<uint64_t>& tickets) {
    for (uint64_t t : tickets) {
        bool dropped = false;
        for (auto it = S->waiting.begin(); it != S->waiting.end(); ++it) {
            if (it->ticket == t) {
                S->done_now.push_back({t, REACH_E_CANCELLED, -1.0});
                S->waiting.erase(it);
                dropped = true;
                break;
            }
        }
        if (dropped) continue;
        auto it = S->slot_of.find(t);
        if (it == S->slot_of.end()) continue;    // already finished
        Running& r = S->run[it->second];
        r.cancel_req = true;
        // an admitted query is always published (mode 0) or launched (mode
        // 1): its sequence is consumed, and its cancel word stops it
        if (S->mode == 0)
            __atomic_store_n(&S->ring[r.seq % S->ring_n].cancel, 1u, __ATOMIC_RELEASE);
        else
            __atomic_store_n(&S->slot_words[2 * it->second + 1], 1u, __ATOMIC_RELEASE);
    }
}

void service(Server* S) {
    hipSetDevice(S->device);
    std::vector<uint64_t> cancels;
    for (;;) {
        bool progress = false;
        bool quit = false;
        cancels.clear();
        {
            std::lock_guard<std::mutex> g(S->in_mu);
            while (!S->incoming.empty()) {
                S->waiting.push_back(std::move(S->incoming.front()));
                S->incoming.pop_front();
            }
            cancels.swap(S->cancels);
            quit = S->quit;
        }
        if (!cancels.empty()) {
            take_cancels(S, cancels);
            progress = true;
        }
        // 1. completions
        for (int32_t k = 0; k < S->slots; ++k) {
            Running& r = S->run[k];
            if (!r.used || !r.published) continue;
            if (S->mode == 0) {
                ServeSlot* sl = &S->ring[r.seq % S->ring_n];
                const uint64_t d0 = __atomic_load_n(&sl->done[0], __ATOMIC_ACQUIRE);
                const uint64_t d1 = __atomic_load_n(&sl->done[1], __ATOMIC_ACQUIRE);
                if (d0 == r.seq + 1 && d1 == r.seq + 1) {
                    const unsigned fl = __atomic_load_n(&sl->flags[0], __ATOMIC_ACQUIRE) |
                                        __atomic_load_n(&sl->flags[1], __ATOMIC_ACQUIRE);
                    finish(S, k, fl);
                    progress = true;
                }
            } else if (hipEventQuery(r.ev) == hipSuccess) {
                finish(S, k, __atomic_load_n(&S->slot_words[2 * k], __ATOMIC_ACQUIRE));
                progress = true;
            }
        }
        // 2. a grid that left on its idle limit is replaced before new work
        if (S->mode == 0) {
            bool inflight = false;
            for (int32_t k = 0; k < S->slots && !inflight; ++k) inflight = S->run[k].used;
            const double t = now_us();
            if ((!S->waiting.empty() && !S->free_slots.empty()) ||
                (inflight && t - S->last_probe_us > 1000.0)) {
                S->last_probe_us = t;
                revive_kernel(S);
            }
        }
        // 3. admission, in submission order
        while (!S->waiting.empty() && !S->free_slots.empty()) {
            Waiting& w = S->waiting.front();
            const int64_t n = w.q.sys.n;
            const size_t len = align256(sizeof(double) * (2 * (size_t)n + 2));
            if (S->mode == 0 && S->ring_busy[S->next_seq % S->ring_n] != 0) break;
            size_t off = 0;
            if (!S->alloc.alloc(len, &off)) break;
            const int32_t k = S->free_slots.back();
            S->free_slots.pop_back();
            Running& r = S->run[k];
            r.used = true;
            r.published = false;
            r.cancel_req = false;
            r.ticket = w.ticket;
            r.pool_off = off;
            r.pool_len = len;
            r.n = n;
            r.r_lo = (double*)w.q.r_lo;
            r.r_hi = (double*)w.q.r_hi;
            r.t_arrive = w.t_arrive;
            S->slot_of[w.ticket] = k;
            double* in = S->stage_in + (size_t)k * kInDoubles;
            std::memcpy(in, w.lo.data(), sizeof(double) * n);
            std::memcpy(in + n, w.hi.data(), sizeof(double) * n);
            in[2 * n] = w.u_lo;
            in[2 * n + 1] = w.u_hi;
            double* dlo = (double*)(S->pool + off);   // pool block: x_lo, x_hi, u_lo, u_hi
            QDesc& d = r.d;
            std::memset(&d, 0, sizeof d);
            d.kind = w.q.sys.kind;
            d.E = batch_cells_per_lane(n);
            d.n = n;
            d.nsteps = w.q.nsteps;
            kernel_params(w.q.sys.kind, w.q.sys.prm, d.prm);
            d.h2 = w.q.dt / 2.0; d.dt = w.q.dt; d.dt6 = w.q.dt / 6.0;
            d.r_lo = S->stage_out + (size_t)k * kOutDoubles;
            d.r_hi = S->stage_out + (size_t)k * kOutDoubles + 512;
            d.tag = k;
            if (S->mode == 0) {
                // the kernel reads the box from the slot's pinned staging and
                // parks it in the pool block
                d.x_lo = in; d.x_hi = in + n;
                if (w.q.sys.n_in == 1) { d.p_lo = in + 2 * n; d.p_hi = in + 2 * n + 1; }
                d.park = dlo;
                r.seq = S->next_seq++;
                S->ring_busy[r.seq % S->ring_n] = r.seq + 1;
                publish(S, k);
            } else {
                d.x_lo = dlo; d.x_hi = dlo + n;
                if (w.q.sys.n_in == 1) { d.p_lo = dlo + 2 * n; d.p_hi = dlo + 2 * n + 1; }
                hipStream_t cs = S->lstreams[k % S->lstreams.size()];
                hipMemcpyAsync(dlo, in, sizeof(double) * (2 * n + 2), hipMemcpyHostToDevice, cs);
                unsigned int* words = S->slot_words + 2 * k;
                __atomic_store_n(&words[0], 0u, __ATOMIC_RELAXED);
                __atomic_store_n(&words[1], 0u, __ATOMIC_RELEASE);
                d.cancel = &words[1];
                launch_single(d, nullptr, &words[0], cs);
                hipEventRecord(r.ev, cs);
                r.published = true;
            }
            S->waiting.pop_front();
            progress = true;
        }
        flush_done(S);
        bool busy = false;
        for (int32_t k = 0; k < S->slots && !busy; ++k) busy = S->run[k].used;
        if (quit && !busy && S->waiting.empty()) {
            std::lock_guard<std::mutex> g(S->in_mu);
            if (S->incoming.empty()) break;
            continue;
        }
        if (progress) S->last_progress_us = now_us();
        if (quit && now_us() - S->last_progress_us > S->drain_limit_us) {
            // bounded drain: whatever has not finished is reported as timed out
            std::lock_guard<std::mutex> g(S->out_mu);
            for (int32_t k = 0; k < S->slots; ++k) {
                Running& r = S->run[k];
                if (!r.used) continue;
                S->finished[r.ticket] = REACH_E_TIMEOUT;
                r.used = false;
            }
            for (auto& w : S->waiting) S->finished[w.ticket] = REACH_E_TIMEOUT;
            S->waiting.clear();
            break;
        }
        if (!progress) {
            if (busy || !S->waiting.empty()) {
                std::this_thread::yield();
            } else {
                std::unique_lock<std::mutex> lk(S->in_mu);
                if (S->incoming.empty() && S->cancels.empty() && !S->quit)
                    S->in_cv.wait_for(lk, std::chrono::microseconds(200));
            }
        }
    }
}

reach_status check_query(const reach_query* q) {
    const reach_system& s = q->sys;
    if (s.kind == REACH_HEAT3D) return REACH_E_UNSUPPORTED;   // served queries are chains
    if (s.kind != REACH_CTM && s.kind != REACH_RD && s.kind != REACH_LIN3) return REACH_E_INVAL;
    if (s.bc != REACH_BC_DEFAULT) return REACH_E_UNSUPPORTED;
    if (q->dtype != REACH_F64) return REACH_E_UNSUPPORTED;
    if (s.n < 1) return REACH_E_INVAL;
    if (s.n > 512) return REACH_E_UNSUPPORTED;
    if (s.n_in != 0 && s.n_in != 1) return REACH_E_UNSUPPORTED;
    if (s.kind == REACH_CTM && s.n_in != 0) return REACH_E_UNSUPPORTED;
    if (s.kind == REACH_RD && !(s.prm[0] > 0)) return REACH_E_INVAL;
    if (!(std::isfinite(q->dt) && q->dt > 0) || q->nsteps < 0) return REACH_E_INVAL;
    if (!q->x_lo || !q->x_hi || !q->r_lo || !q->r_hi) return REACH_E_INVAL;
    if (s.n_in == 1 && (!q->p_lo || !q->p_hi)) return REACH_E_INVAL;
    return REACH_OK;
}

}  // namespace

extern "C" {

double reach_clock_us(void) { return now_us(); }

reach_status reach_server_start(reach_ctx* c, void* pool, size_t pool_bytes, int32_t max_slots,
                                void* stream) {
    if (!c) return REACH_E_INVAL;
    if (srv_of(c)) return REACH_E_BUSY;
    if (!pool || pool_bytes < 256 || max_slots < 1 || max_slots > 65536) return REACH_E_INVAL;
    int dev = 0;
    hipGetDevice(&dev);
    Server* S = new Server();
    S->device = dev;
    S->mode = (int)reach_get_option(c, "serve.mode");
    S->pool = (char*)pool;
    S->pool_bytes = pool_bytes;
    S->alloc.init(pool_bytes);
    S->slots = max_slots;
    S->ring_n = std::max<int32_t>(4 * max_slots, 1024);
    S->kstream = (hipStream_t)stream;   // NULL: an internal stream is made below
    int cus = 256;
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t w = reach_get_option(c, "serve.waves");
    S->grid = w > 0 ? w : std::min<int64_t>((int64_t)cus * 4, 2 * (int64_t)max_slots);
    double idle_s = 120.0;
    if (const char* e = std::getenv("REACH_SERVER_IDLE_S")) idle_s = std::max(1.0, std::atof(e));
    int rate_khz = 0;   // wall_clock64 tick rate
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
        rate_khz <= 0)
        rate_khz = 100000;
    S->idle_cycles = (int64_t)(idle_s * 1000.0 * (double)rate_khz);
    bool ok = true;
    if (!S->kstream) {
        ok &= hipStreamCreateWithFlags(&S->kstream, hipStreamNonBlocking) == hipSuccess;
        S->own_kstream = true;
    }
    ok &= hipHostMalloc((void**)&S->ring, sizeof(ServeSlot) * S->ring_n,
                        hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess;
    ok &= hipHostMalloc((void**)&S->stop, 256, hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess;
    ok &= hipHostMalloc((void**)&S->slot_words, sizeof(unsigned int) * 2 * (size_t)max_slots,
                        hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess;
    ok &= hipHostMalloc((void**)&S->stage_in, sizeof(double) * kInDoubles * (size_t)max_slots,
                        hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess;
    ok &= hipHostMalloc((void**)&S->stage_out, sizeof(double) * kOutDoubles * (size_t)max_slots,
                        hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess;
    ok &= hipMalloc((void**)&S->dctl, 256) == hipSuccess;
    if (ok) {
        std::memset(S->ring, 0, sizeof(ServeSlot) * S->ring_n);
        std::memset(S->stop, 0, 256);
        std::memset(S->slot_words, 0, sizeof(unsigned int) * 2 * (size_t)max_slots);
        S->run.resize(max_slots);
        for (int32_t k = max_slots - 1; k >= 0; --k) S->free_slots.push_back(k);
        S->ring_busy.assign(S->ring_n, 0);
        if (S->mode == 1) {
            for (int i = 0; i < 8 && ok; ++i) {
                hipStream_t s;
                ok &= hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
                if (ok) S->lstreams.push_back(s);
            }
            for (auto& r : S->run)
                ok &= hipEventCreateWithFlags(&r.ev, hipEventDisableTiming) == hipSuccess;
            if (ok) ok &= hipMemset(S->dctl, 0, 256) == hipSuccess;
        } else {
            launch_kernel(S, 0);
            ok &= hipGetLastError() == hipSuccess;
        }
    }
    if (!ok) {
        // nothing launched that could still run: the kernel launch is the last step
        if (S->mode == 0 && S->stop) { *(volatile unsigned int*)S->stop = 1u; hipStreamSynchronize(S->kstream); }
        for (auto s : S->lstreams) hipStreamDestroy(s);
        for (auto& r : S->run) if (r.ev) hipEventDestroy(r.ev);
        if (S->ring) hipHostFree(S->ring);
        if (S->stop) hipHostFree(S->stop);
        if (S->slot_words) hipHostFree(S->slot_words);
        if (S->stage_in) hipHostFree(S->stage_in);
        if (S->stage_out) hipHostFree(S->stage_out);
        if (S->dctl) hipFree(S->dctl);
        if (S->own_kstream && S->kstream) hipStreamDestroy(S->kstream);
        delete S;
        return REACH_E_DEVICE;
    }
    S->last_progress_us = now_us();
    S->th = std::thread(service, S);
    std::lock_guard<std::mutex> g(g_srv_mu);
    g_srv[c] = S;
    return REACH_OK;
}

reach_status reach_submit_at(reach_ctx* c, const reach_query* q, double arrival_us,
                             uint64_t* ticket) {
    Server* S = c ? srv_of(c) : nullptr;
    if (!S) return REACH_E_BUSY;
    if (!q || !ticket || !std::isfinite(arrival_us)) return REACH_E_INVAL;
    reach_status st = check_query(q);
    if (st != REACH_OK) return st;
    const int64_t n = q->sys.n;
    const size_t len = align256(sizeof(double) * (2 * (size_t)n + 2));
    if (len > S->pool_bytes) return REACH_E_NOMEM;
    Waiting w;
    w.q = *q;
    w.lo.assign((const double*)q->x_lo, (const double*)q->x_lo + n);
    w.hi.assign((const double*)q->x_hi, (const double*)q->x_hi + n);
    if (q->sys.n_in == 1) { w.u_lo = *(const double*)q->p_lo; w.u_hi = *(const double*)q->p_hi; }
    w.t_arrive = arrival_us;
    uint64_t t;
    {
        std::lock_guard<std::mutex> g(S->out_mu);
        // the ticket is reserved here so that reach_poll knows it at once
        std::lock_guard<std::mutex> g2(S->in_mu);
        if (S->draining) return REACH_E_BUSY;
        t = S->next_ticket++;
        w.ticket = t;
        S->known.insert(t);
        S->incoming.push_back(std::move(w));
    }
    *ticket = t;
    S->in_cv.notify_one();
    return REACH_OK;
}

reach_status reach_submit(reach_ctx* c, const reach_query* q, uint64_t* ticket) {
    return reach_submit_at(c, q, now_us(), ticket);
}

reach_status reach_poll(reach_ctx* c, uint64_t ticket, reach_status* result) {
    Server* S = c ? srv_of(c) : nullptr;
    if (!S) return REACH_E_BUSY;
    std::lock_guard<std::mutex> g(S->out_mu);
    if (!S->known.count(ticket)) return REACH_E_INVAL;
    auto it = S->finished.find(ticket);
    if (it == S->finished.end()) return REACH_PENDING;
    if (result) *result = it->second;
    S->finished.erase(it);
    S->known.erase(ticket);
    return REACH_OK;
}

reach_status reach_cancel(reach_ctx* c, uint64_t ticket) {
    Server* S = c ? srv_of(c) : nullptr;
    if (!S) return REACH_E_BUSY;
    {
        std::lock_guard<std::mutex> g(S->out_mu);
        if (!S->known.count(ticket)) return REACH_E_INVAL;
        if (S->finished.count(ticket)) return REACH_E_BUSY;
    }
    {
        std::lock_guard<std::mutex> g(S->in_mu);
        S->cancels.push_back(ticket);
    }
    S->in_cv.notify_one();
    return REACH_OK;
}

reach_status reach_server_stats(reach_ctx* c, double* p50, double* p99, double* mx, int64_t* count) {
    Server* S = c ? srv_of(c) : nullptr;
    if (!S) return REACH_E_BUSY;
    std::vector<double> v;
    {
        std::lock_guard<std::mutex> g(S->out_mu);
        v = S->lat;
    }
    if (count) *count = (int64_t)v.size();
    if (v.empty()) {
        if (p50) *p50 = 0; if (p99) *p99 = 0; if (mx) *mx = 0;
        return REACH_OK;
    }
    std::sort(v.begin(), v.end());
    auto q = [&](double f) { return v[std::min(v.size() - 1, (size_t)std::floor(f * (v.size() - 1) + 0.5))]; };
    if (p50) *p50 = q(0.50);
    if (p99) *p99 = q(0.99);
    if (mx) *mx = v.back();
    return REACH_OK;
}

reach_status reach_server_stop(reach_ctx* c) {
    Server* S = c ? srv_of(c) : nullptr;
    if (!S) return REACH_E_BUSY;
    {
        std::lock_guard<std::mutex> g(S->in_mu);
        S->draining = true;
        S->quit = true;
        if (const char* e = std::getenv("REACH_SERVER_DRAIN_S"))
            S->drain_limit_us = std::max(1.0, std::atof(e)) * 1.0e6;
    }
    S->in_cv.notify_one();
    S->th.join();                    // every admitted and waiting query has completed
    *(volatile unsigned int*)S->stop = 1u;
    __atomic_thread_fence(__ATOMIC_SEQ_CST);
    hipSetDevice(S->device);
    hipError_t e = hipStreamSynchronize(S->kstream);
    for (auto s : S->lstreams) { hipStreamSynchronize(s); hipStreamDestroy(s); }
    for (auto& r : S->run) if (r.ev) hipEventDestroy(r.ev);
    hipHostFree(S->ring);
    hipHostFree(S->stop);
    hipHostFree(S->slot_words);
    hipHostFree(S->stage_in);
    hipHostFree(S->stage_out);
    hipFree(S->dctl);
    if (S->own_kstream) hipStreamDestroy(S->kstream);
    {
        std::lock_guard<std::mutex> g(g_srv_mu);
        g_srv.erase(c);
    }
    delete S;
    return e == hipSuccess ? REACH_OK : REACH_E_DEVICE;
}

__attribute__((visibility("hidden"))) void reach_server_destroy_internal(reach_ctx* c) {
    if (srv_of(c)) reach_server_stop(c);
}

}  // extern "C"
