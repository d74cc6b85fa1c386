// C-ABI runtime of the reachability library: argument validation, launch
// planning (tile shape, steps per HBM pass, ping-pong buffers), the batch
// path with its captured hipGraph, the one-launch-per-query baseline, the
// autotuner and the continuous-batching server.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <condition_variable>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/reach.h"
#include "kernels.hpp"

using namespace reach;

void reach::kernel_params(int kind, const double* prm, double out[5]) {
    for (int i = 0; i < 5; ++i) out[i] = 0.0;
    if (kind == REACH_CTM) {
        out[0] = prm[0]; out[1] = prm[1]; out[2] = prm[1] * prm[2]; out[3] = prm[3];
    } else if (kind == REACH_RD) {
        const double ih2 = 1.0 / (prm[0] * prm[0]);
        out[0] = ih2;
        out[1] = 2.0 * ih2;
    } else {
        out[0] = prm[0]; out[1] = prm[1]; out[2] = prm[2]; out[3] = prm[3];
    }
}

namespace {

constexpr int64_t kMaxN = (int64_t)1 << 40;
constexpr int64_t kBatchMaxN = 512;

struct GraphKey {
    int64_t nq;
    void* ws;
    void* staging;
    int64_t grid;
    hipStream_t stream;
    bool operator<(const GraphKey& o) const {
        return std::tie(nq, ws, staging, grid, stream) < std::tie(o.nq, o.ws, o.staging, o.grid, o.stream);
    }
};

struct TuneEntry { int E; int K; int S; };

}  // namespace

// Host worker threads kept for the life of a context (starting threads per
// call costs more than the work they share on a batch of 10^5 queries).
// run(nth, fn) calls fn(0) on the caller and fn(1 .. nth-1) on workers and
// returns when all have finished.  A batch plan runs five such phases back to
// back, so a worker that finishes one watches the job counter for up to
// kSpinUs before it sleeps on the condition variable (a wake-up from sleep
// costs tens of microseconds per phase), and the caller likewise watches for
// the last worker before it sleeps.  A worker that sees the new job while
// watching takes it without the mutex (the job is published before the
// counter, release / acquire), so that the workers of a phase do not queue on
// one lock.
class HostPool {
  public:
    explicit HostPool(int n) : n_(n) {
        for (int i = 1; i < n; ++i) th_.emplace_back([this, i] { loop(i); });
    }
    ~HostPool() {
        {
            std::lock_guard<std::mutex> g(m_);
            stop_.store(true, std::memory_order_relaxed);
            ++gen_;
            agen_.store(gen_, std::memory_order_release);
        }
        start_.notify_all();
        for (auto& t : th_) t.join();
    }
    int size() const { return n_; }
    void run(int nth, const std::function<void(int)>& fn) {
        if (nth <= 1 || n_ <= 1) {
            fn(0);
            return;
        }
        {
            std::lock_guard<std::mutex> g(m_);
            job_.store(&fn, std::memory_order_relaxed);
            job_n_.store(std::min(nth, n_), std::memory_order_relaxed);
            pending_.store(n_ - 1, std::memory_order_relaxed);
            ++gen_;
            agen_.store(gen_, std::memory_order_release);
        }
        start_.notify_all();
        fn(0);
        spin([&] { return pending_.load(std::memory_order_acquire) == 0; });
        std::unique_lock<std::mutex> lk(m_);
        done_.wait(lk, [&] { return pending_.load(std::memory_order_acquire) == 0; });
    }

  private:
    static constexpr int kSpinUs = 200;
    template <class P>
    static void spin(P&& ready) {
        const auto until = std::chrono::steady_clock::now() + std::chrono::microseconds(kSpinUs);
        while (!ready()) {
            for (int k = 0; k < 64 && !ready(); ++k) __builtin_ia32_pause();
            if (ready() || std::chrono::steady_clock::now() > until) return;
        }
    }
    void loop(int id) {
        uint64_t seen = 0;
        for (;;) {
            spin([&] { return agen_.load(std::memory_order_acquire) != seen; });
            uint64_t g = agen_.load(std::memory_order_acquire);
            if (g == seen) {
                std::unique_lock<std::mutex> lk(m_);
                start_.wait(lk, [&] { return gen_ != seen; });
                g = gen_;
            }
            seen = g;
            if (stop_.load(std::memory_order_acquire)) return;
            const std::function<void(int)>* job = job_.load(std::memory_order_relaxed);
            const int jn = job_n_.load(std::memory_order_relaxed);
            if (id < jn) (*job)(id);
            if (pending_.fetch_sub(1, std::memory_order_acq_rel) == 1) {
                std::lock_guard<std::mutex> g(m_);
                done_.notify_one();
            }
        }
    }
    int n_;
    std::vector<std::thread> th_;
    std::mutex m_;
    std::condition_variable start_, done_;
    std::atomic<const std::function<void(int)>*> job_{nullptr};
    std::atomic<int> job_n_{0};
    std::atomic<int> pending_{0};
    uint64_t gen_ = 0;               // under m_; agen_ mirrors it for watchers
    std::atomic<uint64_t> agen_{0};
    std::atomic<bool> stop_{false};
};

struct reach_ctx {
    int device = 0;
    int cus = 256;
    std::string arch;
    unsigned int* status = nullptr;      // device status word
    std::string err;
    std::map<std::string, int64_t> opt;
    // (kind, dtype, log2 n bucket, per-cell inputs)
    std::map<std::tuple<int, int, int, int>, TuneEntry> tune;
    std::map<std::pair<int, int>, int> batch_tune;        // (kind, log2 n bucket) -> pack E cap
    int64_t batch_waves[2] = {0, 0};                     // autotuned resident waves of the
                                                         // narrow / wide packing kernel (0 = none)
    int batch_cap = 0;                                   // autotuned pack E cap of all buckets (0 = none)
    int last_packed = 0;                                 // kernel of the last batch (launch_batch)
    // batch staging (pinned host) and graph cache
    QDesc* staging = nullptr;            // [nq] descriptors, [nq] items, item count
    int64_t staging_cap = 0;
    hipEvent_t staging_ev = nullptr;     // the last batch's uploads from the staging are done
    hipEvent_t batch_ev = nullptr;       // the last batch's kernel is done
    hipEvent_t block_ev[2] = {nullptr, nullptr};   // the last kernel that read workspace block b
    bool batch_ev_recorded = false;
    bool block_ev_recorded[2] = {false, false};
    int next_block = 0;                  // workspace block of the next batch
    void* last_ws = nullptr;             // workspace and query count of the last batch
    int64_t last_nq = 0;
    hipStream_t copy_stream = nullptr;   // batch uploads, beside the previous batch's kernel
    std::map<GraphKey, hipGraphExec_t> graphs;
    std::vector<hipStream_t> each_streams;
    bool log = false;                    // REACH_LOG: one JSON line per call on stderr
    std::unique_ptr<HostPool> pool;      // batch preparation threads (on first large batch)
};

namespace {

reach_status fail(reach_ctx* c, reach_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return st;
}

// One "reach: {...}" line on stderr when the context logs (REACH_LOG).
void log_call(const reach_ctx* c, const char* fmt, ...) {
    if (!c || !c->log) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "reach: {%s}\n", buf);
}

const char* dtype_name(reach_dtype d) { return d == REACH_F64 ? "f64" : "f32"; }

reach_status hip_fail(reach_ctx* c, hipError_t e, const char* what) {
    return fail(c, REACH_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(c, expr)                                          \
    do {                                                         \
        hipError_t _e = (expr);                                  \
        if (_e != hipSuccess) return hip_fail((c), _e, #expr);   \
    } while (0)

size_t dsize(reach_dtype d) { return d == REACH_F64 ? 8 : 4; }

int64_t opt_get(const reach_ctx* c, const char* k) {
    auto it = c->opt.find(k);
    return it == c->opt.end() ? 0 : it->second;
}

reach_status check_system_kind(reach_ctx* c, const reach_system* s, reach_dtype dtype,
                               bool user) {
    if (!s) return fail(c, REACH_E_INVAL, "system is NULL");
    if (s->bc != REACH_BC_DEFAULT)
        return fail(c, REACH_E_UNSUPPORTED, "bc = %d: only each kind's own boundary conditions "
                    "(REACH_BC_DEFAULT) are built", s->bc);
    if (s->kind == REACH_USER && !user)
        return fail(c, REACH_E_INVAL, "REACH_USER systems run through reach_embed_rk4_user");
    if (s->kind != REACH_CTM && s->kind != REACH_RD && s->kind != REACH_LIN3 &&
        s->kind != REACH_HEAT3D && s->kind != REACH_USER)
        return fail(c, REACH_E_INVAL, "unknown system kind %d", s->kind);
    if (user && s->kind != REACH_USER)
        return fail(c, REACH_E_INVAL, "reach_embed_rk4_user takes a REACH_USER system");
    if (dtype != REACH_F64 && dtype != REACH_F32) return fail(c, REACH_E_INVAL, "bad dtype %d", dtype);
    if (s->n < 1 || s->n >= kMaxN) return fail(c, REACH_E_INVAL, "n = %lld out of range", (long long)s->n);
    if (s->n_in != 0 && s->n_in != 1 && s->n_in != s->n)
        return fail(c, REACH_E_INVAL, "n_in must be 0, 1 or n");
    if (s->kind == REACH_CTM && s->n_in != 0)
        return fail(c, REACH_E_UNSUPPORTED, "the CTM chain takes no inputs");
    for (int i = 0; i < 8; ++i)
        if (!std::isfinite(s->prm[i])) return fail(c, REACH_E_INVAL, "parameter %d not finite", i);
    if (s->kind == REACH_RD && !(s->prm[0] > 0.0)) return fail(c, REACH_E_INVAL, "RD spacing h must be > 0");
    if (s->kind == REACH_HEAT3D) {
        if (s->n_in != 0) return fail(c, REACH_E_UNSUPPORTED, "the 3-D heat grid takes no inputs");
        int64_t prod = 1;
        for (int d = 0; d < 3; ++d) {
            const double g = s->prm[d];
            if (!(g >= 1.0 && g < 2147483648.0 && g == std::floor(g)))
                return fail(c, REACH_E_INVAL, "heat grid extent %d must be an integer in [1, 2^31)", d);
            prod *= (int64_t)g;
            if (prod > s->n) break;
        }
        if (prod != s->n) return fail(c, REACH_E_INVAL, "n must equal nx * ny * nz");
        if (!(s->prm[3] >= 0.0)) return fail(c, REACH_E_INVAL, "heat diffusivity must be >= 0");
        if (!(s->prm[4] > 0.0)) return fail(c, REACH_E_INVAL, "heat grid spacing must be > 0");
    }
    return REACH_OK;
}

reach_status check_system(reach_ctx* c, const reach_system* s, reach_dtype dtype) {
    return check_system_kind(c, s, dtype, false);
}

// Steps of every launch that only the chain kernels implement.
reach_status chains_only(reach_ctx* c, const reach_system* s, const char* what) {
    if (s->kind == REACH_HEAT3D)
        return fail(c, REACH_E_UNSUPPORTED, "%s runs the chain systems only", what);
    return REACH_OK;
}

void kernel_prm(const reach_system* s, double out[5]) { kernel_params(s->kind, s->prm, out); }

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

int ceil_pow2_E(int64_t n) {
    int E = 1;
    while ((int64_t)64 * E < n) E *= 2;
    return E;
}

// ------------------------------------------------------------ planning --
struct EmbedPlan {
    int E = 1;
    int S = 2;           // sides per wave
    int K = 1;           // steps per pass
    int64_t W = 1;       // tiles
    int64_t OUT = 0;
    int H = 0;
    int64_t passes = 1;
};

// Defaults measured on MI355X for the 2^26-cell chains (overridden by the
// autotuner or its cache).  Cooperative chains run one side per wave.
// Measured defaults per system, dtype, input mode (cell_in: per-cell inputs)
// and size.
TuneEntry default_tune(int kind, int dtype, bool cell_in, int64_t n) {
    if (kind == REACH_HEAT3D) return TuneEntry{2, 1, 1};   // rows per wave, 16 waves per block
    if (kind == REACH_LIN3) return dtype == REACH_F64 ? TuneEntry{12, 12, 2} : TuneEntry{16, 8, 2};
    if (dtype == REACH_F32) return TuneEntry{48, 12, 1};
    // RD with shared inputs fits 28 cells per lane in 256 VGPRs (the CTM
    // chain and per-cell inputs need more there).  The wider tile pays on
    // long chains (2^26: 1.5% faster); below that its fewer waves leave a
    // larger share of the last round empty (2^24: 5% slower than 24).
    if (kind == REACH_RD && !cell_in && n >= ((int64_t)1 << 26)) return TuneEntry{28, 24, 1};
    return TuneEntry{24, 20, 1};
}
int n_bucket(int64_t n) {
    int b = 0;
    while (((int64_t)1 << (b + 1)) <= n) ++b;
    return b;
}

TuneEntry tuned(const reach_ctx* c, int kind, int dtype, int64_t n, bool cell_in) {
    auto it = c->tune.find({kind, dtype, n_bucket(n), cell_in ? 1 : 0});
    if (it != c->tune.end()) return it->second;
    return default_tune(kind, dtype, cell_in, n);
}

int smallest_E(int kind, int dtype, int S, int64_t n) {
    for (int E : {1, 2, 4, 8, 12, 16, 24, 28, 32, 48, 64})
        if (embed_has_shape(kind, dtype, E, S) && (int64_t)64 * E >= n) return E;
    return 0;
}

reach_status plan_embed(reach_ctx* c, const reach_system* s, reach_dtype dtype, int64_t nsteps,
                        EmbedPlan* p) {
    const int64_t n = s->n;
    const int64_t oE = opt_get(c, "embed.E"), oK = opt_get(c, "embed.K"), oS = opt_get(c, "embed.S");
    const TuneEntry te = tuned(c, s->kind, dtype, n, s->n_in > 1);
    int S = oS ? (int)oS : (oE ? (s->kind == REACH_LIN3 ? 2 : te.S) : te.S);
    if (s->kind == REACH_LIN3 && S == 1)
        return fail(c, REACH_E_INVAL, "the coupled LIN3 chain needs both sides per wave");
    int E = oE ? (int)oE : 0;
    if (E && !embed_has_shape(s->kind, dtype, E, S))
        return fail(c, REACH_E_INVAL, "tile shape E = %d, S = %d not built", E, S);
    if (!E) {
        const int small = smallest_E(s->kind, dtype, S, n);
        E = (small && !oK) ? small : te.E;
        if (!embed_has_shape(s->kind, dtype, E, S)) E = embed_max_E(dtype, S);
    }
    p->E = E;
    p->S = S;
    const int64_t span = (int64_t)64 * E;
    if (n <= span && !oK) {
        // one window covers the chain: both ends are true boundaries, no halo
        p->K = (int)std::min<int64_t>(std::max<int64_t>(nsteps, 1), INT32_MAX);
        p->W = 1; p->OUT = 0; p->H = 0;
        p->passes = nsteps > 0 ? 1 : 0;
        return REACH_OK;
    }
    int K = oK ? (int)oK : te.K;
    if (K < 1) K = 1;
    if ((int64_t)8 * K >= span) return fail(c, REACH_E_INVAL, "K = %d too large for E = %d", K, E);
    if (!oK && nsteps > 0) {
        // the same number of passes with the steps spread evenly: a smaller
        // halo (e.g. 100 steps at K = 24 run as 5 passes of 20, not 4 x 24 + 4)
        const int64_t passes = (nsteps + K - 1) / K;
        K = (int)((nsteps + passes - 1) / passes);
    }
    p->K = K;
    p->H = 4 * K;
    p->OUT = span - 2 * p->H;
    p->W = (n <= span) ? 1 : 1 + (n - span + p->OUT - 1) / p->OUT;
    p->passes = (nsteps + K - 1) / K;
    return REACH_OK;
}

// ------------------------------------------------------------ 3-D heat --
struct HeatPlan {
    int P = 4, WV = 8;        // rows per wave, waves per block
    int OX = 0, OY = 0;       // output cells of a tile along x / y
    int64_t TX = 0, TY = 0;   // tiles per side along x / y
};

// Level j of a step: w <- y + cw[j] (s - 6 w), cw[j] = a dt / (4 - j)
// (the RK4 stability polynomial in nested form, see the heat kernel).
void heat_level_constants(HeatPass* a) {
    for (int l = 0; l < 4; ++l) {
        const double cl = a->a * a->dt / (double)(4 - l);
        a->cw[l] = cl;
        a->m6cw[l] = -6.0 * cl;
        a->cwf[l] = (float)cl;
        a->m6cwf[l] = (float)(-6.0 * cl);
    }
}

int heat_waves(int P) {
    return P == 4 ? 8 : P == 5 ? 8 : P == 2 ? 16 : P == 8 ? 4 : P == 3 ? 12 : 0;
}

reach_status plan_heat(reach_ctx* c, const reach_system* s, reach_dtype dtype, HeatPlan* p) {
    int P = (int)opt_get(c, "heat.P");
    if (!P) P = tuned(c, REACH_HEAT3D, dtype, s->n, false).E;
    const int WV = heat_waves(P);
    if (!WV || !heat_has_shape(dtype == REACH_F64 ? 0 : 1, P, WV))
        return fail(c, REACH_E_INVAL, "heat.P = %d not built for this dtype", P);
    p->P = P;
    p->WV = WV;
    p->OX = 64 - 8;
    p->OY = WV * P - 8;
    const int64_t nx = (int64_t)s->prm[0], ny = (int64_t)s->prm[1];
    p->TX = (nx + p->OX - 1) / p->OX;
    p->TY = (ny + p->OY - 1) / p->OY;
    return REACH_OK;
}

// Which buffer each of `passes` passes reads and writes: 0 = x, 1 = r,
// 2 = workspace.  The last pass writes r unless r aliases x and the pass
// count makes the ping-pong end in the workspace (then final_copy).
void plan_io(int64_t passes, bool inplace_ok, bool alias, std::vector<std::pair<int, int>>* io,
             bool* final_copy) {
    std::vector<int> dst(passes);
    *final_copy = false;
    if (inplace_ok) {
        for (auto& d : dst) d = 1;
    } else {
        for (int64_t p = passes - 1, k = 0; p >= 0; --p, ++k) dst[p] = (k % 2 == 0) ? 1 : 2;
        if (alias && dst[0] == 1) {
            for (int64_t p = 0; p < passes; ++p) dst[p] = (p % 2 == 0) ? 2 : 1;
            *final_copy = (dst[passes - 1] == 2);
        }
    }
    int src = 0;
    io->clear();
    for (int64_t p = 0; p < passes; ++p) {
        io->push_back({src, dst[p]});
        src = dst[p];
    }
}

reach_status embed_heat3d(reach_ctx* c, const reach_system* s, reach_dtype dtype,
                          const void* x_lo, const void* x_hi, double dt, int64_t nsteps,
                          void* r_lo, void* r_hi, void* ws, size_t ws_bytes, hipStream_t hs) {
    HeatPlan hp;
    reach_status st = plan_heat(c, s, dtype, &hp);
    if (st != REACH_OK) return st;
    log_call(c, "\"call\": \"embed\", \"kind\": %d, \"dtype\": \"%s\", \"n\": %lld, "
                "\"nsteps\": %lld, \"rows_per_wave\": %d, \"tiles\": %lld, \"passes\": %lld",
             s->kind, dtype_name(dtype), (long long)s->n, (long long)nsteps, hp.P,
             (long long)(2 * hp.TX * hp.TY), (long long)nsteps);
    const size_t bytes = (size_t)s->n * dsize(dtype);
    const bool alias = (r_lo == x_lo) || (r_hi == x_hi) || (r_lo == x_hi) || (r_hi == x_lo);
    const int64_t passes = nsteps;   // one RK4 step per pass
    const bool need_ws = passes >= 2 || alias;
    void *w_lo = nullptr, *w_hi = nullptr;
    if (need_ws) {
        if (!ws || ws_bytes < 2 * bytes)
            return fail(c, REACH_E_INVAL, "workspace of %zu bytes needed", 2 * bytes);
        w_lo = ws;
        w_hi = (char*)ws + bytes;
    }
    std::vector<std::pair<int, int>> io;
    bool final_copy = false;
    plan_io(passes, false, alias, &io, &final_copy);
    const void* lo_of[3] = {x_lo, r_lo, w_lo};
    const void* hi_of[3] = {x_hi, r_hi, w_hi};
    HeatPass a{};
    a.nx = (int64_t)s->prm[0]; a.ny = (int64_t)s->prm[1]; a.nz = (int64_t)s->prm[2];
    a.TX = (int32_t)hp.TX; a.TY = (int32_t)hp.TY; a.OX = hp.OX; a.OY = hp.OY;
    a.sides = 2;
    const int64_t tiles = 2 * hp.TX * hp.TY;
    a.per_xcd = (int32_t)((tiles + 7) / 8);
    a.a = s->prm[3] / (s->prm[4] * s->prm[4]);
    a.h2 = dt / 2.0; a.dt = dt; a.dt6 = dt / 6.0;
    heat_level_constants(&a);
    a.status = c->status;
    const int64_t grid = 8 * (int64_t)a.per_xcd;
    const int dt_id = dtype == REACH_F64 ? 0 : 1;
    for (int64_t p = 0; p < passes; ++p) {
        a.src[0] = lo_of[io[p].first];
        a.src[1] = hi_of[io[p].first];
        a.dst[0] = (void*)lo_of[io[p].second];
        a.dst[1] = (void*)hi_of[io[p].second];
        hipError_t e = launch_heat3d(dt_id, hp.P, hp.WV, a, grid, hs);
        if (e != hipSuccess) return hip_fail(c, e, "3-D heat kernel launch");
    }
    hipError_t e = launch_order_check(dt_id, lo_of[io.back().second], hi_of[io.back().second],
                                      s->n, c->status, hs);
    if (e != hipSuccess) return hip_fail(c, e, "order check launch");
    if (final_copy) {
        HIPCHK(c, hipMemcpyAsync(r_lo, w_lo, bytes, hipMemcpyDeviceToDevice, hs));
        HIPCHK(c, hipMemcpyAsync(r_hi, w_hi, bytes, hipMemcpyDeviceToDevice, hs));
    }
    return REACH_OK;
}

// Growth bound of the heat grid: the system is linear with non-negative
// couplings, so its own matrix is a contraction matrix and the half-width
// follows the heat equation too; both runs share each launch.
reach_status gb_heat3d(reach_ctx* c, const reach_system* s, reach_dtype dtype, const void* x_lo,
                       const void* x_hi, double dt, int64_t nsteps, void* r_lo, void* r_hi,
                       void* ws, hipStream_t hs) {
    HeatPlan hp;
    reach_status st = plan_heat(c, s, dtype, &hp);
    if (st != REACH_OK) return st;
    log_call(c, "\"call\": \"growth_bound\", \"kind\": %d, \"dtype\": \"%s\", \"n\": %lld, "
                "\"nsteps\": %lld, \"rows_per_wave\": %d, \"tiles\": %lld, \"passes\": %lld",
             s->kind, dtype_name(dtype), (long long)s->n, (long long)nsteps, hp.P,
             (long long)(2 * hp.TX * hp.TY), (long long)nsteps);
    const size_t bytes = (size_t)s->n * dsize(dtype);
    const int dt_id = dtype == REACH_F64 ? 0 : 1;
    char* A = (char*)ws;
    char* B = (char*)ws + 2 * bytes;
    hipError_t e = launch_center_radius(dt_id, x_lo, x_hi, s->n, B, B + bytes, hs);
    if (e != hipSuccess) return hip_fail(c, e, "center / radius launch");
    HeatPass a{};
    a.nx = (int64_t)s->prm[0]; a.ny = (int64_t)s->prm[1]; a.nz = (int64_t)s->prm[2];
    a.TX = (int32_t)hp.TX; a.TY = (int32_t)hp.TY; a.OX = hp.OX; a.OY = hp.OY;
    a.sides = 2;
    const int64_t tiles = 2 * hp.TX * hp.TY;
    a.per_xcd = (int32_t)((tiles + 7) / 8);
    a.a = s->prm[3] / (s->prm[4] * s->prm[4]);
    a.h2 = dt / 2.0; a.dt = dt; a.dt6 = dt / 6.0;
    heat_level_constants(&a);
    a.status = c->status;
    const int64_t grid = 8 * (int64_t)a.per_xcd;
    char* cur = B;
    for (int64_t p = 0; p < nsteps; ++p) {
        char* dst = (cur == A) ? B : A;
        a.src[0] = cur; a.src[1] = cur + bytes;
        a.dst[0] = dst; a.dst[1] = dst + bytes;
        e = launch_heat3d(dt_id, hp.P, hp.WV, a, grid, hs);
        if (e != hipSuccess) return hip_fail(c, e, "3-D heat kernel launch");
        cur = dst;
    }
    e = launch_gb_combine(dt_id, cur, cur + bytes, s->n, r_lo, r_hi, c->status, hs);
    if (e != hipSuccess) return hip_fail(c, e, "growth-bound combine launch");
    return REACH_OK;
}

void save_tune_entry(const reach_ctx* c, int kind, int dtype, int bucket, int cell_in, TuneEntry t,
                     double ps);

// Times every built (rows, waves) shape of the heat kernel, keeps the fastest.
reach_status autotune_heat3d(reach_ctx* c, const reach_system* s, reach_dtype dtype,
                             const void* x_lo, const void* x_hi, double dt, int64_t trial_steps,
                             void* r_lo, void* r_hi, void* ws, size_t ws_bytes, hipStream_t hs,
                             int64_t* best) {
    const int64_t saveP = opt_get(c, "heat.P");
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    double best_ps = 1e300;
    int bestP = 0;
    reach_status st = REACH_OK;
    for (int P : {2, 3, 4, 5, 8}) {
        if (!heat_has_shape(dtype == REACH_F64 ? 0 : 1, P, heat_waves(P))) continue;
        c->opt["heat.P"] = P;
        st = embed_heat3d(c, s, dtype, x_lo, x_hi, dt, trial_steps, r_lo, r_hi, ws, ws_bytes, hs);
        if (st != REACH_OK) break;
        if (hipEventRecord(e0, hs) != hipSuccess) { st = REACH_E_DEVICE; break; }
        for (int rep = 0; rep < 2 && st == REACH_OK; ++rep)
            st = embed_heat3d(c, s, dtype, x_lo, x_hi, dt, trial_steps, r_lo, r_hi, ws, ws_bytes,
                              hs);
        if (st != REACH_OK) break;
        if (hipEventRecord(e1, hs) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            st = REACH_E_DEVICE;
            break;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { st = REACH_E_DEVICE; break; }
        const double ps = (double)ms * 1e9 / (2.0 * 2.0 * (double)s->n * (double)trial_steps);
        if (ps < best_ps) { best_ps = ps; bestP = P; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    c->opt["heat.P"] = saveP;
    if (st != REACH_OK) return st;
    const int bucket = n_bucket(s->n);
    const TuneEntry bt{bestP, 1, 1};
    c->tune[{s->kind, dtype, bucket, 0}] = bt;
    save_tune_entry(c, s->kind, dtype, bucket, 0, bt, best_ps);
    best[0] = bestP;
    best[1] = 1;
    best[2] = (int64_t)std::llround(best_ps * 1000.0);
    best[3] = 1;
    return REACH_OK;
}

size_t embed_ws_bytes(reach_ctx* c, const reach_system* s, reach_dtype dtype) {
    if (s->kind == REACH_HEAT3D) return (size_t)2 * (size_t)s->n * dsize(dtype);
    EmbedPlan p;
    if (plan_embed(c, s, dtype, 2 * (int64_t)std::max(1, (int)opt_get(c, "embed.K")), &p) != REACH_OK)
        return (size_t)-1;
    if (p.W == 1) return 0;
    return (size_t)2 * (size_t)s->n * dsize(dtype);
}

// ------------------------------------------------------------- Monte Carlo
int mc_E(int dtype, int64_t n) {
    const int E = ceil_pow2_E(n);
    return E <= mc_max_E(dtype) ? E : -1;
}

int64_t mc_waves(const reach_ctx* c, int64_t m) {
    int64_t w = opt_get(c, "mc.waves");
    if (w <= 0) w = (int64_t)c->cus * 8;
    return std::max<int64_t>(1, std::min<int64_t>(std::min(w, kMcMaxWaves), m));
}

size_t mc_ws_bytes(const reach_ctx* c, const reach_system* s, reach_dtype dtype, int64_t m) {
    const int E = mc_E(dtype, s->n);
    if (E < 0) return (size_t)-1;
    return (size_t)2 * (size_t)mc_waves(c, m) * (size_t)(64 * E) * dsize(dtype);
}


// Autotune cache: one line per entry, each tagged with the format "reach2":
//   reach2 embed <arch> <kind> <dtype> <log2 n bucket> <per-cell inputs 0/1> <E> <K> <S> <ps per state-step>
//   reach2 batch <arch> <kind> <log2 n bucket> <pack E cap> <ns per batch>
// Lines of any other form (an older format without the input mode among
// them) are ignored.
void load_tune_cache(reach_ctx* c) {
    const char* path = std::getenv("REACH_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        char arch[64];
        int kind, dtype, bucket, cell, E, K, S, cap;
        double ps;
        if (std::sscanf(line, "reach2 embed %63s %d %d %d %d %d %d %d %lf", arch, &kind, &dtype,
                        &bucket, &cell, &E, &K, &S, &ps) == 9) {
            const bool heat_ok = kind == REACH_HEAT3D && heat_waves(E) &&
                                 heat_has_shape(dtype == REACH_F64 ? 0 : 1, E, heat_waves(E));
            if (c->arch == arch && (cell == 0 || cell == 1) &&
                (heat_ok || (embed_has_shape(kind, dtype, E, S) && K >= 1 && 8 * K < 64 * E)))
                c->tune[{kind, dtype, bucket, cell}] = TuneEntry{E, K, S};
        } else if (std::sscanf(line, "reach2 batch %63s %d %d %d %lf", arch, &kind, &bucket, &cap,
                               &ps) == 5) {
            const bool cap_ok = cap == 2 || cap == 4 || cap == 8 || cap == 16;
            if (c->arch == arch && cap_ok && kind == -1 && bucket == -1)
                c->batch_cap = cap;   // the whole batch's width
            else if (c->arch == arch && cap_ok)
                c->batch_tune[{kind, bucket}] = cap;
        }
    }
    std::fclose(f);
}

void save_tune_entry(const reach_ctx* c, int kind, int dtype, int bucket, int cell_in, TuneEntry t,
                     double ps) {
    const char* path = std::getenv("REACH_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "reach2 embed %s %d %d %d %d %d %d %d %.3f\n",
                 c->arch.empty() ? "unknown" : c->arch.c_str(), kind, dtype, bucket, cell_in, t.E,
                 t.K, t.S, ps);
    std::fclose(f);
}

void save_batch_tune_entry(const reach_ctx* c, int kind, int bucket, int cap, double ns) {
    const char* path = std::getenv("REACH_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "reach2 batch %s %d %d %d %.0f\n", c->arch.empty() ? "unknown" : c->arch.c_str(),
                 kind, bucket, cap, ns);
    std::fclose(f);
}
}  // namespace

// =================================================================== ABI ==

extern "C" {

reach_status reach_ctx_create(int device, reach_ctx** out) {
    if (!out) return REACH_E_INVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return REACH_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return REACH_E_DEVICE;
    reach_ctx* c = new reach_ctx();
    c->device = device;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->cus = cus;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        c->arch = prop.gcnArchName;
        const size_t colon = c->arch.find(':');
        if (colon != std::string::npos) c->arch.resize(colon);
    }
    load_tune_cache(c);
    // the no-allocation Monte Carlo's scratch address on this device (its
    // failure is reported by that entry point, not here)
    (void)noalloc_setup(device);
    if (const char* e = std::getenv("REACH_LOG")) c->log = e[0] && std::strcmp(e, "0") != 0;
    if (hipMalloc((void**)&c->status, 256) != hipSuccess) { delete c; return REACH_E_DEVICE; }
    if (hipMemset(c->status, 0, 256) != hipSuccess) { hipFree(c->status); delete c; return REACH_E_DEVICE; }
    if (hipEventCreateWithFlags(&c->staging_ev, hipEventDisableTiming) != hipSuccess) {
        hipFree(c->status); delete c; return REACH_E_DEVICE;
    }
    bool ok = hipEventCreateWithFlags(&c->batch_ev, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; k < 2 && ok; ++k)
        ok = hipEventCreateWithFlags(&c->block_ev[k], hipEventDisableTiming) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        for (hipEvent_t e : {c->staging_ev, c->batch_ev, c->block_ev[0], c->block_ev[1]})
            if (e) hipEventDestroy(e);
        hipFree(c->status);
        delete c;
        return REACH_E_DEVICE;
    }
    *out = c;
    return REACH_OK;
}

__attribute__((visibility("hidden"))) void reach_server_destroy_internal(reach_ctx* c);

void reach_ctx_destroy(reach_ctx* c) {
    if (!c) return;
    hipSetDevice(c->device);
    reach_server_destroy_internal(c);
    hipDeviceSynchronize();
    for (auto& kv : c->graphs) hipGraphExecDestroy(kv.second);
    for (auto s : c->each_streams) hipStreamDestroy(s);
    if (c->staging) hipHostFree(c->staging);
    if (c->staging_ev) hipEventDestroy(c->staging_ev);
    if (c->batch_ev) hipEventDestroy(c->batch_ev);
    for (hipEvent_t e : c->block_ev)
        if (e) hipEventDestroy(e);
    if (c->copy_stream) hipStreamDestroy(c->copy_stream);
    if (c->status) hipFree(c->status);
    c->pool.reset();
    delete c;
}

const char* reach_last_error(const reach_ctx* c) { return c ? c->err.c_str() : "no context"; }

reach_status reach_set_option(reach_ctx* c, const char* key, int64_t value) {
    if (!c || !key) return REACH_E_INVAL;
    static const char* keys[] = {"embed.K", "embed.E", "embed.S", "mc.waves", "batch.waves",
                                 "batch.split", "batch.pack", "batch.E",
                                 "serve.mode", "serve.waves", "gb.E", "gb.K", "heat.P",
                                 "user.E", "user.K"};
    bool known = false;
    for (const char* k : keys) known |= (std::strcmp(k, key) == 0);
    if (!known) return fail(c, REACH_E_INVAL, "unknown option %s", key);
    if (value < 0) return fail(c, REACH_E_INVAL, "option %s must be >= 0", key);
    if (!std::strcmp(key, "embed.E") && value && !embed_has_shape(REACH_CTM, REACH_F32, (int)value, 2) &&
        !embed_has_shape(REACH_CTM, REACH_F32, (int)value, 1) &&
        !embed_has_shape(REACH_CTM, REACH_F64, (int)value, 1))
        return fail(c, REACH_E_INVAL, "embed.E = %lld not built", (long long)value);
    if (!std::strcmp(key, "embed.S") && value != 0 && value != 1 && value != 2)
        return fail(c, REACH_E_INVAL, "embed.S must be 0, 1 or 2");
    if (!std::strcmp(key, "batch.pack") && value > 2)
        return fail(c, REACH_E_INVAL, "batch.pack must be 0 (auto), 1 (always) or 2 (never)");
    if (!std::strcmp(key, "batch.E") && value && value != 2 && value != 4 && value != 8 &&
        value != 16)
        return fail(c, REACH_E_INVAL, "batch.E must be 0, 2, 4, 8 or 16");
    if (!std::strcmp(key, "heat.P") && value && !heat_waves((int)value))
        return fail(c, REACH_E_INVAL, "heat.P must be 0, 2, 3, 4, 5 or 8");
    c->opt[key] = value;
    return REACH_OK;
}

int64_t reach_get_option(const reach_ctx* c, const char* key) {
    return (c && key) ? opt_get(c, key) : 0;
}

reach_status reach_plan_embed(reach_ctx* c, const reach_system* s, reach_dtype dtype,
                              int64_t nsteps, int64_t* out) {
    if (!c || !out) return REACH_E_INVAL;
    reach_status st = check_system(c, s, dtype);
    if (st != REACH_OK) return st;
    if (nsteps < 0) return fail(c, REACH_E_INVAL, "nsteps < 0");
    if (s->kind == REACH_HEAT3D) {
        HeatPlan hp;
        st = plan_heat(c, s, dtype, &hp);
        if (st != REACH_OK) return st;
        out[0] = hp.P; out[1] = 1; out[2] = hp.TX * hp.TY; out[3] = hp.OX; out[4] = 4;
        out[5] = nsteps; out[6] = 1;
        return REACH_OK;
    }
    EmbedPlan p;
    st = plan_embed(c, s, dtype, nsteps, &p);
    if (st != REACH_OK) return st;
    out[0] = p.E; out[1] = p.K; out[2] = p.W; out[3] = p.OUT; out[4] = p.H; out[5] = p.passes;
    out[6] = p.S;
    return REACH_OK;
}

size_t reach_workspace_bytes(reach_ctx* c, const reach_system* s, reach_dtype dtype, int64_t m) {
    if (!c || check_system(c, s, dtype) != REACH_OK || m < 0) return (size_t)-1;
    return m > 0 ? mc_ws_bytes(c, s, dtype, m) : embed_ws_bytes(c, s, dtype);
}

reach_status reach_sync(reach_ctx* c, void* stream) {
    if (!c) return REACH_E_INVAL;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
    unsigned int st = 0;
    HIPCHK(c, hipMemcpy(&st, c->status, sizeof st, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemset(c->status, 0, sizeof st));
    if (st & STATUS_NONFINITE) return fail(c, REACH_E_NONFINITE, "a result was not finite");
    if (st & STATUS_ORDER) return fail(c, REACH_E_ORDER, "a lower bound exceeded its upper bound");
    return REACH_OK;
}

reach_status reach_embed_rk4(reach_ctx* c, const reach_system* s, reach_dtype dtype,
                             const void* x_lo, const void* x_hi, const void* p_lo,
                             const void* p_hi, double t0, double dt, int64_t nsteps, void* r_lo,
                             void* r_hi, void* ws, size_t ws_bytes, void* stream) {
    if (!c) return REACH_E_INVAL;
    reach_status st = check_system(c, s, dtype);
    if (st != REACH_OK) return st;
    if (!x_lo || !x_hi || !r_lo || !r_hi) return fail(c, REACH_E_INVAL, "NULL state pointer");
    if (s->n_in > 0 && (!p_lo || !p_hi)) return fail(c, REACH_E_INVAL, "NULL input pointer");
    if (!(std::isfinite(dt) && dt > 0.0)) return fail(c, REACH_E_INVAL, "dt must be finite and > 0");
    if (!std::isfinite(t0)) return fail(c, REACH_E_INVAL, "t0 must be finite");
    if (nsteps < 0) return fail(c, REACH_E_INVAL, "nsteps < 0");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t hs = (hipStream_t)stream;
    const size_t bytes = (size_t)s->n * dsize(dtype);
    if (nsteps == 0) {
        if (r_lo != x_lo) HIPCHK(c, hipMemcpyAsync(r_lo, x_lo, bytes, hipMemcpyDeviceToDevice, hs));
        if (r_hi != x_hi) HIPCHK(c, hipMemcpyAsync(r_hi, x_hi, bytes, hipMemcpyDeviceToDevice, hs));
        return REACH_OK;
    }
    if (s->kind == REACH_HEAT3D)
        return embed_heat3d(c, s, dtype, x_lo, x_hi, dt, nsteps, r_lo, r_hi, ws, ws_bytes, hs);
    EmbedPlan pl;
    st = plan_embed(c, s, dtype, nsteps, &pl);
    if (st != REACH_OK) return st;
    log_call(c, "\"call\": \"embed\", \"kind\": %d, \"dtype\": \"%s\", \"n\": %lld, "
                "\"nsteps\": %lld, \"E\": %d, \"K\": %d, \"S\": %d, \"tiles\": %lld, "
                "\"passes\": %lld",
             s->kind, dtype_name(dtype), (long long)s->n, (long long)nsteps, pl.E, pl.K, pl.S,
             (long long)(pl.S == 1 ? 2 * pl.W : pl.W), (long long)pl.passes);

    // buffers: the last pass writes r; multi-tile passes never run in place
    const bool alias = (r_lo == x_lo) || (r_hi == x_hi) || (r_lo == x_hi) || (r_hi == x_lo);
    const bool inplace_ok = (pl.W == 1);
    const bool need_ws = !inplace_ok && (pl.passes >= 2 || alias);
    void *w_lo = nullptr, *w_hi = nullptr;
    if (need_ws) {
        if (!ws || ws_bytes < 2 * bytes)
            return fail(c, REACH_E_INVAL, "workspace of %zu bytes needed", 2 * bytes);
        w_lo = ws;
        w_hi = (char*)ws + bytes;
    }
    bool final_copy = false;
    std::vector<std::pair<int, int>> io;  // per pass: (src id, dst id); 0 = x, 1 = r, 2 = ws
    plan_io(pl.passes, inplace_ok, alias, &io, &final_copy);
    const void* lo_of[3] = {x_lo, r_lo, w_lo};
    const void* hi_of[3] = {x_hi, r_hi, w_hi};

    EmbedPass a{};
    a.p_lo = p_lo; a.p_hi = p_hi;
    a.n = s->n; a.W = pl.W; a.OUT = pl.OUT; a.H = pl.H;
    a.aligned = aligned16(x_lo) && aligned16(x_hi) && aligned16(r_lo) && aligned16(r_hi) &&
                (!need_ws || (aligned16(w_lo) && aligned16(w_hi)));
    const int64_t tiles = pl.S == 1 ? 2 * pl.W : pl.W;
    a.per_xcd = (int32_t)((tiles + 7) / 8);
    kernel_prm(s, a.prm);
    a.h2 = dt / 2.0; a.dt = dt; a.dt6 = dt / 6.0;
    a.status = c->status;
    const int mode = s->n_in > 1 ? 1 : 0;   // per-cell inputs
    if (s->n_in == 0) { a.p_lo = nullptr; a.p_hi = nullptr; }
    const int64_t grid = 8 * (int64_t)a.per_xcd;
    // one window, one side per wave: both waves in one block, which checks
    // the order itself
    const bool pair = pl.S == 1 && pl.W == 1;
    int64_t done = 0;
    for (int64_t p = 0; p < pl.passes; ++p) {
        a.src_lo = lo_of[io[p].first];
        a.src_hi = hi_of[io[p].first];
        a.dst_lo = (void*)lo_of[io[p].second];
        a.dst_hi = (void*)hi_of[io[p].second];
        a.ksteps = std::min<int64_t>(pl.K, nsteps - done);
        a.check = (p == pl.passes - 1) ? 1 : 0;
        // a one-step pass is a pure stream: its reads and writes bypass the
        // caches' retention (non-temporal), 1.8% faster at 2^26 cells
        a.nt = a.ksteps == 1 ? 1 : 0;
        hipError_t e = launch_embed(s->kind, mode, dtype == REACH_F64 ? 0 : 1, pl.E, pl.S, pair,
                                    a, grid, hs);
        if (e != hipSuccess) return hip_fail(c, e, "embedding kernel launch");
        done += a.ksteps;
    }
    if (pl.S == 1 && !pair) {
        hipError_t e = launch_order_check(dtype == REACH_F64 ? 0 : 1, lo_of[io.back().second],
                                          hi_of[io.back().second], s->n, c->status, hs);
        if (e != hipSuccess) return hip_fail(c, e, "order check launch");
    }
    if (final_copy) {
        HIPCHK(c, hipMemcpyAsync(r_lo, w_lo, bytes, hipMemcpyDeviceToDevice, hs));
        HIPCHK(c, hipMemcpyAsync(r_hi, w_hi, bytes, hipMemcpyDeviceToDevice, hs));
    }
    return REACH_OK;
}


reach_status reach_embed_rk4_tube(reach_ctx* c, const reach_system* s, reach_dtype dtype,
                                  const void* x_lo, const void* x_hi, const void* p_lo,
                                  const void* p_hi, double t0, double dt, int64_t nsteps,
                                  int64_t every, void* tube_lo, void* tube_hi, void* ws,
                                  size_t ws_bytes, void* stream) {
    if (!c) return REACH_E_INVAL;
    reach_status st = check_system(c, s, dtype);
    if (st != REACH_OK) return st;
    if (every < 1 || nsteps < 1 || nsteps % every != 0)
        return fail(c, REACH_E_INVAL, "nsteps must be a positive multiple of every");
    if (!tube_lo || !tube_hi) return fail(c, REACH_E_INVAL, "NULL tube pointer");
    const size_t bytes = (size_t)s->n * dsize(dtype);
    const int64_t slots = nsteps / every;
    const void* src_lo = x_lo;
    const void* src_hi = x_hi;
    for (int64_t k = 0; k < slots; ++k) {
        void* dlo = (char*)tube_lo + (size_t)k * bytes;
        void* dhi = (char*)tube_hi + (size_t)k * bytes;
        // each slot continues from the previous one: resumed runs are bitwise
        // the same as one run
        st = reach_embed_rk4(c, s, dtype, src_lo, src_hi, p_lo, p_hi, t0 + (double)(k * every) * dt,
                             dt, every, dlo, dhi, ws, ws_bytes, stream);
        if (st != REACH_OK) return st;
        src_lo = dlo;
        src_hi = dhi;
    }
    return REACH_OK;
}

reach_status reach_autotune_embed(reach_ctx* c, const reach_system* s, reach_dtype dtype,
                                  const void* x_lo, const void* x_hi, const void* p_lo,
                                  const void* p_hi, double dt, int64_t trial_steps, void* r_lo,
                                  void* r_hi, void* ws, size_t ws_bytes, void* stream,
                                  int64_t* best) {
    if (!c || !best) return REACH_E_INVAL;
    reach_status st = check_system(c, s, dtype);
    if (st != REACH_OK) return st;
    if (trial_steps < 1) return fail(c, REACH_E_INVAL, "trial_steps must be >= 1");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t hs = (hipStream_t)stream;
    if (s->kind == REACH_HEAT3D)
        return autotune_heat3d(c, s, dtype, x_lo, x_hi, dt, trial_steps, r_lo, r_hi, ws, ws_bytes,
                               hs, best);
    const int64_t saveE = opt_get(c, "embed.E"), saveK = opt_get(c, "embed.K");
    static const int Es[] = {4, 8, 12, 16, 24, 28, 32, 48, 64};
    static const int Ks[] = {2, 4, 6, 8, 10, 12, 16, 20, 24};
    const int64_t saveS = opt_get(c, "embed.S");
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    // picoseconds per state-step of one shape: `reps` timed calls of `steps`
    // steps after one untimed call, the fastest call counted (the least
    // disturbed by anything else on the device)
    auto time_shape = [&](const TuneEntry& t, int64_t steps, int reps, double* ps) -> reach_status {
        c->opt["embed.E"] = t.E;
        c->opt["embed.K"] = t.K;
        c->opt["embed.S"] = t.S;
        reach_status r = reach_embed_rk4(c, s, dtype, x_lo, x_hi, p_lo, p_hi, 0.0, dt, steps,
                                         r_lo, r_hi, ws, ws_bytes, stream);
        double best_ms = 1e300;
        for (int rep = 0; rep < reps && r == REACH_OK; ++rep) {
            if (hipEventRecord(e0, hs) != hipSuccess) return REACH_E_DEVICE;
            r = reach_embed_rk4(c, s, dtype, x_lo, x_hi, p_lo, p_hi, 0.0, dt, steps, r_lo, r_hi,
                                ws, ws_bytes, stream);
            if (hipEventRecord(e1, hs) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                return REACH_E_DEVICE;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return REACH_E_DEVICE;
            best_ms = std::min(best_ms, (double)ms);
        }
        *ps = best_ms * 1e9 / (2.0 * (double)s->n * (double)steps);
        return r;
    };
    // coarse scan of every built shape, then the four fastest and the default
    // shape again with ten times the steps
    std::vector<std::pair<double, TuneEntry>> scan;
    st = REACH_OK;
    for (int S : {2, 1})
    for (int E : Es) {
        if (st != REACH_OK) break;
        if (!embed_has_shape(s->kind, dtype, E, S) || (int64_t)64 * E >= 4 * s->n) continue;
        for (int K : Ks) {
            if (8 * K >= 64 * E) continue;
            double ps = 0;
            st = time_shape(TuneEntry{E, K, S}, trial_steps, 2, &ps);
            if (st != REACH_OK) break;
            scan.push_back({ps, TuneEntry{E, K, S}});
        }
    }
    double best_ps = 1e300;
    TuneEntry bt{0, 0, 0};
    if (st == REACH_OK && !scan.empty()) {
        std::stable_sort(scan.begin(), scan.end(),
                         [](const auto& a, const auto& b) { return a.first < b.first; });
        std::vector<TuneEntry> finals;
        for (size_t q = 0; q < scan.size() && q < 4; ++q) finals.push_back(scan[q].second);
        const TuneEntry d = default_tune(s->kind, dtype, s->n_in > 1, s->n);
        bool have_d = false;
        for (const auto& f : finals) have_d |= (f.E == d.E && f.K == d.K && f.S == d.S);
        for (const auto& q : scan)
            if (!have_d && q.second.E == d.E && q.second.K == d.K && q.second.S == d.S) {
                finals.push_back(d);
                have_d = true;
            }
        // the finals in three rounds, each shape once per round (a warm-up and
        // two timed calls), so that a drift of the clock over the trials
        // favours none of them; the measured default stays unless a shape
        // beats it by more than 2%: shapes within run-to-run noise of each
        // other (at 2^26 FP64 RD, K = 16, 20 and 24) would otherwise take
        // turns from run to run
        constexpr double kKeepDefault = 0.02;
        std::vector<double> fps(finals.size(), 1e300);
        for (int round = 0; round < 3 && st == REACH_OK; ++round)
            for (size_t k = 0; k < finals.size() && st == REACH_OK; ++k) {
                double ps = 0;
                st = time_shape(finals[k], 10 * trial_steps, 2, &ps);
                fps[k] = std::min(fps[k], ps);
            }
        double d_ps = 1e300;
        for (size_t k = 0; k < finals.size() && st == REACH_OK; ++k) {
            if (fps[k] < best_ps) { best_ps = fps[k]; bt = finals[k]; }
            if (finals[k].E == d.E && finals[k].K == d.K && finals[k].S == d.S) d_ps = fps[k];
        }
        if (st == REACH_OK && d_ps <= best_ps * (1.0 + kKeepDefault)) {
            best_ps = d_ps;
            bt = d;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    c->opt["embed.E"] = saveE;
    c->opt["embed.K"] = saveK;
    c->opt["embed.S"] = saveS;
    if (st != REACH_OK) return st;
    if (bt.E == 0) return fail(c, REACH_E_UNSUPPORTED, "n too small to tile: nothing to tune");
    const int bucket = n_bucket(s->n);
    const int cell_in = s->n_in > 1 ? 1 : 0;
    c->tune[{s->kind, dtype, bucket, cell_in}] = bt;
    save_tune_entry(c, s->kind, dtype, bucket, cell_in, bt, best_ps);
    best[0] = bt.E;
    best[1] = bt.K;
    best[2] = (int64_t)std::llround(best_ps * 1000.0);
    best[3] = bt.S;
    return REACH_OK;
}

reach_status reach_montecarlo_range(reach_ctx* c, const reach_system* s, reach_dtype dtype,
                                    const void* x_lo, const void* x_hi, const void* p_lo,
                                    const void* p_hi, double t0, double dt, int64_t nsteps,
                                    int64_t s0, int64_t m, uint64_t seed, void* r_min,
                                    void* r_max, void* ws, size_t ws_bytes, void* stream) {
    if (!c) return REACH_E_INVAL;
    reach_status st = check_system(c, s, dtype);
    if (st != REACH_OK) return st;
    st = chains_only(c, s, "Monte Carlo");
    if (st != REACH_OK) return st;
    if (!x_lo || !x_hi || !r_min || !r_max) return fail(c, REACH_E_INVAL, "NULL pointer");
    if (s->n_in > 0 && (!p_lo || !p_hi)) return fail(c, REACH_E_INVAL, "NULL input pointer");
    if (!(std::isfinite(dt) && dt > 0.0)) return fail(c, REACH_E_INVAL, "dt must be finite and > 0");
    if (!std::isfinite(t0)) return fail(c, REACH_E_INVAL, "t0 must be finite");
    if (nsteps < 0) return fail(c, REACH_E_INVAL, "nsteps < 0");
    if (m < 1) return fail(c, REACH_E_INVAL, "m must be >= 1");
    if (s0 < 0) return fail(c, REACH_E_INVAL, "s0 must be >= 0");
    const int E = mc_E(dtype, s->n);
    if (E < 0)
        return fail(c, REACH_E_UNSUPPORTED, "Monte Carlo holds a sample in one wave: n <= %d",
                    64 * mc_max_E(dtype));
    const size_t need = mc_ws_bytes(c, s, dtype, m);
    if (!ws || ws_bytes < need) return fail(c, REACH_E_INVAL, "workspace of %zu bytes needed", need);
    HIPCHK(c, hipSetDevice(c->device));
    McArgs a{};
    a.x_lo = x_lo; a.x_hi = x_hi; a.p_lo = p_lo; a.p_hi = p_hi;
    a.nw = mc_waves(c, m);
    a.part_min = ws;
    a.part_max = (char*)ws + need / 2;
    a.n = s->n; a.n_in = s->n_in; a.nsteps = nsteps; a.s0 = s0; a.m = m; a.seed = seed;
    a.aligned = 1;
    kernel_prm(s, a.prm);
    a.h2 = dt / 2.0; a.dt = dt; a.dt6 = dt / 6.0;
    const int mode = s->n_in > 1 ? 1 : 0;
    const int dt_id = dtype == REACH_F64 ? 0 : 1;
    hipStream_t hs = (hipStream_t)stream;
    log_call(c, "\"call\": \"montecarlo\", \"kind\": %d, \"dtype\": \"%s\", \"n\": %lld, "
                "\"nsteps\": %lld, \"s0\": %lld, \"m\": %lld, \"E\": %d, \"waves\": %lld",
             s->kind, dtype_name(dtype), (long long)s->n, (long long)nsteps, (long long)s0,
             (long long)m, E, (long long)a.nw);
    hipError_t e = launch_mc(s->kind, mode, dt_id, E, a, hs);
    if (e != hipSuccess) return hip_fail(c, e, "Monte Carlo kernel launch");
    e = launch_mc_reduce(dt_id, E, a.part_min, a.part_max, a.nw, mc_waves_per_group(), s->n, r_min,
                         r_max, c->status, hs);
    if (e != hipSuccess) return hip_fail(c, e, "Monte Carlo reduction launch");
    return REACH_OK;
}

reach_status reach_montecarlo(reach_ctx* c, const reach_system* s, reach_dtype dtype,
                              const void* x_lo, const void* x_hi, const void* p_lo,
                              const void* p_hi, double t0, double dt, int64_t nsteps, int64_t m,
                              uint64_t seed, void* r_min, void* r_max, void* ws, size_t ws_bytes,
                              void* stream) {
    return reach_montecarlo_range(c, s, dtype, x_lo, x_hi, p_lo, p_hi, t0, dt, nsteps, 0, m, seed,
                                  r_min, r_max, ws, ws_bytes, stream);
}

int64_t reach_mc_samples(int64_t n, double eps, double delta) {
    if (n < 1 || !(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 1.0)) return -1;
    const double nn = 2.0 * (double)n;
    const double m = std::ceil((nn / eps) * std::log(nn / delta));
    if (!(m < 9.0e18)) return -1;
    return (int64_t)m;
}

}  // extern "C"


// ---------------------------------------------------------- growth bound --
namespace {

void contraction_params(const reach_system* s, double out[5]) {
    for (int i = 0; i < 5; ++i) out[i] = 0.0;
    if (s->kind == REACH_CTM) {
        out[0] = s->prm[0]; out[1] = 0.0; out[2] = s->prm[1]; out[3] = 0.0;
    } else if (s->kind == REACH_RD) {
        const double h2 = s->prm[0] * s->prm[0];
        out[0] = 1.0 / h2; out[1] = -2.0 / h2; out[2] = 1.0 / h2; out[3] = 1.0;
    } else {
        out[0] = std::fabs(s->prm[0]); out[1] = s->prm[1]; out[2] = std::fabs(s->prm[2]);
        out[3] = std::fabs(s->prm[3]);
    }
}

}  // namespace

extern "C" {

size_t reach_growth_bound_workspace_bytes(reach_ctx* c, const reach_system* s, reach_dtype dtype) {
    if (!c || check_system(c, s, dtype) != REACH_OK) return (size_t)-1;
    return (size_t)4 * (size_t)s->n * dsize(dtype);
}

reach_status reach_growth_bound(reach_ctx* c, const reach_system* s, reach_dtype dtype,
                                const void* x_lo, const void* x_hi, const void* p_lo,
                                const void* p_hi, double t0, double dt, int64_t nsteps,
                                void* r_lo, void* r_hi, void* ws, size_t ws_bytes, void* stream) {
    if (!c) return REACH_E_INVAL;
    reach_status st = check_system(c, s, dtype);
    if (st != REACH_OK) return st;
    if (!x_lo || !x_hi || !r_lo || !r_hi) return fail(c, REACH_E_INVAL, "NULL state pointer");
    if (s->n_in > 0 && (!p_lo || !p_hi)) return fail(c, REACH_E_INVAL, "NULL input pointer");
    if (!(std::isfinite(dt) && dt > 0.0)) return fail(c, REACH_E_INVAL, "dt must be finite and > 0");
    if (!std::isfinite(t0)) return fail(c, REACH_E_INVAL, "t0 must be finite");
    if (nsteps < 0) return fail(c, REACH_E_INVAL, "nsteps < 0");
    const size_t bytes = (size_t)s->n * dsize(dtype);
    if (!ws || ws_bytes < 4 * bytes) return fail(c, REACH_E_INVAL, "workspace of %zu bytes needed", 4 * bytes);
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t hs = (hipStream_t)stream;
    if (s->kind == REACH_HEAT3D)
        return gb_heat3d(c, s, dtype, x_lo, x_hi, dt, nsteps, r_lo, r_hi, ws, hs);
    // plan: one side per wave, as the one-side embedding tiles
    int E = (int)opt_get(c, "gb.E");
    int K = (int)opt_get(c, "gb.K");
    if (E && !gb_has_E(E)) return fail(c, REACH_E_INVAL, "gb.E = %d not built", E);
    const int64_t n = s->n;
    bool single = false;
    if (!E) {
        for (int e : {1, 4, 8, 16, 24, 28, 32})
            if ((int64_t)64 * e >= n) { E = e; break; }
        if (E && !K) single = true;
        // FP64 with shared inputs fits 28 cells per lane in 256 VGPRs (two
        // waves per SIMD; per-cell inputs need more there), which pays on long
        // chains only (see default_tune)
        if (!E) E = dtype == REACH_F64 ? (s->n_in > 1 || n < ((int64_t)1 << 26) ? 24 : 28) : 32;
    } else if ((int64_t)64 * E >= n && !K) {
        single = true;
    }
    const int64_t span = (int64_t)64 * E;
    GbPass a{};
    a.x_lo = x_lo; a.x_hi = x_hi;
    a.p_lo = s->n_in ? p_lo : nullptr;
    a.p_hi = s->n_in ? p_hi : nullptr;
    a.n = n;
    kernel_prm(s, a.prm);
    contraction_params(s, a.prm_r);
    a.h2 = dt / 2.0; a.dt = dt; a.dt6 = dt / 6.0;
    int64_t passes;
    if (single) {
        K = (int)std::min<int64_t>(std::max<int64_t>(nsteps, 1), INT32_MAX);
        a.W = 1; a.OUT = 0; a.H = 0;
        passes = 1;
    } else {
        // steps per pass, measured on the 2^26 RD chain (FP64, 1000 steps): at
        // E = 24, K = 20 (104.1 ms; K = 12 is 5% slower, K = 24 ties); at E = 28,
        // K = 24 (101.1 ms against 102.3 at K = 20 and 104.1 at K = 16)
        if (!K) K = E == 28 ? 24 : 20;
        if ((int64_t)8 * K >= span) return fail(c, REACH_E_INVAL, "gb.K = %d too large for E = %d", K, E);
        a.H = 4 * K;
        a.OUT = span - 2 * a.H;
        a.W = (n <= span) ? 1 : 1 + (n - span + a.OUT - 1) / a.OUT;
        passes = std::max<int64_t>(1, (nsteps + K - 1) / K);
    }
    a.per_xcd = (int32_t)((2 * a.W + 7) / 8);
    const int64_t grid = 8 * (int64_t)a.per_xcd;
    log_call(c, "\"call\": \"growth_bound\", \"kind\": %d, \"dtype\": \"%s\", \"n\": %lld, "
                "\"nsteps\": %lld, \"E\": %d, \"K\": %d, \"tiles\": %lld, \"passes\": %lld",
             s->kind, dtype_name(dtype), (long long)n, (long long)nsteps, E, K,
             (long long)(2 * a.W), (long long)passes);
    // (c, r) ping-pong in the workspace; the last pass writes buffer A
    char* A = (char*)ws;
    char* B = (char*)ws + 2 * bytes;
    const int mode = s->n_in > 1 ? 1 : 0;
    const int dt_id = dtype == REACH_F64 ? 0 : 1;
    int64_t done = 0;
    for (int64_t p = 0; p < passes; ++p) {
        char* dst = ((passes - 1 - p) % 2 == 0) ? A : B;
        char* src = ((passes - 1 - p) % 2 == 0) ? B : A;
        a.first = (p == 0) ? 1 : 0;
        a.src_c = src; a.src_r = src + bytes;
        a.dst_c = dst; a.dst_r = dst + bytes;
        a.ksteps = std::min<int64_t>(K, nsteps - done);
        hipError_t e = launch_gb(s->kind, mode, dt_id, E, a, grid, hs);
        if (e != hipSuccess) return hip_fail(c, e, "growth-bound kernel launch");
        done += a.ksteps;
    }
    hipError_t e = launch_gb_combine(dt_id, A, A + bytes, n, r_lo, r_hi, c->status, hs);
    if (e != hipSuccess) return hip_fail(c, e, "growth-bound combine launch");
    return REACH_OK;
}

}  // extern "C"

// ================================================================ batch ==

namespace {

reach_status make_desc(reach_ctx* c, const reach_query& q, int64_t tag, QDesc* d) {
    reach_status st = check_system(c, &q.sys, q.dtype);
    if (st != REACH_OK) return st;
    st = chains_only(c, &q.sys, "the batch path");
    if (st != REACH_OK) return st;
    if (q.dtype != REACH_F64) return fail(c, REACH_E_UNSUPPORTED, "batched queries are FP64");
    if (q.sys.n > kBatchMaxN) return fail(c, REACH_E_UNSUPPORTED, "batched queries need n <= 512");
    if (q.sys.n_in > 1) return fail(c, REACH_E_UNSUPPORTED, "batched queries take n_in 0 or 1");
    if (!(std::isfinite(q.dt) && q.dt > 0.0)) return fail(c, REACH_E_INVAL, "dt must be finite and > 0");
    if (!std::isfinite(q.t0)) return fail(c, REACH_E_INVAL, "t0 must be finite");
    if (q.nsteps < 0) return fail(c, REACH_E_INVAL, "nsteps < 0");
    if (!q.x_lo || !q.x_hi || !q.r_lo || !q.r_hi) return fail(c, REACH_E_INVAL, "NULL state pointer");
    if (q.sys.n_in == 1 && (!q.p_lo || !q.p_hi)) return fail(c, REACH_E_INVAL, "NULL input pointer");
    std::memset(d, 0, sizeof *d);
    d->kind = q.sys.kind;
    d->E = batch_cells_per_lane(q.sys.n);
    d->n = q.sys.n;
    d->nsteps = q.nsteps;
    kernel_prm(&q.sys, d->prm);
    d->h2 = q.dt / 2.0; d->dt = q.dt; d->dt6 = q.dt / 6.0;
    d->x_lo = (const double*)q.x_lo; d->x_hi = (const double*)q.x_hi;
    d->r_lo = (double*)q.r_lo; d->r_hi = (double*)q.r_hi;
    d->tag = tag;
    if (q.sys.n_in == 1) {
        d->p_lo = (const double*)q.p_lo;
        d->p_hi = (const double*)q.p_hi;
    }
    return REACH_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Host threads for preparing a batch of nq queries (1 below 16384 queries,
// at most kMaxHostThreads).
constexpr int64_t kMaxHostThreads = 16;
int batch_host_threads(int64_t nq) {
    if (nq < 16384) return 1;
    const unsigned hw = std::thread::hardware_concurrency();
    const int64_t by_size = nq / 4096;
    return (int)std::max<int64_t>(
        1, std::min<int64_t>({by_size, kMaxHostThreads, hw ? (int64_t)hw : 1}));
}

// fn(t) for t in [0, nth): t = 0 on the calling thread, the rest on the pool's
// workers (nth <= the pool's size; without a pool nth must be 1).
template <class F>
void run_threads(HostPool* pool, int nth, F&& fn) {
    if (nth <= 1 || !pool) {
        for (int t = 0; t < nth; ++t) fn(t);
        return;
    }
    pool->run(nth, std::function<void(int)>(fn));
}

// fn(u) for every u in [0, nu) on nth threads, each thread taking the next
// unclaimed u: a thread the system holds back delays only the unit it holds,
// and the outputs, kept per unit, do not depend on which thread ran which.
template <class F>
void run_units(HostPool* pool, int nth, int nu, F&& fn) {
    std::atomic<int> next{0};
    run_threads(pool, std::min(nth, nu), [&](int) {
        for (int u = next.fetch_add(1); u < nu; u = next.fetch_add(1)) fn(u);
    });
}

// The context's pool, started on first use with batch_host_threads' maximum.
HostPool* host_pool(reach_ctx* c) {
    if (!c) return nullptr;
    if (!c->pool) {
        const unsigned hw = std::thread::hardware_concurrency();
        c->pool.reset(new HostPool(
            (int)std::max<int64_t>(1, std::min<int64_t>(kMaxHostThreads, hw ? hw : 1))));
    }
    return c->pool.get();
}

// Descriptors (the caller's order), work items, the item count and the items'
// query indices, uploaded as one block.
size_t batch_block_bytes(int64_t nq) {
    return (sizeof(QDesc) + sizeof(BatchItem) + sizeof(uint32_t)) * (size_t)nq + sizeof(uint64_t);
}
struct BatchBlock {
    QDesc* desc;
    BatchItem* items;
    uint64_t* count;
    uint32_t* members;
};
BatchBlock batch_block(void* base, int64_t nq) {
    BatchBlock b;
    b.desc = (QDesc*)base;
    b.items = (BatchItem*)(b.desc + nq);
    b.count = (uint64_t*)(b.items + nq);
    b.members = (uint32_t*)(b.count + 1);
    return b;
}

// 1/16-octave class of a wave time, larger for shorter work (the launch
// order takes classes in increasing order: longest first).
int wave_time_bucket(uint64_t cost) {
    constexpr int kBuckets = 64 * 16;
    const uint64_t c1 = cost + 1u;      // never 0
    const int msb = 63 - __builtin_clzll(c1);
    const int frac = msb >= 4 ? (int)((c1 >> (msb - 4)) & 15u) : (int)((c1 << (4 - msb)) & 15u);
    return kBuckets - 1 - (msb * 16 + frac);
}

// Segment packing of a batch.  A query of n cells in a pack at E cells per
// lane takes L = ceil(n / E) lanes and needs the balanced layout
// n >= (E - 1) L; its estimated issue cost per cell is (kCellOps + kSegLaneOps
// / E) L E / n (arithmetic per cell and stage, plus the lane shifts and
// boundary selects per lane and stage, over the cells the lanes hold).
// seg_E picks the cheapest E of kSegE up to cap (ties to the wider), or the
// narrowest valid E above cap when none up to it is valid.
constexpr double kCellOps = 6.0, kSegLaneOps = 12.0;
// Default cap on E before the batch autotuner has run.
constexpr int kSegECap = 16;

int seg_E(int64_t n, int cap) {
    double best = 1e300;
    int bestE = 0, above = 0;
    for (int E : kSegE) {
        const int64_t L = (n + E - 1) / E;
        if (L > 64 || n < (int64_t)(E - 1) * L) continue;
        if (E > cap) {
            if (!above) above = E;
            continue;
        }
        const double cost = (kCellOps + kSegLaneOps / E) * (double)(L * E) / (double)n;
        if (cost <= best) { best = cost; bestE = E; }
    }
    return bestE ? bestE : above;
}

// Whether a batch packs: option batch.pack 1 always, 2 never, 0 (default)
// when it has more queries than twice the resident waves (below that every
// query gets a wave of its own and packing would only lengthen the longest).
bool batch_packs(const reach_ctx* c, int64_t nq) {
    const int64_t mode = c ? opt_get(c, "batch.pack") : 0;
    if (mode == 1) return true;
    if (mode == 2) return false;
    int64_t waves = c ? opt_get(c, "batch.waves") : 0;
    if (waves <= 0) waves = (int64_t)(c ? c->cus : 256) * 8;
    return nq > 2 * waves;
}

// Largest cells per lane of a pack for (kind, size bucket): option batch.E,
// else the bucket's autotuned cap, else the autotuned cap of the whole batch
// (reach_autotune_batch), else kSegECap.
int batch_ecap(const reach_ctx* c, int kind, int bucket) {
    if (c) {
        const int64_t e = opt_get(c, "batch.E");
        if (e > 0) return (int)e;
        auto it = c->batch_tune.find({kind, bucket});
        if (it != c->batch_tune.end()) return it->second;
        if (c->batch_cap) return c->batch_cap;
    }
    return kSegECap;
}

// The schedule of a batch: the descriptors descs[nq] in the caller's order
// and the work items in launch order (items[k] covers members[start .. start
// + count), indices into q, contiguous in launch order).
//
// Two parallel passes over nu work units (up to two per thread, claimed
// dynamically; every output is kept per unit, so the plan does not depend on
// which thread ran which unit).  First each unit reads a contiguous chunk of
// the caller's array once: it validates every query (without touching the
// context; the first bad query, lowest index, is re-checked with the context
// afterwards to set the error message).  When the batch does not pack
// (batch_packs), every query is an item of its own, run alone over a whole
// wave.  When it packs, every item is a segment pack, and each query gets a
// pack key: its constants class (bitwise equal kind, dt and parameters),
// cells per lane E (seg_E under the bucket's cap) and 1/16-octave step
// bucket.  Then unit u owns the keys of the (E, bucket) pairs r with r mod
// nu = u and scans the queries of its keys in caller order, placing each in
// the first of up to kOpen open packs of its key with room (at most 64 lanes
// and kPackMax queries; when none has room the fullest is closed); the packs
// still open at the end are packed again per key, widest query first into
// the first pack with room.  Items are then ordered longest first by the wave
// time (E * steps of the longest member; ceil(n / 64) * steps alone) at 1/16
// octave, ties in unit order.
struct PlanTimes {
    double pass1_ms = 0, pass_ms = 0, order_ms = 0, members_ms = 0;
};

reach_status plan_batch(reach_ctx* c, HostPool* pool, const reach_query* q, int64_t nq,
                        int split, int nth, QDesc* descs, std::vector<uint32_t>* members_out,
                        std::vector<BatchItem>* items_out, int* packed,
                        PlanTimes* times = nullptr,
                        const std::function<void()>& descs_done = nullptr) {
    using clk = std::chrono::steady_clock;
    auto since = [](clk::time_point t0) {
        return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    };
    auto t0 = clk::now();
    int nu = 1;   // work units (set below)
    auto chunk = [&](int t, int64_t total, int64_t* lo, int64_t* hi) {
        *lo = total * t / nu;
        *hi = total * (t + 1) / nu;
    };
    constexpr int kBuckets = 64 * 16;
    constexpr int kLanes = 64;
    constexpr int kOpen = 8;             // open packs per key
    constexpr int kNE = (int)(sizeof(kSegE) / sizeof(kSegE[0]));
    constexpr int kNB = 10;              // size buckets floor(log2 n), n <= 512
    constexpr int kMaxClasses = 16;      // per thread (4 bits of a key); further classes run alone
    struct Item {
        uint32_t first;    // into the thread's member list
        uint16_t count;
        uint16_t E;
        int16_t bucket;
    };
    struct Consts {
        int32_t kind;
        double dt;
        double prm[8];
        bool operator==(const Consts& o) const {
            return kind == o.kind && std::memcmp(&dt, &o.dt, sizeof dt) == 0 &&
                   std::memcmp(prm, o.prm, sizeof prm) == 0;
        }
    };
    struct Open {
        int lanes = 0;
        int count = 0;
        int E = 0;
        int64_t max_steps = 0;
        uint32_t mem[kPackMax];
    };
    const bool packs = !split && batch_packs(c, nq);
    *packed = packs ? 1 : 0;
    int ecap[4][kNB];
    for (int k = 0; k < 4; ++k)
        for (int b = 0; b < kNB; ++b) ecap[k][b] = batch_ecap(c, k, b);
    auto push_alone = [&](std::vector<Item>& items, std::vector<uint32_t>& members, uint32_t i) {
        const QDesc& d = descs[i];
        const uint64_t cost = (uint64_t)d.E * (uint64_t)std::min<int64_t>(d.nsteps, (int64_t)1 << 40);
        items.push_back(Item{(uint32_t)members.size(), 1, 0, (int16_t)wave_time_bucket(cost)});
        members.push_back(i);
    };
    auto push_pack = [&](std::vector<Item>& items, std::vector<uint32_t>& members, Open& o) {
        if (o.count >= 1) {
            const uint64_t cost = (uint64_t)o.E * (uint64_t)std::min<int64_t>(o.max_steps, (int64_t)1 << 40);
            items.push_back(Item{(uint32_t)members.size(), (uint16_t)o.count, (uint16_t)o.E,
                                 (int16_t)wave_time_bucket(cost)});
            for (int m = 0; m < o.count; ++m) members.push_back(o.mem[m]);
        }
        o.count = 0;
        o.lanes = 0;
        o.max_steps = 0;
    };
    // work units: contiguous chunks of the queries in pass 1, (E, step bucket)
    // partitions in pass 2, item ranges after; several per thread, claimed
    // dynamically (run_units)
    nu = nth > 1 ? (int)std::min<int64_t>(2 * (int64_t)nth, std::max<int64_t>(nth, nq / 2048)) : 1;
    std::vector<std::vector<Item>> titems((size_t)nu);
    std::vector<std::vector<uint32_t>> tmembers((size_t)nu);
    std::vector<int64_t> bad((size_t)nu, nq);
    // cells per lane of a packed query by cap (2, 4, 8, 16) and size
    int8_t etab[4][513];
    for (int ci = 0; ci < 4; ++ci)
        for (int64_t n = 1; n <= 512; ++n) etab[ci][n] = (int8_t)seg_E(n, 2 << ci);
    // pass 1: descriptors, validation, pack keys (class ids local to the
    // chunk); a chunk's packed queries are listed by the partition owning
    // their (E, step bucket) pair, r mod nu
    // what pass 2 needs of a query, carried in the lists so that it never
    // reads the descriptors other chunks wrote
    struct QRef {
        uint32_t i;
        int32_t key;       // (E index, step bucket) << 4 | chunk-local class
        int64_t nsteps;
        int32_t L;         // lanes at the key's E
    };
    std::vector<std::vector<Consts>> tclasses((size_t)nu);
    std::vector<std::vector<QRef>> lists((size_t)nu);          // by partition, caller order within
    std::vector<std::vector<uint32_t>> list_at((size_t)nu);    // partition p: [at[p], at[p + 1])
    run_units(pool, nth, nu, [&](int t) {
        int64_t lo, hi;
        chunk(t, nq, &lo, &hi);
        std::vector<Item> items;
        std::vector<uint32_t> members;
        int64_t my_bad = nq;
        std::vector<Consts> classes;
        std::vector<QRef> mine;
        for (int64_t i = lo; i < hi; ++i) {
            QDesc& d = descs[i];
            if (make_desc(nullptr, q[i], i, &d) != REACH_OK) {
                my_bad = std::min(my_bad, i);
                continue;
            }
            if (!packs) {
                push_alone(items, members, (uint32_t)i);
                continue;
            }
            const int cap = ecap[d.kind & 3][std::min(n_bucket(d.n), kNB - 1)];
            const int E = etab[cap >= 16 ? 3 : cap >= 8 ? 2 : cap >= 4 ? 1 : 0][d.n];
            int cls = -1;
            Consts cs;
            std::memset(&cs, 0, sizeof cs);
            cs.kind = q[i].sys.kind;
            cs.dt = q[i].dt;
            std::memcpy(cs.prm, q[i].sys.prm, sizeof cs.prm);
            for (size_t u = 0; u < classes.size(); ++u)
                if (classes[u] == cs) { cls = (int)u; break; }
            if (cls < 0 && (int)classes.size() < kMaxClasses) {
                classes.push_back(cs);
                cls = (int)classes.size() - 1;
            }
            if (cls < 0) {
                // a class beyond the thread's table: a pack of its own
                Open o;
                o.E = E;
                o.mem[o.count++] = (uint32_t)i;
                o.lanes = (int)((d.n + E - 1) / E);
                o.max_steps = d.nsteps;
                push_pack(items, members, o);
                continue;
            }
            int ei = 0;
            while (kSegE[ei] != E) ++ei;
            const int b = wave_time_bucket((uint64_t)std::min<int64_t>(d.nsteps, (int64_t)1 << 40));
            const int r = ei * kBuckets + b;
            mine.push_back(QRef{(uint32_t)i, (r << 4) | cls, d.nsteps, (int32_t)((d.n + E - 1) / E)});
        }
        // by partition (counting sort, caller order kept within a partition)
        std::vector<uint32_t>& at = list_at[(size_t)t];
        at.assign((size_t)nu + 1, 0);
        for (const QRef& qr : mine) ++at[(size_t)((qr.key >> 4) % nu) + 1];
        for (int u = 0; u < nu; ++u) at[(size_t)u + 1] += at[(size_t)u];
        std::vector<QRef>& sorted_refs = lists[(size_t)t];
        sorted_refs.resize(mine.size());
        {
            std::vector<uint32_t> put(at.begin(), at.end() - 1);
            for (const QRef& qr : mine) sorted_refs[put[(size_t)((qr.key >> 4) % nu)]++] = qr;
        }
        titems[(size_t)t] = std::move(items);
        tmembers[(size_t)t] = std::move(members);
        tclasses[(size_t)t] = std::move(classes);
        bad[(size_t)t] = my_bad;
    });
    const int64_t first_bad = *std::min_element(bad.begin(), bad.end());
    if (first_bad < nq) {
        QDesc tmp;
        return make_desc(c, q[first_bad], first_bad, &tmp);
    }
    // every descriptor is written: the caller may start moving them while
    // the items are formed
    if (descs_done) descs_done();
    if (times) times->pass1_ms = since(t0);
    if (packs) {
        // global class ids (the chunks' tables merged in chunk order)
        std::vector<Consts> global;
        std::vector<std::vector<int32_t>> remap((size_t)nu);
        for (int t = 0; t < nu; ++t)
            for (const Consts& cs : tclasses[(size_t)t]) {
                int g = -1;
                for (size_t u = 0; u < global.size(); ++u)
                    if (global[u] == cs) { g = (int)u; break; }
                if (g < 0) {
                    global.push_back(cs);
                    g = (int)global.size() - 1;
                }
                remap[(size_t)t].push_back(g);
            }
        const size_t G = global.size();
        // key = (E index, step bucket) * G + global class; partition t owns
        // the (E index, step bucket) pairs r with r mod nu == t
        std::vector<uint32_t> local((size_t)kNE * kBuckets);
        std::vector<uint32_t> owned((size_t)nu, 0);
        for (size_t r = 0; r < local.size(); ++r) local[r] = owned[r % (size_t)nu]++;
        // pass 2: partition t packs the keys it owns, scanning the queries in
        // caller order.  The scan only assigns each query a pack (fill levels
        // in a small table, a key's kOpen current packs side by side); the
        // packs' member lists are then formed by a counting sort on the pack.
        run_units(pool, nth, nu, [&](int t) {
            std::vector<Item>& items = titems[(size_t)t];
            std::vector<uint32_t>& members = tmembers[(size_t)t];
            struct Pack {
                int32_t lanes, count, E, key;
                int64_t max_steps;
            };
            std::vector<Pack> packs;
            std::vector<int32_t> slot((size_t)owned[(size_t)t] * G * kOpen, -1);
            std::vector<const QRef*> refs;
            std::vector<int32_t> assign;
            for (int u = 0; u < nu; ++u) {
                const std::vector<int32_t>& rm = remap[(size_t)u];
                const std::vector<uint32_t>& at = list_at[(size_t)u];
                for (uint32_t k = at[(size_t)t]; k < at[(size_t)t + 1]; ++k) {
                    const QRef& qr = lists[(size_t)u][k];
                    const size_t r = (size_t)(qr.key >> 4);
                    const int E = kSegE[r / kBuckets];
                    const int L = qr.L;
                    const size_t key = (size_t)local[r] * G + (size_t)rm[(size_t)(qr.key & 15)];
                    int32_t* sl = &slot[key * kOpen];
                    if (sl[0] < 0)
                        for (int j = 0; j < kOpen; ++j) {
                            sl[j] = (int32_t)packs.size();
                            packs.push_back(Pack{0, 0, E, (int32_t)key, 0});
                        }
                    int j = 0;
                    while (j < kOpen && packs[(size_t)sl[j]].lanes + L > kLanes) ++j;
                    if (j == kOpen) {
                        // every open pack is too full for this query: close the
                        // fullest and open a new one in its place
                        j = 0;
                        for (int k = 1; k < kOpen; ++k)
                            if (packs[(size_t)sl[k]].lanes > packs[(size_t)sl[j]].lanes) j = k;
                        sl[j] = (int32_t)packs.size();
                        packs.push_back(Pack{0, 0, E, (int32_t)key, 0});
                    }
                    Pack& pk = packs[(size_t)sl[j]];
                    pk.lanes += L;
                    pk.max_steps = std::max(pk.max_steps, qr.nsteps);
                    refs.push_back(&qr);
                    assign.push_back(sl[j]);
                    if (++pk.count == kPackMax || pk.lanes == kLanes) {
                        sl[j] = (int32_t)packs.size();
                        packs.push_back(Pack{0, 0, E, (int32_t)key, 0});
                    }
                }
            }
            // members by pack (counting sort, scan order kept within a pack)
            std::vector<int32_t> start(packs.size() + 1, 0);
            for (const int32_t p : assign) ++start[(size_t)p + 1];
            for (size_t p = 0; p < packs.size(); ++p) start[p + 1] += start[p];
            std::vector<const QRef*> by_pack(refs.size());
            {
                std::vector<int32_t> at(start.begin(), start.end() - 1);
                for (size_t k = 0; k < refs.size(); ++k) by_pack[(size_t)at[(size_t)assign[k]]++] = refs[k];
            }
            // packs still open at the end (those the slots point to) are packed
            // again per key below; every other pack is final
            std::vector<uint8_t> open_now(packs.size(), 0);
            for (const int32_t p : slot)
                if (p >= 0) open_now[(size_t)p] = 1;
            for (size_t p = 0; p < packs.size(); ++p) {
                const Pack& pk = packs[p];
                if (open_now[p] || pk.count == 0) continue;
                const uint64_t cost = (uint64_t)pk.E * (uint64_t)std::min<int64_t>(pk.max_steps, (int64_t)1 << 40);
                items.push_back(Item{(uint32_t)members.size(), (uint16_t)pk.count, (uint16_t)pk.E,
                                     (int16_t)wave_time_bucket(cost)});
                for (int32_t k = start[p]; k < start[p + 1]; ++k) members.push_back(by_pack[(size_t)k]->i);
            }
            // each key's open packs: their queries again, widest first into
            // the first pack with room (first fit decreasing)
            std::vector<const QRef*> rest;
            std::vector<Open> merged;
            for (size_t k = 0; k < slot.size(); k += kOpen) {
                if (slot[k] < 0) continue;
                rest.clear();
                int E = 0;
                for (int j = 0; j < kOpen; ++j) {
                    const size_t p = (size_t)slot[k + (size_t)j];
                    E = packs[p].E;
                    for (int32_t m = start[p]; m < start[p + 1]; ++m) rest.push_back(by_pack[(size_t)m]);
                }
                if (rest.empty()) continue;
                std::sort(rest.begin(), rest.end(), [](const QRef* x, const QRef* y) {
                    return x->L != y->L ? x->L > y->L : x->i < y->i;
                });
                merged.clear();
                for (const QRef* rr : rest) {
                    Open* o = nullptr;
                    for (Open& oj : merged)
                        if (oj.lanes + rr->L <= kLanes && oj.count < kPackMax) { o = &oj; break; }
                    if (!o) {
                        merged.emplace_back();
                        o = &merged.back();
                        o->E = E;
                    }
                    o->mem[o->count++] = rr->i;
                    o->lanes += rr->L;
                    o->max_steps = std::max(o->max_steps, rr->nsteps);
                }
                for (Open& o : merged) push_pack(items, members, o);
            }
        });
    }
    if (times) times->pass_ms = since(t0);
    t0 = clk::now();
    // launch order: bucket-major, then unit, then the unit's item order.  A
    // count of items and of their members per (unit, bucket), one prefix over
    // (bucket, unit), then every unit places its own items and members.
    // (the counts live in buffers kept by the calling thread: fresh ones of this
    // size would cost page faults on every call)
    thread_local std::vector<int64_t> hist_buf, mhist_buf;
    if (hist_buf.size() < (size_t)nu * kBuckets) {
        hist_buf.resize((size_t)nu * kBuckets);
        mhist_buf.resize((size_t)nu * kBuckets);
    }
    int64_t* hist = hist_buf.data();
    int64_t* mhist = mhist_buf.data();
    std::vector<int> blo((size_t)nu, kBuckets), bhi((size_t)nu, -1);   // buckets in use
    run_units(pool, nth, nu, [&](int t) {
        int64_t* h = &hist[(size_t)t * kBuckets];
        int64_t* mh = &mhist[(size_t)t * kBuckets];
        std::fill(h, h + kBuckets, 0);
        std::fill(mh, mh + kBuckets, 0);
        for (const Item& it : titems[(size_t)t]) {
            ++h[it.bucket];
            mh[it.bucket] += it.count;
            blo[(size_t)t] = std::min<int>(blo[(size_t)t], it.bucket);
            bhi[(size_t)t] = std::max<int>(bhi[(size_t)t], it.bucket);
        }
    });
    const int b0 = *std::min_element(blo.begin(), blo.end());
    const int b1 = *std::max_element(bhi.begin(), bhi.end());
    int64_t ni = 0, nm = 0;
    for (int b = b0; b <= b1; ++b)
        for (int t = 0; t < nu; ++t) {
            const size_t x = (size_t)t * kBuckets + b;
            const int64_t v = hist[x], mv = mhist[x];
            hist[x] = ni;
            mhist[x] = nm;
            ni += v;
            nm += mv;
        }
    if (times) times->order_ms = since(t0);
    t0 = clk::now();
    std::vector<BatchItem>& io = *items_out;
    std::vector<uint32_t>& mo = *members_out;
    io.resize((size_t)ni);
    mo.resize((size_t)nq);
    std::vector<uint8_t> wide((size_t)nu, 0);
    run_units(pool, nth, nu, [&](int t) {
        int64_t* h = &hist[(size_t)t * kBuckets];
        int64_t* mh = &mhist[(size_t)t * kBuckets];
        for (const Item& it : titems[(size_t)t]) {
            const int64_t k = h[it.bucket]++;
            const int64_t m = mh[it.bucket];
            mh[it.bucket] += it.count;
            io[(size_t)k] = BatchItem{(uint32_t)m, it.count, it.E};
            std::memcpy(&mo[(size_t)m], &tmembers[(size_t)t][it.first], sizeof(uint32_t) * it.count);
            if (it.E > 8) wide[(size_t)t] = 1;
        }
    });
    if (std::find(wide.begin(), wide.end(), 1) != wide.end()) *packed = 2;
    if (times) times->members_ms = since(t0);
    return REACH_OK;
}

}  // namespace

extern "C" {

// batch workspace: [work counter][per-query flags][per-query side counters]
// and two blocks of [descriptors, items, item count, members], used by turns
size_t reach_batch_workspace_bytes(int64_t nq) {
    if (nq < 0) return (size_t)-1;
    return align256(8) + 2 * align256(4 * (size_t)nq) + 2 * align256(batch_block_bytes(nq));
}

reach_status reach_plan_batch(reach_ctx* c, const reach_query* q, int64_t nq,
                              int64_t* item_start, int32_t* item_count, int32_t* item_E,
                              int64_t* member, int64_t* n_items) {
    if (nq < 0 || !n_items || (nq > 0 && (!q || !item_start || !item_count || !item_E || !member)))
        return c ? fail(c, REACH_E_INVAL, "bad arguments") : REACH_E_INVAL;
    *n_items = 0;
    if (nq == 0) return REACH_OK;
    const int split = (c && opt_get(c, "batch.split")) ? 1 : 0;
    std::vector<QDesc> descs((size_t)nq);
    std::vector<uint32_t> members;
    std::vector<BatchItem> items;
    // without a context a large plan gets a pool of its own for this call,
    // so the schedule is computed the same way as for the batch
    std::unique_ptr<HostPool> local;
    HostPool* pool = host_pool(c);
    if (!pool && batch_host_threads(nq) > 1) {
        local.reset(new HostPool(batch_host_threads(nq)));
        pool = local.get();
    }
    const int nth = pool ? std::min(batch_host_threads(nq), pool->size()) : 1;
    int packed = 0;
    const reach_status st = plan_batch(c, pool, q, nq, split, nth, descs.data(), &members, &items,
                                       &packed);
    if (st != REACH_OK) return st;
    for (size_t k = 0; k < items.size(); ++k) {
        item_start[k] = items[k].start;
        item_count[k] = (int32_t)items[k].count;
        item_E[k] = (int32_t)items[k].E;
    }
    for (int64_t p = 0; p < nq; ++p) member[p] = members[(size_t)p];
    *n_items = (int64_t)items.size();
    return REACH_OK;
}

reach_status reach_embed_rk4_batch(reach_ctx* c, const reach_query* q, int64_t nq, void* ws,
                                   size_t ws_bytes, void* stream) {
    if (!c) return REACH_E_INVAL;
    if (nq < 0 || (nq > 0 && !q)) return fail(c, REACH_E_INVAL, "bad query array");
    if (nq == 0) return REACH_OK;
    const size_t need = reach_batch_workspace_bytes(nq);
    if (!ws || ws_bytes < need) return fail(c, REACH_E_NOMEM, "workspace of %zu bytes needed", need);
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t hs = (hipStream_t)stream;
    // whole queries per wave by default (most work per wave, best throughput);
    // batch.split = 1 gives each side of a cooperative query its own wave
    const int split = opt_get(c, "batch.split") ? 1 : 0;
    HostPool* pool = batch_host_threads(nq) > 1 ? host_pool(c) : nullptr;
    const int nth = pool ? std::min(batch_host_threads(nq), pool->size()) : 1;
    // pinned staging (reused; wait for the previous upload from it, which
    // ends before that batch's kernel starts).  Growing it drops the cached
    // graphs, after every launched one has finished.
    if (c->staging_cap < nq) {
        HIPCHK(c, hipDeviceSynchronize());
        if (c->staging) HIPCHK(c, hipHostFree(c->staging));
        c->staging = nullptr;
        for (auto& kv : c->graphs) hipGraphExecDestroy(kv.second);
        c->graphs.clear();
        int64_t cap = std::max<int64_t>(nq, 1024);
        HIPCHK(c, hipHostMalloc((void**)&c->staging, batch_block_bytes(cap), hipHostMallocDefault));
        c->staging_cap = cap;
    } else {
        HIPCHK(c, hipEventSynchronize(c->staging_ev));
    }
    const BatchBlock hb = batch_block(c->staging, nq);
    char* base = (char*)ws;
    auto* counter = (unsigned long long*)base;
    auto* qflags = (unsigned int*)(base + align256(8));
    auto* pair = (unsigned int*)(base + align256(8) + align256(4 * (size_t)nq));
    // two blocks of descriptors and work items, used by turns: this batch's
    // upload (on the context's copy stream) waits only for the kernel that
    // read its block two batches ago, so it runs beside the previous batch's
    // kernel; the counter reset and the kernel wait for that kernel, on any
    // stream, and for the upload
    const int blk = c->next_block;
    const BatchBlock db = batch_block(base + align256(8) + 2 * align256(4 * (size_t)nq) +
                                      (size_t)blk * align256(batch_block_bytes(nq)), nq);
    hipStream_t cs = c->copy_stream;
    if (c->block_ev_recorded[blk]) HIPCHK(c, hipStreamWaitEvent(cs, c->block_ev[blk], 0));
    // another workspace or query count moves the blocks, which may then
    // overlap what the previous batch's kernel still uses: wait for it too
    if (c->batch_ev_recorded && (ws != c->last_ws || nq != c->last_nq))
        HIPCHK(c, hipStreamWaitEvent(cs, c->batch_ev, 0));
    const auto t_start = std::chrono::steady_clock::now();
    std::vector<uint32_t> members;
    std::vector<BatchItem> items;
    PlanTimes pt;
    int packed = 0;
    // the descriptors go up as soon as they are written, while the host forms
    // the work items
    hipError_t desc_err = hipSuccess;
    const size_t desc_bytes = sizeof(QDesc) * (size_t)nq;
    reach_status pst = plan_batch(c, pool, q, nq, split, nth, hb.desc, &members, &items, &packed,
                                  &pt, [&] {
        desc_err = hipMemcpyAsync(db.desc, hb.desc, desc_bytes, hipMemcpyHostToDevice, cs);
    });
    if (pst != REACH_OK) return pst;
    if (desc_err != hipSuccess) return hip_fail(c, desc_err, "descriptor upload");
    const int64_t ni = (int64_t)items.size();
    std::memcpy(hb.items, items.data(), sizeof(BatchItem) * (size_t)ni);
    std::memcpy(hb.members, members.data(), sizeof(uint32_t) * (size_t)nq);
    *hb.count = (uint64_t)ni;
    const auto t_plan = std::chrono::steady_clock::now();

    int64_t grid = opt_get(c, "batch.waves");
    if (grid <= 0) {
        if (packed) grid = c->batch_waves[packed - 1];
        if (grid <= 0)
            grid = (int64_t)c->cus * (packed == 2 ? kWideWavesPerCU
                                      : packed == 1 ? kPackWavesPerCU : kBatchWavesPerCU);
        // the wide packing kernel holds at most two waves per SIMD
        if (packed == 2) grid = std::min<int64_t>(grid, (int64_t)c->cus * 8);
    }
    c->last_packed = packed;
    grid = std::min<int64_t>(grid, split ? 2 * ni : ni);

    if (c->log) {
        using ms = std::chrono::duration<double, std::milli>;
        log_call(c, "\"call\": \"batch\", \"queries\": %lld, \"items\": %lld, \"packed\": %lld, "
                    "\"waves\": %lld, \"split\": %d, \"host_threads\": %d, \"plan_ms\": %.3f, "
                    "\"plan_pass1_ms\": %.3f, \"plan_pass_ms\": %.3f, \"plan_order_ms\": %.3f, "
                    "\"plan_members_ms\": %.3f",
                 (long long)nq, (long long)ni, (long long)(nq - (int64_t)std::count_if(
                     items.begin(), items.end(), [](const BatchItem& x) { return x.count == 1; })),
                 (long long)grid, split, nth, ms(t_plan - t_start).count(), pt.pass1_ms,
                 pt.pass_ms, pt.order_ms, pt.members_ms);
    }
    // the rest of the block (items, their count, the members) follows; the
    // staging is free for the next call once both copies are done, so the
    // next call plans while this batch's kernel runs
    HIPCHK(c, hipMemcpyAsync(db.items, hb.items, batch_block_bytes(nq) - desc_bytes,
                             hipMemcpyHostToDevice, cs));
    HIPCHK(c, hipEventRecord(c->staging_ev, cs));
    HIPCHK(c, hipStreamWaitEvent(hs, c->staging_ev, 0));
    if (c->batch_ev_recorded) HIPCHK(c, hipStreamWaitEvent(hs, c->batch_ev, 0));
    auto enqueue = [&](hipStream_t s) -> hipError_t {
        hipError_t e = launch_zero(base, (int64_t)(align256(8) + 2 * align256(4 * (size_t)nq)) / 4, s);
        if (e != hipSuccess) return e;
        return launch_batch(db.desc, db.items, db.members, db.count, counter, qflags, pair,
                            c->status, split, packed, grid, s);
    };

    if (hs == nullptr) {
        hipError_t e = enqueue(hs);
        if (e != hipSuccess) return hip_fail(c, e, "batch launch");
    } else {
        GraphKey key{nq, ws, c->staging, (((grid * 2 + split) * 3 + packed) * 2 + blk), hs};
        auto it = c->graphs.find(key);
        if (it == c->graphs.end()) {
            hipGraph_t g = nullptr;
            HIPCHK(c, hipStreamBeginCapture(hs, hipStreamCaptureModeRelaxed));
            hipError_t e = enqueue(hs);
            hipError_t e2 = hipStreamEndCapture(hs, &g);
            if (e != hipSuccess) { if (g) hipGraphDestroy(g); return hip_fail(c, e, "batch capture"); }
            if (e2 != hipSuccess) return hip_fail(c, e2, "hipStreamEndCapture");
            hipGraphExec_t ge = nullptr;
            e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            hipGraphDestroy(g);
            if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
            it = c->graphs.emplace(key, ge).first;
        }
        HIPCHK(c, hipGraphLaunch(it->second, hs));
    }
    HIPCHK(c, hipEventRecord(c->batch_ev, hs));
    HIPCHK(c, hipEventRecord(c->block_ev[blk], hs));
    c->batch_ev_recorded = true;
    c->block_ev_recorded[blk] = true;
    c->next_block = 1 - blk;
    c->last_ws = ws;
    c->last_nq = nq;
    (void)counter;
    return REACH_OK;
}

// Batch autotuner, on the caller's whole batch (a bucket's queries alone
// would be too few to fill the device, and their timing would favour short
// items over dense ones).  After kTuneWarm untimed calls, every comparison
// times the batch (one warm-up and four timed calls, fastest kept) with the
// candidate setting and then again with the current one, and takes the
// candidate only when it is faster by more than kTuneGain.  In order: the
// width of the whole batch (every bucket's cap 16, the wide kernel, against
// 8, the narrow one); then, bucket by bucket, most queries first, for every
// (kind, size bucket) with at least kTuneMinQueries queries, the narrower
// caps 8, 4 and 2; then 4, 8 and (narrow kernel only) 12 resident waves per
// compute unit.  Results are those of the batch at any setting (bitwise).
reach_status reach_autotune_batch(reach_ctx* c, const reach_query* q, int64_t nq, void* ws,
                                  size_t ws_bytes, void* stream, int64_t* best) {
    if (!c) return REACH_E_INVAL;
    if (!best || nq < 1 || !q) return fail(c, REACH_E_INVAL, "bad arguments");
    constexpr int64_t kTuneMinQueries = 256;
    constexpr double kTuneGain = 0.01;
    constexpr int kTuneWarm = 8;
    constexpr int kNB = 10;
    hipStream_t hs = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return fail(c, REACH_E_DEVICE, "hipEventCreate failed");
    }
    // fastest of four timed calls after a warm-up, in nanoseconds (host
    // planning and the descriptor upload included)
    auto time_batch = [&](double* ns) -> reach_status {
        double bestms = 1e300;
        for (int r = 0; r < 5; ++r) {
            if (hipEventRecord(e0, hs) != hipSuccess) return fail(c, REACH_E_DEVICE, "event");
            const reach_status st = reach_embed_rk4_batch(c, q, nq, ws, ws_bytes, stream);
            if (st != REACH_OK) return st;
            if (hipEventRecord(e1, hs) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                return fail(c, REACH_E_DEVICE, "event");
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return fail(c, REACH_E_DEVICE, "event");
            if (r > 0) bestms = std::min(bestms, (double)ms);
        }
        *ns = bestms * 1e6;
        return REACH_OK;
    };
    const int64_t save_E = opt_get(c, "batch.E"), save_waves = opt_get(c, "batch.waves");
    c->opt["batch.E"] = 0;
    // widths are timed at each packing kernel's default wave count
    c->batch_waves[0] = c->batch_waves[1] = 0;
    // a few untimed calls first, so that the device clock has left its idle
    // level before anything is compared
    reach_status st = REACH_OK;
    for (int w = 0; w < kTuneWarm && st == REACH_OK; ++w)
        st = reach_embed_rk4_batch(c, q, nq, ws, ws_bytes, stream);
    if (st == REACH_OK && hipStreamSynchronize(hs) != hipSuccess)
        st = fail(c, REACH_E_DEVICE, "batch warm-up");
    double cur = 0;
    if (st == REACH_OK) st = time_batch(&cur);
    // a setting replaces the current one only when the batch timed with it is
    // faster by kTuneGain than the batch timed again with the current one
    // right after (drift of the device clock hits both alike)
    auto trial = [&](const std::function<void()>& cand, const std::function<void()>& keep,
                     bool* won) -> reach_status {
        double tc = 0, tk = 0;
        cand();
        reach_status r = time_batch(&tc);
        keep();
        if (r == REACH_OK) r = time_batch(&tk);
        if (r != REACH_OK) return r;
        *won = tc < tk * (1.0 - kTuneGain);
        if (*won) {
            cand();
            cur = tc;
        } else {
            cur = tk;
        }
        return REACH_OK;
    };
    const bool packs = !opt_get(c, "batch.split") && batch_packs(c, nq);
    if (st == REACH_OK && packs) {
        // (kind, bucket) groups, most queries first
        std::map<std::pair<int, int>, int64_t> count;
        for (int64_t i = 0; i < nq; ++i) {
            const reach_system& sy = q[i].sys;
            ++count[{sy.kind, std::min(n_bucket(sy.n), kNB - 1)}];
        }
        std::vector<std::pair<int64_t, std::pair<int, int>>> order;
        for (const auto& kv : count)
            if (kv.second >= kTuneMinQueries) order.push_back({-kv.second, kv.first});
        std::sort(order.begin(), order.end());
        // the whole batch's width first: every bucket at 8 cells per lane (the
        // narrow kernel, two waves per SIMD) against 16 (the wide kernel, one)
        for (const auto& kv : count) c->batch_tune.erase(kv.first);
        const int first = c->batch_cap ? c->batch_cap : kSegECap;
        const int other = first == 16 ? 8 : 16;
        bool won = false;
        st = trial([&] { c->batch_cap = other; }, [&] { c->batch_cap = first; }, &won);
        if (st == REACH_OK) save_batch_tune_entry(c, -1, -1, c->batch_cap, cur);
        // then narrower caps bucket by bucket
        for (size_t k = 0; k < order.size() && st == REACH_OK; ++k) {
            const auto key = order[k].second;
            const int keep = batch_ecap(c, key.first, key.second);
            for (int cap : {8, 4, 2}) {
                if (cap >= batch_ecap(c, key.first, key.second)) continue;
                const int now = batch_ecap(c, key.first, key.second);
                st = trial([&] { c->batch_tune[key] = cap; }, [&] { c->batch_tune[key] = now; },
                           &won);
                if (st != REACH_OK) break;
            }
            if (st == REACH_OK && batch_ecap(c, key.first, key.second) != keep)
                save_batch_tune_entry(c, key.first, key.second,
                                      batch_ecap(c, key.first, key.second), cur);
        }
    }
    int64_t best_waves = save_waves;
    if (st == REACH_OK && packs && save_waves == 0) {
        // from the kernel's default (one wave per SIMD for the wide kernel,
        // two for the narrow one), which the last timed call used
        const bool wide = c->last_packed == 2;
        int64_t& tuned = c->batch_waves[wide ? 1 : 0];
        int64_t now = (int64_t)c->cus * (wide ? kWideWavesPerCU : kPackWavesPerCU);
        for (int64_t per_cu : {4, 8, 12}) {
            const int64_t w = per_cu * c->cus;
            // the wide packing kernel holds at most two waves per SIMD
            if (w == now || (wide && per_cu > 8)) continue;
            bool won = false;
            const int64_t was = now;
            st = trial([&] { tuned = w; }, [&] { tuned = was; }, &won);
            if (st != REACH_OK) break;
            if (won) now = w;
        }
        best_waves = now;
    }
    c->opt["batch.E"] = save_E;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != REACH_OK) return st;
    best[0] = best_waves;
    best[1] = (int64_t)std::llround(cur);
    return REACH_OK;
}

reach_status reach_embed_rk4_each(reach_ctx* c, const reach_query* q, int64_t nq, int32_t nstreams) {
    if (!c) return REACH_E_INVAL;
    if (nq < 0 || (nq > 0 && !q)) return fail(c, REACH_E_INVAL, "bad query array");
    if (nstreams < 1 || nstreams > 16) return fail(c, REACH_E_INVAL, "nstreams must be 1..16");
    HIPCHK(c, hipSetDevice(c->device));
    while ((int32_t)c->each_streams.size() < nstreams) {
        hipStream_t s;
        HIPCHK(c, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        c->each_streams.push_back(s);
    }
    std::vector<QDesc> d(nq);
    for (int64_t i = 0; i < nq; ++i) {
        reach_status st = make_desc(c, q[i], i, &d[i]);
        if (st != REACH_OK) return st;
    }
    for (int64_t i = 0; i < nq; ++i) {
        hipError_t e = launch_single(d[i], c->status, nullptr, c->each_streams[i % nstreams]);
        if (e != hipSuccess) return hip_fail(c, e, "single-query launch");
    }
    for (int32_t k = 0; k < nstreams; ++k) HIPCHK(c, hipStreamSynchronize(c->each_streams[k]));
    return REACH_OK;
}

}  // extern "C"


// ------------------------------------------------ services for user.cpp --
namespace reach {
namespace rt {

int ctx_device(const reach_ctx* c) { return c->device; }
int ctx_cus(const reach_ctx* c) { return c->cus; }
unsigned int* ctx_status(reach_ctx* c) { return c->status; }
int64_t option(const reach_ctx* c, const char* key) { return opt_get(c, key); }
reach_status set_error(reach_ctx* c, reach_status st, const std::string& msg) {
    return fail(c, st, "%s", msg.c_str());
}
reach_status validate_user(reach_ctx* c, const reach_system* s, reach_dtype dtype) {
    return check_system_kind(c, s, dtype, true);
}
void pass_buffers(int64_t passes, bool inplace_ok, bool alias,
                  std::vector<std::pair<int, int>>* io, bool* final_copy) {
    plan_io(passes, inplace_ok, alias, io, final_copy);
}

}  // namespace rt
}  // namespace reach
