// Many small embedding queries on gfx950: offline batches and online serving.
//
// Every query (FP64, n <= 512 cells, scalar input) is run by one wavefront
// with its whole lower/upper state in registers (E = ceil(n / 64) cells per
// lane, 1..8, spread so that every lane is busy), all N RK4 steps in one go:
// no halo, no HBM traffic inside the step loop; short cooperative queries
// share a wavefront, one cell per lane.  The arithmetic per cell is the
// large-n embedding kernel's, so a query gives the same box alone, in a batch,
// or served.
//
//   batch_kernel   persistent grid; each wave pops the next work item (a whole
//                  query, a pack of short ones, or with `split` one side of a
//                  cooperative query) from a device counter until the batch is
//                  exhausted.
//   single_kernel  one query per launch (the baseline the batch is compared with).
//   serve_kernel   persistent grid fed through a ring of descriptors in pinned
//                  host memory; each wave claims the next work item (sequence
//                  number and side), waits (bounded) until the host publishes
//                  it, runs it and publishes that side's completion.  The grid
//                  leaves as a whole when the host sets the stop flag or when
//                  any wave reaches the idle limit, so it always drains.  A
//                  served query reads its host-written cancel word every
//                  kCancelEvery steps and stops early when it is set.
#include "dev.hpp"
#include "kernels.hpp"

namespace reach {

// Cancel word of the queries that have none (batches, single launches).
__device__ unsigned int g_never_cancelled = 0u;

__device__ __forceinline__ uint64_t wave_bcast(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Balanced layout of a query's n cells over the 64 lanes: E = ceil(n / 64)
// (1..8), the first F = n - 64 (E - 1) lanes hold E consecutive cells and the
// others ("short" lanes) E - 1.  For E >= 2 every lane holds cells and the
// chain's last cell sits in lane 63, so no cell of the window is a ghost and
// no stage needs a per-cell select: a short lane's last cell is slot E - 2,
// whose right neighbour (and the value its left neighbour lane reads) is
// picked once per stage; slot E - 1 of a short lane computes a value nobody
// reads.  For E = 1 the lanes past cell n-1 are empty and the right neighbour
// of cell n-1 is set to the ghost.  The arithmetic per cell is the
// large-chain kernel's, operation for operation, so a query's box is the
// same alone, batched or served.
struct Lanes {
    bool shortl;   // this lane holds E - 1 cells
    bool end;      // this lane holds cell n-1
    int cnt;       // cells held
    int64_t first; // index of the first cell held
};

template <int E>
__device__ __forceinline__ Lanes lanes_of(int64_t n) {
    const int lane = threadIdx.x;
    const int64_t F = n - (int64_t)WAVE * (E - 1);   // lanes holding E cells
    Lanes L;
    L.shortl = lane >= F;
    L.cnt = L.shortl ? E - 1 : E;
    L.first = (int64_t)lane * E - (L.shortl ? (int64_t)lane - F : 0);
    L.end = (E == 1) ? (lane == n - 1) : (lane == WAVE - 1);
    return L;
}

// Right neighbour of slot e, given the value shifted in from the next lane.
template <int E, class T>
__device__ __forceinline__ T right_of(const T (&in)[E], int e, T rn, bool shortl) {
    if (e == E - 1) return rn;
    if (e == E - 2) return shortl ? rn : in[E - 1];
    return in[e + 1];
}
// The value lane l + 1 needs from this lane: its last held cell.
template <int E, class T>
__device__ __forceinline__ T last_of(const T (&in)[E], bool shortl) {
    if constexpr (E == 1) return in[0];
    else return shortl ? in[E - 2] : in[E - 1];
}

template <int KIND, int STAGE, int E, int S>
__device__ __forceinline__ void bal_stage(double (&y)[S][E], double (&acc)[S][E],
                                          double (&t)[S][E], const SysPrm<double>& P,
                                          const Inputs<double, E, S, IN_SCALAR>& U,
                                          const Steps<double>& st, const Lanes& L) {
    using T = double;
    T (&in)[S][E] = (STAGE == 1) ? y : t;
    if constexpr (KIND == K_CTM) {
        // F_e = min(v y_e, wc - w y_{e+1}, q), k_e = F_{e-1} - F_e; ghost -inf
        // right of cell n-1 (free outflow), zero flux into cell 0 (lane 0
        // receives 0 from the shift)
        const T v = P.a0, w = P.a1, wc = P.a2, q = P.a3;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            T rn = from_right(in[s][0]);
            rn = L.end ? neg_inf<T>() : rn;
            T F[E];
#pragma unroll
            for (int e = 0; e < E; ++e)
                F[e] = minT(minT(v * in[s][e], fmaT(-w, right_of<E>(in[s], e, rn, L.shortl), wc)), q);
            T Fprev = from_left(last_of<E>(F, L.shortl));
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const T k = Fprev - F[e];
                Fprev = F[e];
                rk_update<STAGE>(k, y[s][e], acc[s][e], t[s][e], st);
            }
        }
    } else if constexpr (KIND == K_RD) {
        // k = (y_{e-1} + y_{e+1}) / h^2 + (u - y_e (y_e^2 + 2 / h^2)), ghosts 0
        const T ih2 = P.a0, two_ih2 = P.a1;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const T ln = from_left(last_of<E>(in[s], L.shortl));
            T rn = from_right(in[s][0]);
            if (E == 1) rn = L.end ? T(0) : rn;
            T left = ln;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const T mid = in[s][e];
                const T right = right_of<E>(in[s], e, rn, L.shortl);
                const T loc = fmaT(-mid, fmaT(mid, mid, two_ih2), U.at(s, e));
                const T k = fmaT(left + right, ih2, loc);
                left = mid;
                rk_update<STAGE>(k, y[s][e], acc[s][e], t[s][e], st);
            }
        }
    } else {
        // LIN3, both sides (S == 2): the sign split of aL, aR, b
        const T aL = P.a0, aD = P.a1, aR = P.a2, b = P.a3;
        const T aLp = aL > T(0) ? aL : T(0), aLn = aL < T(0) ? aL : T(0);
        const T aRp = aR > T(0) ? aR : T(0), aRn = aR < T(0) ? aR : T(0);
        const T bp = b > T(0) ? b : T(0), bn = b < T(0) ? b : T(0);
        T ln[2], rn[2], left[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            ln[s] = from_left(last_of<E>(in[s], L.shortl));
            rn[s] = from_right(in[s][0]);
            if (E == 1) rn[s] = L.end ? T(0) : rn[s];
            left[s] = ln[s];
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            T mid[2], right[2], k[2];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                mid[s] = in[s][e];
                right[s] = right_of<E>(in[s], e, rn[s], L.shortl);
            }
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int o = 1 - s;
                T acc0 = aD * mid[s];
                acc0 = fmaT(aLp, left[s], acc0);
                acc0 = fmaT(aLn, left[o], acc0);
                acc0 = fmaT(aRp, right[s], acc0);
                acc0 = fmaT(aRn, right[o], acc0);
                acc0 = fmaT(bp, U.at(s, e), acc0);
                k[s] = fmaT(bn, U.at(o, e), acc0);
            }
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                left[s] = mid[s];
                rk_update<STAGE>(k[s], y[s][e], acc[s][e], t[s][e], st);
            }
        }
    }
}

// One query, or one side of it: S = 2 runs both sides in this wave, S = 1
// only side `side` (cooperative systems, whose sides do not interact).
template <int KIND, int E, int S>
__device__ __noinline__ unsigned run_query_E(const QDesc& d, int side) {
    using T = double;
    const int64_t n = d.n;
    const Lanes L = lanes_of<E>(n);
    const double* src[2] = {d.x_lo, d.x_hi};
    double* dst[2] = {d.r_lo, d.r_hi};
    const double* pin[2] = {d.p_lo, d.p_hi};
    T y[S][E];
    Inputs<T, E, S, IN_SCALAR> U;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int sd = S == 1 ? side : s;
#pragma unroll
        for (int e = 0; e < E; ++e)
            y[s][e] = (e < L.cnt) ? src[sd][L.first + e] : ghost<KIND, T>();
        U.u[s] = pin[sd] ? *pin[sd] : T(0);
    }
    SysPrm<T> P;
    P.a0 = d.prm[0]; P.a1 = d.prm[1]; P.a2 = d.prm[2]; P.a3 = d.prm[3]; P.a4 = d.prm[4];
    const Steps<T> st = {d.h2, d.dt, d.dt6};
    T acc[S][E], t[S][E];
    // Steps in blocks of kCancelEvery.  A served query reads its cancel word
    // at the start of a block and looks at the value only after the block's
    // steps, so the host-memory read never stalls the arithmetic.  Queries
    // without one read a device word that is always 0 (no branch around the
    // load, so nothing has to wait for it before the steps).
    const unsigned int* cw = d.cancel ? d.cancel : &g_never_cancelled;
    bool cancelled = false;
    for (int64_t k0 = 0; k0 < d.nsteps; k0 += kCancelEvery) {
        const unsigned stop = __hip_atomic_load(cw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        const int64_t k1 = k0 + kCancelEvery < d.nsteps ? k0 + kCancelEvery : d.nsteps;
        for (int64_t k = k0; k < k1; ++k) {
            bal_stage<KIND, 1, E, S>(y, acc, t, P, U, st, L);
            bal_stage<KIND, 2, E, S>(y, acc, t, P, U, st, L);
            bal_stage<KIND, 3, E, S>(y, acc, t, P, U, st, L);
            bal_stage<KIND, 4, E, S>(y, acc, t, P, U, st, L);
        }
        if (wave_bcast(stop)) {
            cancelled = true;
            break;
        }
    }
    if (cancelled) return ST_CANCELLED;
    unsigned bits = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (e < L.cnt) {
            const int64_t j = L.first + e;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                dst[S == 1 ? side : s][j] = y[s][e];
                if (!finiteT(y[s][e])) bits |= ST_NONFINITE;
            }
            if constexpr (S == 2) {
                if (y[0][e] > y[1][e]) bits |= ST_ORDER;
            }
        }
    }
    const unsigned long long nf = __ballot(bits & ST_NONFINITE);
    const unsigned long long od = __ballot(bits & ST_ORDER);
    return (nf ? (unsigned)ST_NONFINITE : 0u) | (od ? (unsigned)ST_ORDER : 0u);
}

template <int KIND, int S>
__device__ __forceinline__ unsigned run_query_kind(const QDesc& d, int side) {
    switch (d.E) {
        case 1: return run_query_E<KIND, 1, S>(d, side);
        case 2: return run_query_E<KIND, 2, S>(d, side);
        case 3: return run_query_E<KIND, 3, S>(d, side);
        case 4: return run_query_E<KIND, 4, S>(d, side);
        case 5: return run_query_E<KIND, 5, S>(d, side);
        case 6: return run_query_E<KIND, 6, S>(d, side);
        case 7: return run_query_E<KIND, 7, S>(d, side);
        default: return run_query_E<KIND, 8, S>(d, side);
    }
}

// Packed short queries: up to kPackMax cooperative queries (CTM or RD) of at
// most kPackMaxN cells with the same system constants and dt share one wave,
// query m on a contiguous segment of n_m lanes (one cell per lane, both
// sides).  A segment's first lane takes the left boundary value (ghost 0;
// zero inflow for the CTM) and its last lane the right ghost (0; -inf, free
// outflow, for the CTM) instead of the neighbouring segment's values; the
// wave runs the longest member's step count and a member's lanes keep their
// state once its own steps are done.  Per cell this is the arithmetic of the
// single-query path, so the results are bitwise those of the query run alone.
template <int KIND, int STAGE>
__device__ __forceinline__ void pack_stage(double (&y)[2], double (&acc)[2], double (&t)[2],
                                           const SysPrm<double>& P, const double (&u)[2],
                                           const Steps<double>& st, bool first, bool last,
                                           bool live) {
    using T = double;
    T (&in)[2] = (STAGE == 1) ? y : t;
    if constexpr (KIND == K_CTM) {
        const T v = P.a0, w = P.a1, wc = P.a2, q = P.a3;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            T rn = from_right(in[s]);
            rn = last ? neg_inf<T>() : rn;
            const T F = minT(minT(v * in[s], fmaT(-w, rn, wc)), q);
            T Fprev = from_left(F);
            Fprev = first ? T(0) : Fprev;
            const T y0 = y[s];
            rk_update<STAGE>(Fprev - F, y[s], acc[s], t[s], st);
            if (STAGE == 4) y[s] = live ? y[s] : y0;
        }
    } else {
        const T ih2 = P.a0, two_ih2 = P.a1;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            T ln = from_left(in[s]);
            ln = first ? T(0) : ln;
            T rn = from_right(in[s]);
            rn = last ? T(0) : rn;
            const T mid = in[s];
            const T loc = fmaT(-mid, fmaT(mid, mid, two_ih2), u[s]);
            const T y0 = y[s];
            rk_update<STAGE>(fmaT(ln + rn, ih2, loc), y[s], acc[s], t[s], st);
            if (STAGE == 4) y[s] = live ? y[s] : y0;
        }
    }
}

template <int KIND>
__device__ __noinline__ void run_pack(const QDesc* __restrict__ desc,
                                      const uint32_t* __restrict__ mem_idx, int count,
                                      unsigned int* qflags, unsigned int* status) {
    using T = double;
    const int lane = threadIdx.x;
    const QDesc* d = desc + mem_idx[0];
    int mem = -1;
    int64_t c = 0;
    int off = 0;
    int64_t steps = 0;   // the longest member's
    for (int m = 0; m < count; ++m) {
        const QDesc* dm = desc + mem_idx[m];
        const int nm = (int)dm->n;
        if (lane >= off && lane < off + nm) {
            mem = m;
            c = lane - off;
        }
        off += nm;
        steps = dm->nsteps > steps ? dm->nsteps : steps;
    }
    const bool valid = mem >= 0;
    const QDesc* me = desc + mem_idx[valid ? mem : 0];
    const int64_t n = me->n;
    const bool first = valid && c == 0;
    const bool last = valid && c == n - 1;
    T y[2], u[2], acc[2], t[2];
    const double* src[2] = {me->x_lo, me->x_hi};
    const double* pin[2] = {me->p_lo, me->p_hi};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        y[s] = valid ? src[s][c] : ghost<KIND, T>();
        u[s] = (valid && pin[s]) ? *pin[s] : T(0);
    }
    SysPrm<T> P;
    P.a0 = d->prm[0]; P.a1 = d->prm[1]; P.a2 = d->prm[2]; P.a3 = d->prm[3]; P.a4 = d->prm[4];
    const Steps<T> st = {d->h2, d->dt, d->dt6};
    const int64_t my_steps = me->nsteps;
    for (int64_t k = 0; k < steps; ++k) {
        const bool live = k < my_steps;
        pack_stage<KIND, 1>(y, acc, t, P, u, st, first, last, live);
        pack_stage<KIND, 2>(y, acc, t, P, u, st, first, last, live);
        pack_stage<KIND, 3>(y, acc, t, P, u, st, first, last, live);
        pack_stage<KIND, 4>(y, acc, t, P, u, st, first, last, live);
    }
    if (valid) {
        me->r_lo[c] = y[0];
        me->r_hi[c] = y[1];
        unsigned bits = 0;
        if (!finiteT(y[0]) || !finiteT(y[1])) bits |= ST_NONFINITE;
        if (y[0] > y[1]) bits |= ST_ORDER;
        if (bits) {
            atomicOr(&qflags[me->tag], bits);
            atomicOr(status, bits);
        }
    }
}

// Whole query in one wave (descriptor fields are wave-uniform; the host
// validated kind and E).
__device__ __forceinline__ unsigned run_query(const QDesc& d) {
    if (d.kind == K_CTM) return run_query_kind<K_CTM, 2>(d, 0);
    if (d.kind == K_RD) return run_query_kind<K_RD, 2>(d, 0);
    return run_query_kind<K_LIN3, 2>(d, 0);
}

// Work item (query, side).  Cooperative queries split into two waves, one per
// side, which halves the dependent chain of a query; the coupled LIN3 query
// runs whole in its side-0 item and its side-1 item is empty.
__device__ __forceinline__ bool item_is_empty(const QDesc& d, int side) {
    return d.kind == K_LIN3 && side == 1;
}
__device__ __forceinline__ bool item_is_whole(const QDesc& d) { return d.kind == K_LIN3; }
__device__ __forceinline__ unsigned run_item(const QDesc& d, int side) {
    if (d.kind == K_CTM) return run_query_kind<K_CTM, 1>(d, side);
    if (d.kind == K_RD) return run_query_kind<K_RD, 1>(d, side);
    return run_query_kind<K_LIN3, 2>(d, 0);
}

// lower > upper check of a finished query, by the wave that finished last
__device__ __forceinline__ unsigned order_bits(const QDesc& d) {
    unsigned bits = 0;
    for (int64_t j = threadIdx.x; j < d.n; j += WAVE)
        if (d.r_lo[j] > d.r_hi[j]) bits = ST_ORDER;
    return __ballot(bits) ? (unsigned)ST_ORDER : 0u;
}

__global__ __launch_bounds__(64) void batch_kernel(const QDesc* __restrict__ desc,
                                                   const BatchItem* __restrict__ items,
                                                   const uint32_t* __restrict__ members,
                                                   const uint64_t* n_items,
                                                   unsigned long long* counter,
                                                   unsigned int* qflags, unsigned int* pair,
                                                   unsigned int* status, int split) {
    const int lane = threadIdx.x;
    const uint64_t ni = wave_bcast(*n_items);
    const uint64_t total = split ? 2 * ni : ni;
    for (;;) {
        uint64_t u = 0;
        if (lane == 0) u = atomicAdd(counter, 1ULL);
        u = wave_bcast(u);
        if (u >= total) break;
        if (!split) {
            // whole queries (both sides in one wave, most work per wave) or a
            // pack of short ones
            const BatchItem it = items[u];
            if (it.count > 1) {
                const int kind = desc[members[it.start]].kind;
                if (kind == K_CTM)
                    run_pack<K_CTM>(desc, members + it.start, (int)it.count, qflags, status);
                else
                    run_pack<K_RD>(desc, members + it.start, (int)it.count, qflags, status);
                continue;
            }
            const QDesc d = desc[members[it.start]];
            const unsigned bits = run_query(d);
            if (lane == 0 && bits) {
                atomicOr(&qflags[d.tag], bits);
                atomicOr(status, bits);
            }
            continue;
        }
        // one side of item i (items are single queries when split)
        const uint64_t i = u >> 1;
        const int side = (int)(u & 1);
        const QDesc d = desc[members[items[i].start]];
        if (item_is_empty(d, side)) continue;
        unsigned bits = run_item(d, side);
        if (!item_is_whole(d)) {
            // publish this side, then the second side to finish checks the order
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            uint64_t old = 0;
            if (lane == 0)
                old = __hip_atomic_fetch_add(&pair[i], 1u, __ATOMIC_ACQ_REL,
                                             __HIP_MEMORY_SCOPE_AGENT);
            old = wave_bcast(old);
            if (old == 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                bits |= order_bits(d);
            }
        }
        if (lane == 0 && bits) {
            atomicOr(&qflags[d.tag], bits);
            atomicOr(status, bits);
        }
    }
}

__global__ __launch_bounds__(64) void single_kernel(QDesc d, unsigned int* status,
                                                    unsigned int* flags) {
    const unsigned bits = run_query(d);
    if (threadIdx.x == 0) {
        if (flags) *flags = bits;
        else if (bits) atomicOr(status, bits);
    }
}

__global__ __launch_bounds__(256) void zero_kernel(unsigned int* p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

// ctl[0]: claim counter (work items: two per sequence number, one per side),
// ctl[1]: status bits, ctl[2]: watermark (every sequence below it has been
// seen published), ctl[3]: grid quit word.  Only the waves holding the
// sequence at the watermark read the host ring; the others wait on device
// memory, so idle waves do not flood the host link with polls.  The first wave
// to reach the idle limit sets the quit word, and every other wave leaves at
// its next wait iteration or claim: the grid exits as a whole, and the host
// moves any query published to a sequence no wave will run to a new grid.
__global__ __launch_bounds__(64) void serve_kernel(ServeSlot* ring, int32_t slots,
                                                   unsigned long long* ctl,
                                                   volatile unsigned int* stop,
                                                   unsigned int* status, int64_t idle_cycles) {
    const int lane = threadIdx.x;
    unsigned long long* claim = ctl;
    unsigned long long* seen = ctl + 2;
    unsigned long long* quitw = ctl + 3;
    for (;;) {
        uint64_t u = 0, gq = 0;
        if (lane == 0) {
            gq = __hip_atomic_load(quitw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!gq) u = atomicAdd(claim, 1ULL);
        }
        if (wave_bcast(gq)) return;
        u = wave_bcast(u);
        const uint64_t t = u >> 1;
        const int side = (int)(u & 1);
        ServeSlot* sl = &ring[t % (uint64_t)slots];
        // Wait until the host publishes sequence t in this slot, the host asks
        // to stop, another wave ends the grid, or the idle limit passes.
        // Every branch ends the wait.
        const uint64_t t_start = wall_clock64();
        int quit = 0;
        for (uint32_t it = 0;; ++it) {
            uint64_t seq = 0, w = 0, q = 0;
            unsigned st = 0;
            if (lane == 0) {
                w = __hip_atomic_load(seen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                q = __hip_atomic_load(quitw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (w >= t)
                    seq = __hip_atomic_load(&sl->seq, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
                if ((it & 63u) == 0u)
                    st = __hip_atomic_load((unsigned int*)stop, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM);
            }
            seq = wave_bcast(seq);
            w = wave_bcast(w);
            q = wave_bcast(q);
            st = (unsigned)wave_bcast(st);
            if (seq == t + 1) break;
            if (st || q) { quit = 1; break; }
            if ((int64_t)(wall_clock64() - t_start) > idle_cycles) {
                if (lane == 0)
                    __hip_atomic_store(quitw, 1ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                quit = 1;
                break;
            }
            if (w >= t) __builtin_amdgcn_s_sleep(2);
            else __builtin_amdgcn_s_sleep(32);
        }
        if (quit) return;
        if (lane == 0) atomicMax(seen, (unsigned long long)(t + 1));
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
        const QDesc d = sl->d;
        const unsigned bits = item_is_empty(d, side) ? 0u : run_item(d, side);
        if (lane == 0) {
            sl->flags[side] = bits;
            if (bits & (ST_NONFINITE | ST_ORDER)) atomicOr(status, bits & (ST_NONFINITE | ST_ORDER));
            __hip_atomic_store(&sl->done[side], t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

hipError_t launch_batch(const QDesc* d, const BatchItem* items, const uint32_t* members,
                        const uint64_t* n_items, unsigned long long* counter,
                        unsigned int* qflags, unsigned int* pair, unsigned int* status,
                        int split, int64_t grid, hipStream_t s) {
    hipLaunchKernelGGL(batch_kernel, dim3((unsigned)grid), dim3(WAVE), 0, s, d, items, members,
                       n_items, counter, qflags, pair, status, split);
    return hipGetLastError();
}

hipError_t launch_single(const QDesc& d, unsigned int* status, unsigned int* flags,
                         hipStream_t s) {
    hipLaunchKernelGGL(single_kernel, dim3(1), dim3(WAVE), 0, s, d, status, flags);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, int64_t count, hipStream_t s) {
    const unsigned grid = (unsigned)((count + 255) / 256);
    hipLaunchKernelGGL(zero_kernel, dim3(grid > 0 ? grid : 1), dim3(256), 0, s,
                       (unsigned int*)p, count);
    return hipGetLastError();
}

hipError_t launch_server(ServeSlot* ring, int32_t slots, unsigned long long* ctl,
                         volatile unsigned int* stop, unsigned int* status, int64_t idle_cycles,
                         int64_t grid, hipStream_t s) {
    hipLaunchKernelGGL(serve_kernel, dim3((unsigned)grid), dim3(WAVE), 0, s, ring, slots, ctl,
                       stop, status, idle_cycles);
    return hipGetLastError();
}

}  // namespace reach
