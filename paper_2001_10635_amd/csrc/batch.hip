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
//                  query, or with `split` one side of a cooperative query) from
//                  a device counter until the batch is exhausted.
//   pack_kernel    the same for a packed batch, whose items are segment packs:
//                  queries sharing a wave at E cells per lane.
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
    bool begin;    // this lane holds cell 0 (read by segment packs only)
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
    L.begin = lane == 0;
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

// SEG: the query occupies a run of lanes inside the wave (a segment pack), so
// its first lane takes the left boundary value and its last lane the right
// ghost by a select, where a query spanning the whole wave gets them from the
// shifts' zero fill.
template <int KIND, int STAGE, int E, int S, bool SEG = false>
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
            if (SEG) Fprev = L.begin ? T(0) : Fprev;
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
            T ln = from_left(last_of<E>(in[s], L.shortl));
            if (SEG) ln = L.begin ? T(0) : ln;
            T rn = from_right(in[s][0]);
            if (E == 1 || SEG) rn = L.end ? T(0) : rn;
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
            if (SEG) ln[s] = L.begin ? T(0) : ln[s];
            rn[s] = from_right(in[s][0]);
            if (E == 1 || SEG) rn[s] = L.end ? T(0) : rn[s];
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

// Segment packs: several queries of one kind with bitwise equal constants and
// dt share a wave, E cells per lane (E = 2, 4, 8 or 16, one E per pack).  Member m
// runs on the L_m = ceil(n_m / E) lanes after the previous members', in the
// balanced layout of those lanes: the first F_m = n_m - L_m (E - 1) lanes hold
// E cells and the others E - 1 (the planner packs a query at this E only when
// F_m >= 0).  A member's first and last lanes take the chain's boundary values
// by a select, so members never read each other's cells; lanes past the last
// member hold ghosts and stay masked off.  The wave runs the longest member's
// steps, a member's lanes masked off once its own steps are done.  Per cell
// this is the single-query arithmetic, so every box is bitwise the one the
// query gets alone.
template <int KIND, int E>
__device__ __forceinline__ void run_seg(const QDesc* __restrict__ desc,
                                     const uint32_t* __restrict__ mem_idx, int count,
                                     unsigned int* qflags, unsigned int* status) {
    using T = double;
    constexpr int S = 2;
    const int lane = threadIdx.x;
    const QDesc* d0 = desc + mem_idx[0];
    int mem = -1, off = 0, base = 0, len = 0;
    int64_t steps = 0;   // the longest member's
    for (int m = 0; m < count; ++m) {
        const QDesc* dm = desc + mem_idx[m];
        const int l = (int)((dm->n + E - 1) / E);
        if (lane >= off && lane < off + l) {
            mem = m;
            base = off;
            len = l;
        }
        off += l;
        steps = dm->nsteps > steps ? dm->nsteps : steps;
    }
    const bool valid = mem >= 0;
    const QDesc* me = desc + mem_idx[valid ? mem : 0];
    const int64_t n = me->n;
    const int rel = lane - base;
    const int64_t F = n - (int64_t)len * (E - 1);   // lanes holding E cells
    Lanes L;
    L.shortl = rel >= F;
    L.cnt = !valid ? 0 : (L.shortl ? E - 1 : E);
    L.first = (int64_t)rel * E - (L.shortl ? (int64_t)rel - F : 0);
    L.begin = valid && rel == 0;
    L.end = valid && rel == len - 1;
    const double* src[2] = {me->x_lo, me->x_hi};
    const double* pin[2] = {me->p_lo, me->p_hi};
    T y[S][E];
    Inputs<T, E, S, IN_SCALAR> U;
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int e = 0; e < E; ++e)
            y[s][e] = (e < L.cnt) ? src[s][L.first + e] : ghost<KIND, T>();
        U.u[s] = (valid && pin[s]) ? *pin[s] : T(0);
    }
    SysPrm<T> P;
    P.a0 = d0->prm[0]; P.a1 = d0->prm[1]; P.a2 = d0->prm[2]; P.a3 = d0->prm[3]; P.a4 = d0->prm[4];
    const Steps<T> st = {d0->h2, d0->dt, d0->dt6};
    T acc[S][E], t[S][E];
    const int64_t mine = valid ? me->nsteps : 0;
    for (int64_t k = 0; k < steps; ++k) {
        if (k < mine) {
            bal_stage<KIND, 1, E, S, true>(y, acc, t, P, U, st, L);
            bal_stage<KIND, 2, E, S, true>(y, acc, t, P, U, st, L);
            bal_stage<KIND, 3, E, S, true>(y, acc, t, P, U, st, L);
            bal_stage<KIND, 4, E, S, true>(y, acc, t, P, U, st, L);
        }
    }
    unsigned bits = 0;
    double* dst[2] = {me->r_lo, me->r_hi};
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (e < L.cnt) {
            const int64_t j = L.first + e;
            dst[0][j] = y[0][e];
            dst[1][j] = y[1][e];
            if (!finiteT(y[0][e]) || !finiteT(y[1][e])) bits |= ST_NONFINITE;
            if (y[0][e] > y[1][e]) bits |= ST_ORDER;
        }
    }
    if (bits) {
        atomicOr(&qflags[me->tag], bits);
        atomicOr(status, bits);
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
            // a whole query over the wave (both sides, E = ceil(n / 64))
            const BatchItem it = items[u];
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

// Persistent worker of a packed batch: every item is a segment pack.  The
// packs' bodies are inlined into this one kernel (no calls).  EMAX is the
// widest pack it runs: with EMAX = 8 its registers are capped for three waves
// per SIMD (it runs fastest at two); the 16-cell bodies need ~240 registers,
// so EMAX = 16 fits two waves per SIMD and runs fastest at one, whose 32
// independent cell-sides per stage keep the SIMD issuing.
template <int EMAX>
__global__ __launch_bounds__(64, EMAX > 8 ? 2 : 3) void pack_kernel(
        const QDesc* __restrict__ desc, const BatchItem* __restrict__ items,
        const uint32_t* __restrict__ members, const uint64_t* n_items,
        unsigned long long* counter, unsigned int* qflags, unsigned int* status) {
    const int lane = threadIdx.x;
    const uint64_t ni = wave_bcast(*n_items);
    for (;;) {
        uint64_t u = 0;
        if (lane == 0) u = atomicAdd(counter, 1ULL);
        u = wave_bcast(u);
        if (u >= ni) break;
        const BatchItem it = items[u];
        const int kind = desc[members[it.start]].kind;
        const uint32_t* mi = members + it.start;
        const int cnt = it.count;
        const int ki = kind == K_CTM ? 0 : kind == K_RD ? 1 : 2;
        const int ei = it.E == 2 ? 0 : it.E == 4 ? 1 : it.E == 8 ? 2 : 3;
        switch (4 * ki + ei) {
            case 0: run_seg<K_CTM, 2>(desc, mi, cnt, qflags, status); break;
            case 1: run_seg<K_CTM, 4>(desc, mi, cnt, qflags, status); break;
            case 2: run_seg<K_CTM, 8>(desc, mi, cnt, qflags, status); break;
            case 4: run_seg<K_RD, 2>(desc, mi, cnt, qflags, status); break;
            case 5: run_seg<K_RD, 4>(desc, mi, cnt, qflags, status); break;
            case 6: run_seg<K_RD, 8>(desc, mi, cnt, qflags, status); break;
            case 8: run_seg<K_LIN3, 2>(desc, mi, cnt, qflags, status); break;
            case 9: run_seg<K_LIN3, 4>(desc, mi, cnt, qflags, status); break;
            case 10: run_seg<K_LIN3, 8>(desc, mi, cnt, qflags, status); break;
            default:   // E = 16 (the host gives such packs to EMAX = 16 only)
                if constexpr (EMAX > 8) {
                    if (ki == 0) run_seg<K_CTM, 16>(desc, mi, cnt, qflags, status);
                    else if (ki == 1) run_seg<K_RD, 16>(desc, mi, cnt, qflags, status);
                    else run_seg<K_LIN3, 16>(desc, mi, cnt, qflags, status);
                }
                break;
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

// A served item's box arrives in pinned host staging; the wave that runs it
// copies what it reads (its side, or both sides of a coupled LIN3 query) into
// the query's device pool block, points its copy of the descriptor there, and
// runs from it.  The fences make the lanes' stores visible to the wave's own
// loads of other lanes' cells (agent-scope release, then acquire: the vector
// L1 may hold the block from an earlier query).
__device__ __forceinline__ void park_box(QDesc& d, int side) {
    const int lane = threadIdx.x;
    const int64_t n = d.n;
    double* blk = d.park;
    const bool both = item_is_whole(d);
    for (int s = 0; s < 2; ++s) {
        if (!both && s != side) continue;
        const double* src = s ? d.x_hi : d.x_lo;
        double* dst = blk + (int64_t)s * n;
        for (int64_t j = lane; j < n; j += WAVE) dst[j] = src[j];
        if (d.p_lo && lane == 0) blk[2 * n + s] = s ? *d.p_hi : *d.p_lo;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    d.x_lo = blk;
    d.x_hi = blk + n;
    if (d.p_lo) {
        d.p_lo = blk + 2 * n;
        d.p_hi = blk + 2 * n + 1;
    }
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
        QDesc d = sl->d;
        const bool empty = item_is_empty(d, side);
        if (d.park && !empty) park_box(d, side);
        const unsigned bits = empty ? 0u : run_item(d, side);
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
                        int split, int packed, int64_t grid, hipStream_t s) {
    if (packed == 2)
        hipLaunchKernelGGL(pack_kernel<16>, dim3((unsigned)grid), dim3(WAVE), 0, s, d, items,
                           members, n_items, counter, qflags, status);
    else if (packed)
        hipLaunchKernelGGL(pack_kernel<8>, dim3((unsigned)grid), dim3(WAVE), 0, s, d, items,
                           members, n_items, counter, qflags, status);
    else
        hipLaunchKernelGGL(batch_kernel, dim3((unsigned)grid), dim3(WAVE), 0, s, d, items,
                           members, n_items, counter, qflags, pair, status, split);
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
