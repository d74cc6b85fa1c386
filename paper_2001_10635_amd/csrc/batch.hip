// Many small embedding queries on gfx950: offline batches and online serving.
//
// Every query (FP64, n <= 512 cells, scalar input) is run by one wavefront
// with its whole lower/upper state in registers (E = 1, 2, 4 or 8 cells per
// lane), all N RK4 steps in one go: no halo, no HBM traffic inside the step
// loop.  The arithmetic per cell is the same code the large-n embedding kernel
// runs, so a query gives the same box alone, in a batch, or served.
//
//   batch_kernel   persistent grid; each wave pops the next work item (a whole
//                  query, or with `split` one side of a cooperative query) from
//                  a device counter until the batch is exhausted.
//   single_kernel  one query per launch (the baseline the batch is compared with).
//   serve_kernel   persistent grid fed through a ring of descriptors in pinned
//                  host memory; each wave claims the next work item (sequence
//                  number and side), waits (bounded) until the host publishes
//                  it, runs it and publishes that side's completion.  Waves leave when the host sets the stop
//                  flag or after an idle limit, so the grid always drains.
#include "dev.hpp"
#include "kernels.hpp"

namespace reach {

__device__ __forceinline__ uint64_t wave_bcast(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// One query, or one side of it: S = 2 runs both sides in this wave, S = 1
// only side `side` (cooperative systems, whose sides do not interact).
template <int KIND, int E, bool MASKED, int S>
__device__ __noinline__ unsigned run_query_E(const QDesc& d, int side) {
    using T = double;
    const int lane = threadIdx.x;
    const int64_t n = d.n;
    const double* src[2] = {d.x_lo, d.x_hi};
    double* dst[2] = {d.r_lo, d.r_hi};
    const double* pin[2] = {d.p_lo, d.p_hi};
    T y[S][E];
    Inputs<T, E, S, IN_SCALAR> U;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int sd = S == 1 ? side : s;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t j = (int64_t)lane * E + e;
            y[s][e] = (j < n) ? src[sd][j] : ghost<KIND, T>();
        }
        U.u[s] = pin[sd] ? *pin[sd] : T(0);
    }
    SysPrm<T> P;
    P.a0 = d.prm[0]; P.a1 = d.prm[1]; P.a2 = d.prm[2]; P.a3 = d.prm[3]; P.a4 = d.prm[4];
    const Steps<T> st = {d.h2, d.dt, d.dt6};
    const int64_t left = n - (int64_t)lane * E;
    Mask<E, MASKED, true> M{(int)(left < 0 ? 0 : (left > E ? E : left))};
    rk4_steps<KIND, T, E, S, IN_SCALAR>(y, d.nsteps, P, U, st, M);
    unsigned bits = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t j = (int64_t)lane * E + e;
        if (j < n) {
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

template <int KIND, int E, int S>
__device__ __forceinline__ unsigned run_query_k(const QDesc& d, int side) {
    if (d.n == (int64_t)WAVE * E) return run_query_E<KIND, E, false, S>(d, side);
    return run_query_E<KIND, E, true, S>(d, side);
}

template <int KIND, int S>
__device__ __forceinline__ unsigned run_query_kind(const QDesc& d, int side) {
    switch (d.E) {
        case 1: return run_query_k<KIND, 1, S>(d, side);
        case 2: return run_query_k<KIND, 2, S>(d, side);
        case 4: return run_query_k<KIND, 4, S>(d, side);
        default: return run_query_k<KIND, 8, S>(d, side);
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

__global__ __launch_bounds__(64) void batch_kernel(const QDesc* __restrict__ desc, int64_t nq,
                                                   unsigned long long* counter,
                                                   unsigned int* qflags, unsigned int* pair,
                                                   unsigned int* status, int split) {
    const int lane = threadIdx.x;
    const uint64_t items = split ? 2 * (uint64_t)nq : (uint64_t)nq;
    for (;;) {
        uint64_t u = 0;
        if (lane == 0) u = atomicAdd(counter, 1ULL);
        u = wave_bcast(u);
        if (u >= items) break;
        if (!split) {
            // whole queries: both sides in one wave (most work per wave)
            const QDesc d = desc[u];
            const unsigned bits = run_query(d);
            if (lane == 0 && bits) {
                atomicOr(&qflags[d.tag], bits);
                atomicOr(status, bits);
            }
            continue;
        }
        const uint64_t i = u >> 1;
        const int side = (int)(u & 1);
        const QDesc d = desc[i];
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

__global__ __launch_bounds__(64) void single_kernel(QDesc d, unsigned int* status) {
    const unsigned bits = run_query(d);
    if (threadIdx.x == 0 && bits) atomicOr(status, bits);
}

__global__ __launch_bounds__(256) void zero_kernel(unsigned int* p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

// ctl[0]: claim counter (work items: two per sequence number, one per side),
// ctl[1]: status bits, ctl[2]: watermark (every sequence below it has been
// seen published).  Only the waves holding the sequence at the watermark read
// the host ring; the others wait on device memory, so idle waves do not flood
// the host link with polls.
__global__ __launch_bounds__(64) void serve_kernel(ServeSlot* ring, int32_t slots,
                                                   unsigned long long* ctl,
                                                   volatile unsigned int* stop,
                                                   unsigned int* status, int64_t idle_cycles) {
    const int lane = threadIdx.x;
    unsigned long long* claim = ctl;
    unsigned long long* seen = ctl + 2;
    for (;;) {
        uint64_t u = 0;
        if (lane == 0) u = atomicAdd(claim, 1ULL);
        u = wave_bcast(u);
        const uint64_t t = u >> 1;
        const int side = (int)(u & 1);
        ServeSlot* sl = &ring[t % (uint64_t)slots];
        // Wait until the host publishes sequence t in this slot, the host asks
        // to stop, or the idle limit passes.  Every branch ends the wait.
        const uint64_t t_start = wall_clock64();
        int quit = 0;
        for (uint32_t it = 0;; ++it) {
            uint64_t seq = 0, w = 0;
            unsigned st = 0;
            if (lane == 0) {
                w = __hip_atomic_load(seen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (w >= t)
                    seq = __hip_atomic_load(&sl->seq, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
                if ((it & 63u) == 0u)
                    st = __hip_atomic_load((unsigned int*)stop, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM);
            }
            seq = wave_bcast(seq);
            w = wave_bcast(w);
            st = (unsigned)wave_bcast(st);
            if (seq == t + 1) break;
            if (st) { quit = 1; break; }
            if ((int64_t)(wall_clock64() - t_start) > idle_cycles) { quit = 1; break; }
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
            if (bits) atomicOr(status, bits);
            __hip_atomic_store(&sl->done[side], t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

hipError_t launch_batch(const QDesc* d, int64_t nq, unsigned long long* counter,
                        unsigned int* qflags, unsigned int* pair, unsigned int* status,
                        int split, int64_t grid, hipStream_t s) {
    hipLaunchKernelGGL(batch_kernel, dim3((unsigned)grid), dim3(WAVE), 0, s, d, nq, counter,
                       qflags, pair, status, split);
    return hipGetLastError();
}

hipError_t launch_single(const QDesc& d, unsigned int* status, hipStream_t s) {
    hipLaunchKernelGGL(single_kernel, dim3(1), dim3(WAVE), 0, s, d, status);
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
