// Many small embedding queries on gfx950: offline batches and online serving.
//
// Every query (FP64, n <= 512 cells, scalar input) is run by one wavefront
// with its whole lower/upper state in registers (E = 1, 2, 4 or 8 cells per
// lane), all N RK4 steps in one go: no halo, no HBM traffic inside the step
// loop.  The arithmetic per cell is the same code the large-n embedding kernel
// runs, so a query gives the same box alone, in a batch, or served.
//
//   batch_kernel   persistent grid; each wave pops the next descriptor from a
//                  device counter until the batch is exhausted.
//   single_kernel  one query per launch (the baseline the batch is compared with).
//   serve_kernel   persistent grid fed through a ring of descriptors in pinned
//                  host memory; each wave claims the next ring sequence number,
//                  waits (bounded) until the host publishes it, runs it and
//                  publishes completion.  Waves leave when the host sets the stop
//                  flag or after an idle limit, so the grid always drains.
#include "dev.hpp"
#include "kernels.hpp"

namespace reach {

__device__ __forceinline__ uint64_t wave_bcast(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

template <int KIND, int E, bool MASKED>
__device__ __noinline__ unsigned run_query_E(const QDesc& d) {
    using T = double;
    const int lane = threadIdx.x;
    const int64_t n = d.n;
    T y[2][E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t j = (int64_t)lane * E + e;
        y[0][e] = (j < n) ? d.x_lo[j] : ghost<KIND, T>();
        y[1][e] = (j < n) ? d.x_hi[j] : ghost<KIND, T>();
    }
    Inputs<T, E, 2, IN_SCALAR> U;
    U.u[0] = d.p_lo ? *d.p_lo : T(0);
    U.u[1] = d.p_hi ? *d.p_hi : T(0);
    SysPrm<T> P;
    P.a0 = d.prm[0]; P.a1 = d.prm[1]; P.a2 = d.prm[2]; P.a3 = d.prm[3]; P.a4 = d.prm[4];
    const Steps<T> st = {d.h2, d.dt, d.dt6};
    const int64_t left = n - (int64_t)lane * E;
    Mask<E, MASKED, true> M{(int)(left < 0 ? 0 : (left > E ? E : left))};
    rk4_steps<KIND, T, E, 2, IN_SCALAR>(y, d.nsteps, P, U, st, M);
    unsigned bits = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t j = (int64_t)lane * E + e;
        if (j < n) {
            d.r_lo[j] = y[0][e];
            d.r_hi[j] = y[1][e];
            if (!finiteT(y[0][e]) || !finiteT(y[1][e])) bits |= ST_NONFINITE;
            if (y[0][e] > y[1][e]) bits |= ST_ORDER;
        }
    }
    const unsigned long long nf = __ballot(bits & ST_NONFINITE);
    const unsigned long long od = __ballot(bits & ST_ORDER);
    return (nf ? (unsigned)ST_NONFINITE : 0u) | (od ? (unsigned)ST_ORDER : 0u);
}

template <int KIND, int E>
__device__ __forceinline__ unsigned run_query_k(const QDesc& d) {
    if (d.n == (int64_t)WAVE * E) return run_query_E<KIND, E, false>(d);
    return run_query_E<KIND, E, true>(d);
}

template <int KIND>
__device__ __forceinline__ unsigned run_query_kind(const QDesc& d) {
    switch (d.E) {
        case 1: return run_query_k<KIND, 1>(d);
        case 2: return run_query_k<KIND, 2>(d);
        case 4: return run_query_k<KIND, 4>(d);
        default: return run_query_k<KIND, 8>(d);
    }
}

// The descriptor fields are wave-uniform; the host validated kind and E.
__device__ __forceinline__ unsigned run_query(const QDesc& d) {
    if (d.kind == K_CTM) return run_query_kind<K_CTM>(d);
    if (d.kind == K_RD) return run_query_kind<K_RD>(d);
    return run_query_kind<K_LIN3>(d);
}

__global__ __launch_bounds__(64) void batch_kernel(const QDesc* __restrict__ desc, int64_t nq,
                                                   unsigned long long* counter,
                                                   unsigned int* qflags, unsigned int* status) {
    const int lane = threadIdx.x;
    for (;;) {
        uint64_t i = 0;
        if (lane == 0) i = atomicAdd(counter, 1ULL);
        i = wave_bcast(i);
        if (i >= (uint64_t)nq) break;
        const QDesc d = desc[i];
        const unsigned bits = run_query(d);
        if (lane == 0) {
            qflags[d.tag] = bits;
            if (bits) atomicOr(status, bits);
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

// ctl[0]: claim counter, ctl[1]: status bits, ctl[2]: watermark (every
// sequence below it has been seen published).  Only the wave holding the
// sequence at the watermark reads the host ring; the others wait on device
// memory, so idle waves do not flood the host link with polls.
__global__ __launch_bounds__(64) void serve_kernel(ServeSlot* ring, int32_t slots,
                                                   unsigned long long* ctl,
                                                   volatile unsigned int* stop,
                                                   unsigned int* status, int64_t idle_cycles) {
    const int lane = threadIdx.x;
    unsigned long long* claim = ctl;
    unsigned long long* seen = ctl + 2;
    for (;;) {
        uint64_t t = 0;
        if (lane == 0) t = atomicAdd(claim, 1ULL);
        t = wave_bcast(t);
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
        const unsigned bits = run_query(d);
        if (lane == 0) {
            sl->flags = bits;
            if (bits) atomicOr(status, bits);
            __hip_atomic_store(&sl->done, t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

hipError_t launch_batch(const QDesc* d, int64_t nq, unsigned long long* counter,
                        unsigned int* qflags, unsigned int* status, int64_t grid,
                        hipStream_t s) {
    hipLaunchKernelGGL(batch_kernel, dim3((unsigned)grid), dim3(WAVE), 0, s, d, nq, counter,
                       qflags, status);
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
