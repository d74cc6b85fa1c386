// HBM ceiling probe for the embedding pass: a plain stream that reads two
// arrays and writes two (the byte pattern of one embedding pass, x_lo and
// x_hi in, r_lo and r_hi out) with no arithmetic, in the launch shapes a
// streaming kernel on gfx950 can take.  It measures the rate the device
// sustains for that traffic, against which the one-step embedding pass is
// judged; it is not part of the reachability method.
//
// Each thread moves U 16-byte vectors of each input per round (2U loads in
// flight before the first store), rounds strided over a grid of `blocks`
// workgroups of 256 threads; NT selects non-temporal loads and stores.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/reach_probe.h"

namespace {

typedef double V2 __attribute__((ext_vector_type(2)));

template <int U, bool NT>
__global__ __launch_bounds__(256) void stream2_kernel(const V2* __restrict__ a0,
                                                      const V2* __restrict__ a1,
                                                      V2* __restrict__ b0, V2* __restrict__ b1,
                                                      int64_t nvec) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; base < nvec;
         base += stride * U) {
        V2 x[U], y[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = base + u * stride;
            if (i < nvec) {
                if (NT) {
                    x[u] = __builtin_nontemporal_load(a0 + i);
                    y[u] = __builtin_nontemporal_load(a1 + i);
                } else {
                    x[u] = a0[i];
                    y[u] = a1[i];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = base + u * stride;
            if (i < nvec) {
                if (NT) {
                    __builtin_nontemporal_store(x[u], b0 + i);
                    __builtin_nontemporal_store(y[u], b1 + i);
                } else {
                    b0[i] = x[u];
                    b1[i] = y[u];
                }
            }
        }
    }
}

template <int U, bool NT>
hipError_t go(const void* a0, const void* a1, void* b0, void* b1, int64_t nvec, int64_t blocks,
              hipStream_t s) {
    hipLaunchKernelGGL((stream2_kernel<U, NT>), dim3((unsigned)blocks), dim3(256), 0, s,
                       (const V2*)a0, (const V2*)a1, (V2*)b0, (V2*)b1, nvec);
    return hipGetLastError();
}

}  // namespace

extern "C" int reach_probe_stream2(const void* in0, const void* in1, void* out0, void* out1,
                                   int64_t bytes, int32_t unroll, int32_t nontemporal,
                                   int64_t blocks, void* stream) {
    if (!in0 || !in1 || !out0 || !out1 || bytes <= 0 || bytes % 16 != 0) return -1;
    if (((uintptr_t)in0 | (uintptr_t)in1 | (uintptr_t)out0 | (uintptr_t)out1) & 15) return -1;
    if (blocks < 1 || blocks > (int64_t)1 << 31) return -1;
    const int64_t nvec = bytes / 16;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    const bool nt = nontemporal != 0;
    switch (unroll) {
        case 1: e = nt ? go<1, true>(in0, in1, out0, out1, nvec, blocks, s)
                       : go<1, false>(in0, in1, out0, out1, nvec, blocks, s); break;
        case 2: e = nt ? go<2, true>(in0, in1, out0, out1, nvec, blocks, s)
                       : go<2, false>(in0, in1, out0, out1, nvec, blocks, s); break;
        case 4: e = nt ? go<4, true>(in0, in1, out0, out1, nvec, blocks, s)
                       : go<4, false>(in0, in1, out0, out1, nvec, blocks, s); break;
        case 8: e = nt ? go<8, true>(in0, in1, out0, out1, nvec, blocks, s)
                       : go<8, false>(in0, in1, out0, out1, nvec, blocks, s); break;
        default: return -1;
    }
    return e == hipSuccess ? 0 : -3;
}
