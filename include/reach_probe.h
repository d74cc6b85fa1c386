/*
 * reach_probe.h -- measurement probe shipped beside the reachability library
 * (libreach_probe.so).  Not part of the method: it gives the HBM rate the
 * device sustains for the traffic of one embedding pass (two arrays read, two
 * written), the ceiling the one-step embedding pass is compared with.
 */
#ifndef REACH_PROBE_H
#define REACH_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* out0 = in0 and out1 = in1 over `bytes` bytes each, by a streaming kernel
   launched on `stream` (a hipStream_t; NULL = the default stream).
   All four are DEVICE pointers, 16-byte aligned, caller-owned, not overlapping.
   unroll: 16-byte vectors per thread and input in flight per round (1, 2, 4
   or 8); nontemporal: nonzero for non-temporal loads and stores; blocks:
   workgroups of 256 threads (grid-stride rounds).  Returns 0 when launched,
   -1 for bad arguments (bytes not a positive multiple of 16, misaligned or
   NULL pointers, unroll not built, blocks outside [1, 2^31]), -3 when the
   launch fails.  Stream-ordered: completion is the stream's. */
int reach_probe_stream2(const void* in0, const void* in1, void* out0, void* out1,
                        int64_t bytes, int32_t unroll, int32_t nontemporal, int64_t blocks,
                        void* stream);

#ifdef __cplusplus
}
#endif
#endif /* REACH_PROBE_H */
