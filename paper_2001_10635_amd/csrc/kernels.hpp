// Host-side interface between the C-ABI runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace reach {

// Bits of a context's device status word (the kernels use the same values).
enum { STATUS_NONFINITE = 1, STATUS_ORDER = 2 };

// Kernel-side parameters of a system (CTM {v, w, w*c, q}, RD {1/h^2, 2/h^2},
// LIN3 {aL, aD, aR, b}) from the C-ABI parameter array.
void kernel_params(int kind, const double* prm, double out[5]);

// One HBM pass of the embedding: `ksteps` RK4 steps on every tile.
// Tile w reads cells [w*OUT, w*OUT + 64E) of src and writes the cells it
// owns to dst: [0, 64E - H) for tile 0, [w*OUT + H, w*OUT + 64E - H) for
// the others, up to n for the tile whose window reaches the chain's end.
struct EmbedPass {
    const void* src_lo;
    const void* src_hi;
    void* dst_lo;
    void* dst_hi;
    const void* p_lo;
    const void* p_hi;
    int64_t n;        // cells in the chain
    int64_t W;        // tiles
    int64_t OUT;      // tile stride (64E - 2H); 0 when W == 1
    int64_t ksteps;   // RK4 steps this pass
    int32_t H;        // halo cells per cut edge (4 * steps per pass)
    int32_t aligned;  // every array 16-byte aligned
    int32_t check;    // last pass: report non-finite / lower > upper
    int32_t per_xcd;  // tiles per XCD in the blockIdx -> tile map
    int32_t nt;       // non-temporal global accesses (a pass whose data is not reused soon)
    double prm[5];
    double h2, dt, dt6;
    unsigned int* status;
};

// kind: 1 CTM, 2 RD, 3 LIN3; mode: 0 scalar input, 1 per-cell input;
// dtype: 0 f64, 1 f32.  Returns hipErrorInvalidValue for an E the library
// does not instantiate.
// S: sides per wave (2 = lower and upper together, 1 = one side per wave;
// 1 only for the cooperative CTM and RD chains).  W counts tiles per side.
// pair (S = 1, W = 1 only): one block of two waves, lower and upper, that
// also checks lower <= upper (no order-check launch needed); grid unused.
hipError_t launch_embed(int kind, int mode, int dtype, int E, int S, bool pair,
                        const EmbedPass& a, int64_t grid, hipStream_t stream);
bool embed_has_shape(int kind, int dtype, int E, int S);
int embed_max_E(int dtype, int S);
// Flags lower > upper anywhere in a finished box.
hipError_t launch_order_check(int dtype, const void* lo, const void* hi, int64_t n,
                              unsigned int* status, hipStream_t stream);

// One pass of the growth-bound method: tiles [0, W) advance the center, tiles
// [W, 2W) the half-width; `first` forms them from the box (x_lo, x_hi).
struct GbPass {
    const void* x_lo;
    const void* x_hi;
    const void* src_c;
    const void* src_r;
    void* dst_c;
    void* dst_r;
    const void* p_lo;
    const void* p_hi;
    int64_t n, W, OUT, ksteps;
    int32_t H, first, per_xcd, pad;
    double prm[5];     // the system (kernel_params)
    double prm_r[5];   // the growth dynamics: {C_sub, C_diag, C_sup, |b|}
    double h2, dt, dt6;
};
hipError_t launch_gb(int kind, int mode, int dtype, int E, const GbPass& a, int64_t grid,
                     hipStream_t stream);
hipError_t launch_gb_combine(int dtype, const void* c, const void* r, int64_t n, void* lo,
                             void* hi, unsigned int* status, hipStream_t stream);
bool gb_has_E(int E);

// One RK4 step of the 3-D heat grid for `sides` independent states
// (lower / upper, or center / half-width).  Tiles are x-y columns of 64 by
// WV * P cells streaming through z; TX * TY tiles per side, each writing its
// OX by OY output cells (64 - 8 and WV * P - 8: a 4-cell halo per cut face).
struct HeatPass {
    const void* src[2];
    void* dst[2];
    int64_t nx, ny, nz;
    int32_t TX, TY, OX, OY;
    int32_t sides;
    int32_t per_xcd;    // tiles per XCD in the blockIdx -> tile map
    double a;           // alpha / dx^2
    double h2, dt, dt6;
    // level j of a step updates w <- y + cw[j] (s - 6 w), cw[j] = a dt / (4 - j)
    double cw[4], m6cw[4];     // cw and -6 cw
    float cwf[4], m6cwf[4];    // the same in FP32
    unsigned int* status;
};
hipError_t launch_heat3d(int dtype, int P, int WV, const HeatPass& a, int64_t grid,
                         hipStream_t stream);
bool heat_has_shape(int dtype, int P, int WV);
// c = (lo + hi) / 2, r = (hi - lo) / 2 elementwise (growth-bound start).
hipError_t launch_center_radius(int dtype, const void* lo, const void* hi, int64_t n, void* c,
                                void* r, hipStream_t stream);

struct McArgs {
    const void* x_lo;
    const void* x_hi;
    const void* p_lo;
    const void* p_hi;
    void* part_min;     // [nw][E][64] interleaved partials of the kernel's type
    void* part_max;
    int64_t n;
    int64_t n_in;
    int64_t nsteps;
    int64_t s0;
    int64_t m;
    int64_t nw;         // resident waves (= grid)
    uint64_t seed;
    int32_t aligned;
    double prm[5];
    double h2, dt, dt6;
};
hipError_t launch_mc(int kind, int mode, int dtype, int E, const McArgs& a, hipStream_t stream);
// r_min / r_max [n] from the partials of `nw` <= kMcMaxWaves waves of which
// every group-th slot holds a partial (mc_kernel folds each workgroup's waves
// into the group's first slot: group = mc_waves_per_group(); one wave per
// slot: group = 1).  The partials are overwritten (chunk results are written in
// place); reports non-finite values.
constexpr int64_t kMcMaxWaves = 4096;
hipError_t launch_mc_reduce(int dtype, int E, void* part_min, void* part_max,
                            int64_t nw, int64_t group, int64_t n, void* r_min, void* r_max,
                            unsigned int* status, hipStream_t stream);
int mc_waves_per_group();
bool mc_has_E(int dtype, int E);
int mc_max_E(int dtype);

// Batch / serving descriptor of one FP64 query (n <= 512).
struct QDesc {
    int32_t kind;
    int32_t E;          // cells per lane: batch_cells_per_lane(n), 1..8
    int64_t n;
    int64_t nsteps;
    double prm[5];
    const double* p_lo;  // scalar input interval (NULL when n_in == 0), device-visible
    const double* p_hi;
    double h2, dt, dt6;
    const double* x_lo;
    const double* x_hi;
    double* r_lo;
    double* r_hi;
    int64_t tag;        // caller's index (batch) or ticket slot (serving)
    // Served queries: a host-written word (pinned, coherent host memory) that
    // the kernel reads every kCancelEvery steps; nonzero ends the query early
    // with the ST_CANCELLED bit.  NULL for batches.
    const unsigned int* cancel;
    // Served queries (persistent kernel): the query's device pool block
    // [x_lo | x_hi | u_lo | u_hi] (2n + 2 values).  x_lo .. p_hi then point
    // into pinned host staging, and the wave that runs a side first copies
    // that side's box (both for the coupled LIN3) into the block and runs
    // from there.  NULL otherwise.
    double* park;
};

// Status bit of a served query that stopped on its cancel word.
enum { STATUS_CANCELLED = 4 };
constexpr int64_t kCancelEvery = 64;

// Cells per lane of a batched query: ceil(n / 64) (lanes hold E or E - 1).
inline int batch_cells_per_lane(int64_t n) { return (int)((n + 63) / 64); }

// Segment packs: queries of one kind, constants and dt sharing a wave at
// E cells per lane (kSegE), member m on ceil(n_m / E) lanes, at most 64 lanes
// and so at most 64 members.
constexpr int kSegE[] = {2, 4, 8, 16};
constexpr int kPackMax = 64;

// One work item of a batch: the queries members[start .. start + count) --
// a single query spread over the whole wave (E = 0, count 1) or a segment
// pack at E cells per lane.
struct BatchItem {
    uint32_t start;
    uint16_t count;
    uint16_t E;
};

// Persistent batch worker: `grid` waves pull work items through *counter:
// items[0 .. *n_items) (d[] in the caller's order, members[] the query
// indices of the items in launch order).  packed 1: every item is a segment
// pack of at most 8 cells per lane (E > 0), run by the packing kernel (room
// for three waves per SIMD); packed 2: some pack has 16 cells per lane, all
// run by the wide packing kernel (room for two); packed 0:
// every item is one query (E = 0), or with `split` two per item (one per side
// of a cooperative chain), pair[i] counting the finished sides of item i.
hipError_t launch_batch(const QDesc* d, const BatchItem* items, const uint32_t* members,
                        const uint64_t* n_items, unsigned long long* counter,
                        unsigned int* qflags, unsigned int* pair, unsigned int* status,
                        int split, int packed, int64_t grid, hipStream_t stream);
// Default waves per compute unit of the batch kernels: the one-query kernel
// and the narrow packing kernel two per SIMD (the narrow one fits three, which
// measures slower), the wide packing kernel one per SIMD (16 cells give one
// wave enough independent work to keep its SIMD issuing; two measure slower).
constexpr int kBatchWavesPerCU = 8;
constexpr int kPackWavesPerCU = 8;
constexpr int kWideWavesPerCU = 4;
// Zero `count` 32-bit words (a kernel, so it can sit in a captured graph).
hipError_t launch_zero(void* p, int64_t count, hipStream_t stream);
// One query with a plain launch (the one-launch-per-query baseline).  With
// `flags` non-NULL, lane 0 stores the query's status bits there (a served
// query's own word) instead of OR-ing them into `status`.
hipError_t launch_single(const QDesc& d, unsigned int* status, unsigned int* flags,
                         hipStream_t stream);

// Serving ring (see server.cpp): slots live in pinned host memory.
struct ServeSlot {
    QDesc d;
    unsigned long long seq;      // sequence published in this slot (+1), 0 = empty
    unsigned long long done[2];  // sequence whose lower / upper side completed (+1)
    unsigned int flags[2];       // status bits of each side
    unsigned int cancel;         // set by the host to stop the query (d.cancel points here)
    unsigned int pad;
};
// ctl: device words [claim counter, status, published watermark, grid quit].
// A wave that reaches the idle limit sets the quit word and every other wave
// leaves at its next wait or claim, so the grid always exits as a whole.
hipError_t launch_server(ServeSlot* ring, int32_t slots, unsigned long long* ctl,
                         volatile unsigned int* stop, unsigned int* status,
                         int64_t idle_cycles, int64_t grid, hipStream_t stream);

// With `device` current: looks up, once per device, the device address of
// the fixed scratch array of reach_montecarlo_noalloc.
hipError_t noalloc_setup(int device);

}  // namespace reach
