/*
 * reach.h -- C ABI of the MI355X (gfx950) interval-reachability library.
 *
 * The library computes interval reachable sets of a nonlinear system
 * x' = f(t, x, p) from an interval initial set and constant inputs drawn from
 * an interval, following PIRK (Devonport, Khaled, Arcak, Zamani, arXiv
 * 2001.10635):
 *   - reach_embed_rk4: the mixed-monotonicity method.  The embedding system
 *     of Sec. 2.1 (state (x, xh) of dimension 2n, right-hand side
 *     (d(x, p, xh, ph), d(xh, ph, x, p)) for a decomposition function d with
 *     d(x, p, x, p) = f(x, p)) is integrated by classical RK4 from
 *     (lower, upper) with inputs (lower, upper), Algorithm 3 with Algorithm 1
 *     as integrator.  The result [r_lo, r_hi] over-approximates the reachable
 *     set (Sec. 2.1).
 *   - reach_montecarlo: the Monte Carlo method of Sec. 2.1 / Algorithm 4:
 *     uniform samples of the initial box (and input box) integrated by RK4,
 *     reduced to the per-dimension min / max.
 *   - reach_mc_samples: the sample count m = ceil((2n/eps) ln(2n/delta)) of
 *     the Monte Carlo guarantee (Sec. 2.1, Algorithm 4).
 *   - reach_embed_rk4_batch, reach_server_*: many small embeddings at once,
 *     by a persistent kernel (offline batch) or by a continuously fed request
 *     loop (online serving).  These answer the "many reachable sets" use of
 *     the paper's vehicle study and its reachability-as-a-service interface
 *     (Sec. 1); each query is the same computation as reach_embed_rk4.
 *
 * Integrator (Algorithm 1, read as the classical method): for step k,
 * t = t0 + k dt (computed, not accumulated), stages at t, t + dt/2,
 * t + dt/2, t + dt with inputs z, z + dt/2 K1, z + dt/2 K2, z + dt K3, and
 * z <- z + dt/6 (K1 + 2 K2 + 2 K3 + K4).  All built-in systems are autonomous.
 *
 * Built-in systems (one-dimensional chains, cell i couples to i-1 and i+1):
 *   REACH_CTM  prm = {v, w, c, q}: cell transmission model of the n-link road
 *              (Sec. 5.1): F_i = min(v y_i, w (c - y_{i+1}), q) for i < n-1,
 *              F_{n-1} = min(v y_{n-1}, q) (free outflow), zero inflow into
 *              cell 0, f_i = F_{i-1} - F_i.  Cooperative: d = f.  n_in = 0.
 *   REACH_RD   prm = {h}: reaction-diffusion, f_i = (y_{i-1} - 2 y_i +
 *              y_{i+1}) / h^2 - y_i^3 + u, Dirichlet ghosts 0.  Cooperative and
 *              increasing in u: d = f.  n_in = 0, 1 (shared u) or n.
 *   REACH_LIN3 prm = {aL, aD, aR, b}: f_i = aL y_{i-1} + aD y_i + aR y_{i+1}
 *              + b u, ghosts 0, with the sign-split decomposition function
 *              d_i = aD x_i + aL+ x_{i-1} + aL- xh_{i-1} + aR+ x_{i+1}
 *                    + aR- xh_{i+1} + b+ p_i + b- ph_i.
 *              n_in = 0, 1 or n.
 *
 * Built-in grid system (heat diffusion case study, Sec. 5):
 *   REACH_HEAT3D prm = {nx, ny, nz, alpha, dx}: the heat equation on an
 *              nx * ny * nz grid of spacing dx, n = nx ny nz, cell (x, y, z)
 *              at index x + nx (y + ny z).  f = alpha / dx^2 times the sum
 *              over the six directions of (neighbour - own).  Every face is
 *              insulated (a direction leaving the grid adds nothing) except
 *              x = nx - 1, whose outside is held at temperature 0.  Linear
 *              with non-negative couplings (alpha >= 0): d = f.  n_in = 0.
 *              nx, ny, nz are integers >= 1, nx < 2^31, dx > 0.
 *              Entry points: reach_embed_rk4 (and its tube, plan, autotune
 *              and workspace queries) and reach_growth_bound; the Monte Carlo,
 *              batch and serving calls return REACH_E_UNSUPPORTED.
 *
 * Conventions (all entry points):
 *   - Array pointers are DEVICE pointers (hipMalloc / torch tensors on the
 *     GPU) unless stated otherwise, owned by the caller.  The library never
 *     allocates or frees caller memory; its own allocations are a few status
 *     words per context, pinned host staging for batch descriptors, and the
 *     serving ring.
 *   - Arrays are contiguous SoA vectors of n elements of the call's dtype
 *     (double for REACH_F64, float for REACH_F32); input arrays have n_in
 *     elements.  Element i is cell i.
 *   - Calls that take a `stream` (a hipStream_t, NULL = the default stream)
 *     are stream-ordered and return only argument or launch errors; what the
 *     device detects (a non-finite result, lower > upper) is accumulated in
 *     the context's status word and returned by reach_sync.
 *   - Returned status codes: REACH_OK, or a negative REACH_E_*; the context's
 *     reach_last_error() then describes the failure.
 *   - A context is not thread-safe, except reach_submit / reach_poll /
 *     reach_cancel, which may be called from any thread while a server runs.
 */
#ifndef REACH_H
#define REACH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t reach_status;
enum {
    REACH_OK = 0,
    REACH_PENDING = 1,          /* reach_poll: the query has not finished */
    REACH_E_INVAL = -1,         /* bad argument (sizes, pointers, parameters) */
    REACH_E_NOMEM = -2,         /* workspace / pool / slots too small */
    REACH_E_DEVICE = -3,        /* HIP runtime error */
    REACH_E_UNSUPPORTED = -4,   /* valid request outside what the library runs */
    REACH_E_NONFINITE = -5,     /* device saw a non-finite result */
    REACH_E_ORDER = -6,         /* device saw r_lo > r_hi */
    REACH_E_CANCELLED = -7,     /* the query was cancelled */
    REACH_E_BUSY = -8,          /* server state does not allow the call */
    REACH_E_TIMEOUT = -9        /* a bounded wait ran out */
};

typedef int32_t reach_dtype;
enum { REACH_F64 = 0, REACH_F32 = 1 };

enum { REACH_CTM = 1, REACH_RD = 2, REACH_LIN3 = 3, REACH_HEAT3D = 4, REACH_USER = 5 };

/* Boundary conditions of a system: each kind has its own, stated with it above
   (zero ghosts for RD, LIN3 and USER chains, zero inflow and free outflow for
   the CTM, insulated faces and one open face for HEAT3D).  No other set is
   built: any other value of reach_system.bc is REACH_E_UNSUPPORTED. */
enum { REACH_BC_DEFAULT = 0 };

/* A system of the list above. */
typedef struct reach_system {
    int32_t kind;
    int32_t bc;       /* REACH_BC_DEFAULT */
    int64_t n;        /* number of cells (state dimension), 1 <= n < 2^40 */
    int64_t n_in;     /* input dimension: 0, 1 or n (64-bit, since n_in = n may
                         exceed 2^31) */
    double prm[8];    /* parameters, layout per kind (unused entries ignored) */
} reach_system;

/* One embedding query for the batch and serving entry points.  For
   reach_embed_rk4_batch all pointers are device pointers; for reach_submit
   they are HOST pointers (inputs are copied before reach_submit returns,
   r_lo / r_hi are written before reach_poll reports completion). */
typedef struct reach_query {
    reach_system sys;
    reach_dtype dtype;     /* REACH_F64 (the batch and serving kernels are FP64) */
    int32_t reserved;
    const void* x_lo;
    const void* x_hi;
    const void* p_lo;      /* NULL when sys.n_in == 0 */
    const void* p_hi;
    void* r_lo;
    void* r_hi;
    double t0;
    double dt;
    int64_t nsteps;
} reach_query;

typedef struct reach_ctx reach_ctx;

/* ------------------------------------------------------------ context -- */

/* Create a context on HIP device `device` (made current for the call).
   Allocates the context's status words on that device.  With the environment
   variable REACH_LOG set (and not "0") when the context is created, every
   embedding, Monte Carlo, growth-bound and batch call on it writes one line
   "reach: {...}" to stderr: a JSON object with the call, system kind, dtype,
   sizes and the launch plan (tile shape, tiles, passes, waves). */
reach_status reach_ctx_create(int device, reach_ctx** out);

/* Destroy a context (stops a running server first).  NULL is a no-op. */
void reach_ctx_destroy(reach_ctx* ctx);

/* Text of the last error on this context; valid until the next call on it. */
const char* reach_last_error(const reach_ctx* ctx);

/* Tuning overrides, mainly for tests and the autotuner:
     "embed.K"    steps fused per HBM pass (0 = tuned default)
     "embed.E"    cells per lane of the embedding kernel (0 = tuned default)
     "embed.S"    sides per wavefront, 1 or 2 (0 = tuned default)
     "gb.E", "gb.K"  cells per lane / steps per pass of the growth-bound kernel
     "heat.P"     rows per wavefront of the 3-D heat kernel: 2, 3, 4, 5 or 8
                  (with 16, 12, 8, 8 or 4 wavefronts per block; FP64 builds 2, 3,
                  4 and 5, FP32 2, 3, 4 and 8; 0 = tuned default)
     "mc.waves"   resident waves of the Monte Carlo kernel (0 = default, at most 4096)
     "batch.split" 1: one wave per side of each cooperative query (shorter
                  latency per query); 0 (default): one wave per query or pack
     "batch.pack" 0 (default): segment packs when the batch has more queries
                  than twice the resident waves; 1: always; 2: never
     "batch.E"    largest cells per lane of a segment pack: 2, 4, 8 or 16 (0 =
                  the autotuned cap of the query's bucket, else that of the
                  whole batch, else 16)
     "batch.waves" resident waves of the batch kernels (0 = default: the
                  count the autotuner chose for that packing kernel, else 8
                  per compute unit, 4 when a pack has 16 cells per lane)
     "serve.mode" 0 (default): persistent serving kernel; 1: one launch per
                  served query (read by reach_server_start)
     "serve.waves" resident waves of the serving kernel (0 = default)
   Returns REACH_E_INVAL for an unknown key or a value out of range. */
reach_status reach_set_option(reach_ctx* ctx, const char* key, int64_t value);
int64_t reach_get_option(const reach_ctx* ctx, const char* key);

/* Launch plan reach_embed_rk4 would use for this system, dtype and step
   count with the context's current tuning: out[0] = E (cells per lane),
   out[1] = K (RK4 steps per HBM pass), out[2] = tiles (one wavefront each),
   out[3] = tile stride in cells, out[4] = halo cells per cut edge,
   out[5] = passes (kernel launches), out[6] = S, sides per wavefront (2: lower
   and upper together; 1: one side per wavefront, twice the tiles, for the
   cooperative CTM and RD chains).  `out` is a host array of 7.  For
   REACH_HEAT3D: out[0] = rows per wavefront, out[1] = 1, out[2] = tiles per
   side (x-y tiles of 64 by rows x waves cells), out[3] = output cells of a
   tile along x, out[4] = 4, out[5] = nsteps, out[6] = 1. */
reach_status reach_plan_embed(reach_ctx* ctx, const reach_system* sys, reach_dtype dtype,
                              int64_t nsteps, int64_t* out);

/* Autotuner for reach_embed_rk4: times every built tile shape (E cells per
   lane) and steps-per-pass K on the caller's own buffers (trial_steps RK4
   steps per trial, one warm-up and two timed calls, HIP events on `stream`),
   re-times the four fastest and the built-in default over ten times the
   steps (three rounds, each shape once per round), and records the fastest
   (the default unless a shape beats it by more than 2%) for this system kind, dtype and power-of-two size bucket of
   n in the context; later calls of that bucket use it.  Arguments
   are those of reach_embed_rk4 (r_lo / r_hi receive scratch results).
   best[0] = E, best[1] = K, best[2] = femtoseconds per state-step (2n per
   step), best[3] = S (sides per wavefront).  `best` is a host array of 4.
   For REACH_HEAT3D it times the built heat kernel shapes instead ("heat.P"):
   best[0] = rows per wavefront, best[1] = 1, best[3] = 1.  With REACH_AUTOTUNE_CACHE set to a file name, results are appended
   there and read back by reach_ctx_create on the same device architecture. */
reach_status reach_autotune_embed(reach_ctx* ctx, const reach_system* sys, reach_dtype dtype,
                                  const void* x_lo, const void* x_hi,
                                  const void* p_lo, const void* p_hi, double dt,
                                  int64_t trial_steps, void* r_lo, void* r_hi,
                                  void* workspace, size_t workspace_bytes, void* stream,
                                  int64_t* best);

/* Bytes of device workspace reach_embed_rk4 (m = 0) or reach_montecarlo
   (m = sample count) needs for this system and dtype with the context's
   current tuning; 0 if none is needed; (size_t)-1 on invalid arguments. */
size_t reach_workspace_bytes(reach_ctx* ctx, const reach_system* sys, reach_dtype dtype,
                             int64_t m);

/* Wait for all work on `stream`, then return and clear the device status
   word: REACH_E_NONFINITE or REACH_E_ORDER if a kernel since the last
   reach_sync saw such a result, REACH_E_DEVICE on a HIP error, else OK. */
reach_status reach_sync(reach_ctx* ctx, void* stream);

/* ---------------------------------------------------------- embedding --
 * Mixed-monotonicity reachable box (Sec. 2.1, Algorithm 3): integrate the
 * embedding system nsteps RK4 steps of size dt from t0, starting at
 * (x_lo, x_hi) with inputs (p_lo, p_hi), and write the box (r_lo, r_hi).
 *   x_lo, x_hi  n elements, x_lo <= x_hi expected (not checked)
 *   p_lo, p_hi  n_in elements (NULL iff n_in == 0)
 *   r_lo, r_hi  n elements; may be the same arrays as x_lo, x_hi
 *   workspace   device memory of reach_workspace_bytes(ctx, sys, dtype, 0)
 *               bytes (may be NULL when that is 0); must not overlap the
 *               other arrays
 * nsteps = 0 copies the box.  Errors: REACH_E_INVAL for n < 1, n_in not in
 * {0, 1, n}, dt not finite or <= 0, nsteps < 0, NULL required pointers,
 * unknown kind or nonzero reserved field, workspace too small;
 * REACH_E_UNSUPPORTED for CTM with inputs.
 */
reach_status reach_embed_rk4(reach_ctx* ctx, const reach_system* sys, reach_dtype dtype,
                             const void* x_lo, const void* x_hi,
                             const void* p_lo, const void* p_hi,
                             double t0, double dt, int64_t nsteps,
                             void* r_lo, void* r_hi,
                             void* workspace, size_t workspace_bytes, void* stream);

/* Reach tube: the embedding box after every `every` steps, as in the paper's
 * vehicle study, which computes a reach set per time step (Sec. 5).  Slot k
 * (0 <= k < nsteps / every) of tube_lo / tube_hi (device arrays of
 * (nsteps / every) x n elements, slot-major) receives the box at step
 * (k + 1) * every, bitwise equal to reach_embed_rk4 run for that many steps.
 * nsteps must be a positive multiple of every.  Other arguments as
 * reach_embed_rk4 (the same workspace). */
reach_status reach_embed_rk4_tube(reach_ctx* ctx, const reach_system* sys, reach_dtype dtype,
                                  const void* x_lo, const void* x_hi,
                                  const void* p_lo, const void* p_hi,
                                  double t0, double dt, int64_t nsteps, int64_t every,
                                  void* tube_lo, void* tube_hi,
                                  void* workspace, size_t workspace_bytes, void* stream);

/* -------------------------------------------------------- growth bound --
 * Contraction / growth-bound box (Sec. 2.1, Algorithm 2): the center
 * c = (x_lo + x_hi)/2 follows x' = f(x, p*) at the center input
 * p* = (p_lo + p_hi)/2, the half-width r = (x_hi - x_lo)/2 follows the growth
 * dynamics r' = C r + |b| [p] with [p] = (p_hi - p_lo)/2 and the tridiagonal
 * contraction matrix C (C_ii >= J_ii, C_ij >= |J_ij| over all states):
 *   CTM  C = (v, 0, w) (sub, diagonal, super), no input;
 *   RD   C = (1/h^2, -2/h^2, 1/h^2), input factor 1;
 *   LIN3 C = (|aL|, aD, |aR|), input factor |b|.
 * Both runs use the same RK4 as reach_embed_rk4; the result is
 * [c - r, c + r] in (r_lo, r_hi).  Arguments as reach_embed_rk4; workspace:
 * reach_growth_bound_workspace_bytes bytes (4 n elements). */
size_t reach_growth_bound_workspace_bytes(reach_ctx* ctx, const reach_system* sys,
                                          reach_dtype dtype);
reach_status reach_growth_bound(reach_ctx* ctx, const reach_system* sys, reach_dtype dtype,
                                const void* x_lo, const void* x_hi,
                                const void* p_lo, const void* p_hi,
                                double t0, double dt, int64_t nsteps,
                                void* r_lo, void* r_hi,
                                void* workspace, size_t workspace_bytes, void* stream);

/* --------------------------------------------------------- Monte Carlo --
 * Monte Carlo box (Sec. 2.1, Algorithm 4) over samples s = s0 .. s0+m-1:
 *   x0_j = x_lo_j + U(s, j) (x_hi_j - x_lo_j),  p_k = p_lo_k + U(s, n+k) (p_hi_k - p_lo_k)
 * where U(s, j) is word j mod 4 of Philox4x64-10 (Salmon et al., SC'11) at
 * key (seed, 0), counter (floor(j/4), s, 2, 0), taken as its top 53 bits
 * (REACH_F64) or top 24 bits (REACH_F32) over 2^53 or 2^24.  Each sample is
 * integrated nsteps RK4 steps of x' = f(x, p); r_min / r_max (n elements)
 * receive the per-dimension min / max over the samples, NaN-propagating.
 * Sample ranges compose: the min / max of two ranges is that of their union.
 * workspace: reach_workspace_bytes(ctx, sys, dtype, m) bytes.
 * Errors as reach_embed_rk4, plus REACH_E_INVAL for m < 1 or s0 < 0, and
 * REACH_E_UNSUPPORTED when n exceeds the register-resident limit
 * (4096 cells for REACH_F32, 2048 for REACH_F64).
 */
reach_status reach_montecarlo(reach_ctx* ctx, const reach_system* sys, reach_dtype dtype,
                              const void* x_lo, const void* x_hi,
                              const void* p_lo, const void* p_hi,
                              double t0, double dt, int64_t nsteps,
                              int64_t m, uint64_t seed,
                              void* r_min, void* r_max,
                              void* workspace, size_t workspace_bytes, void* stream);

/* Same as reach_montecarlo over samples s0 .. s0+m-1 (resumable MC). */
reach_status reach_montecarlo_range(reach_ctx* ctx, const reach_system* sys, reach_dtype dtype,
                                    const void* x_lo, const void* x_hi,
                                    const void* p_lo, const void* p_hi,
                                    double t0, double dt, int64_t nsteps,
                                    int64_t s0, int64_t m, uint64_t seed,
                                    void* r_min, void* r_max,
                                    void* workspace, size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same as
 * reach_montecarlo_range, with no workspace argument.  The per-wave partials
 * live in a fixed array of reach_noalloc_scratch_bytes() = 64 MiB of device
 * memory that the library holds on each device it runs on until the process
 * ends; the call allocates nothing.  Every call on one device shares that
 * device's array, so calls that overlap on one device (two streams, two host
 * threads) race and must be serialised by the caller.  Results are those of
 * reach_montecarlo_range with the same arguments.  Errors: those of
 * reach_montecarlo_range, and REACH_E_NOMEM when the partials
 * (reach_workspace_bytes(ctx, sys, dtype, m)) exceed the array: only with more
 * waves than the default, option "mc.waves". */
reach_status reach_montecarlo_noalloc(reach_ctx* ctx, const reach_system* sys, reach_dtype dtype,
                                      const void* x_lo, const void* x_hi,
                                      const void* p_lo, const void* p_hi,
                                      double t0, double dt, int64_t nsteps,
                                      int64_t s0, int64_t m, uint64_t seed,
                                      void* r_min, void* r_max, void* stream);
size_t reach_noalloc_scratch_bytes(void);

/* Sample count of the Monte Carlo guarantee (Sec. 2.1): with
   m = ceil((2n/eps) ln(2n/delta)) samples, with probability 1 - delta the
   box leaves out at most probability eps of the reachable set.
   Returns -1 unless n >= 1, 0 < eps < 1 and 0 < delta < 1.  Host only. */
int64_t reach_mc_samples(int64_t n, double eps, double delta);

/* --------------------------------------------------------------- batch --
 * Many small embeddings (n <= 512, FP64, n_in 0 or 1) in one persistent
 * kernel: each wave takes the next work item from a device work counter
 * (longest first; the schedule is reach_plan_batch's) and integrates it with
 * its whole state in registers.  A work item is one query spread over the
 * wave, or a segment pack of queries sharing it (E cells per lane).
 * `q` is a HOST array of nq queries whose pointers are device pointers; it is
 * read during the call only.  workspace: reach_batch_workspace_bytes(nq)
 * bytes of device memory.  Results are identical to nq separate
 * reach_embed_rk4 calls.  The workspace holds two blocks of descriptors
 * and work items, used by turns.  The query descriptors are copied into this
 * call's block on the context's own copy stream as soon as the host has
 * written them, while it forms the work items, which follow; the upload waits
 * for the kernel that read the block two batches before (and for the previous
 * batch's kernel when the workspace or nq differs from the previous call's).  The counter
 * reset and the worker kernel (replayed from a captured hipGraph when the
 * same nq capacity, block and stream repeat) run on `stream` after the upload
 * and after the context's previous batch kernel, on whichever stream that ran.
 * The call returns once the uploads are issued, so batches issued back to
 * back overlap the host's planning and the upload of one batch with the
 * previous batch's kernel.
 * Errors: as reach_embed_rk4 for each query, REACH_E_UNSUPPORTED for n > 512,
 * REACH_F32 or per-cell inputs, REACH_E_NOMEM for a short workspace.
 */
size_t reach_batch_workspace_bytes(int64_t nq);

/* The schedule reach_embed_rk4_batch launches for these queries, computed on
 * the host only (no device call; the query pointers are not dereferenced).
 * A batch with more queries than twice the resident waves of the unpacked
 * kernel (option "batch.pack": 0 = that rule, 1 = always, 2 = never) is
 * packed: every work item is then a segment pack, queries of one kind with
 * bitwise equal parameters and dt, step counts in the same 1/16 octave and
 * the same cells per lane E (2, 4, 8 or 16, chosen per query by the least
 * estimated issue cost, at most option "batch.E" or else the (kind, size)
 * bucket's autotuned cap) sharing a wavefront, query m on ceil(n_m / E)
 * lanes, at most 64 lanes and 64 queries.  An unpacked batch runs every
 * query alone, spread over a whole wavefront (E = ceil(n / 64)).  Items come
 * longest first (wave time E * nsteps of the longest member).
 * On return *n_items holds the item count and item k runs the queries
 * member[item_start[k] .. item_start[k] + item_count[k]) (indices into q) at
 * item_E[k] cells per lane (0: alone); item_start, item_count, item_E and
 * member are host arrays of nq entries.  ctx may be NULL (then the default
 * options apply with 256 compute units, a large plan runs on host threads
 * started for the call, and errors carry no message); with a context its
 * "batch.split" option turns packing off as it does for the batch.
 * Errors: those of reach_embed_rk4_batch's query checks, REACH_E_INVAL for
 * NULL arrays. */
reach_status reach_plan_batch(reach_ctx* ctx, const reach_query* q, int64_t nq,
                              int64_t* item_start, int32_t* item_count, int32_t* item_E,
                              int64_t* member, int64_t* n_items);
reach_status reach_embed_rk4_batch(reach_ctx* ctx, const reach_query* q, int64_t nq,
                                   void* workspace, size_t workspace_bytes, void* stream);

/* Autotuner of the batch (its pack widths and resident waves), on the
   caller's whole batch.  After a few untimed calls, every comparison times
   the batch (one warm-up and four timed calls, HIP events on `stream`,
   fastest kept, host planning included) with the candidate setting and again
   with the current one, and keeps the candidate only if it is more than 1%
   faster.  In order: the width of the whole batch (largest pack width 16,
   the wide kernel at one wavefront per SIMD, against 8, the narrow kernel at
   two); then, for every (kind, log2 n bucket) with at least 256 queries, most
   queries first, the narrower widths 8, 4 and 2 for that bucket; then,
   unless option "batch.waves" is set, 4, 8 and (without 16-cell packs) 12
   resident waves per compute unit.  A batch that does not pack is only
   timed.  The widths are recorded in the context (used while option
   "batch.E" is 0).  Arguments as reach_embed_rk4_batch, whose results the
   queries' r_lo / r_hi hold afterwards; every setting gives the same boxes
   bit for bit.  best[0] = resident waves (0: the default), best[1] =
   nanoseconds of the whole batch at the chosen settings.  `best` is a host
   array of 2.  With REACH_AUTOTUNE_CACHE set, the widths are appended there
   and read back by reach_ctx_create on the same device architecture. */
reach_status reach_autotune_batch(reach_ctx* ctx, const reach_query* q, int64_t nq,
                                  void* workspace, size_t workspace_bytes, void* stream,
                                  int64_t* best);

/* Baseline for the batch: one kernel launch per query, round-robin over
   `nstreams` internal streams (1..16).  Same results; host-blocking. */
reach_status reach_embed_rk4_each(reach_ctx* ctx, const reach_query* q, int64_t nq,
                                  int32_t nstreams);

/* ------------------------------------------------------------- serving --
 * Continuous batching.  reach_server_start launches a persistent kernel on
 * `stream` that keeps `max_slots` query slots; queries submitted while others
 * run are admitted as soon as a slot and enough bytes of the device `pool`
 * (caller-owned device memory, first-fit, 2 n + 2 doubles per query, 256-byte
 * aligned) are free, and run concurrently with them.  Admission order is
 * submission order.  A service thread started by reach_server_start does the
 * admission and completion work; the client calls below only append to its
 * inbox or read its outbox under short locks, so they never wait for it.
 *   reach_submit: HOST pointers in *q (inputs copied before return);
 *     *ticket receives the query's id.  The query arrives at the call.
 *     REACH_E_NOMEM if the query can never fit the pool; REACH_E_BUSY if no
 *     server runs or it is stopping; REACH_E_INVAL / REACH_E_UNSUPPORTED as
 *     reach_embed_rk4_batch for the query itself.
 *   reach_submit_at: the same, with the query's arrival time given by the
 *     caller in microseconds on the reach_clock_us() clock (for a client that
 *     submits queries of a planned arrival schedule: their latency then counts
 *     any delay of the client itself).  REACH_E_INVAL if it is not finite.
 *   reach_poll: REACH_PENDING until the query is done, then REACH_OK with its
 *     final status in *result (REACH_OK, REACH_E_NONFINITE, REACH_E_ORDER,
 *     REACH_E_CANCELLED or, after a drain that ran out of time,
 *     REACH_E_TIMEOUT); r_lo / r_hi hold the box when *result is REACH_OK.
 *     A ticket is forgotten once it has been reported done (REACH_E_INVAL
 *     afterwards and for unknown tickets).
 *   reach_cancel: request that a query stop.  A waiting query is dropped; a
 *     running one stops within kCancelEvery = 64 RK4 steps (the kernel reads
 *     the query's host-written cancel word between blocks of steps).  Returns
 *     REACH_OK when the request is recorded, REACH_E_BUSY if the query has
 *     already finished, REACH_E_INVAL for an unknown ticket.  A query that
 *     completes before the request takes effect reports its own status;
 *     otherwise reach_poll reports REACH_E_CANCELLED and r_lo / r_hi are not
 *     written.
 *   reach_server_stop: drain every admitted and waiting query (bounded by
 *     REACH_SERVER_DRAIN_S seconds without progress, default 60), stop the
 *     kernel and join the service thread.
 *   reach_server_stats: latency in microseconds from arrival (see
 *     reach_submit / reach_submit_at) to the box being in the caller's
 *     arrays, of the queries completed so far, cancelled ones excepted
 *     (p50, p99, max) and their count.
 * The serving grid leaves as a whole when the host sets its stop flag or
 * after `REACH_SERVER_IDLE_S` seconds (default 120) in which some wave saw no
 * work, so the kernel always drains; the service thread starts a new grid
 * for the next arrival and moves admitted queries to it.
 * With the option "serve.mode" = 1 at reach_server_start, each admitted query
 * is one kernel launch instead (the baseline of the persistent kernel).
 */
reach_status reach_server_start(reach_ctx* ctx, void* pool, size_t pool_bytes,
                                int32_t max_slots, void* stream);
reach_status reach_submit(reach_ctx* ctx, const reach_query* q, uint64_t* ticket);
reach_status reach_submit_at(reach_ctx* ctx, const reach_query* q, double arrival_us,
                             uint64_t* ticket);
/* Microseconds on the steady clock the server stamps latencies with.  Host only. */
double reach_clock_us(void);
reach_status reach_poll(reach_ctx* ctx, uint64_t ticket, reach_status* result);
reach_status reach_cancel(reach_ctx* ctx, uint64_t ticket);
reach_status reach_server_stop(reach_ctx* ctx);
reach_status reach_server_stats(reach_ctx* ctx, double* p50_us, double* p99_us,
                                double* max_us, int64_t* completed);

/* ---------------------------------------------------- user-defined systems
 * A chain system given by its decomposition function as C source text (the
 * embedding of Sec. 2.1 exists for any system with a decomposition function;
 * PIRK takes the system dynamics as a C function).  The text defines
 *
 *   REACH_DEVICE real reach_d(real xm, real x, real xp, real hm, real h, real hp,
 *                             real u, real uh, const real* prm, long long i,
 *                             long long n);
 *
 * returning d_i(x, p, xh, ph) for cell i of an n-cell chain in which cell i
 * couples only to cells i-1 and i+1: (xm, x, xp) are x_{i-1}, x_i, x_{i+1},
 * (hm, h, hp) the same cells of xh, u = p_i and uh = ph_i (0 without inputs,
 * the shared value for n_in = 1), prm the system's 8 parameters.  Neighbours
 * past the chain's ends read as 0 (boundary conditions go in d, using i and
 * n).  d must equal f on the diagonal (d(x, p, x, p) = f(x, p)) and be
 * nondecreasing in x_j (j != i) and p and nonincreasing in xh and ph; the
 * library cannot check this, and a d that breaks it gives no guarantee.
 * `real` is double in FP64 runs and float in FP32 runs; helper functions
 * must be declared REACH_DEVICE; the device math functions (sin, exp, fmin,
 * ceil, ...) are available; names starting with reach_ are reserved.
 *
 * reach_user_create compiles the text with hipRTC for the context's device
 * (no floating-point contraction, as the built-in kernels) and loads it;
 * REACH_E_INVAL with the compiler's log in reach_last_error() when it does
 * not compile.  Kernels are built per precision and input kind (none or
 * scalar, per cell): the FP64 scalar set at creation, every other set on
 * the first call that needs it (that call blocks for the compile and may
 * fail with REACH_E_INVAL / REACH_E_DEVICE like creation).  The handle is
 * owned by the caller (reach_user_destroy), valid on the context's device
 * only, and like the context not safe for concurrent calls.
 *
 * reach_embed_rk4_user: Algorithm 3 (embedding RK4) for the user system.
 * `sys` has kind REACH_USER, n, n_in and prm; the other arguments and the
 * workspace rule are those of reach_embed_rk4 (2n elements of workspace
 * when the chain spans several tiles and more than one pass).  Options
 * "user.E" (cells per lane: 1, 2, 4, 8) and "user.K" (steps per pass). */
typedef struct reach_user reach_user;

reach_status reach_user_create(reach_ctx* ctx, const char* source, reach_user** out);
void reach_user_destroy(reach_user* user);
reach_status reach_embed_rk4_user(reach_ctx* ctx, reach_user* user,
                                  const reach_system* sys, reach_dtype dtype,
                                  const void* x_lo, const void* x_hi, const void* p_lo,
                                  const void* p_hi, double t0, double dt, int64_t nsteps,
                                  void* r_lo, void* r_hi, void* workspace,
                                  size_t workspace_bytes, void* stream);

/* reach_montecarlo_user: Algorithm 4 for the user system (samples s0 ..
 * s0+m-1 integrated with f(x, p) = d(x, p, x, p)); arguments, sampling and
 * results as reach_montecarlo_range.  n <= 512 (a sample lives in one
 * wavefront), else REACH_E_UNSUPPORTED.
 * reach_user_workspace_bytes: workspace of reach_embed_rk4_user (m = 0) or
 * reach_montecarlo_user with m samples; (size_t)-1 on bad arguments. */
size_t reach_user_workspace_bytes(reach_ctx* ctx, const reach_system* sys, reach_dtype dtype,
                                  int64_t m);
reach_status reach_montecarlo_user(reach_ctx* ctx, reach_user* user,
                                   const reach_system* sys, reach_dtype dtype,
                                   const void* x_lo, const void* x_hi, const void* p_lo,
                                   const void* p_hi, double t0, double dt, int64_t nsteps,
                                   int64_t s0, int64_t m, uint64_t seed, void* r_min,
                                   void* r_max, void* workspace, size_t workspace_bytes,
                                   void* stream);

#ifdef __cplusplus
}
#endif
#endif /* REACH_H */
