// Device building blocks for the gfx950 reachability kernels.
//
// Layout convention shared by every kernel: one wavefront (64 lanes) owns a
// window of 64*E consecutive cells of a chain, lane l holding cells
// [l*E, l*E + E) of the window in registers.  A three-point stencil then
// needs only two cross-lane values per stage (the last cell of lane l-1 and
// the first cell of lane l+1), moved with DPP whole-wave shifts; every other
// neighbour is a register of the same lane.  Lanes past either end of the
// wave receive zero, which is how the chain's boundary conditions enter when
// the window starts at cell 0 or ends at cell n-1 (see Mask below).
//
// The four stages of classical RK4 (Algorithm 1, read as the classical
// method: stage inputs z + dt/2 K1, z + dt/2 K2, z + dt K3, update
// z + dt/6 (K1 + 2 K2 + 2 K3 + K4)) run on registers: per cell and side the
// state y, the running sum acc = K1 + 2 K2 + 2 K3 + K4 and the current stage
// input t.  No stage value ever leaves the register file.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace reach {

constexpr int WAVE = 64;

// DPP controls of the GFX9 family: shift the whole wavefront by one lane.
constexpr int DPP_WAVE_SHL1 = 0x130;  // lane l reads lane l+1
constexpr int DPP_WAVE_SHR1 = 0x138;  // lane l reads lane l-1

// Lane l receives x of lane l-1; lane 0 receives 0 (DPP bound control: the
// out-of-wave source reads as zero, so no fill value has to be staged).
__device__ __forceinline__ float from_left(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), DPP_WAVE_SHR1, 0xF,
                                                      0xF, true));
}
// Lane l receives x of lane l+1; lane 63 receives 0.
__device__ __forceinline__ float from_right(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), DPP_WAVE_SHL1, 0xF,
                                                      0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp64(double x) {
    const uint64_t xi = (uint64_t)__double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)xi, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(xi >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ __forceinline__ double from_left(double x) { return dpp64<DPP_WAVE_SHR1>(x); }
__device__ __forceinline__ double from_right(double x) { return dpp64<DPP_WAVE_SHL1>(x); }

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float minT(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double minT(double a, double b) { return __builtin_fmin(a, b); }

template <class T> __device__ __forceinline__ T neg_inf();
template <> __device__ __forceinline__ float neg_inf<float>() { return -__builtin_inff(); }
template <> __device__ __forceinline__ double neg_inf<double>() { return -__builtin_inf(); }

// ------------------------------------------------------------- systems --
// Kind tags (match the C ABI) and input modes.
enum { K_CTM = 1, K_RD = 2, K_LIN3 = 3 };
enum { IN_SCALAR = 0, IN_CELL = 1 };

// Per-launch system constants, already converted to the kernel's type.
template <class T> struct SysPrm {
    T a0, a1, a2, a3, a4;   // CTM: v, w, c*w, q  RD: 1/h^2, 2/h^2  LIN3: aL, aD, aR, b
};

// Inputs seen by one lane: scalar (same for every cell) or one per cell.
template <class T, int E, int S, int MODE> struct Inputs;
template <class T, int E, int S> struct Inputs<T, E, S, IN_SCALAR> {
    T u[S];
    __device__ __forceinline__ T at(int s, int) const { return u[s]; }
};
template <class T, int E, int S> struct Inputs<T, E, S, IN_CELL> {
    T u[S][E];
    __device__ __forceinline__ T at(int s, int e) const { return u[s][e]; }
};

// Stage update applied to cell e of side s once its derivative k is known.
// STAGE 1..4 of classical RK4; h2 = dt/2, dt, dt6 = dt/6.
template <class T> struct Steps { T h2, dt, dt6; };

template <int STAGE, class T>
__device__ __forceinline__ void rk_update(T k, T& y, T& acc, T& t, const Steps<T>& st) {
    if (STAGE == 1) { acc = k;                 t = fmaT(st.h2, k, y); }
    if (STAGE == 2) { acc = fmaT(T(2), k, acc); t = fmaT(st.h2, k, y); }
    if (STAGE == 3) { acc = fmaT(T(2), k, acc); t = fmaT(st.dt, k, y); }
    if (STAGE == 4) { acc = acc + k;           y = fmaT(st.dt6, acc, y); }
}

// Where a window sits relative to the chain's right end.
//   PAD : the window runs past cell n-1; cells at or beyond n hold the
//         boundary's ghost value at every stage (nvalid cells of this lane are
//         inside the chain): a select per cell.
//   ONE : (with PAD; the Monte Carlo kernel, whose every wave may pad) only
//         cell n, the right neighbour of cell n-1, is set to the ghost after
//         each stage: slot `en` of the lane holding it, en the same in every
//         lane, so one indexed register move per stage replaces the per-cell
//         selects.  Cells beyond n then hold values that reach no cell of the
//         chain and that no caller reads or checks.  Only for lane arrays of
//         up to 128 bytes: an index into longer ones (or into both sides of a
//         window) made the compiler move them to scratch memory.
//   END : the window contains cell n-1, so lane 63's right neighbour is the
//         ghost.  Zero-filled lane shifts already give the Dirichlet ghost 0;
//         only the CTM's free outflow (ghost -inf) needs an explicit value.
// A window's left end at cell 0 needs nothing: lane 0 receives 0 from the
// left, which is both the Dirichlet ghost and the CTM's zero inflow flux.
template <int E, bool PAD, bool END, bool ONE = false> struct Mask {
    int nvalid;  // cells of this lane inside the chain
    int en;      // slot of cell n in its lane (wave-uniform; ONE only)
    bool mine;   // this lane holds cell n (ONE only)
    template <class T> static constexpr bool indexed() { return PAD && ONE && E * sizeof(T) <= 128; }
    template <class T> static constexpr bool per_cell() { return PAD && !indexed<T>(); }
    __device__ __forceinline__ bool ok(int e) const { return !PAD || e < nvalid; }
    template <class T>
    __device__ __forceinline__ void fix(T (&v)[E], T ghost) const {
        if constexpr (indexed<T>()) {
            const T cur = v[en];
            v[en] = mine ? ghost : cur;
        }
    }
};

// The mask of a window whose first n_rel cells (1 <= n_rel <= 64 E) are the
// chain's (cell n is the window's cell n_rel).
template <int E, bool END, bool ONE = false>
__device__ __forceinline__ Mask<E, true, END, ONE> chain_end_mask(int64_t n_rel) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t left = n_rel - (int64_t)lane * E;
    Mask<E, true, END, ONE> M;
    M.nvalid = (int)(left < 0 ? 0 : (left > E ? E : left));
    M.en = 0;
    M.mine = false;
    if constexpr (ONE) {
        M.en = __builtin_amdgcn_readfirstlane((int)(n_rel % E));
        M.mine = lane == (int)(n_rel / E);
    }
    return M;
}

// One RK4 stage for all cells of the lane, for every side s < S.
//   in  : the stage input (y for stage 1, t otherwise)
// For S == 2 the sides are (lower, upper) of the embedding; for S == 1 the
// kernel integrates f itself (Monte Carlo).
template <int KIND, int STAGE, class T, int E, int S, int MODE, bool MASKED, bool END, bool ONE>
__device__ __forceinline__ void rk_stage(T (&y)[S][E], T (&acc)[S][E], T (&t)[S][E],
                                         const SysPrm<T>& P, const Inputs<T, E, S, MODE>& U,
                                         const Steps<T>& st, const Mask<E, MASKED, END, ONE>& M)
{
    T (&in)[S][E] = (STAGE == 1) ? y : t;
    if constexpr (KIND == K_CTM) {
        // Flux form: F_e = min(v y_e, w (c - y_{e+1}), q) = min(v y_e, wc - w y_{e+1}, q),
        // k_e = F_{e-1} - F_e.  Right ghost past the chain's end is -inf, so
        // the supply term becomes +inf (free outflow); the flux into the
        // window's first cell arrives from the left lane, 0 at lane 0 (zero
        // inflow into cell 0).
        const T v = P.a0, w = P.a1, wc = P.a2, q = P.a3;
        const bool last_lane = (threadIdx.x & (WAVE - 1)) == WAVE - 1;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            T rn = from_right(in[s][0]);
            if (END) rn = last_lane ? neg_inf<T>() : rn;
            const T Flast = minT(minT(v * in[s][E - 1], fmaT(-w, rn, wc)), q);
            T Fprev = from_left(Flast);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const T F = (e == E - 1) ? Flast : minT(minT(v * in[s][e], fmaT(-w, in[s][e + 1], wc)), q);
                const T k = Fprev - F;
                Fprev = F;
                if (STAGE == 4) {
                    rk_update<4>(k, y[s][e], acc[s][e], t[s][e], st);
                    if (M.template per_cell<T>() && !M.ok(e)) y[s][e] = neg_inf<T>();
                } else {
                    rk_update<STAGE>(k, y[s][e], acc[s][e], t[s][e], st);
                    if (M.template per_cell<T>() && !M.ok(e)) t[s][e] = neg_inf<T>();
                }
            }
            if constexpr (MASKED) M.fix(STAGE == 4 ? y[s] : t[s], neg_inf<T>());
        }
    } else if constexpr (KIND == K_RD) {
        // k = (y_{e-1} - 2 y_e + y_{e+1}) / h^2 - y_e^3 + u, Dirichlet ghosts 0,
        // regrouped into four fused operations:
        //   k = (y_{e-1} + y_{e+1}) / h^2 + (u - y_e (y_e^2 + 2 / h^2)).
        const T ih2 = P.a0, two_ih2 = P.a1;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const T ln = from_left(in[s][E - 1]);
            const T rn = from_right(in[s][0]);
            T left = ln;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const T mid = in[s][e];
                const T right = (e == E - 1) ? rn : in[s][e + 1];
                const T loc = fmaT(-mid, fmaT(mid, mid, two_ih2), U.at(s, e));
                const T k = fmaT(left + right, ih2, loc);
                left = mid;
                if (STAGE == 4) {
                    rk_update<4>(k, y[s][e], acc[s][e], t[s][e], st);
                    if (M.template per_cell<T>() && !M.ok(e)) y[s][e] = T(0);
                } else {
                    rk_update<STAGE>(k, y[s][e], acc[s][e], t[s][e], st);
                    if (M.template per_cell<T>() && !M.ok(e)) t[s][e] = T(0);
                }
            }
            if constexpr (MASKED) M.fix(STAGE == 4 ? y[s] : t[s], T(0));
        }
    } else {
        // LIN3.  S == 1: f = aL y_{e-1} + aD y_e + aR y_{e+1} + b u.
        // S == 2: d(x, p, xh, ph) with the sign split of aL, aR, b; both sides
        // of a cell are computed from the old values before either is updated.
        const T aL = P.a0, aD = P.a1, aR = P.a2, b = P.a3;
        T ln[S], rn[S], left[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            ln[s] = from_left(in[s][E - 1]);
            rn[s] = from_right(in[s][0]);
            left[s] = ln[s];
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            T mid[S], right[S], k[S];
#pragma unroll
            for (int s = 0; s < S; ++s) {
                mid[s] = in[s][e];
                right[s] = (e == E - 1) ? rn[s] : in[s][e + 1];
            }
            if constexpr (S == 1) {
                k[0] = fmaT(b, U.at(0, e), fmaT(aR, right[0], fmaT(aD, mid[0], aL * left[0])));
            } else {
                const T aLp = aL > T(0) ? aL : T(0), aLn = aL < T(0) ? aL : T(0);
                const T aRp = aR > T(0) ? aR : T(0), aRn = aR < T(0) ? aR : T(0);
                const T bp = b > T(0) ? b : T(0), bn = b < T(0) ? b : T(0);
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
            }
#pragma unroll
            for (int s = 0; s < S; ++s) {
                left[s] = mid[s];
                if (STAGE == 4) {
                    rk_update<4>(k[s], y[s][e], acc[s][e], t[s][e], st);
                    if (M.template per_cell<T>() && !M.ok(e)) y[s][e] = T(0);
                } else {
                    rk_update<STAGE>(k[s], y[s][e], acc[s][e], t[s][e], st);
                    if (M.template per_cell<T>() && !M.ok(e)) t[s][e] = T(0);
                }
            }
        }
        if constexpr (MASKED) {
#pragma unroll
            for (int s = 0; s < S; ++s) M.fix(STAGE == 4 ? y[s] : t[s], T(0));
        }
    }
}

// `nsteps` classical RK4 steps on the lane's registers.
template <int KIND, class T, int E, int S, int MODE, bool MASKED, bool END, bool ONE>
__device__ __forceinline__ void rk4_steps(T (&y)[S][E], int64_t nsteps, const SysPrm<T>& P,
                                          const Inputs<T, E, S, MODE>& U, const Steps<T>& st,
                                          const Mask<E, MASKED, END, ONE>& M)
{
    T acc[S][E], t[S][E];
    for (int64_t k = 0; k < nsteps; ++k) {
        rk_stage<KIND, 1>(y, acc, t, P, U, st, M);
        rk_stage<KIND, 2>(y, acc, t, P, U, st, M);
        rk_stage<KIND, 3>(y, acc, t, P, U, st, M);
        rk_stage<KIND, 4>(y, acc, t, P, U, st, M);
    }
}

// Ghost value of a system past the chain's right end.
template <int KIND, class T> __device__ __forceinline__ T ghost() {
    if constexpr (KIND == K_CTM) return neg_inf<T>();
    else return T(0);
}

// ------------------------------------------------------------ status --
// Bits OR-ed into the context's device status word (ST_CANCELLED: only in a
// served query's own flags, never in the context's word).
enum { ST_NONFINITE = 1, ST_ORDER = 2, ST_CANCELLED = 4 };

__device__ __forceinline__ bool finiteT(float x) { return __builtin_isfinite(x); }
__device__ __forceinline__ bool finiteT(double x) { return __builtin_isfinite(x); }

// One lane per wave ORs `bits` (wave-reduced) into *status with a vector atomic.
__device__ __forceinline__ void report_status(unsigned int* status, unsigned int bits) {
    const unsigned long long nf = __ballot(bits & ST_NONFINITE);
    const unsigned long long od = __ballot(bits & ST_ORDER);
    if ((nf | od) && (threadIdx.x & 63) == 0)
        atomicOr(status, (nf ? (unsigned)ST_NONFINITE : 0u) | (od ? (unsigned)ST_ORDER : 0u));
}

// ------------------------------------------------------------ Philox --
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two
// 64x64->128 multiplications with the published multipliers and Weyl key
// increments.  Used for the Monte Carlo samples.
struct U4 { uint64_t x[4]; };

__device__ __forceinline__ U4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                            uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    U4 o; o.x[0] = c0; o.x[1] = c1; o.x[2] = c2; o.x[3] = c3;
    return o;
}

// Word q (0..3) of a block, chosen by selects: indexing r.x with a lane-varying
// q would put the block in a per-thread array, which the compiler moves to LDS
// and addresses through the dispatch packet, one host-memory read per wave at
// start-up (about 14 us of serialized reads for a 1000-wave launch).
__device__ __forceinline__ uint64_t philox_word(const U4& r, int q) {
    return q == 0 ? r.x[0] : q == 1 ? r.x[1] : q == 2 ? r.x[2] : r.x[3];
}

constexpr uint64_t MC_STREAM = 2;

// Uniform from one 64-bit word: top 53 bits / 2^53 (double), top 24 / 2^24 (float).
__device__ __forceinline__ double unif(uint64_t r, double) { return (double)(r >> 11) * 0x1.0p-53; }
__device__ __forceinline__ float unif(uint64_t r, float) { return (float)(uint32_t)(r >> 40) * 0x1.0p-24f; }

}  // namespace reach
