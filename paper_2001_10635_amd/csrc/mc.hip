// Monte Carlo reachable box on gfx950 (PIRK Sec. 2.1, Algorithm 4).
//
// Each wavefront integrates whole samples: the full n-cell state of one sample
// lives in the wave's registers (E cells per lane, n <= 64E), so a sample's
// N RK4 steps touch no memory at all.  Waves (four per workgroup, each on its
// own) are persistent: wave w takes
// samples s0 + w, s0 + w + nw, ... and folds each final state into its own
// running min / max kept in the workspace (read-modify-write once per sample,
// interleaved [w][e][lane] so those accesses are coalesced).  At the end the
// first wave of each workgroup folds its group's partials into its own slot,
// and a second kernel reduces those ceil(nw / 4) partials per dimension.
//
// Sampling: x0_j = x_lo_j + U(s, j) (x_hi_j - x_lo_j) and, for inputs,
// p_k = p_lo_k + U(s, n + k) (p_hi_k - p_lo_k), with U(s, j) word j mod 4 of
// Philox4x64-10 at key (seed, 0), counter (floor(j/4), s, 2, 0): counter-based,
// so any sample can be drawn independently and sample ranges compose.
#include "dev.hpp"
#include "kernels.hpp"

namespace reach {

template <class T>
__device__ __forceinline__ T nan_min(T m, T x) {
    // NaN-propagating: once either side is NaN the result stays NaN.
    return (m != m) ? m : ((x < m || x != x) ? x : m);
}
template <class T>
__device__ __forceinline__ T nan_max(T m, T x) {
    return (m != m) ? m : ((x > m || x != x) ? x : m);
}

// Waves per workgroup.  Each wave is independent; grouping four makes the
// dispatcher give a small launch (a few hundred samples) one wave per SIMD
// instead of stacking single-wave groups on the same SIMDs.
constexpr int MC_WPB = 4;

// Balanced layout of a chain that ends inside the wave, for lane arrays too
// long for the indexed ghost fix-up of the other padded waves: the chain
// fills lanes 0 .. L-1 (L = ceil(n / E)), the first F = n - L (E - 1) of them
// with E cells and the others ("short" lanes) with E - 1, so that cell n-1 is
// the last cell of lane L-1 and no cell of the chain has a padded neighbour
// inside its lane.  Per stage a short lane takes its last cell's right
// neighbour, and the value it hands to the lane on its left, by a select, and
// lane L-1 takes the ghost as its right neighbour: a few selects per stage
// instead of one per cell.  Lanes past L-1 and a short lane's unused slot
// compute values that reach no cell of the chain.  Per cell the arithmetic is
// the general stage's (rk_stage).
template <int E, class T>
__device__ __forceinline__ T mc_right_of(const T (&in)[E], int e, T rn, bool shortl) {
    if (e == E - 1) return rn;
    if (e == E - 2) return shortl ? rn : in[E - 1];
    return in[e + 1];
}
template <int E, class T>
__device__ __forceinline__ T mc_last_of(const T (&in)[E], bool shortl) {
    return shortl ? in[E - 2] : in[E - 1];
}

template <int KIND, int STAGE, class T, int E, int MODE>
__device__ __forceinline__ void mc_bal_stage(T (&y)[E], T (&acc)[E], T (&t)[E],
                                             const SysPrm<T>& P, const Inputs<T, E, 1, MODE>& U,
                                             const Steps<T>& st, bool shortl, bool endl) {
    T (&in)[E] = (STAGE == 1) ? y : t;
    if constexpr (KIND == K_CTM) {
        // free outflow past cell n-1 (ghost -inf), zero inflow into cell 0
        // (lane 0 receives 0 from the shift)
        const T v = P.a0, w = P.a1, wc = P.a2, q = P.a3;
        T rn = from_right(in[0]);
        rn = endl ? neg_inf<T>() : rn;
        T F[E];
#pragma unroll
        for (int e = 0; e < E; ++e)
            F[e] = minT(minT(v * in[e], fmaT(-w, mc_right_of<E>(in, e, rn, shortl), wc)), q);
        T Fprev = from_left(mc_last_of<E>(F, shortl));
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const T k = Fprev - F[e];
            Fprev = F[e];
            rk_update<STAGE>(k, y[e], acc[e], t[e], st);
        }
    } else if constexpr (KIND == K_RD) {
        // Dirichlet ghosts 0
        const T ih2 = P.a0, two_ih2 = P.a1;
        T left = from_left(mc_last_of<E>(in, shortl));
        T rn = from_right(in[0]);
        rn = endl ? T(0) : rn;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const T mid = in[e];
            const T right = mc_right_of<E>(in, e, rn, shortl);
            const T loc = fmaT(-mid, fmaT(mid, mid, two_ih2), U.at(0, e));
            const T k = fmaT(left + right, ih2, loc);
            left = mid;
            rk_update<STAGE>(k, y[e], acc[e], t[e], st);
        }
    } else {
        // LIN3 integrating f itself: aL y_{e-1} + aD y_e + aR y_{e+1} + b u, ghosts 0
        const T aL = P.a0, aD = P.a1, aR = P.a2, b = P.a3;
        T left = from_left(mc_last_of<E>(in, shortl));
        T rn = from_right(in[0]);
        rn = endl ? T(0) : rn;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const T mid = in[e];
            const T right = mc_right_of<E>(in, e, rn, shortl);
            const T k = fmaT(b, U.at(0, e), fmaT(aR, right, fmaT(aD, mid, aL * left)));
            left = mid;
            rk_update<STAGE>(k, y[e], acc[e], t[e], st);
        }
    }
}

template <int KIND, class T, int E, int MODE>
__device__ __forceinline__ void mc_bal_steps(T (&y)[E], int64_t nsteps, const SysPrm<T>& P,
                                             const Inputs<T, E, 1, MODE>& U, const Steps<T>& st,
                                             bool shortl, bool endl) {
    T acc[E], t[E];
    for (int64_t k = 0; k < nsteps; ++k) {
        mc_bal_stage<KIND, 1>(y, acc, t, P, U, st, shortl, endl);
        mc_bal_stage<KIND, 2>(y, acc, t, P, U, st, shortl, endl);
        mc_bal_stage<KIND, 3>(y, acc, t, P, U, st, shortl, endl);
        mc_bal_stage<KIND, 4>(y, acc, t, P, U, st, shortl, endl);
    }
}

template <int KIND, class T, int E, int MODE, bool BAL = false>
__global__ __launch_bounds__(WAVE * MC_WPB) void mc_kernel(McArgs a) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = threadIdx.x / WAVE;
    const int64_t wb = (int64_t)blockIdx.x * MC_WPB;
    const int64_t w = wb + wv;
    const int64_t n = a.n;
    const bool masked = (int64_t)WAVE * E > n;
    // BAL (chosen by the host): a padded wave whose lane arrays are too long
    // for the indexed ghost fix-up, in the balanced layout (n >= (E - 1) L)
    const int64_t Lb = (n + E - 1) / E;
    const int64_t Fb = n - Lb * (E - 1);               // lanes holding E cells
    const bool shortl = lane >= Fb;
    const int cnt = lane >= Lb ? 0 : (shortl ? E - 1 : E);
    const int64_t first_j = (int64_t)lane * E - (shortl ? (int64_t)lane - Fb : 0);
    const bool endl = lane == Lb - 1;

    const T* __restrict__ xlo = (const T*)a.x_lo;
    const T* __restrict__ xhi = (const T*)a.x_hi;
    T* __restrict__ pmin = (T*)a.part_min + (size_t)w * E * WAVE;
    T* __restrict__ pmax = (T*)a.part_max + (size_t)w * E * WAVE;
    const SysPrm<T> P = {(T)a.prm[0], (T)a.prm[1], (T)a.prm[2], (T)a.prm[3], (T)a.prm[4]};
    const Steps<T> st = {(T)a.h2, (T)a.dt, (T)a.dt6};
    const uint64_t k0 = a.seed, k1 = 0;

    bool first = true;
    // waves past nw (in the last workgroup) draw nothing but join the fold
    for (int64_t s = w < a.nw ? a.s0 + w : a.s0 + a.m; s < a.s0 + a.m; s += a.nw) {
        T y[1][E];
        Inputs<T, E, 1, MODE> U;
        if constexpr (BAL) {
            {
                // balanced layout: slot e of this lane is cell first_j + e
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int64_t j = first_j + e;
                    const U4 r = philox4x64_10((uint64_t)(j >> 2), (uint64_t)s, MC_STREAM, 0, k0, k1);
                    const T u = unif(philox_word(r, (int)(j & 3)), T(0));
                    y[0][e] = ghost<KIND, T>();
                    if (e < cnt) y[0][e] = fmaT(u, xhi[j] - xlo[j], xlo[j]);
                }
                if constexpr (MODE == IN_SCALAR) {
                    if (a.n_in == 0) {
                        U.u[0] = T(0);
                    } else {
                        const U4 r = philox4x64_10((uint64_t)(n >> 2), (uint64_t)s, MC_STREAM, 0, k0, k1);
                        const T u = unif(philox_word(r, (int)(n & 3)), T(0));
                        const T pl = ((const T*)a.p_lo)[0], ph = ((const T*)a.p_hi)[0];
                        U.u[0] = fmaT(u, ph - pl, pl);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const int64_t c = first_j + e;
                        const int64_t j = n + c;
                        const U4 r = philox4x64_10((uint64_t)(j >> 2), (uint64_t)s, MC_STREAM, 0, k0, k1);
                        const T u = unif(philox_word(r, (int)(j & 3)), T(0));
                        U.u[0][e] = T(0);
                        if (e < cnt) {
                            const T pl = ((const T*)a.p_lo)[c], ph = ((const T*)a.p_hi)[c];
                            U.u[0][e] = fmaT(u, ph - pl, pl);
                        }
                    }
                }
                mc_bal_steps<KIND, T, E, MODE>(y[0], a.nsteps, P, U, st, shortl, endl);
                // each cell's running min / max in the slot of the plain
                // layout (slot j mod E of lane j / E), which the reduction reads
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if (e < cnt) {
                        const int64_t j = first_j + e;
                        const size_t idx = (size_t)(j % E) * WAVE + (size_t)(j / E);
                        if (first) {
                            pmin[idx] = y[0][e];
                            pmax[idx] = y[0][e];
                        } else {
                            pmin[idx] = nan_min(pmin[idx], y[0][e]);
                            pmax[idx] = nan_max(pmax[idx], y[0][e]);
                        }
                    }
                }
                first = false;
                continue;
            }
        }
        // initial state: one Philox block per 4 consecutive cells
        if constexpr (E % 4 == 0) {
#pragma unroll
            for (int g = 0; g < E / 4; ++g) {
                const int64_t j0 = (int64_t)lane * E + 4 * g;
                const U4 r = philox4x64_10((uint64_t)(j0 >> 2), (uint64_t)s, MC_STREAM, 0, k0, k1);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t j = j0 + q;
                    const T u = unif(r.x[q], T(0));
                    y[0][4 * g + q] = (j < n) ? fmaT(u, xhi[j] - xlo[j], xlo[j]) : ghost<KIND, T>();
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t j = (int64_t)lane * E + e;
                const U4 r = philox4x64_10((uint64_t)(j >> 2), (uint64_t)s, MC_STREAM, 0, k0, k1);
                const T u = unif(philox_word(r, (int)(j & 3)), T(0));
                y[0][e] = (j < n) ? fmaT(u, xhi[j] - xlo[j], xlo[j]) : ghost<KIND, T>();
            }
        }
        // inputs, drawn per sample at coordinates n + k
        if constexpr (MODE == IN_SCALAR) {
            if (a.n_in == 0) {
                U.u[0] = T(0);
            } else {
                const int64_t j = n;
                const U4 r = philox4x64_10((uint64_t)(j >> 2), (uint64_t)s, MC_STREAM, 0, k0, k1);
                const T u = unif(philox_word(r, (int)(j & 3)), T(0));
                const T pl = ((const T*)a.p_lo)[0], ph = ((const T*)a.p_hi)[0];
                U.u[0] = fmaT(u, ph - pl, pl);
            }
        } else if constexpr (E % 4 == 0) {
            // cells c = lane E + 4g + q sit at coordinates n + c; with o = n mod 4
            // (the same in every lane) the four of group g fall in blocks b and
            // b + 1, b = (n + lane E + 4g) / 4, at words o + q counted on from b
            const int o = (int)(n & 3);
            const int64_t b0 = (n + (int64_t)lane * E) >> 2;
            U4 cur = philox4x64_10((uint64_t)b0, (uint64_t)s, MC_STREAM, 0, k0, k1);
#pragma unroll
            for (int g = 0; g < E / 4; ++g) {
                U4 nxt = cur;
                if (o != 0 || g + 1 < E / 4)
                    nxt = philox4x64_10((uint64_t)(b0 + g + 1), (uint64_t)s, MC_STREAM, 0, k0, k1);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int k = o + q;
                    const uint64_t word = k < 4 ? philox_word(cur, k) : philox_word(nxt, k - 4);
                    const T u = unif(word, T(0));
                    const int64_t c = (int64_t)lane * E + 4 * g + q;
                    if (c < n) {
                        const T pl = ((const T*)a.p_lo)[c], ph = ((const T*)a.p_hi)[c];
                        U.u[0][4 * g + q] = fmaT(u, ph - pl, pl);
                    } else {
                        U.u[0][4 * g + q] = T(0);
                    }
                }
                cur = nxt;
            }
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t c = (int64_t)lane * E + e;
                const int64_t j = n + c;
                const U4 r = philox4x64_10((uint64_t)(j >> 2), (uint64_t)s, MC_STREAM, 0, k0, k1);
                const T u = unif(philox_word(r, (int)(j & 3)), T(0));
                if (c < n) {
                    const T pl = ((const T*)a.p_lo)[c], ph = ((const T*)a.p_hi)[c];
                    U.u[0][e] = fmaT(u, ph - pl, pl);
                } else {
                    U.u[0][e] = T(0);
                }
            }
        }

        // the wave holds the whole chain: its window always contains cell n-1
        if (masked) {
            const auto M = chain_end_mask<E, true, true>(n);
            rk4_steps<KIND, T, E, 1, MODE>(y, a.nsteps, P, U, st, M);
        } else {
            Mask<E, false, true> M{E};
            rk4_steps<KIND, T, E, 1, MODE>(y, a.nsteps, P, U, st, M);
        }

#pragma unroll
        for (int e = 0; e < E; ++e) {
            const size_t idx = (size_t)e * WAVE + lane;
            if (first) {
                pmin[idx] = y[0][e];
                pmax[idx] = y[0][e];
            } else {
                pmin[idx] = nan_min(pmin[idx], y[0][e]);
                pmax[idx] = nan_max(pmax[idx], y[0][e]);
            }
        }
        first = false;
    }

    // fold the group's partials (waves wb .. wb + live - 1, each of which drew
    // at least one sample since nw <= m) into slot wb
    __syncthreads();
    const int64_t rest = a.nw - wb;
    const int live = (int)(rest < MC_WPB ? rest : MC_WPB);
    if (wv != 0 || live <= 1) return;
    T* bmin = (T*)a.part_min + (size_t)wb * E * WAVE;   // wave 0's own slot: may alias pmin
    T* bmax = (T*)a.part_max + (size_t)wb * E * WAVE;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const size_t idx = (size_t)e * WAVE + lane;
        T mn = bmin[idx], mx = bmax[idx];
        for (int k = 1; k < live; ++k) {
            mn = nan_min(mn, bmin[(size_t)k * E * WAVE + idx]);
            mx = nan_max(mx, bmax[(size_t)k * E * WAVE + idx]);
        }
        bmin[idx] = mn;
        bmax[idx] = mx;
    }
}

// Reduction of np partials lying wstep slots apart (slot = one wave's [e][lane]
// block), in two launches when np > RED_CHUNK.  Block (e, g) owns the 64 values
// [e][0..63] (cells j = lane * E + e) of partials w in [g RED_CHUNK,
// (g + 1) RED_CHUNK): its RED_WAVES waves issue RED_CHUNK / RED_WAVES
// independent loads each, then combine through LDS.  The first launch writes
// each chunk's result over the chunk's first partial; the second (wstep times
// RED_CHUNK) reduces those and writes the box.  Min and max (NaN-propagating)
// are exact, so the split changes no value (signed zeros aside), and every
// block reads only its own chunk.
constexpr int RED_WAVES = 16;
constexpr int RED_CHUNK = 256;
constexpr int RED_PER_WAVE = RED_CHUNK / RED_WAVES;

template <class T, int E>
__global__ __launch_bounds__(WAVE * RED_WAVES) void mc_reduce_kernel(
    T* __restrict__ pmin, T* __restrict__ pmax, int64_t nw, int64_t wstep, int64_t n,
    T* __restrict__ rmin, T* __restrict__ rmax, unsigned int* status, int final_pass) {
    __shared__ T smin[RED_WAVES][WAVE];
    __shared__ T smax[RED_WAVES][WAVE];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = threadIdx.x / WAVE;
    const size_t off = (size_t)blockIdx.x * WAVE + (size_t)lane;
    const size_t stride = (size_t)E * WAVE;
    const int64_t w0 = (int64_t)blockIdx.y * RED_CHUNK;
    const int64_t w1 = w0 + RED_CHUNK < nw ? w0 + RED_CHUNK : nw;
    // indices past the chunk load nothing and stand in with the identities
    // +inf / -inf (nan_min(x, +inf) = x for every x, NaN included; the
    // chunk's first partial always exists)
    T a[RED_PER_WAVE], b[RED_PER_WAVE];
#pragma unroll
    for (int u = 0; u < RED_PER_WAVE; ++u) {
        const int64_t w = w0 + wv + (int64_t)u * RED_WAVES;
        a[u] = T(__builtin_inf());
        b[u] = -T(__builtin_inf());
        if (w < w1) {   // the same in every lane of the wave
            const size_t idx = (size_t)(w * wstep) * stride + off;
            a[u] = pmin[idx];
            b[u] = pmax[idx];
        }
    }
    T mn = a[0], mx = b[0];
#pragma unroll
    for (int u = 1; u < RED_PER_WAVE; ++u) {
        mn = nan_min(mn, a[u]);
        mx = nan_max(mx, b[u]);
    }
    smin[wv][lane] = mn;
    smax[wv][lane] = mx;
    __syncthreads();
    if (wv != 0) return;
    mn = smin[0][lane];
    mx = smax[0][lane];
#pragma unroll
    for (int k = 1; k < RED_WAVES; ++k) {
        mn = nan_min(mn, smin[k][lane]);
        mx = nan_max(mx, smax[k][lane]);
    }
    if (!final_pass) {
        const size_t idx = (size_t)(w0 * wstep) * stride + off;
        pmin[idx] = mn;
        pmax[idx] = mx;
        return;
    }
    const int64_t j = (int64_t)lane * E + blockIdx.x;
    unsigned bits = 0;
    if (j < n) {
        rmin[j] = mn;
        rmax[j] = mx;
        if (!finiteT(mn) || !finiteT(mx)) bits = ST_NONFINITE;
    }
    report_status(status, bits);
}

template <int KIND, class T, int E, int MODE>
static hipError_t go(const McArgs& a, hipStream_t s) {
    const unsigned grid = (unsigned)((a.nw + MC_WPB - 1) / MC_WPB);
    // the balanced layout for padded waves with lane arrays over 128 bytes
    const int64_t L = (a.n + E - 1) / E;
    const bool bal = E * sizeof(T) > 128 && (int64_t)WAVE * E > a.n && a.n >= (int64_t)(E - 1) * L;
    if constexpr (E * sizeof(T) > 128) {
        if (bal) {
            hipLaunchKernelGGL((mc_kernel<KIND, T, E, MODE, true>), dim3(grid), dim3(WAVE * MC_WPB),
                               0, s, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((mc_kernel<KIND, T, E, MODE>), dim3(grid), dim3(WAVE * MC_WPB), 0, s, a);
    return hipGetLastError();
}

template <int KIND, class T, int MODE>
static hipError_t by_E(int E, const McArgs& a, hipStream_t s) {
    switch (E) {
        case 1: return go<KIND, T, 1, MODE>(a, s);
        case 2: return go<KIND, T, 2, MODE>(a, s);
        case 4: return go<KIND, T, 4, MODE>(a, s);
        case 8: return go<KIND, T, 8, MODE>(a, s);
        case 16: return go<KIND, T, 16, MODE>(a, s);
        case 32: return go<KIND, T, 32, MODE>(a, s);
        case 64:
            if constexpr (sizeof(T) == 4) return go<KIND, T, 64, MODE>(a, s);
            else return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

bool mc_has_E(int dtype, int E) {
    return E == 1 || E == 2 || E == 4 || E == 8 || E == 16 || E == 32 || (dtype == 1 && E == 64);
}
int mc_max_E(int dtype) { return dtype == 1 ? 64 : 32; }

hipError_t launch_mc(int kind, int mode, int dtype, int E, const McArgs& a, hipStream_t s) {
    if (dtype == 0) {
        if (kind == K_CTM) return by_E<K_CTM, double, IN_SCALAR>(E, a, s);
        if (kind == K_RD) return mode ? by_E<K_RD, double, IN_CELL>(E, a, s)
                                      : by_E<K_RD, double, IN_SCALAR>(E, a, s);
        if (kind == K_LIN3) return mode ? by_E<K_LIN3, double, IN_CELL>(E, a, s)
                                        : by_E<K_LIN3, double, IN_SCALAR>(E, a, s);
    } else {
        if (kind == K_CTM) return by_E<K_CTM, float, IN_SCALAR>(E, a, s);
        if (kind == K_RD) return mode ? by_E<K_RD, float, IN_CELL>(E, a, s)
                                      : by_E<K_RD, float, IN_SCALAR>(E, a, s);
        if (kind == K_LIN3) return mode ? by_E<K_LIN3, float, IN_CELL>(E, a, s)
                                        : by_E<K_LIN3, float, IN_SCALAR>(E, a, s);
    }
    return hipErrorInvalidValue;
}

template <class T, int E>
static hipError_t reduce_E(void* pmin, void* pmax, int64_t nw, int64_t group, int64_t n,
                           void* rmin, void* rmax, unsigned int* status, hipStream_t s) {
    const dim3 block(WAVE * RED_WAVES);
    const int64_t np = (nw + group - 1) / group;
    const int64_t chunks = (np + RED_CHUNK - 1) / RED_CHUNK;
    if (chunks > 1) {
        hipLaunchKernelGGL((mc_reduce_kernel<T, E>), dim3(E, (unsigned)chunks), block, 0, s,
                           (T*)pmin, (T*)pmax, np, group, n, (T*)rmin, (T*)rmax, status, 0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        static_assert(RED_CHUNK * RED_CHUNK >= kMcMaxWaves, "two passes cover every wave count");
        hipLaunchKernelGGL((mc_reduce_kernel<T, E>), dim3(E, 1), block, 0, s, (T*)pmin, (T*)pmax,
                           chunks, group * RED_CHUNK, n, (T*)rmin, (T*)rmax, status, 1);
    } else {
        hipLaunchKernelGGL((mc_reduce_kernel<T, E>), dim3(E, 1), block, 0, s, (T*)pmin, (T*)pmax,
                           np, group, n, (T*)rmin, (T*)rmax, status, 1);
    }
    return hipGetLastError();
}

template <class T>
static hipError_t reduce_T(int E, void* pmin, void* pmax, int64_t nw, int64_t group, int64_t n,
                           void* rmin, void* rmax, unsigned int* status, hipStream_t s) {
    switch (E) {
        case 1: return reduce_E<T, 1>(pmin, pmax, nw, group, n, rmin, rmax, status, s);
        case 2: return reduce_E<T, 2>(pmin, pmax, nw, group, n, rmin, rmax, status, s);
        case 4: return reduce_E<T, 4>(pmin, pmax, nw, group, n, rmin, rmax, status, s);
        case 8: return reduce_E<T, 8>(pmin, pmax, nw, group, n, rmin, rmax, status, s);
        case 16: return reduce_E<T, 16>(pmin, pmax, nw, group, n, rmin, rmax, status, s);
        case 32: return reduce_E<T, 32>(pmin, pmax, nw, group, n, rmin, rmax, status, s);
        case 64: return reduce_E<T, 64>(pmin, pmax, nw, group, n, rmin, rmax, status, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_mc_reduce(int dtype, int E, void* pmin, void* pmax, int64_t nw, int64_t group,
                            int64_t n, void* rmin, void* rmax, unsigned int* status,
                            hipStream_t s) {
    if (group < 1) return hipErrorInvalidValue;
    return dtype == 0 ? reduce_T<double>(E, pmin, pmax, nw, group, n, rmin, rmax, status, s)
                      : reduce_T<float>(E, pmin, pmax, nw, group, n, rmin, rmax, status, s);
}

int mc_waves_per_group() { return MC_WPB; }

}  // namespace reach
