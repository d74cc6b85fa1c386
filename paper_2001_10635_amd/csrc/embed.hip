// Embedding-system RK4 on gfx950: the mixed-monotonicity method of PIRK
// (Sec. 2.1; Algorithm 3 with Algorithm 1 as integrator), fused and
// temporally blocked.
//
// One wavefront owns a window of 64*E cells of both the lower and the upper
// vector (E cells per lane, both sides in the same lane so the coupled LIN3
// decomposition function sees x and xh of its neighbours).  A pass loads the
// window once, runs `ksteps` RK4 steps entirely in registers (four stages per
// step, neighbour values by DPP lane shifts), and writes back only the cells
// that are still exact: each stage lets a cut window edge corrupt one more
// cell, so a pass of K steps keeps a halo of H = 4K cells per cut edge.
// Windows that start at cell 0 or reach cell n-1 use the chain's own boundary
// conditions there and lose nothing on that side.  HBM traffic is one read
// and one write of 2n values per pass, i.e. per K steps.
//
// Global <-> register transfers go through LDS so that every global access is
// a coalesced 16-byte vector access even though each lane owns E consecutive
// cells (rows padded by 16 bytes to keep the LDS reads conflict-free).
#include <algorithm>

#include "dev.hpp"
#include "kernels.hpp"

namespace reach {

template <class T> struct Vec16;
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); };

template <class T, int E> struct TileIO {
    static constexpr int VEC = 16 / (int)sizeof(T);
    static constexpr bool STAGED = (E % VEC) == 0;
    static constexpr int ROW = E + VEC;
    static constexpr int LDS_ELEMS = STAGED ? WAVE * ROW : 1;
    using V = typename Vec16<T>::type;

    template <bool NT>
    static __device__ __forceinline__ V ld(const T* p) {
        const V* q = reinterpret_cast<const V*>(p);
        if constexpr (NT) return __builtin_nontemporal_load(q);
        else return *q;
    }
    template <bool NT>
    static __device__ __forceinline__ void st(T* p, V v) {
        V* q = reinterpret_cast<V*>(p);
        if constexpr (NT) __builtin_nontemporal_store(v, q);
        else *q = v;
    }
    // the window's global reads into LDS rows (NT: non-temporal)
    template <bool NT>
    static __device__ __forceinline__ void gather(const T* __restrict__ src, int64_t ts, T* lds) {
        const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
        for (int j = 0; j < E / VEC; ++j) {
            const int el = (j * WAVE + lane) * VEC;
            const V v = ld<NT>(src + ts + el);
            *reinterpret_cast<V*>(lds + (el / E) * ROW + (el % E)) = v;
        }
    }
    // LDS rows to the window's global cells [olo, ohi) (NT: non-temporal)
    template <bool NT>
    static __device__ __forceinline__ void scatter(T* __restrict__ dst, int64_t ts, int olo, int ohi,
                                                   const T* lds) {
        const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
        for (int j = 0; j < E / VEC; ++j) {
            const int el = (j * WAVE + lane) * VEC;
            const V x = *reinterpret_cast<const V*>(lds + (el / E) * ROW + (el % E));
            if (el >= olo && el + VEC <= ohi) {
                st<NT>(dst + ts + el, x);
            } else {
#pragma unroll
                for (int q = 0; q < VEC; ++q)
                    if (el + q >= olo && el + q < ohi) dst[ts + el + q] = x[q];
            }
        }
    }

    // Cells [ts, ts + 64E) of src into lane registers; cells >= n get `ghost`.
    // `fast`: the window lies inside the chain and src is 16-byte aligned;
    // `nt`: its global accesses are non-temporal.
    static __device__ __forceinline__ void load(T (&dst)[E], const T* __restrict__ src, int64_t ts,
                                                int64_t n, T ghost, bool fast, bool nt, T* lds) {
        const int lane = threadIdx.x & (WAVE - 1);
        if constexpr (STAGED) {
            if (fast) {
                constexpr int CPL = E / VEC;
                if (nt) gather<true>(src, ts, lds);
                else gather<false>(src, ts, lds);
                __syncthreads();
#pragma unroll
                for (int j = 0; j < CPL; ++j) {
                    const V v = *reinterpret_cast<const V*>(lds + lane * ROW + j * VEC);
#pragma unroll
                    for (int q = 0; q < VEC; ++q) dst[j * VEC + q] = v[q];
                }
                __syncthreads();
                return;
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t g = ts + (int64_t)lane * E + e;
            dst[e] = (g < n) ? src[g] : ghost;
        }
    }

    // Window cells [olo, ohi) of the lane registers to dst[ts + ...].
    static __device__ __forceinline__ void store(const T (&v)[E], T* __restrict__ dst, int64_t ts,
                                                 int olo, int ohi, bool fast, bool nt, T* lds) {
        const int lane = threadIdx.x & (WAVE - 1);
        if constexpr (STAGED) {
            if (fast) {
                constexpr int CPL = E / VEC;
#pragma unroll
                for (int j = 0; j < CPL; ++j) {
                    V x;
#pragma unroll
                    for (int q = 0; q < VEC; ++q) x[q] = v[j * VEC + q];
                    *reinterpret_cast<V*>(lds + lane * ROW + j * VEC) = x;
                }
                __syncthreads();
                if (nt) scatter<true>(dst, ts, olo, ohi, lds);
                else scatter<false>(dst, ts, olo, ohi, lds);
                __syncthreads();
                return;
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int el = lane * E + e;
            if (el >= olo && el < ohi) dst[ts + el] = v[e];
        }
    }
};

template <class T> __device__ __forceinline__ SysPrm<T> make_prm(const double (&p)[5]) {
    SysPrm<T> P;
    P.a0 = (T)p[0]; P.a1 = (T)p[1]; P.a2 = (T)p[2]; P.a3 = (T)p[3]; P.a4 = (T)p[4];
    return P;
}

// S = 2: a wave holds both sides of its window (any system, including the
// coupled LIN3).  S = 1: a wave holds one side (cooperative systems only, whose
// decomposition function reads one side), so the same registers cover twice
// the cells and the halo share halves; tiles [0, W) are the lower side and
// [W, 2W) the upper side.  PAIR (S = 1, one window): one block of two waves,
// the lower and the upper side, which compare their boxes through LDS at the
// end instead of a separate order-check launch.
template <int KIND, class T, int E, int MODE, int S, bool PAIR>
__global__ __launch_bounds__(PAIR ? 2 * WAVE : WAVE) void embed_tile_kernel(EmbedPass a) {
    using IO = TileIO<T, E>;
    __shared__ __attribute__((aligned(16))) T lds[IO::LDS_ELEMS * (PAIR ? 2 : 1)];
    const int lane = threadIdx.x & (WAVE - 1);

    // blockIdx -> tile: consecutive tiles on one XCD share halos in its L2.
    int64_t g;
    if constexpr (PAIR) {
        g = (int64_t)(threadIdx.x / WAVE);   // W = 1: tile 0 lower, tile 1 upper
    } else {
        const int64_t b = blockIdx.x;
        g = (b & 7) * (int64_t)a.per_xcd + (b >> 3);
        if (g >= (S == 1 ? 2 * a.W : a.W)) return;
    }
    const int side = (S == 1 && g >= a.W) ? 1 : 0;
    T* const my_lds = lds + (PAIR ? side * IO::LDS_ELEMS : 0);
    const int64_t w = g - side * a.W;

    const int64_t span = (int64_t)WAVE * E;
    const int64_t ts = w * a.OUT;
    const bool reaches_end = ts + span >= a.n;
    const bool fast = a.aligned && ts + span <= a.n;
    const T* src[2] = {(const T*)a.src_lo, (const T*)a.src_hi};
    T* dst[2] = {(T*)a.dst_lo, (T*)a.dst_hi};
    const T* pin[2] = {(const T*)a.p_lo, (const T*)a.p_hi};

    T y[S][E];
#pragma unroll
    for (int s = 0; s < S; ++s)
        IO::load(y[s], src[S == 1 ? side : s], ts, a.n, ghost<KIND, T>(), fast, a.nt, my_lds);

    Inputs<T, E, S, MODE> U;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const T* p = pin[S == 1 ? side : s];
        if constexpr (MODE == IN_SCALAR) {
            U.u[s] = p ? p[0] : T(0);
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t c = ts + (int64_t)lane * E + e;
                U.u[s][e] = (c < a.n) ? p[c] : T(0);
            }
        }
    }
    const SysPrm<T> P = make_prm<T>(a.prm);
    const Steps<T> st = {(T)a.h2, (T)a.dt, (T)a.dt6};

    bool exact = false;
    if constexpr (PAIR) {
        // a single window filled exactly (n = 64E): the chain's end is lane
        // 63's last cell and no cell is padding, so no per-stage masking (the
        // latency path: every select saved shortens the dependent chain)
        exact = a.n - ts == span;
        if (exact) {
            Mask<E, false, true> M{E};
            rk4_steps<KIND, T, E, S, MODE>(y, a.ksteps, P, U, st, M);
        }
    }
    if (!exact) {
        if (reaches_end) {
            // the window holding cell n-1 (cells past it, if any, are ghosts)
            const int64_t left = a.n - (ts + (int64_t)lane * E);
            Mask<E, true, true> M{(int)(left < 0 ? 0 : (left > E ? E : left))};
            rk4_steps<KIND, T, E, S, MODE>(y, a.ksteps, P, U, st, M);
        } else {
            Mask<E, false, false> M{E};
            rk4_steps<KIND, T, E, S, MODE>(y, a.ksteps, P, U, st, M);
        }
    }

    const int olo = (w == 0) ? 0 : a.H;
    const int ohi = reaches_end ? (int)(a.n - ts) : (int)(span - a.H);
#pragma unroll
    for (int s = 0; s < S; ++s)
        IO::store(y[s], dst[S == 1 ? side : s], ts, olo, ohi, fast, a.nt, my_lds);

    if (a.check) {
        unsigned bits = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int el = lane * E + e;
            if (el >= olo && el < ohi) {
#pragma unroll
                for (int s = 0; s < S; ++s)
                    if (!finiteT(y[s][e])) bits |= ST_NONFINITE;
                if constexpr (S == 2) {
                    if (y[0][e] > y[1][e]) bits |= ST_ORDER;
                }
            }
        }
        if constexpr (PAIR) {
            // the upper wave hands its box to the lower one
            __shared__ T upper[PAIR ? WAVE * E : 1];
            if (side == 1) {
#pragma unroll
                for (int e = 0; e < E; ++e) upper[lane * E + e] = y[0][e];
            }
            __syncthreads();
            if (side == 0) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int el = lane * E + e;
                    if (el >= olo && el < ohi && y[0][e] > upper[el]) bits |= ST_ORDER;
                }
            }
        }
        report_status(a.status, bits);
    }
}

// Lower > upper check of a finished box (used after single-side passes, where
// no wave sees both sides of a cell).
template <class T>
__global__ __launch_bounds__(256) void order_check_kernel(const T* __restrict__ lo,
                                                          const T* __restrict__ hi, int64_t n,
                                                          unsigned int* status) {
    unsigned bits = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (lo[i] > hi[i]) bits = ST_ORDER;
    report_status(status, bits);
}

template <int KIND, class T, int E, int MODE, int S, bool PAIR = false>
static hipError_t go(const EmbedPass& a, int64_t grid, hipStream_t s) {
    if constexpr (PAIR)
        hipLaunchKernelGGL((embed_tile_kernel<KIND, T, E, MODE, S, true>), dim3(1), dim3(2 * WAVE),
                           0, s, a);
    else
        hipLaunchKernelGGL((embed_tile_kernel<KIND, T, E, MODE, S, false>), dim3((unsigned)grid),
                           dim3(WAVE), 0, s, a);
    return hipGetLastError();
}
template <int KIND, class T, int E, int MODE>
static hipError_t go_one_side(bool pair, const EmbedPass& a, int64_t grid, hipStream_t s) {
    return pair ? go<KIND, T, E, MODE, 1, true>(a, grid, s) : go<KIND, T, E, MODE, 1, false>(a, grid, s);
}

// Shapes built: S = 2 (both sides per wave) for every system, S = 1 (one side
// per wave, wider tiles) for the cooperative CTM and RD chains.
template <int KIND, class T, int MODE>
static hipError_t by_E(int E, int S, bool pair, const EmbedPass& a, int64_t grid, hipStream_t s) {
    constexpr bool F32 = sizeof(T) == 4;
    constexpr bool COOP = KIND != K_LIN3;
    if (S == 2) {
        switch (E) {
            case 1: return go<KIND, T, 1, MODE, 2>(a, grid, s);
            case 2: return go<KIND, T, 2, MODE, 2>(a, grid, s);
            case 4: return go<KIND, T, 4, MODE, 2>(a, grid, s);
            case 8: return go<KIND, T, 8, MODE, 2>(a, grid, s);
            case 12: return go<KIND, T, 12, MODE, 2>(a, grid, s);
            case 16: return go<KIND, T, 16, MODE, 2>(a, grid, s);
            case 32:
                if constexpr (F32) return go<KIND, T, 32, MODE, 2>(a, grid, s);
                else return hipErrorInvalidValue;
            default: return hipErrorInvalidValue;
        }
    }
    if constexpr (COOP) {
        if (S == 1) {
            switch (E) {
                case 1: return go_one_side<KIND, T, 1, MODE>(pair, a, grid, s);
                case 2: return go_one_side<KIND, T, 2, MODE>(pair, a, grid, s);
                case 4: return go_one_side<KIND, T, 4, MODE>(pair, a, grid, s);
                case 8: return go_one_side<KIND, T, 8, MODE>(pair, a, grid, s);
                case 16: return go_one_side<KIND, T, 16, MODE>(pair, a, grid, s);
                case 24: return go_one_side<KIND, T, 24, MODE>(pair, a, grid, s);
                case 28:   // FP64: the widest one-side tile within 256 VGPRs
                    if constexpr (!F32) return go_one_side<KIND, T, 28, MODE>(pair, a, grid, s);
                    else return hipErrorInvalidValue;
                case 32: return go_one_side<KIND, T, 32, MODE>(pair, a, grid, s);
                case 48:
                    if constexpr (F32) return go_one_side<KIND, T, 48, MODE>(pair, a, grid, s);
                    else return hipErrorInvalidValue;
                case 64:
                    if constexpr (F32) return go_one_side<KIND, T, 64, MODE>(pair, a, grid, s);
                    else return hipErrorInvalidValue;
                default: return hipErrorInvalidValue;
            }
        }
    }
    return hipErrorInvalidValue;
}

bool embed_has_shape(int kind, int dtype, int E, int S) {
    if (S == 2)
        return E == 1 || E == 2 || E == 4 || E == 8 || E == 12 || E == 16 || (dtype == 1 && E == 32);
    if (S == 1 && kind != K_LIN3)
        return E == 1 || E == 2 || E == 4 || E == 8 || E == 16 || E == 24 || E == 32 ||
               (dtype == 0 && E == 28) || (dtype == 1 && (E == 48 || E == 64));
    return false;
}
int embed_max_E(int dtype, int S) {
    if (S == 1) return dtype == 1 ? 64 : 32;
    return dtype == 1 ? 32 : 16;
}

hipError_t launch_embed(int kind, int mode, int dtype, int E, int S, bool pair,
                        const EmbedPass& a, int64_t grid, hipStream_t s) {
    if (pair && (S != 1 || a.W != 1)) return hipErrorInvalidValue;
    if (dtype == 0) {
        if (kind == K_CTM) return by_E<K_CTM, double, IN_SCALAR>(E, S, pair, a, grid, s);
        if (kind == K_RD) return mode ? by_E<K_RD, double, IN_CELL>(E, S, pair, a, grid, s)
                                      : by_E<K_RD, double, IN_SCALAR>(E, S, pair, a, grid, s);
        if (kind == K_LIN3) return mode ? by_E<K_LIN3, double, IN_CELL>(E, S, pair, a, grid, s)
                                        : by_E<K_LIN3, double, IN_SCALAR>(E, S, pair, a, grid, s);
    } else {
        if (kind == K_CTM) return by_E<K_CTM, float, IN_SCALAR>(E, S, pair, a, grid, s);
        if (kind == K_RD) return mode ? by_E<K_RD, float, IN_CELL>(E, S, pair, a, grid, s)
                                      : by_E<K_RD, float, IN_SCALAR>(E, S, pair, a, grid, s);
        if (kind == K_LIN3) return mode ? by_E<K_LIN3, float, IN_CELL>(E, S, pair, a, grid, s)
                                        : by_E<K_LIN3, float, IN_SCALAR>(E, S, pair, a, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_order_check(int dtype, const void* lo, const void* hi, int64_t n,
                              unsigned int* status, hipStream_t s) {
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    if (dtype == 0)
        hipLaunchKernelGGL(order_check_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const double*)lo, (const double*)hi, n, status);
    else
        hipLaunchKernelGGL(order_check_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const float*)lo, (const float*)hi, n, status);
    return hipGetLastError();
}

}  // namespace reach
