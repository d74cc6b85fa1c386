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

    // Cells [ts, ts + 64E) of src into lane registers; cells >= n get `ghost`.
    // `fast`: the window lies inside the chain and src is 16-byte aligned.
    static __device__ __forceinline__ void load(T (&dst)[E], const T* __restrict__ src, int64_t ts,
                                                int64_t n, T ghost, bool fast, T* lds) {
        const int lane = threadIdx.x;
        if constexpr (STAGED) {
            if (fast) {
                constexpr int CPL = E / VEC;
#pragma unroll
                for (int j = 0; j < CPL; ++j) {
                    const int el = (j * WAVE + lane) * VEC;
                    const V v = *reinterpret_cast<const V*>(src + ts + el);
                    *reinterpret_cast<V*>(lds + (el / E) * ROW + (el % E)) = v;
                }
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
                                                 int olo, int ohi, bool fast, T* lds) {
        const int lane = threadIdx.x;
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
#pragma unroll
                for (int j = 0; j < CPL; ++j) {
                    const int el = (j * WAVE + lane) * VEC;
                    const V x = *reinterpret_cast<const V*>(lds + (el / E) * ROW + (el % E));
                    if (el >= olo && el + VEC <= ohi) {
                        *reinterpret_cast<V*>(dst + ts + el) = x;
                    } else {
#pragma unroll
                        for (int q = 0; q < VEC; ++q)
                            if (el + q >= olo && el + q < ohi) dst[ts + el + q] = x[q];
                    }
                }
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

template <int KIND, class T, int E, int MODE>
__global__ __launch_bounds__(64) void embed_tile_kernel(EmbedPass a) {
    using IO = TileIO<T, E>;
    __shared__ __attribute__((aligned(16))) T lds[IO::LDS_ELEMS];
    const int lane = threadIdx.x;

    // blockIdx -> tile: consecutive tiles on one XCD share halos in its L2.
    const int64_t b = blockIdx.x;
    const int64_t w = (b & 7) * (int64_t)a.per_xcd + (b >> 3);
    if (w >= a.W) return;

    const int64_t span = (int64_t)WAVE * E;
    const int64_t ts = w * a.OUT;
    const bool reaches_end = ts + span >= a.n;
    const bool masked = ts + span > a.n;
    const bool fast = a.aligned && !masked;

    T y[2][E];
    IO::load(y[0], (const T*)a.src_lo, ts, a.n, ghost<KIND, T>(), fast, lds);
    IO::load(y[1], (const T*)a.src_hi, ts, a.n, ghost<KIND, T>(), fast, lds);

    Inputs<T, E, 2, MODE> U;
    if constexpr (MODE == IN_SCALAR) {
        U.u[0] = a.p_lo ? ((const T*)a.p_lo)[0] : T(0);
        U.u[1] = a.p_hi ? ((const T*)a.p_hi)[0] : T(0);
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t g = ts + (int64_t)lane * E + e;
            U.u[0][e] = (g < a.n) ? ((const T*)a.p_lo)[g] : T(0);
            U.u[1][e] = (g < a.n) ? ((const T*)a.p_hi)[g] : T(0);
        }
    }
    const SysPrm<T> P = make_prm<T>(a.prm);
    const Steps<T> st = {(T)a.h2, (T)a.dt, (T)a.dt6};

    if (masked) {
        const int64_t left = a.n - (ts + (int64_t)lane * E);
        Mask<E, true> M{(int)(left < 0 ? 0 : (left > E ? E : left))};
        rk4_steps<KIND, T, E, 2, MODE, true>(y, a.ksteps, P, U, st, M);
    } else {
        Mask<E, false> M{E};
        rk4_steps<KIND, T, E, 2, MODE, false>(y, a.ksteps, P, U, st, M);
    }

    const int olo = (w == 0) ? 0 : a.H;
    const int ohi = reaches_end ? (int)(a.n - ts) : (int)(span - a.H);
    IO::store(y[0], (T*)a.dst_lo, ts, olo, ohi, fast, lds);
    IO::store(y[1], (T*)a.dst_hi, ts, olo, ohi, fast, lds);

    if (a.check) {
        unsigned bits = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int el = lane * E + e;
            if (el >= olo && el < ohi) {
                if (!finiteT(y[0][e]) || !finiteT(y[1][e])) bits |= ST_NONFINITE;
                if (y[0][e] > y[1][e]) bits |= ST_ORDER;
            }
        }
        report_status(a.status, bits);
    }
}

template <int KIND, class T, int E, int MODE>
static hipError_t go(const EmbedPass& a, int64_t grid, hipStream_t s) {
    hipLaunchKernelGGL((embed_tile_kernel<KIND, T, E, MODE>), dim3((unsigned)grid), dim3(WAVE), 0, s, a);
    return hipGetLastError();
}

template <int KIND, class T, int MODE>
static hipError_t by_E(int E, const EmbedPass& a, int64_t grid, hipStream_t s) {
    switch (E) {
        case 1: return go<KIND, T, 1, MODE>(a, grid, s);
        case 2: return go<KIND, T, 2, MODE>(a, grid, s);
        case 4: return go<KIND, T, 4, MODE>(a, grid, s);
        case 8: return go<KIND, T, 8, MODE>(a, grid, s);
        case 16: return go<KIND, T, 16, MODE>(a, grid, s);
        case 32:
            if constexpr (sizeof(T) == 4) return go<KIND, T, 32, MODE>(a, grid, s);
            else return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

bool embed_has_E(int dtype, int E) {
    return E == 1 || E == 2 || E == 4 || E == 8 || E == 16 || (dtype == 1 && E == 32);
}
int embed_max_E(int dtype) { return dtype == 1 ? 32 : 16; }

hipError_t launch_embed(int kind, int mode, int dtype, int E, const EmbedPass& a, int64_t grid,
                        hipStream_t s) {
    if (dtype == 0) {
        if (kind == K_CTM) return by_E<K_CTM, double, IN_SCALAR>(E, a, grid, s);
        if (kind == K_RD) return mode ? by_E<K_RD, double, IN_CELL>(E, a, grid, s)
                                      : by_E<K_RD, double, IN_SCALAR>(E, a, grid, s);
        if (kind == K_LIN3) return mode ? by_E<K_LIN3, double, IN_CELL>(E, a, grid, s)
                                        : by_E<K_LIN3, double, IN_SCALAR>(E, a, grid, s);
    } else {
        if (kind == K_CTM) return by_E<K_CTM, float, IN_SCALAR>(E, a, grid, s);
        if (kind == K_RD) return mode ? by_E<K_RD, float, IN_CELL>(E, a, grid, s)
                                      : by_E<K_RD, float, IN_SCALAR>(E, a, grid, s);
        if (kind == K_LIN3) return mode ? by_E<K_LIN3, float, IN_CELL>(E, a, grid, s)
                                        : by_E<K_LIN3, float, IN_SCALAR>(E, a, grid, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace reach
