// Contraction / growth-bound reachable box on gfx950 (PIRK Sec. 2.1,
// Algorithm 2).
//
// Two RK4 runs share every launch: tiles [0, W) integrate the center of the
// box with the system's own f at the center input, tiles [W, 2W) integrate the
// half-width with the linear growth dynamics r' = C r + |b| [p], C the
// tridiagonal contraction matrix.  Each wave holds one run's window in
// registers, exactly like the one-side embedding tiles (same per-cell code,
// same temporal blocking and halos).  The first pass forms c = (lo + hi) / 2 or
// r = (hi - lo) / 2 as it loads the box; a final elementwise kernel writes
// [c - r, c + r].
#include <algorithm>

#include "dev.hpp"
#include "kernels.hpp"

namespace reach {

template <class T> struct Vec16g;
template <> struct Vec16g<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct Vec16g<float> { typedef float type __attribute__((ext_vector_type(4))); };

// Cells [ts, ts + 64E) of src into registers, cells >= n get `fill`.
template <class T, int E>
__device__ __forceinline__ void gb_load(T (&dst)[E], const T* __restrict__ src, int64_t ts,
                                        int64_t n, T fill) {
    const int lane = threadIdx.x;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t g = ts + (int64_t)lane * E + e;
        dst[e] = (g < n) ? src[g] : fill;
    }
}

template <int KIND, class T, int E, int MODE>
__global__ __launch_bounds__(64) void gb_tile_kernel(GbPass a) {
    const int lane = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int64_t g = (b & 7) * (int64_t)a.per_xcd + (b >> 3);
    if (g >= 2 * a.W) return;
    const int side = g >= a.W ? 1 : 0;          // 0: center run, 1: half-width run
    const int64_t w = g - side * a.W;
    const int64_t span = (int64_t)WAVE * E;
    const int64_t ts = w * a.OUT;
    const bool reaches_end = ts + span >= a.n;

    T y[1][E];
    if (a.first) {
        // c = (lo + hi) / 2, r = (hi - lo) / 2 (ghost cells: the center run's
        // ghost, radius 0)
        T lo[E], hi[E];
        gb_load<T, E>(lo, (const T*)a.x_lo, ts, a.n, T(0));
        gb_load<T, E>(hi, (const T*)a.x_hi, ts, a.n, T(0));
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t c = ts + (int64_t)lane * E + e;
            if (side == 0) y[0][e] = (c < a.n) ? (lo[e] + hi[e]) / T(2) : ghost<KIND, T>();
            else y[0][e] = (c < a.n) ? (hi[e] - lo[e]) / T(2) : T(0);
        }
    } else {
        const T* src = (const T*)(side == 0 ? a.src_c : a.src_r);
        gb_load<T, E>(y[0], src, ts, a.n, side == 0 ? ghost<KIND, T>() : T(0));
    }

    // inputs: center p* = (p_lo + p_hi) / 2, half-width [p] = (p_hi - p_lo) / 2
    Inputs<T, E, 1, MODE> U;
    const T* pl = (const T*)a.p_lo;
    const T* ph = (const T*)a.p_hi;
    if constexpr (MODE == IN_SCALAR) {
        if (pl) U.u[0] = side == 0 ? (pl[0] + ph[0]) / T(2) : (ph[0] - pl[0]) / T(2);
        else U.u[0] = T(0);
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t c = ts + (int64_t)lane * E + e;
            T u = T(0);
            if (c < a.n) u = side == 0 ? (pl[c] + ph[c]) / T(2) : (ph[c] - pl[c]) / T(2);
            U.u[0][e] = u;
        }
    }
    const Steps<T> st = {(T)a.h2, (T)a.dt, (T)a.dt6};
    const int64_t left = a.n - (ts + (int64_t)lane * E);
    const int nvalid = (int)(left < 0 ? 0 : (left > E ? E : left));

    if (side == 0) {
        const SysPrm<T> P = {(T)a.prm[0], (T)a.prm[1], (T)a.prm[2], (T)a.prm[3], (T)a.prm[4]};
        if (reaches_end) {
            Mask<E, true, true> M{nvalid};
            rk4_steps<KIND, T, E, 1, MODE>(y, a.ksteps, P, U, st, M);
        } else {
            Mask<E, false, false> M{E};
            rk4_steps<KIND, T, E, 1, MODE>(y, a.ksteps, P, U, st, M);
        }
    } else {
        const SysPrm<T> P = {(T)a.prm_r[0], (T)a.prm_r[1], (T)a.prm_r[2], (T)a.prm_r[3], T(0)};
        if (reaches_end) {
            Mask<E, true, true> M{nvalid};
            rk4_steps<K_LIN3, T, E, 1, MODE>(y, a.ksteps, P, U, st, M);
        } else {
            Mask<E, false, false> M{E};
            rk4_steps<K_LIN3, T, E, 1, MODE>(y, a.ksteps, P, U, st, M);
        }
    }

    const int olo = (w == 0) ? 0 : a.H;
    const int ohi = reaches_end ? (int)(a.n - ts) : (int)(span - a.H);
    T* dst = (T*)(side == 0 ? a.dst_c : a.dst_r);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int el = lane * E + e;
        if (el >= olo && el < ohi) dst[ts + el] = y[0][e];
    }
}

template <class T>
__global__ __launch_bounds__(256) void gb_combine_kernel(const T* __restrict__ c,
                                                         const T* __restrict__ r, int64_t n,
                                                         T* __restrict__ lo, T* __restrict__ hi,
                                                         unsigned int* status) {
    unsigned bits = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T l = c[i] - r[i], h = c[i] + r[i];
        lo[i] = l;
        hi[i] = h;
        if (!finiteT(l) || !finiteT(h)) bits |= ST_NONFINITE;
        if (l > h) bits |= ST_ORDER;
    }
    report_status(status, bits);
}

template <int KIND, class T, int E, int MODE>
static hipError_t go_gb(const GbPass& a, int64_t grid, hipStream_t s) {
    hipLaunchKernelGGL((gb_tile_kernel<KIND, T, E, MODE>), dim3((unsigned)grid), dim3(WAVE), 0,
                       s, a);
    return hipGetLastError();
}

template <int KIND, class T, int MODE>
static hipError_t gb_by_E(int E, const GbPass& a, int64_t grid, hipStream_t s) {
    switch (E) {
        case 1: return go_gb<KIND, T, 1, MODE>(a, grid, s);
        case 4: return go_gb<KIND, T, 4, MODE>(a, grid, s);
        case 8: return go_gb<KIND, T, 8, MODE>(a, grid, s);
        case 16: return go_gb<KIND, T, 16, MODE>(a, grid, s);
        case 24: return go_gb<KIND, T, 24, MODE>(a, grid, s);
        case 28: return go_gb<KIND, T, 28, MODE>(a, grid, s);
        case 32: return go_gb<KIND, T, 32, MODE>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

bool gb_has_E(int E) {
    return E == 1 || E == 4 || E == 8 || E == 16 || E == 24 || E == 28 || E == 32;
}

hipError_t launch_gb(int kind, int mode, int dtype, int E, const GbPass& a, int64_t grid,
                     hipStream_t s) {
    if (dtype == 0) {
        if (kind == K_CTM) return gb_by_E<K_CTM, double, IN_SCALAR>(E, a, grid, s);
        if (kind == K_RD) return mode ? gb_by_E<K_RD, double, IN_CELL>(E, a, grid, s)
                                      : gb_by_E<K_RD, double, IN_SCALAR>(E, a, grid, s);
        if (kind == K_LIN3) return mode ? gb_by_E<K_LIN3, double, IN_CELL>(E, a, grid, s)
                                        : gb_by_E<K_LIN3, double, IN_SCALAR>(E, a, grid, s);
    } else {
        if (kind == K_CTM) return gb_by_E<K_CTM, float, IN_SCALAR>(E, a, grid, s);
        if (kind == K_RD) return mode ? gb_by_E<K_RD, float, IN_CELL>(E, a, grid, s)
                                      : gb_by_E<K_RD, float, IN_SCALAR>(E, a, grid, s);
        if (kind == K_LIN3) return mode ? gb_by_E<K_LIN3, float, IN_CELL>(E, a, grid, s)
                                        : gb_by_E<K_LIN3, float, IN_SCALAR>(E, a, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_gb_combine(int dtype, const void* c, const void* r, int64_t n, void* lo,
                             void* hi, unsigned int* status, hipStream_t s) {
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    if (dtype == 0)
        hipLaunchKernelGGL(gb_combine_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const double*)c, (const double*)r, n, (double*)lo, (double*)hi, status);
    else
        hipLaunchKernelGGL(gb_combine_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const float*)c, (const float*)r, n, (float*)lo, (float*)hi, status);
    return hipGetLastError();
}

}  // namespace reach
