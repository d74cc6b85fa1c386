// 3-D heat diffusion embedding on gfx950 (heat diffusion case study, Sec. 5,
// integrated by the state-parallel RK4 of Algorithm 1; the system is linear
// with non-negative couplings, so the embedding of Algorithm 3 is RK4 of f
// from the lower and from the upper corner).
//
// State: an nx * ny * nz grid, cell (x, y, z) at x + nx (y + ny z).  Per cell
// and stage, k = a (sum of the six neighbours - 6 u), a = alpha / dx^2.
// Faces are insulated (a neighbour past the face equals the cell itself)
// except x = nx - 1, whose outside neighbour is held at temperature 0.
//
// The grid is linear and autonomous, so one classical RK4 step is exactly the
// stability polynomial R(hA) = I + hA + (hA)^2/2 + (hA)^3/6 + (hA)^4/24 applied
// to the state.  Each of the four stencil applications of a step evaluates it
// in nested form, w <- y + (h/j) A w for j = 4, 3, 2, 1 starting from w = y
// (the same polynomial as the four stages with their running sum, one update
// per level and no running sum to carry).
//
// 2.5-D blocking.  A block owns an x-y tile: 64 lanes along x (DPP shifts give
// the x neighbours) by WV waves of P rows along y (rows of one lane are
// registers; the first and last row of each wave go through LDS to the
// waves above and below).  The block streams through z.  The four stencil
// applications of one step form a pipeline of levels: in iteration z the loader brings in
// plane z + 3, level 0 works on plane z-1, level 1 on z-2, level 2 on z-3,
// level 3 on z-4 and writes the new state of that plane.  Each level keeps
// its input for three consecutive planes (the z neighbours).
// One step costs one read and one write of the state per cell; the tile's
// halo (4 cells on each cut face, one per stage) is recomputed, not
// exchanged.
//
// Boundaries without per-cell tests:
//   - y faces: ghost rows load the mirror image of the grid (even
//     reflection, repeated for grids thinner than the halo).  The mirror
//     evolves exactly like the cells it mirrors (same operands, commuted
//     additions), so the insulated face needs nothing more.
//   - x = 0: ghost lanes load the mirror image the same way.
//   - x = nx - 1: the ghost lane at nx (and its mirror at -1 - nx for grids
//     narrower than the halo) loads 0 and is forced to 0 after every stage,
//     in the tiles that hold it.
//   - z faces: when a stage input of plane 0 is made, it is also copied into
//     the ring slot of plane -1; the slot of plane nz receives plane nz - 1
//     (loaded again for the first stage, copied for the others).
#include <algorithm>

#include "dev.hpp"
#include "kernels.hpp"

namespace reach {

constexpr int HEAT_R = 4;   // halo cells per cut face: one per RK4 stage

constexpr int pmod(int a, int m) { return ((a % m) + m) % m; }

template <class T, int P>
struct HeatRegs {
    T t0[6][P];      // loaded planes (level 0 inputs): z-2 .. z in use, z+1 .. z+3 in flight
    T t[3][3][P];    // level 1..3 inputs, three consecutive planes each
    T y2[2][P];      // step-start state handed to level 2, by plane parity
    T y3[2][P];      // step-start state handed to level 3, by plane parity
};

template <class T, int WV>
struct HeatLds {
    T e[4][2][WV][2][WAVE];   // [level input][plane parity][wave][first/last row][lane]
};

template <class T>
struct HeatCtx {
    const T* src;
    T* dst;
    int64_t plane;       // nx * ny
    int nz;
    int lane, w, wm, wp; // wave index and the waves above / below (clamped)
    int xl;              // x index this lane loads (mirror-mapped), valid if xload
    bool xload;          // lane loads a grid cell (else it holds 0)
    bool zlane;          // lane is a zero ghost (outside the open face)
    bool ztile;          // the tile holds a zero ghost lane (uniform)
    bool xout;           // lane's cell is an output of this tile
    T cw[4], m6cw[4];      // a dt / (4 - j) for level j and -6 times it (uniform)
    unsigned bits;
};

template <class T, int P>
struct HeatRows {
    int64_t off[P];      // row offset (y * nx) of each row, mirror-mapped
    bool out[P];         // row is an output row of this tile
};

template <class T, int P, int WV>
__device__ __forceinline__ void heat_load(T (&dst)[P], const HeatCtx<T>& c,
                                          const HeatRows<T, P>& rows, int z) {
    const T* base = c.src + (int64_t)z * c.plane + c.xl;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const T v = base[rows.off[p]];
        dst[p] = c.xload ? v : T(0);
    }
}

template <class T, int P, int WV>
__device__ __forceinline__ void heat_publish(HeatLds<T, WV>& L, int lvl, int par,
                                             const T (&v)[P], const HeatCtx<T>& c) {
    L.e[lvl][par][c.w][0][c.lane] = v[0];
    L.e[lvl][par][c.w][1][c.lane] = v[P - 1];
}

// Rows of the waves above and below, for the inputs every level works
// on in this iteration: read right after the barrier, all at once.
template <class T>
struct HeatEdges {
    T up[4], dn[4];   // last row of the wave above, first row of the wave below
};

template <int PH, class T, int WV>
__device__ __forceinline__ void heat_read_edges(HeatEdges<T>& E, const HeatLds<T, WV>& L,
                                                const HeatCtx<T>& c) {
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const int par = pmod(PH - 1 - l, 2);
        E.up[l] = L.e[l][par][c.wm][1][c.lane];
        E.dn[l] = L.e[l][par][c.wp][0][c.lane];
    }
}

// One stencil application on one plane, folded into the level's update:
// out = y + (h/j) A w = y + c (s - 6 w) with s the sum of the six neighbours
// and c = a h / j, evaluated as fma(c, s, fma(-6 c, w, y)).
template <class T, int P>
__device__ __forceinline__ void heat_apply(T (&out)[P], const T (&cur)[P], const T (&zm)[P],
                                           const T (&zp)[P], T up, T dn, const T (&y)[P],
                                           T cj, T m6cj) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const T u = cur[p];
        const T xm = from_left(u), xp = from_right(u);
        const T ym = (p > 0) ? cur[p - 1] : up;
        const T yp = (p < P - 1) ? cur[p + 1] : dn;
        T s = (xm + xp) + (ym + yp);
        s = s + (zm[p] + zp[p]);
        out[p] = fmaT(cj, s, fmaT(m6cj, u, y[p]));
    }
}

template <class T, int P>
__device__ __forceinline__ void heat_zero_ghost(T (&v)[P], const HeatCtx<T>& c) {
#pragma unroll
    for (int p = 0; p < P; ++p) v[p] = c.zlane ? T(0) : v[p];
}

template <class T, int P>
__device__ __forceinline__ void copy_rows(T (&d)[P], const T (&s)[P]) {
#pragma unroll
    for (int p = 0; p < P; ++p) d[p] = s[p];
}

// Level LV (stencil application LV + 1 of the step) in the iteration with
// z % 6 == PH, working on plane
// q = z - 1 - LV.  Levels run in every iteration: before their first plane
// and after their last one they compute values nobody reads (they land in
// ring slots, pipes and LDS rows that are rewritten before their next use)
// and store nothing.  STEADY: the caller guarantees 0 <= q < nz and no
// mirror copy due, so the uniform tests drop out.
template <int LV, int PH, bool STEADY, bool ZT, class T, int P, int WV>
__device__ __forceinline__ void heat_level(HeatRegs<T, P>& R, HeatLds<T, WV>& L,
                                           const HeatEdges<T>& E, HeatCtx<T>& c,
                                           const HeatRows<T, P>& rows, int z) {
    const int q = z - 1 - LV;
    constexpr int par = pmod(PH - 1 - LV, 2);
    // the level's input w (three planes), and y: the state at the start of
    // the step, plane q.  Levels 0 and 1 read y from the loader ring; plane
    // z-3 has left the ring by level 2 (its slot holds a plane in flight), so
    // level 1 hands it on in y2 and level 2 in y3.
    const T (&cur)[P] = (LV == 0) ? R.t0[pmod(PH - 1, 6)] : R.t[LV - 1][pmod(PH - 1 - LV, 3)];
    const T (&zm)[P] = (LV == 0) ? R.t0[pmod(PH - 2, 6)] : R.t[LV - 1][pmod(PH - 2 - LV, 3)];
    const T (&zp)[P] = (LV == 0) ? R.t0[pmod(PH, 6)] : R.t[LV - 1][pmod(PH - LV, 3)];
    const T (&y)[P] = (LV == 3) ? R.y3[par] : (LV == 2) ? R.y2[par] : R.t0[pmod(PH - 1 - LV, 6)];
    if constexpr (LV < 3) {
        T (&nt)[P] = R.t[LV][pmod(PH - 1 - LV, 3)];
        if constexpr (LV == 1) copy_rows(R.y2[par], y);
        if constexpr (LV == 2) copy_rows(R.y3[par], y);
        heat_apply<T, P>(nt, cur, zm, zp, E.up[LV], E.dn[LV], y, c.cw[LV], c.m6cw[LV]);
        if (ZT) heat_zero_ghost<T, P>(nt, c);
        heat_publish<T, P, WV>(L, LV + 1, par, nt, c);
        if constexpr (!STEADY) {
            // insulated z faces: plane -1 mirrors plane 0, plane nz mirrors nz - 1
            const bool first = (q == 0), past = (q == c.nz);
            T (&before)[P] = R.t[LV][pmod(PH - 2 - LV, 3)];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const T m = before[p];
                before[p] = first ? nt[p] : m;
                nt[p] = past ? m : nt[p];
            }
        }
    } else {
        T* out = c.dst + (int64_t)q * c.plane;
        const bool live = STEADY || (q >= 0 && q < c.nz);
        T nv[P];
        heat_apply<T, P>(nv, cur, zm, zp, E.up[3], E.dn[3], y, c.cw[3], c.m6cw[3]);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const T v = nv[p];
            if (live && rows.out[p] && c.xout) {
                // the new state is not read again in this pass: non-temporal
                __builtin_nontemporal_store(v, &out[rows.off[p] + c.xl]);
                if (!finiteT(v)) c.bits |= ST_NONFINITE;
            }
        }
    }
}

template <int PH, bool STEADY, bool ZT, class T, int P, int WV>
__device__ __forceinline__ void heat_iter(HeatRegs<T, P>& R, HeatLds<T, WV>& L, HeatCtx<T>& c,
                                          const HeatRows<T, P>& rows, int z) {
    __syncthreads();
    // plane z + 3 into the slot of plane z - 3, which no level reads any more
    // (past the last plane this loads plane nz - 1 again: the mirror image the
    // insulated face needs in the slot of plane nz)
    const int zl = STEADY ? z + 3 : (z + 3 < c.nz ? z + 3 : c.nz - 1);
    heat_load<T, P, WV>(R.t0[pmod(PH + 3, 6)], c, rows, zl);
    HeatEdges<T> E;
    heat_read_edges<PH, T, WV>(E, L, c);
    heat_publish<T, P, WV>(L, 0, pmod(PH, 2), R.t0[PH], c);
    heat_level<0, PH, STEADY, ZT>(R, L, E, c, rows, z);
    heat_level<1, PH, STEADY, ZT>(R, L, E, c, rows, z);
    heat_level<2, PH, STEADY, ZT>(R, L, E, c, rows, z);
    heat_level<3, PH, STEADY, ZT>(R, L, E, c, rows, z);
}

// Six iterations, z0 % 6 == 0 (the ring slots repeat with period 6).
template <bool STEADY, bool ZT, class T, int P, int WV>
__device__ __forceinline__ void heat_group(HeatRegs<T, P>& R, HeatLds<T, WV>& L, HeatCtx<T>& c,
                                           const HeatRows<T, P>& rows, int z0) {
    heat_iter<0, STEADY, ZT>(R, L, c, rows, z0);
    heat_iter<1, STEADY, ZT>(R, L, c, rows, z0 + 1);
    heat_iter<2, STEADY, ZT>(R, L, c, rows, z0 + 2);
    heat_iter<3, STEADY, ZT>(R, L, c, rows, z0 + 3);
    heat_iter<4, STEADY, ZT>(R, L, c, rows, z0 + 4);
    heat_iter<5, STEADY, ZT>(R, L, c, rows, z0 + 5);
}

// Whole z sweep, iterations z = 0 .. nz + 3 (rounded up to whole groups:
// the extra iterations compute nothing that is stored).  A first group with
// the boundary tests, steady groups while each of their iterations z has
// 5 <= z and z + 3 < nz, then the rest with the tests again.
template <bool ZT, class T, int P, int WV>
__device__ __forceinline__ void heat_sweep(HeatRegs<T, P>& R, HeatLds<T, WV>& L, HeatCtx<T>& c,
                                           const HeatRows<T, P>& rows) {
    heat_group<false, ZT>(R, L, c, rows, 0);
    int z = 6;
    for (; z + 6 <= c.nz - 3; z += 6) heat_group<true, ZT>(R, L, c, rows, z);
    for (; z < c.nz + 4; z += 6) heat_group<false, ZT>(R, L, c, rows, z);
}

// Even reflection of grid index g into [0, n) (period 2n).
__device__ __forceinline__ int64_t mirror_index(int64_t g, int64_t n) {
    int64_t r = g % (2 * n);
    if (r < 0) r += 2 * n;
    return r < n ? r : 2 * n - 1 - r;
}

template <class T, int P, int WV>
__global__ __launch_bounds__(WAVE * WV) void heat3d_kernel(HeatPass a) {
    __shared__ HeatLds<T, WV> L;
    const int64_t b = blockIdx.x;
    const int64_t g = (b & 7) * (int64_t)a.per_xcd + (b >> 3);
    const int64_t tiles = (int64_t)a.TX * a.TY;
    if (g >= a.sides * tiles) return;
    const int side = (int)(g / tiles);
    const int64_t t = g - side * tiles;
    const int64_t by = t / a.TX, bx = t - by * a.TX;

    HeatCtx<T> c;
    c.src = (const T*)a.src[side];
    c.dst = (T*)a.dst[side];
    c.plane = a.nx * a.ny;
    c.nz = (int)a.nz;
    c.lane = threadIdx.x & (WAVE - 1);
    c.w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    c.wm = c.w > 0 ? c.w - 1 : c.w;
    c.wp = c.w < WV - 1 ? c.w + 1 : c.w;
    const int64_t gx = bx * a.OX - HEAT_R + c.lane;
    int64_t xl = gx;
    c.xload = true;
    if (gx >= a.nx) c.xload = false;                 // open face: outside is 0
    else if (gx < 0) {
        xl = -1 - gx;                                // mirror about the insulated x = 0 face
        if (xl >= a.nx) { c.xload = false; }         // mirror of the zero ghost (thin grids)
    }
    c.xl = (int)(c.xload ? xl : 0);
    c.zlane = (gx == a.nx) || (gx == -1 - a.nx);
    const int64_t x0 = bx * a.OX - HEAT_R;
    c.ztile = (x0 + WAVE > a.nx) || (x0 <= -1 - a.nx);
    c.xout = c.lane >= HEAT_R && c.lane < WAVE - HEAT_R && gx < a.nx;
    // straight from the kernel arguments (no arithmetic: they stay in scalar
    // registers)
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        if constexpr (sizeof(T) == 8) {
            c.cw[l] = a.cw[l];
            c.m6cw[l] = a.m6cw[l];
        } else {
            c.cw[l] = a.cwf[l];
            c.m6cw[l] = a.m6cwf[l];
        }
    }
    c.bits = 0;

    HeatRows<T, P> rows;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int r = c.w * P + p;                   // row within the tile
        const int64_t gy = by * a.OY - HEAT_R + r;
        rows.off[p] = mirror_index(gy, a.ny) * a.nx;
        rows.out[p] = r >= HEAT_R && r < WV * P - HEAT_R && gy < a.ny;
    }

    HeatRegs<T, P> R;
#pragma unroll
    for (int s = 0; s < 6; ++s)
#pragma unroll
        for (int p = 0; p < P; ++p) R.t0[s][p] = T(0);
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int p = 0; p < P; ++p) R.t[l][0][p] = R.t[l][1][p] = R.t[l][2][p] = T(0);
#pragma unroll
    for (int p = 0; p < P; ++p) R.y2[0][p] = R.y2[1][p] = R.y3[0][p] = R.y3[1][p] = T(0);

    // prologue: planes 0, 1 and 2 in flight (past the last plane, the
    // mirror plane nz - 1 again); plane -1 mirrors plane 0
    heat_load<T, P, WV>(R.t0[0], c, rows, 0);
    heat_load<T, P, WV>(R.t0[1], c, rows, c.nz > 1 ? 1 : c.nz - 1);
    heat_load<T, P, WV>(R.t0[2], c, rows, c.nz > 2 ? 2 : c.nz - 1);
    copy_rows(R.t0[5], R.t0[0]);

    if (c.ztile) heat_sweep<true>(R, L, c, rows);
    else heat_sweep<false>(R, L, c, rows);
    report_status(a.status, c.bits);
}

template <class T>
__global__ __launch_bounds__(256) void center_radius_kernel(const T* __restrict__ lo,
                                                            const T* __restrict__ hi, int64_t n,
                                                            T* __restrict__ c, T* __restrict__ r) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T l = lo[i], h = hi[i];
        c[i] = (l + h) / T(2);
        r[i] = (h - l) / T(2);
    }
}

hipError_t launch_center_radius(int dtype, const void* lo, const void* hi, int64_t n, void* c,
                                void* r, hipStream_t s) {
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    if (dtype == 0)
        hipLaunchKernelGGL(center_radius_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const double*)lo, (const double*)hi, n, (double*)c, (double*)r);
    else
        hipLaunchKernelGGL(center_radius_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const float*)lo, (const float*)hi, n, (float*)c, (float*)r);
    return hipGetLastError();
}

template <class T, int P, int WV>
static hipError_t go_heat(const HeatPass& a, int64_t grid, hipStream_t s) {
    hipLaunchKernelGGL((heat3d_kernel<T, P, WV>), dim3((unsigned)grid), dim3(WAVE * WV), 0, s, a);
    return hipGetLastError();
}

// (P, WV) shapes: rows per wave, waves per block.  FP64 keeps the shapes
// whose registers fit in the steady loop (4 x 8, 5 x 8, 3 x 12, 2 x 16).
bool heat_has_shape(int dtype, int P, int WV) {
    if (dtype == 0)
        return (P == 4 && WV == 8) || (P == 2 && WV == 16) || (P == 5 && WV == 8) ||
               (P == 3 && WV == 12);
    return (P == 4 && WV == 8) || (P == 2 && WV == 16) || (P == 8 && WV == 4) ||
           (P == 3 && WV == 12);
}

hipError_t launch_heat3d(int dtype, int P, int WV, const HeatPass& a, int64_t grid,
                         hipStream_t s) {
    if (dtype == 0) {
        if (P == 4 && WV == 8) return go_heat<double, 4, 8>(a, grid, s);
        if (P == 2 && WV == 16) return go_heat<double, 2, 16>(a, grid, s);
        if (P == 5 && WV == 8) return go_heat<double, 5, 8>(a, grid, s);
        if (P == 3 && WV == 12) return go_heat<double, 3, 12>(a, grid, s);
    } else {
        if (P == 4 && WV == 8) return go_heat<float, 4, 8>(a, grid, s);
        if (P == 2 && WV == 16) return go_heat<float, 2, 16>(a, grid, s);
        if (P == 8 && WV == 4) return go_heat<float, 8, 4>(a, grid, s);
        if (P == 3 && WV == 12) return go_heat<float, 3, 12>(a, grid, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace reach
