/*
 * Seeded synthetic workloads: interval boxes for the cell-transmission (CTM)
 * and reaction-diffusion (RD) chains and the 3-D heat grid.
 *
 * This module only generates inputs.  It holds none of the reachability
 * arithmetic (no dynamics, no decomposition function, no integrator), so both
 * the FP64 oracle and the GPU library can be fed from it.
 *
 * Random source: Philox4x64-10, the counter-based generator of Salmon, Moraes,
 * Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11),
 * written here from that published definition.  One 64-bit word of output
 * becomes a uniform double on [0, 1) by keeping its top 53 bits.
 *
 *   U_stream(i) = (Philox(key = (seed, 0),
 *                         ctr = (floor(i/4), 0, stream, 0))[i mod 4] >> 11) * 2^-53
 *
 * Box recipes (all in FP64, each product and sum rounded separately, no fused
 * multiply-add, so any other implementation of the same recipe is bitwise
 * equal; FP32 boxes are the FP64 boxes rounded to nearest):
 *   CTM_RANDW  : lo = a + a*U0(i),          hi = lo + d*U1(i)
 *   CTM_FIXEDW : lo = a + a*U0(i),          hi = lo + d
 *   SIN        : s  = sin(pi*(i+1)/(n+1)),  w = wmax*U1(i),
 *                lo = s - 0.5*w,            hi = s + 0.5*w
 *   HEAT_CORNER: a grid of nx * ny * nz cells, cell i = a + nx (b + ny c);
 *                the corner block a < f nx, b < f ny, c < f nz is heated:
 *                lo = T - hw*U0(i), hi = T + hw*U1(i); elsewhere
 *                lo = 0, hi = cw*U1(i).   prm = {nx, ny, nz, f, T, hw, cw}
 * The sine profile is the first Dirichlet eigenmode of the chain; sin is the
 * host libm routine and is only ever evaluated here.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <string.h>

#define WL_PI 3.14159265358979323846
#define WL_M0 0xD2E7470EE14C6C93ULL
#define WL_M1 0xCA5A826395121157ULL
#define WL_W0 0x9E3779B97F4A7C15ULL
#define WL_W1 0xBB67AE8584CAA73BULL

void wl_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        unsigned __int128 p0 = (unsigned __int128)WL_M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)WL_M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        x0 = hi1 ^ x1 ^ k0;
        x1 = lo1;
        x2 = hi0 ^ x3 ^ k1;
        x3 = lo0;
        k0 += WL_W0;
        k1 += WL_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Raw 64-bit words of stream `stream` at indices [i0, i0+count). */
void wl_raw(uint64_t seed, uint64_t stream, int64_t i0, int64_t count, uint64_t* out)
{
    const uint64_t key[2] = {seed, 0};
    #pragma omp parallel for schedule(static)
    for (int64_t b = (i0 >> 2); b <= ((i0 + count - 1) >> 2); ++b) {
        uint64_t ctr[4] = {(uint64_t)b, 0, stream, 0}, r[4];
        wl_philox4x64_10(ctr, key, r);
        for (int w = 0; w < 4; ++w) {
            int64_t i = b * 4 + w;
            if (i >= i0 && i < i0 + count) out[i - i0] = r[w];
        }
    }
}

static inline double wl_u53(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

void wl_uniform(uint64_t seed, uint64_t stream, int64_t i0, int64_t count, double* out)
{
    const uint64_t key[2] = {seed, 0};
    #pragma omp parallel for schedule(static)
    for (int64_t b = (i0 >> 2); b <= ((i0 + count - 1) >> 2); ++b) {
        uint64_t ctr[4] = {(uint64_t)b, 0, stream, 0}, r[4];
        wl_philox4x64_10(ctr, key, r);
        for (int w = 0; w < 4; ++w) {
            int64_t i = b * 4 + w;
            if (i >= i0 && i < i0 + count) out[i - i0] = wl_u53(r[w]);
        }
    }
}

enum { WL_CTM_RANDW = 0, WL_CTM_FIXEDW = 1, WL_SIN = 2, WL_HEAT_CORNER = 3 };

/* One cell of a box recipe; `u0`, `u1` are the stream-0 and stream-1 draws. */
static inline void wl_cell(int recipe, const double* prm, int64_t n, int64_t i,
                           double u0, double u1, double* lo, double* hi)
{
    /* Each line below is one rounded IEEE operation; volatile stops the
       compiler from contracting a*b+c into a fused multiply-add. */
    volatile double t;
    if (recipe == WL_CTM_RANDW || recipe == WL_CTM_FIXEDW) {
        const double a = prm[0], d = prm[1];
        t = a * u0;
        double l = a + t;
        double w;
        if (recipe == WL_CTM_RANDW) { t = d * u1; w = t; } else { w = d; }
        *lo = l;
        *hi = l + w;
    } else if (recipe == WL_HEAT_CORNER) {
        const int64_t nx = (int64_t)prm[0], ny = (int64_t)prm[1];
        const int64_t a = i % nx, b = (i / nx) % ny, c = i / (nx * ny);
        const double f = prm[3], T = prm[4], hw = prm[5], cw = prm[6];
        t = f * prm[0];
        const int in_x = (double)a < t;
        t = f * prm[1];
        const int in_y = (double)b < t;
        t = f * prm[2];
        const int in_z = (double)c < t;
        if (in_x && in_y && in_z) {
            t = hw * u0;
            *lo = T - t;
            t = hw * u1;
            *hi = T + t;
        } else {
            *lo = 0.0;
            t = cw * u1;
            *hi = t;
        }
    } else {
        const double wmax = prm[0];
        t = WL_PI * (double)(i + 1);
        double arg = t / (double)(n + 1);
        double s = sin(arg);
        t = wmax * u1;
        double w = t;
        t = 0.5 * w;
        double hw = t;
        *lo = s - hw;
        *hi = s + hw;
    }
}

/*
 * Box cells [i0, i0+count) of an n-cell chain.  out_f32 != 0 writes float
 * arrays (the FP64 values rounded to nearest), else double arrays.
 * Returns 0, or -1 on a bad recipe or range.
 */
int wl_box(int recipe, const double* prm, uint64_t seed, int64_t n,
           int64_t i0, int64_t count, int out_f32, void* lo_out, void* hi_out)
{
    if (recipe < 0 || recipe > 3 || n < 1 || i0 < 0 || count < 0 || i0 + count > n)
        return -1;
    if (count == 0) return 0;
    const uint64_t key[2] = {seed, 0};
    const int64_t b0 = i0 >> 2, b1 = (i0 + count - 1) >> 2;
    #pragma omp parallel for schedule(static)
    for (int64_t b = b0; b <= b1; ++b) {
        uint64_t c0[4] = {(uint64_t)b, 0, 0, 0}, c1[4] = {(uint64_t)b, 0, 1, 0};
        uint64_t r0[4], r1[4];
        wl_philox4x64_10(c0, key, r0);
        wl_philox4x64_10(c1, key, r1);
        for (int w = 0; w < 4; ++w) {
            int64_t i = b * 4 + w;
            if (i < i0 || i >= i0 + count) continue;
            double lo, hi;
            wl_cell(recipe, prm, n, i, wl_u53(r0[w]), wl_u53(r1[w]), &lo, &hi);
            if (out_f32) {
                ((float*)lo_out)[i - i0] = (float)lo;
                ((float*)hi_out)[i - i0] = (float)hi;
            } else {
                ((double*)lo_out)[i - i0] = lo;
                ((double*)hi_out)[i - i0] = hi;
            }
        }
    }
    return 0;
}
