/*
 * FP64 CPU oracle for interval reachability by mixed monotonicity and by
 * Monte Carlo sampling.  TEST INFRASTRUCTURE ONLY: it exists so the GPU
 * library can be checked against a plain, slow, obviously correct
 * implementation.  It shares no code with the GPU library; only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark may call it.
 *
 * Paper: Devonport, Khaled, Arcak, Zamani, "PIRK: Scalable Interval
 * Reachability Analysis for High-Dimensional Nonlinear Systems" (arXiv
 * 2001.10635).  Sections followed:
 *   - Sec. 2 (interval reachability problem; interval sets as lower/upper
 *     vector pairs; constant inputs drawn from an interval).
 *   - Sec. 2.1, mixed monotonicity: the embedding system built from a
 *     decomposition function d with d(t,x,p,x,p) = f(t,x,p); integrating it
 *     from (lower, upper) with inputs (lower, upper) gives an over-approximating
 *     box.
 *   - Sec. 2.1, Monte Carlo: iid uniform samples of the initial set (and of the
 *     input set) integrated forward; elementwise min / max of the final states;
 *     sample count m >= (2n/eps) log(2n/delta).
 *   - Sec. 3.1, Algorithm 1: state-parallel classical RK4 with four parallel
 *     sections per step and a barrier after each (here: one OpenMP parallel
 *     loop per section).  Two misprints of the printed algorithm are read as
 *     the classical method: the fourth stage input is x + h*k3 (not h/2), and
 *     the update carries the factor h (x += h/6 (k1 + 2k2 + 2k3 + k4)).
 *   - Sec. 3.2, Algorithm 3 (mixed monotonicity: one RK4 run on the 2n-state
 *     embedding) and Algorithm 4 (Monte Carlo: m independent RK4 runs, then a
 *     per-dimension min / max).
 *   - Sec. 2.1, contraction / growth bound, and Sec. 3.2, Algorithm 2: the
 *     center of the box follows f at the center input; the half-width follows
 *     the growth dynamics r' = C r + [p], with a contraction matrix C whose
 *     diagonal bounds the Jacobian's diagonal and whose off-diagonal entries
 *     bound the Jacobian's off-diagonal magnitudes; the box is [c - r, c + r].
 *   - Sec. 5.1, the n-link road traffic (cell transmission) chain, and the
 *     3-D heat diffusion case study of Sec. 5.
 *
 * The case-study systems (the paper gives no decomposition functions; these
 * are the tight ones for sign-stable Jacobians):
 *   CTM  (v, w, c, q):  F_i = min(v y_i, w (c - y_{i+1}), q) for i < n-1,
 *        F_{n-1} = min(v y_{n-1}, q) (free outflow), F_{-1} = 0 (zero inflow),
 *        f_i = F_{i-1} - F_i.  Off-diagonal Jacobian entries are >= 0
 *        (cooperative), so d(x, p, xh, ph) = f(x).
 *   RD   (h):  f_i = (y_{i-1} - 2 y_i + y_{i+1}) / h^2 - y_i^3 + u, with
 *        y_{-1} = y_n = 0.  Cooperative and increasing in u, so
 *        d(x, p, xh, ph) = f(x, p).
 *   LIN3 (aL, aD, aR, b):  f_i = aL y_{i-1} + aD y_i + aR y_{i+1} + b u, ghosts
 *        0.  d_i = aD x_i + aL+ x_{i-1} + aL- xh_{i-1} + aR+ x_{i+1}
 *                + aR- xh_{i+1} + b+ p_i + b- ph_i, with a+ = max(a, 0),
 *        a- = min(a, 0).
 *   HEAT3D (nx, ny, nz, alpha, dx):  the heat diffusion case study (Sec. 5):
 *        the heat equation on an nx * ny * nz grid, second differences along
 *        each axis scaled by alpha / dx^2, insulated faces except x = nx - 1,
 *        which touches an outside held at temperature 0.  Linear with
 *        non-negative off-diagonal entries (cooperative), so d = f.  No inputs.
 * Inputs: n_in = 0 (none), 1 (one scalar shared by all cells) or n (per cell).
 *
 * Sub-domains ("windows"): every routine works on cells [g0, g0+len) of an
 * n_total-cell chain.  Boundary conditions are applied only at the chain's true
 * ends; at a cut edge the missing neighbour is taken as 0.  A wrong neighbour
 * can only influence cells within 4 per RK4 step of the cut (one per stage),
 * so cells farther than 4*nsteps from a cut are bitwise those of a run on the
 * whole chain.
 *
 * Precision: FP64 throughout, compiled with -ffp-contract=off (no fused
 * multiply-add), every expression evaluated left to right as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_CTM = 1, OR_RD = 2, OR_LIN3 = 3, OR_HEAT3D = 4, OR_USER = 5 };

/* A caller-supplied decomposition function of a chain (OR_USER):
   d_i(x, p, xh, ph) from the cells i-1, i, i+1 of x and of xh, the inputs
   p_i and ph_i, the system parameters, the global cell index and the chain
   length. */
typedef double (*or_user_fn)(double xm, double x, double xp, double hm, double h, double hp,
                             double u, double uh, const double* prm, long long i, long long n);

/* Threads of the OpenMP loops started from the calling thread (timing only). */
#include <omp.h>
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int or_get_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ RNG --
 * Philox4x64-10 (Salmon et al., SC'11), written from its published
 * definition: two 64x64->128 multiplications per round, 10 rounds, Weyl key
 * schedule.  Used only for the Monte Carlo samples the method draws.
 */
static void or_philox(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    int r;
    for (r = 0; r < 10; ++r) {
        unsigned __int128 a = (unsigned __int128)M0 * x0;
        unsigned __int128 b = (unsigned __int128)M1 * x2;
        uint64_t y0 = (uint64_t)(b >> 64) ^ x1 ^ k0;
        uint64_t y1 = (uint64_t)b;
        uint64_t y2 = (uint64_t)(a >> 64) ^ x3 ^ k1;
        uint64_t y3 = (uint64_t)a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0; k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void or_philox4x64_10(const uint64_t* ctr, const uint64_t* key, uint64_t* out)
{
    or_philox(ctr, key, out);
}

#define OR_MC_STREAM 2

/* Uniform draw U(s, j) for sample s, coordinate j: word j mod 4 of
   Philox(key = (seed, 0), ctr = (j / 4, s, 2, 0)), top `bits` bits (53 or 24)
   as a fraction in [0, 1). */
double or_uniform(uint64_t seed, int64_t s, int64_t j, int bits)
{
    uint64_t key[2] = {seed, 0};
    uint64_t ctr[4] = {(uint64_t)(j / 4), (uint64_t)s, OR_MC_STREAM, 0};
    uint64_t r[4];
    or_philox(ctr, key, r);
    uint64_t w = r[j % 4];
    if (bits == 24) return ldexp((double)(w >> 40), -24);
    return ldexp((double)(w >> 11), -53);
}

/* ------------------------------------------------------------ dynamics -- */

typedef struct {
    int kind;
    const double* prm;
    int64_t n_total, g0, len;
    int64_t n_in;
    /* HEAT3D only: the window is the box of grid cells [org, org + dim) along
       (x, y, z); left zero, it is the whole grid. */
    int64_t org[3], dim[3];
    or_user_fn user;   /* OR_USER only */
} or_sys;

/* Fill in the whole-grid window of a HEAT3D system (no-op for chains). */
static void or_grid_default(or_sys* S)
{
    if (S->kind != OR_HEAT3D || S->dim[0] > 0) return;
    S->org[0] = S->org[1] = S->org[2] = 0;
    S->dim[0] = (int64_t)S->prm[0];
    S->dim[1] = (int64_t)S->prm[1];
    S->dim[2] = (int64_t)S->prm[2];
}

static double or_min2(double a, double b) { return a < b ? a : b; }
static double or_min3(double a, double b, double c) { return or_min2(or_min2(a, b), c); }

/* Input seen by window cell i (global cell g0 + i). */
static double or_input(const or_sys* S, const double* p, int64_t i)
{
    if (S->n_in == 0) return 0.0;
    if (S->n_in == 1) return p[0];
    return p[S->g0 + i];  /* per-cell inputs are indexed globally */
}

/* Neighbour value y_{i+off} (off = -1 or +1) of window cell i, with the
   chain's own boundary value `ghost` past its true ends, and 0 past a cut. */
static double or_nb(const or_sys* S, const double* y, int64_t i, int off, double ghost)
{
    int64_t j = i + off, g = S->g0 + j;
    if (g < 0 || g >= S->n_total) return ghost;
    if (j < 0 || j >= S->len) return 0.0;
    return y[j];
}

/* CTM flux out of window cell i (towards i+1). */
static double or_ctm_flux(const or_sys* S, const double* y, int64_t i)
{
    const double v = S->prm[0], w = S->prm[1], c = S->prm[2], q = S->prm[3];
    int64_t g = S->g0 + i;
    if (g < 0) return 0.0;                           /* zero inflow into cell 0 */
    double yi = (i >= 0) ? y[i] : 0.0;               /* i = -1: cut edge */
    if (g == S->n_total - 1) return or_min2(v * yi, q);  /* free outflow */
    double yn = (i + 1 < S->len) ? y[i + 1] : 0.0;   /* cut edge on the right */
    return or_min3(v * yi, w * (c - yn), q);
}

/* 3-D heat diffusion (Sec. 5, heat diffusion case study): the heat equation
   on a box of nx * ny * nz grid cells of spacing dx, state = the temperature
   of each cell, cell (a, b, c) stored at a + nx (b + ny c).  Each of the six
   directions adds alpha / dx^2 (u_nb - u) (the second difference along each
   axis).  A direction that leaves the grid adds nothing (insulated face),
   except +x at a = nx - 1: that face touches the outside, held at
   temperature 0, and adds alpha / dx^2 (0 - u).  Past a window's cut edge
   the missing neighbour is taken as 0. */
static double or_heat3d_f(const or_sys* S, const double* y, int64_t i)
{
    const int64_t G[3] = {(int64_t)S->prm[0], (int64_t)S->prm[1], (int64_t)S->prm[2]};
    const double alpha = S->prm[3], dx = S->prm[4];
    const int64_t wx = S->dim[0], wy = S->dim[1];
    const int64_t a[3] = {i % wx, (i / wx) % wy, i / (wx * wy)};
    const double u = y[i];
    double sum = 0.0;
    int d, s;
    for (d = 0; d < 3; ++d) {
        for (s = -1; s <= 1; s += 2) {
            int64_t g = S->org[d] + a[d] + s;        /* neighbour's grid coordinate */
            if (g < 0 || g >= G[d]) {
                if (d == 0 && s == 1) sum += 0.0 - u;   /* the face open to the outside */
                continue;                                /* insulated face */
            }
            int64_t b[3] = {a[0], a[1], a[2]};
            b[d] += s;
            double v = (b[d] < 0 || b[d] >= S->dim[d]) ? 0.0
                                                      : y[b[0] + wx * (b[1] + wy * b[2])];
            sum += v - u;
        }
    }
    return alpha / (dx * dx) * sum;
}

static double or_d(const or_sys* S, const double* x, const double* p,
                   const double* xh, const double* ph, int64_t i);

/* f_i(y, p) of the original system at window cell i. */
static double or_f(const or_sys* S, const double* y, const double* p, int64_t i)
{
    if (S->kind == OR_USER) {
        return or_d(S, y, p, y, p, i);   /* a decomposition function equals f on the diagonal */
    } else if (S->kind == OR_HEAT3D) {
        return or_heat3d_f(S, y, i);
    } else if (S->kind == OR_CTM) {
        return or_ctm_flux(S, y, i - 1) - or_ctm_flux(S, y, i);
    } else if (S->kind == OR_RD) {
        const double h = S->prm[0];
        double ym = or_nb(S, y, i, -1, 0.0), yp = or_nb(S, y, i, +1, 0.0), yi = y[i];
        double lap = (ym - 2.0 * yi + yp) / (h * h);
        return lap - yi * yi * yi + or_input(S, p, i);
    } else {
        const double aL = S->prm[0], aD = S->prm[1], aR = S->prm[2], b = S->prm[3];
        double ym = or_nb(S, y, i, -1, 0.0), yp = or_nb(S, y, i, +1, 0.0);
        return aL * ym + aD * y[i] + aR * yp + b * or_input(S, p, i);
    }
}

static double or_pos(double a) { return a > 0.0 ? a : 0.0; }
static double or_neg(double a) { return a < 0.0 ? a : 0.0; }

/* Decomposition function d_i(x, p, xh, ph) at window cell i. */
static double or_d(const or_sys* S, const double* x, const double* p,
                   const double* xh, const double* ph, int64_t i)
{
    if (S->kind == OR_USER) {
        /* neighbours past the chain's ends read as 0 */
        double xm = or_nb(S, x, i, -1, 0.0), xp = or_nb(S, x, i, +1, 0.0);
        double hm = or_nb(S, xh, i, -1, 0.0), hp = or_nb(S, xh, i, +1, 0.0);
        return S->user(xm, x[i], xp, hm, xh[i], hp, or_input(S, p, i), or_input(S, ph, i),
                       S->prm, (long long)(S->g0 + i), (long long)S->n_total);
    }
    if (S->kind == OR_LIN3) {
        const double aL = S->prm[0], aD = S->prm[1], aR = S->prm[2], b = S->prm[3];
        double xm = or_nb(S, x, i, -1, 0.0), xp = or_nb(S, x, i, +1, 0.0);
        double hm = or_nb(S, xh, i, -1, 0.0), hp = or_nb(S, xh, i, +1, 0.0);
        return aD * x[i] + or_pos(aL) * xm + or_neg(aL) * hm + or_pos(aR) * xp
             + or_neg(aR) * hp + or_pos(b) * or_input(S, p, i) + or_neg(b) * or_input(S, ph, i);
    }
    /* CTM, RD and HEAT3D are cooperative: d(x, p, xh, ph) = f(x, p). */
    (void)xh; (void)ph;
    return or_f(S, x, p, i);
}

/* Exposed for tests: out[i] = d_i(x, p, xh, ph) (or f_i(x, p) when use_f). */
void or_rhs(int kind, const double* prm, int64_t n_total, int64_t g0, int64_t len,
            int64_t n_in, const double* x, const double* p, const double* xh,
            const double* ph, int use_f, double* out)
{
    or_sys S = {kind, prm, n_total, g0, len, n_in};
    or_grid_default(&S);
    int64_t i;
    for (i = 0; i < len; ++i)
        out[i] = use_f ? or_f(&S, x, p, i) : or_d(&S, x, p, xh, ph, i);
}

/* ------------------------------------------------------------ embedding --
 * Algorithm 3 with Algorithm 1 as its integrator.  State z = (x, xh) starts
 * at (lower, upper); inputs (p, ph) = (lower, upper).  The embedding vector
 * field is H(z) = (d(x, p, xh, ph), d(xh, ph, x, p)).  For k = 0 .. N-1,
 * t = t0 + k dt (all case-study systems are autonomous, so t is not read):
 *     K1 = H(z)
 *     K2 = H(z + dt/2 K1)
 *     K3 = H(z + dt/2 K2)
 *     K4 = H(z + dt K3)
 *     z  = z + dt/6 (K1 + 2 K2 + 2 K3 + K4)
 * Work arrays k1..k4 and tmp as in Algorithm 1, one parallel loop per section.
 */
static void or_H(const or_sys* S, const double* zx, const double* zh,
                 const double* p, const double* ph, double* kx, double* kh)
{
    int64_t i;
    #pragma omp parallel for schedule(static)
    for (i = 0; i < S->len; ++i) {
        kx[i] = or_d(S, zx, p, zh, ph, i);
        kh[i] = or_d(S, zh, ph, zx, p, i);
    }
}

static void or_axpy(int64_t len, const double* z, double a, const double* k, double* out)
{
    int64_t i;
    #pragma omp parallel for schedule(static)
    for (i = 0; i < len; ++i) out[i] = z[i] + a * k[i];
}

static int or_embed_core(const or_sys* Sp, const double* x_lo, const double* x_hi,
                         const double* p_lo, const double* p_hi, double dt, int64_t nsteps,
                         double* r_lo, double* r_hi)
{
    const or_sys S = *Sp;
    const int64_t len = S.len;
    if (len < 1 || nsteps < 0) return -1;
    const int64_t L = 2 * len;   /* z = [x ; xh] stored back to back */
    double* buf = (double*)malloc(sizeof(double) * (size_t)L * 6);
    if (!buf) return -2;
    double *z = buf, *k1 = buf + L, *k2 = buf + 2 * L, *k3 = buf + 3 * L, *k4 = buf + 4 * L,
           *tmp = buf + 5 * L;
    memcpy(z, x_lo, sizeof(double) * (size_t)len);
    memcpy(z + len, x_hi, sizeof(double) * (size_t)len);
    const double h2 = dt / 2.0, h6 = dt / 6.0;
    int64_t k, i;
    for (k = 0; k < nsteps; ++k) {
        or_H(&S, z, z + len, p_lo, p_hi, k1, k1 + len);          /* section 1 */
        or_axpy(L, z, h2, k1, tmp);
        or_H(&S, tmp, tmp + len, p_lo, p_hi, k2, k2 + len);      /* section 2 */
        or_axpy(L, z, h2, k2, tmp);
        or_H(&S, tmp, tmp + len, p_lo, p_hi, k3, k3 + len);      /* section 3 */
        or_axpy(L, z, dt, k3, tmp);
        or_H(&S, tmp, tmp + len, p_lo, p_hi, k4, k4 + len);      /* section 4 */
        #pragma omp parallel for schedule(static)
        for (i = 0; i < L; ++i)
            z[i] = z[i] + h6 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
    memcpy(r_lo, z, sizeof(double) * (size_t)len);
    memcpy(r_hi, z + len, sizeof(double) * (size_t)len);
    free(buf);
    return 0;
}

int or_embed_rk4(int kind, const double* prm, int64_t n_total, int64_t g0, int64_t len,
                 int64_t n_in, const double* x_lo, const double* x_hi,
                 const double* p_lo, const double* p_hi, double t0, double dt,
                 int64_t nsteps, double* r_lo, double* r_hi)
{
    (void)t0;
    if (kind == OR_HEAT3D && (g0 != 0 || len != n_total)) return -1;  /* use or_embed_rk4_grid */
    or_sys S = {kind, prm, n_total, g0, len, n_in};
    or_grid_default(&S);
    return or_embed_core(&S, x_lo, x_hi, p_lo, p_hi, dt, nsteps, r_lo, r_hi);
}

/* Algorithm 3 for a chain given by a caller-supplied decomposition
   function `d` (window cells [g0, g0+len) of an n_total-cell chain). */
int or_embed_rk4_user(or_user_fn d, const double* prm, int64_t n_total, int64_t g0, int64_t len,
                      int64_t n_in, const double* x_lo, const double* x_hi,
                      const double* p_lo, const double* p_hi, double dt, int64_t nsteps,
                      double* r_lo, double* r_hi)
{
    if (!d) return -1;
    or_sys S = {OR_USER, prm, n_total, g0, len, n_in, {0, 0, 0}, {0, 0, 0}, d};
    return or_embed_core(&S, x_lo, x_hi, p_lo, p_hi, dt, nsteps, r_lo, r_hi);
}

/* Algorithm 3 on the window box [org, org + dim) of a HEAT3D grid (no
   inputs).  Cells farther than 4 * nsteps cells from every cut face of the
   window are bitwise those of a whole-grid run. */
int or_embed_rk4_grid(const double* prm, const int64_t* org, const int64_t* dim,
                      const double* x_lo, const double* x_hi, double dt, int64_t nsteps,
                      double* r_lo, double* r_hi)
{
    const int64_t n = (int64_t)prm[0] * (int64_t)prm[1] * (int64_t)prm[2];
    const int64_t len = dim[0] * dim[1] * dim[2];
    or_sys S = {OR_HEAT3D, prm, n, 0, len, 0, {org[0], org[1], org[2]}, {dim[0], dim[1], dim[2]}};
    int d;
    for (d = 0; d < 3; ++d)
        if (dim[d] < 1 || org[d] < 0 || org[d] + dim[d] > (int64_t)prm[d]) return -1;
    return or_embed_core(&S, x_lo, x_hi, NULL, NULL, dt, nsteps, r_lo, r_hi);
}

/* ----------------------------------------------------------- one trajectory
 * The same classical RK4 on the original system x' = f(x, p) (the integrator
 * Algorithm 4 calls per sample).  Serial over cells; `w` is 6*n doubles of
 * scratch.
 */
static void or_f_all(const or_sys* S, const double* y, const double* p, double* k)
{
    int64_t i;
    for (i = 0; i < S->len; ++i) k[i] = or_f(S, y, p, i);
}

static void or_traj(const or_sys* S, double* z, const double* p, double dt,
                    int64_t nsteps, double* w)
{
    const int64_t n = S->len;
    double *k1 = w, *k2 = w + n, *k3 = w + 2 * n, *k4 = w + 3 * n, *tmp = w + 4 * n;
    const double h2 = dt / 2.0, h6 = dt / 6.0;
    int64_t k, i;
    for (k = 0; k < nsteps; ++k) {
        or_f_all(S, z, p, k1);
        for (i = 0; i < n; ++i) tmp[i] = z[i] + h2 * k1[i];
        or_f_all(S, tmp, p, k2);
        for (i = 0; i < n; ++i) tmp[i] = z[i] + h2 * k2[i];
        or_f_all(S, tmp, p, k3);
        for (i = 0; i < n; ++i) tmp[i] = z[i] + dt * k3[i];
        or_f_all(S, tmp, p, k4);
        for (i = 0; i < n; ++i)
            z[i] = z[i] + h6 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
}

int or_f_rk4(int kind, const double* prm, int64_t n, int64_t n_in, const double* x0,
             const double* p, double t0, double dt, int64_t nsteps, double* out)
{
    (void)t0;
    if (n < 1 || nsteps < 0) return -1;
    or_sys S = {kind, prm, n, 0, n, n_in};
    or_grid_default(&S);
    double* w = (double*)malloc(sizeof(double) * (size_t)n * 5);
    if (!w) return -2;
    memcpy(out, x0, sizeof(double) * (size_t)n);
    or_traj(&S, out, p, dt, nsteps, w);
    free(w);
    return 0;
}

/* One trajectory of x' = f(x, p) = d(x, p, x, p) for a caller-supplied d. */
int or_f_rk4_user(or_user_fn d, const double* prm, int64_t n, int64_t n_in, const double* x0,
                  const double* p, double dt, int64_t nsteps, double* out)
{
    if (!d || n < 1 || nsteps < 0) return -1;
    or_sys S = {OR_USER, prm, n, 0, n, n_in, {0, 0, 0}, {0, 0, 0}, d};
    double* w = (double*)malloc(sizeof(double) * (size_t)n * 5);
    if (!w) return -2;
    memcpy(out, x0, sizeof(double) * (size_t)n);
    or_traj(&S, out, p, dt, nsteps, w);
    free(w);
    return 0;
}

/* ---------------------------------------------------------- Monte Carlo --
 * Algorithm 4 on samples s = s0 .. s0+m-1:
 *     x0_j = x_lo_j + U(s, j) (x_hi_j - x_lo_j)            j < n
 *     p_k  = p_lo_k + U(s, n + k) (p_hi_k - p_lo_k)        k < n_in
 * (inputs are drawn per sample and held constant, as Sec. 2 asks of inputs),
 * then x1 = RK4^N(x0; p) and r_min_j = min_s x1_j, r_max_j = max_s x1_j.
 * The min / max propagate NaN.  `ubits` is 53 (FP64 runs) or 24 (the 24-bit
 * draws an FP32 run uses, so both sides sample the same points).  When
 * `samples` is non-NULL it receives every x1 (m x n, row per sample).
 */
static double or_nmin(double a, double b)
{
    if (a != a) return a;
    if (b != b) return b;
    return b < a ? b : a;
}
static double or_nmax(double a, double b)
{
    if (a != a) return a;
    if (b != b) return b;
    return b > a ? b : a;
}

static int or_montecarlo_core(const or_sys* Sp, const double* x_lo, const double* x_hi,
                              const double* p_lo, const double* p_hi, double dt,
                              int64_t nsteps, int64_t s0, int64_t m, uint64_t seed, int ubits,
                              double* r_min, double* r_max, double* samples)
{
    const or_sys S = *Sp;
    const int64_t n = S.len, n_in = S.n_in;
    if (n < 1 || m < 1 || nsteps < 0 || (n_in != 0 && n_in != 1 && n_in != n)) return -1;
    int64_t j;
    for (j = 0; j < n; ++j) { r_min[j] = INFINITY; r_max[j] = -INFINITY; }
    int failed = 0;
    #pragma omp parallel
    {
        double* z = (double*)malloc(sizeof(double) * (size_t)n * 6);
        double* mn = (double*)malloc(sizeof(double) * (size_t)n * 2);
        double* p = (double*)malloc(sizeof(double) * (size_t)(n_in > 0 ? n_in : 1));
        int ok = (z && mn && p);
        if (!ok) {
            #pragma omp atomic write
            failed = 1;
        }
        double* mx = ok ? mn + n : NULL;
        double* w = ok ? z + n : NULL;
        int64_t i, s;
        if (ok)
            for (i = 0; i < n; ++i) { mn[i] = INFINITY; mx[i] = -INFINITY; }
        #pragma omp for schedule(dynamic, 1)
        for (s = s0; s < s0 + m; ++s) {
            if (!ok) continue;
            for (i = 0; i < n; ++i)
                z[i] = x_lo[i] + or_uniform(seed, s, i, ubits) * (x_hi[i] - x_lo[i]);
            for (i = 0; i < n_in; ++i)
                p[i] = p_lo[i] + or_uniform(seed, s, n + i, ubits) * (p_hi[i] - p_lo[i]);
            or_traj(&S, z, p, dt, nsteps, w);
            for (i = 0; i < n; ++i) {
                mn[i] = or_nmin(mn[i], z[i]);
                mx[i] = or_nmax(mx[i], z[i]);
            }
            if (samples)
                memcpy(samples + (size_t)(s - s0) * (size_t)n, z, sizeof(double) * (size_t)n);
        }
        if (ok) {
            #pragma omp critical
            {
                for (i = 0; i < n; ++i) {
                    r_min[i] = or_nmin(r_min[i], mn[i]);
                    r_max[i] = or_nmax(r_max[i], mx[i]);
                }
            }
        }
        free(z); free(mn); free(p);
    }
    return failed ? -2 : 0;
}

int or_montecarlo(int kind, const double* prm, int64_t n, int64_t n_in,
                  const double* x_lo, const double* x_hi, const double* p_lo,
                  const double* p_hi, double t0, double dt, int64_t nsteps,
                  int64_t s0, int64_t m, uint64_t seed, int ubits,
                  double* r_min, double* r_max, double* samples)
{
    (void)t0;
    or_sys S = {kind, prm, n, 0, n, n_in};
    or_grid_default(&S);
    return or_montecarlo_core(&S, x_lo, x_hi, p_lo, p_hi, dt, nsteps, s0, m, seed, ubits,
                              r_min, r_max, samples);
}

/* Algorithm 4 for a chain given by a caller-supplied decomposition function
   (trajectories of f = d on the diagonal). */
int or_montecarlo_user(or_user_fn d, const double* prm, int64_t n, int64_t n_in,
                       const double* x_lo, const double* x_hi, const double* p_lo,
                       const double* p_hi, double dt, int64_t nsteps, int64_t s0, int64_t m,
                       uint64_t seed, int ubits, double* r_min, double* r_max, double* samples)
{
    if (!d) return -1;
    or_sys S = {OR_USER, prm, n, 0, n, n_in, {0, 0, 0}, {0, 0, 0}, d};
    return or_montecarlo_core(&S, x_lo, x_hi, p_lo, p_hi, dt, nsteps, s0, m, seed, ubits,
                              r_min, r_max, samples);
}

/* ------------------------------------------------------- growth bound --
 * Contraction matrices valid over all states.  HEAT3D is linear with
 * non-negative off-diagonal entries, so its own matrix is one (the radius
 * follows the heat equation too).  For the chains (tridiagonal, as
 * {sub, diag, super}), from their Jacobians:
 *   CTM:  df_i/dy_i = dF_{i-1}/dy_i - dF_i/dy_i lies in {-w-v, -w, -v, 0}, so
 *         C_ii = 0; |df_i/dy_{i-1}| <= v, |df_i/dy_{i+1}| <= w.
 *   RD:   df_i/dy_i = -2/h^2 - 3 y_i^2 <= -2/h^2; off-diagonals 1/h^2.
 *   LIN3: C = (|aL|, aD, |aR|).
 * The input enters additively (RD) or through b (LIN3), so the half-width of
 * the input interval enters r' with the factor |b| (1 for RD).
 */
static void or_contraction(int kind, const double* prm, double C[4])
{
    if (kind == OR_CTM) {
        C[0] = prm[0]; C[1] = 0.0; C[2] = prm[1]; C[3] = 0.0;
    } else if (kind == OR_RD) {
        const double h = prm[0];
        C[0] = 1.0 / (h * h); C[1] = -2.0 / (h * h); C[2] = 1.0 / (h * h); C[3] = 1.0;
    } else {
        C[0] = fabs(prm[0]); C[1] = prm[1]; C[2] = fabs(prm[2]); C[3] = fabs(prm[3]);
    }
}

void or_contraction_matrix(int kind, const double* prm, double* C) { or_contraction(kind, prm, C); }

/* Algorithm 2 on window cells [g0, g0+len) of an n_total-cell chain:
 *   c0 = (lo + hi) / 2, r0 = (hi - lo) / 2         (one parallel loop)
 *   p* = (p_lo + p_hi) / 2, [p] = (p_hi - p_lo) / 2
 *   c1 = RK4^N of x' = f(x, p*) from c0
 *   r1 = RK4^N of r' = C r + |b| [p] from r0 (zero ghosts, as the chain's)
 *   box = [c1 - r1, c1 + r1]
 */
int or_growth_bound(int kind, const double* prm, int64_t n_total, int64_t g0, int64_t len,
                    int64_t n_in, const double* x_lo, const double* x_hi,
                    const double* p_lo, const double* p_hi, double t0, double dt,
                    int64_t nsteps, double* r_lo, double* r_hi)
{
    (void)t0;
    if (len < 1 || nsteps < 0) return -1;
    const int64_t np = n_in > 0 ? n_in : 1;
    double* buf = (double*)malloc(sizeof(double) * ((size_t)len * 7 + 2 * (size_t)np));
    if (!buf) return -2;
    double *c = buf, *r = buf + len, *w = buf + 2 * len;
    double *pc = buf + 7 * len, *pr = pc + np;
    int64_t i;
    #pragma omp parallel for schedule(static)
    for (i = 0; i < len; ++i) {
        c[i] = (x_lo[i] + x_hi[i]) / 2.0;
        r[i] = (x_hi[i] - x_lo[i]) / 2.0;
    }
    for (i = 0; i < np; ++i) {
        pc[i] = n_in > 0 ? (p_lo[i] + p_hi[i]) / 2.0 : 0.0;
        pr[i] = n_in > 0 ? (p_hi[i] - p_lo[i]) / 2.0 : 0.0;
    }
    if (kind == OR_HEAT3D && (g0 != 0 || len != n_total)) { free(buf); return -1; }
    or_sys S = {kind, prm, n_total, g0, len, n_in};
    or_grid_default(&S);
    or_traj(&S, c, pc, dt, nsteps, w);                       /* center run */
    double C[8] = {0};
    or_contraction(kind, prm, C);
    or_sys G = {OR_LIN3, C, n_total, g0, len, n_in};
    if (kind == OR_HEAT3D) G = S;  /* linear and Metzler: C = the system matrix itself */
    or_traj(&G, r, pr, dt, nsteps, w);                       /* radius run */
    #pragma omp parallel for schedule(static)
    for (i = 0; i < len; ++i) {
        r_lo[i] = c[i] - r[i];
        r_hi[i] = c[i] + r[i];
    }
    free(buf);
    return 0;
}

/* Sample count of the Monte Carlo guarantee (Sec. 2.1, Algorithm 4):
   m = ceil((2n/eps) ln(2n/delta)); -1 on arguments outside n >= 1,
   0 < eps < 1, 0 < delta < 1. */
int64_t or_mc_samples(int64_t n, double eps, double delta)
{
    if (n < 1 || !(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 1.0)) return -1;
    double nn = 2.0 * (double)n;
    return (int64_t)ceil((nn / eps) * log(nn / delta));
}
