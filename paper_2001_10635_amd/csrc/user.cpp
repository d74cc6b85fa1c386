// User-defined chain systems: a decomposition function given as source text,
// compiled at run time with hipRTC for the context's device and run through
// a temporally blocked embedding kernel like the built-in chains'
// (Sec. 2.1: the embedding system exists for any system with a decomposition
// function; PIRK likewise takes the system dynamics as a C function).
//
// The program handed to hipRTC is
//   - the user text twice, inside namespaces reach_user_f64 / reach_user_f32
//     with `real` = double / float (so one text serves both precisions);
//   - the tile kernel below, instantiated for FP64 / FP32 and a few tile
//     widths E, looked up by name expression.
// The kernel is the chain embedding of Algorithm 3 with the classical RK4 of
// Algorithm 1: one wavefront owns 64E consecutive cells of both sides in
// registers, neighbours by DPP lane shifts, K steps per pass with a halo of
// 4K cells per cut edge, cells past the chain's end held at 0.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/reach.h"
#include "kernels.hpp"
#include "rt.hpp"

using namespace reach;

namespace {

// Kernel argument block: one field list, stringized for the device program,
// so host and device agree on the layout by construction.
#define REACH_USER_PASS_FIELDS                                                        \
    const void* src_lo; const void* src_hi; void* dst_lo; void* dst_hi;              \
    const void* p_lo; const void* p_hi;                                              \
    long long n; long long W; long long OUT; long long ksteps;                       \
    int H; int in_mode; int check; int per_xcd;                                      \
    double prm[8]; double h2; double dt; double dt6; unsigned int* status;
#define REACH_STR2(...) #__VA_ARGS__
#define REACH_STR(...) REACH_STR2(__VA_ARGS__)

struct UserPass { REACH_USER_PASS_FIELDS };

#define REACH_USER_MC_FIELDS                                                          \
    const void* x_lo; const void* x_hi; const void* p_lo; const void* p_hi;          \
    void* part_min; void* part_max;                                                  \
    long long n; long long nsteps; long long s0; long long m; long long nw;           \
    unsigned long long seed; int in_mode; int pad;                                   \
    double prm[8]; double h2; double dt; double dt6;

struct UserMcPass { REACH_USER_MC_FIELDS };

// Tile widths (cells per lane); wider tiles of arbitrary user code spill.
constexpr int kUserE[] = {1, 2, 4, 8};
constexpr int kNumE = 4;
constexpr int kNumMcE = 4;

const char* kPrelude = R"(
#define REACH_DEVICE __device__ static inline
)";

const char* kKernel = R"(
namespace reach_rtc {

template <int D> struct Real;
template <> struct Real<0> { typedef double T; };
template <> struct Real<1> { typedef float T; };

// whole-wave lane shifts; lanes past the wave's ends receive 0.  The empty
// asm keeps each shifted value a plain register move: some run-time compiler
// versions otherwise fold the shift into the 64-bit arithmetic that uses it,
// which gfx950 only allows for broadcast patterns.
template <int CTRL> __device__ inline float dpp(float x) {
    int v = __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true);
    asm volatile("" : "+v"(v));
    return __int_as_float(v);
}
template <int CTRL> __device__ inline double dpp(double x) {
    const unsigned long long v = (unsigned long long)__double_as_longlong(x);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, 0xF, 0xF, true);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, 0xF, 0xF, true);
    asm volatile("" : "+v"(lo), "+v"(hi));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <class T> __device__ inline T from_left(T x) { return dpp<0x138>(x); }
template <class T> __device__ inline T from_right(T x) { return dpp<0x130>(x); }

template <int D>
__device__ inline typename Real<D>::T call_d(typename Real<D>::T xm, typename Real<D>::T x,
                                            typename Real<D>::T xp, typename Real<D>::T hm,
                                            typename Real<D>::T h, typename Real<D>::T hp,
                                            typename Real<D>::T u, typename Real<D>::T uh,
                                            const typename Real<D>::T* prm, long long i,
                                            long long n) {
    if constexpr (D == 0) return reach_user_f64::reach_d(xm, x, xp, hm, h, hp, u, uh, prm, i, n);
    else return reach_user_f32::reach_d(xm, x, xp, hm, h, hp, u, uh, prm, i, n);
}

// Inputs seen by a lane: M = 0 one value per side (no input, or a scalar
// input interval), M = 1 one value per cell and side.
template <int D, int E, int M> struct UIn;
template <int D, int E> struct UIn<D, E, 0> {
    typename Real<D>::T v[2];
    __device__ inline typename Real<D>::T at(int s, int) const { return v[s]; }
};
template <int D, int E> struct UIn<D, E, 1> {
    typename Real<D>::T v[2][E];
    __device__ inline typename Real<D>::T at(int s, int e) const { return v[s][e]; }
};

// One tile: load, ksteps classical RK4 steps of both sides of the lane's
// cells, store.  MASKED: the tile runs past cell n-1 and cells past it (ok[e]
// false) are held at the zero ghost (the stage input t after stages 1-3, the
// state y after stage 4); a tile inside the chain skips those selects.  The
// whole tile is one function body per variant: splitting the step loop off
// behind reference parameters costs the compiler ~100 extra registers.
template <int D, int E, int M, bool MASKED>
__device__ inline void tile_run(const UserPass& a, long long w) {
    typedef typename Real<D>::T T;
    const int lane = threadIdx.x;
    const long long span = 64LL * E;
    const long long ts = w * a.OUT;
    const T* src[2] = {(const T*)a.src_lo, (const T*)a.src_hi};
    const T* pin[2] = {(const T*)a.p_lo, (const T*)a.p_hi};
    T y[2][E];
    UIn<D, E, M> u;
    bool ok[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const long long i = ts + (long long)lane * E + e;
        ok[e] = i < a.n;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            y[s][e] = ok[e] ? src[s][i] : T(0);
            if constexpr (M == 1) u.v[s][e] = ok[e] ? pin[s][i] : T(0);
        }
    }
    if constexpr (M == 0) {
#pragma unroll
        for (int s = 0; s < 2; ++s) u.v[s] = a.in_mode == 0 ? T(0) : pin[s][0];
    }
    T prm[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) prm[j] = (T)a.prm[j];
    const T h2 = (T)a.h2, dt = (T)a.dt, dt6 = (T)a.dt6;
    for (long long k = 0; k < a.ksteps; ++k) {
        T acc[2][E], t[2][E];
#pragma unroll
        for (int stage = 1; stage <= 4; ++stage) {
            T in[2][E];
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int e = 0; e < E; ++e) in[s][e] = (stage == 1) ? y[s][e] : t[s][e];
            const T ln0 = from_left(in[0][E - 1]), ln1 = from_left(in[1][E - 1]);
            const T rn0 = from_right(in[0][0]), rn1 = from_right(in[1][0]);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const long long i = ts + (long long)lane * E + e;
                const T xm = e == 0 ? ln0 : in[0][e - 1], xp = e == E - 1 ? rn0 : in[0][e + 1];
                const T hm = e == 0 ? ln1 : in[1][e - 1], hp = e == E - 1 ? rn1 : in[1][e + 1];
                T kk[2];
                kk[0] = call_d<D>(xm, in[0][e], xp, hm, in[1][e], hp, u.at(0, e), u.at(1, e), prm, i, a.n);
                kk[1] = call_d<D>(hm, in[1][e], hp, xm, in[0][e], xp, u.at(1, e), u.at(0, e), prm, i, a.n);
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const T kv = kk[s];
                    if (stage == 1) { acc[s][e] = kv; t[s][e] = __builtin_fma(h2, kv, y[s][e]); }
                    else if (stage == 2) { acc[s][e] = __builtin_fma(T(2), kv, acc[s][e]); t[s][e] = __builtin_fma(h2, kv, y[s][e]); }
                    else if (stage == 3) { acc[s][e] = __builtin_fma(T(2), kv, acc[s][e]); t[s][e] = __builtin_fma(dt, kv, y[s][e]); }
                    else { acc[s][e] = acc[s][e] + kv; y[s][e] = __builtin_fma(dt6, acc[s][e], y[s][e]); }
                    if (MASKED && !ok[e]) {
                        if (stage == 4) y[s][e] = T(0);
                        else t[s][e] = T(0);
                    }
                }
            }
        }
    }
    const bool reaches_end = ts + span >= a.n;
    const int olo = (w == 0) ? 0 : a.H;
    const int ohi = reaches_end ? (int)(a.n - ts) : (int)(span - a.H);
    T* dst[2] = {(T*)a.dst_lo, (T*)a.dst_hi};
    unsigned bits = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int el = lane * E + e;
        if (el >= olo && el < ohi) {
            dst[0][ts + el] = y[0][e];
            dst[1][ts + el] = y[1][e];
            if (!__builtin_isfinite(y[0][e]) || !__builtin_isfinite(y[1][e])) bits |= 1u;
            if (y[0][e] > y[1][e]) bits |= 2u;
        }
    }
    if (a.check) {
        const unsigned long long nf = __ballot(bits & 1u), od = __ballot(bits & 2u);
        if ((nf | od) && lane == 0) atomicOr(a.status, (nf ? 1u : 0u) | (od ? 2u : 0u));
    }
}

template <int D, int E, int M>
__global__ __launch_bounds__(64) void user_tile(UserPass a) {
    const long long b = blockIdx.x;
    const long long w = (b & 7) * (long long)a.per_xcd + (b >> 3);
    if (w >= a.W) return;
    if (w * a.OUT + 64LL * E <= a.n) tile_run<D, E, M, false>(a, w);
    else tile_run<D, E, M, true>(a, w);
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64 -> 128-bit products with the published multipliers, Weyl key steps.
struct Philox4 { unsigned long long x[4]; };
__device__ inline Philox4 philox(unsigned long long c0, unsigned long long c1,
                                 unsigned long long c2, unsigned long long c3,
                                 unsigned long long k0, unsigned long long k1) {
    for (int r = 0; r < 10; ++r) {
        const unsigned long long lo0 = 0xD2E7470EE14C6C93ULL * c0;
        const unsigned long long hi0 = __umul64hi(0xD2E7470EE14C6C93ULL, c0);
        const unsigned long long lo1 = 0xCA5A826395121157ULL * c2;
        const unsigned long long hi1 = __umul64hi(0xCA5A826395121157ULL, c2);
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    }
    Philox4 r;
    r.x[0] = c0; r.x[1] = c1; r.x[2] = c2; r.x[3] = c3;
    return r;
}
__device__ inline unsigned long long pick(const Philox4& r, long long q) {
    return q == 0 ? r.x[0] : q == 1 ? r.x[1] : q == 2 ? r.x[2] : r.x[3];
}
// Uniform on [0, 1): top 53 bits (FP64 runs) or top 24 bits (FP32 runs).
__device__ inline double unif(unsigned long long r, double) { return (double)(r >> 11) * 0x1.0p-53; }
__device__ inline float unif(unsigned long long r, float) { return (float)(r >> 40) * 0x1.0p-24f; }

template <class T> __device__ inline T nan_min(T m, T x) {
    return (m != m) ? m : ((x < m || x != x) ? x : m);
}
template <class T> __device__ inline T nan_max(T m, T x) {
    return (m != m) ? m : ((x > m || x != x) ? x : m);
}

// Algorithm 4 on the user system: persistent waves, a whole sample per wave
// (cells lane * E + e, n <= 64 E), f = d on the diagonal, each final state
// folded into the wave's min / max partials [w][e][lane].  Sample s draws
// U(s, j) = word j mod 4 of Philox at key (seed, 0), counter
// (floor(j / 4), s, 2, 0): cells at j < n, inputs at j = n + k.  MASKED as
// for the tiles (n < 64 E).
template <int D, int E, int M, bool MASKED>
__device__ inline void mc_run(const UserMcPass& a, long long w) {
    typedef typename Real<D>::T T;
    const int lane = threadIdx.x;
    const long long n = a.n;
    const T* xlo = (const T*)a.x_lo;
    const T* xhi = (const T*)a.x_hi;
    const T* plo = (const T*)a.p_lo;
    const T* phi = (const T*)a.p_hi;
    T* pmin = (T*)a.part_min + (size_t)w * E * 64;
    T* pmax = (T*)a.part_max + (size_t)w * E * 64;
    T prm[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) prm[j] = (T)a.prm[j];
    const T h2 = (T)a.h2, dt = (T)a.dt, dt6 = (T)a.dt6;
    bool ok[E];
#pragma unroll
    for (int e = 0; e < E; ++e) ok[e] = (long long)lane * E + e < n;
    bool first = true;
    for (long long s = a.s0 + w; s < a.s0 + a.m; s += a.nw) {
        T y[E];
        UIn<D, E, M> u;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const long long j = (long long)lane * E + e;
            const Philox4 r = philox((unsigned long long)(j >> 2), (unsigned long long)s, 2ULL, 0ULL,
                                     a.seed, 0ULL);
            const T uu = unif(pick(r, j & 3), T(0));
            y[e] = ok[e] ? __builtin_fma(uu, xhi[j] - xlo[j], xlo[j]) : T(0);
        }
        if constexpr (M == 0) {
            if (a.in_mode == 1) {
                const long long j = n;
                const Philox4 r = philox((unsigned long long)(j >> 2), (unsigned long long)s, 2ULL,
                                         0ULL, a.seed, 0ULL);
                const T uu = unif(pick(r, j & 3), T(0));
                u.v[0] = __builtin_fma(uu, phi[0] - plo[0], plo[0]);
            } else {
                u.v[0] = T(0);
            }
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const long long c = (long long)lane * E + e;
                const long long j = n + c;
                const Philox4 r = philox((unsigned long long)(j >> 2), (unsigned long long)s, 2ULL,
                                         0ULL, a.seed, 0ULL);
                const T uu = unif(pick(r, j & 3), T(0));
                u.v[0][e] = ok[e] ? __builtin_fma(uu, phi[c] - plo[c], plo[c]) : T(0);
            }
        }
        for (long long k = 0; k < a.nsteps; ++k) {
            T acc[E], t[E];
#pragma unroll
            for (int stage = 1; stage <= 4; ++stage) {
                T in[E];
#pragma unroll
                for (int e = 0; e < E; ++e) in[e] = (stage == 1) ? y[e] : t[e];
                const T ln = from_left(in[E - 1]), rn = from_right(in[0]);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const long long i = (long long)lane * E + e;
                    const T xm = e == 0 ? ln : in[e - 1], xp = e == E - 1 ? rn : in[e + 1];
                    const T uu = u.at(0, e);
                    const T kv = call_d<D>(xm, in[e], xp, xm, in[e], xp, uu, uu, prm, i, n);
                    if (stage == 1) { acc[e] = kv; t[e] = __builtin_fma(h2, kv, y[e]); }
                    else if (stage == 2) { acc[e] = __builtin_fma(T(2), kv, acc[e]); t[e] = __builtin_fma(h2, kv, y[e]); }
                    else if (stage == 3) { acc[e] = __builtin_fma(T(2), kv, acc[e]); t[e] = __builtin_fma(dt, kv, y[e]); }
                    else { acc[e] = acc[e] + kv; y[e] = __builtin_fma(dt6, acc[e], y[e]); }
                    if (MASKED && !ok[e]) {
                        if (stage == 4) y[e] = T(0);
                        else t[e] = T(0);
                    }
                }
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const size_t idx = (size_t)e * 64 + lane;
            pmin[idx] = first ? y[e] : nan_min(pmin[idx], y[e]);
            pmax[idx] = first ? y[e] : nan_max(pmax[idx], y[e]);
        }
        first = false;
    }
}

template <int D, int E, int M>
__global__ __launch_bounds__(64) void user_mc(UserMcPass a) {
    if (a.n < 64LL * E) mc_run<D, E, M, true>(a, blockIdx.x);
    else mc_run<D, E, M, false>(a, blockIdx.x);
}

}  // namespace reach_rtc
)";

std::string name_expr(int dtype, int E, int M, bool mc) {
    return std::string(mc ? "reach_rtc::user_mc<" : "reach_rtc::user_tile<") +
           std::to_string(dtype) + ", " + std::to_string(E) + ", " + std::to_string(M) + ">";
}

}  // namespace

struct reach_user {
    int device = 0;
    std::string text;                       // the whole program handed to hipRTC
    std::string arch;                       // --offload-arch=... of the device
    // one module per (precision, input mode), compiled on first use
    hipModule_t mod[2][2] = {};
    hipFunction_t fn[2][2][kNumE] = {};     // embedding tiles [dtype][mode][E]
    hipFunction_t mc[2][2][kNumMcE] = {};   // Monte Carlo samples
};

namespace {

// Compile and load the kernels of one precision d and input mode m.
reach_status compile_set(reach_ctx* c, reach_user* u, int d, int m) {
    if (u->mod[d][m]) return REACH_OK;
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, u->text.c_str(), "reach_user.hip", 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS)
        return rt::set_error(c, REACH_E_NOMEM, "hiprtcCreateProgram failed");
    std::vector<std::string> names;
    for (int e = 0; e < kNumE; ++e) names.push_back(name_expr(d, kUserE[e], m, false));
    for (int e = 0; e < kNumMcE; ++e) names.push_back(name_expr(d, kUserE[e], m, true));
    for (const auto& nm : names) hiprtcAddNameExpression(prog, nm.c_str());
    const char* opts[] = {u->arch.c_str(), "-O3", "-std=c++17", "-ffp-contract=off",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult cr = hiprtcCompileProgram(prog, 8, opts);
    if (cr != HIPRTC_SUCCESS) {
        size_t ln = 0;
        hiprtcGetProgramLogSize(prog, &ln);
        std::string log(ln, '\0');
        if (ln) hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        if (log.size() > 400) log = log.substr(0, 400) + " ...";
        return rt::set_error(c, REACH_E_INVAL, "user source does not compile: " + log);
    }
    size_t code_size = 0;
    hiprtcGetCodeSize(prog, &code_size);
    std::vector<char> code(code_size);
    hiprtcGetCode(prog, code.data());
    std::vector<std::string> lowered;
    for (const auto& nm : names) {
        const char* low = nullptr;
        hiprtcGetLoweredName(prog, nm.c_str(), &low);
        lowered.push_back(low ? low : "");
    }
    hiprtcDestroyProgram(&prog);
    hipModule_t mod = nullptr;
    if (hipSetDevice(u->device) != hipSuccess || hipModuleLoadData(&mod, code.data()) != hipSuccess)
        return rt::set_error(c, REACH_E_DEVICE, "loading the compiled user module failed");
    hipFunction_t f[kNumE + kNumMcE];
    for (size_t q = 0; q < names.size(); ++q) {
        if (hipModuleGetFunction(&f[q], mod, lowered[q].c_str()) != hipSuccess) {
            hipModuleUnload(mod);
            return rt::set_error(c, REACH_E_DEVICE, "user kernel " + names[q] + " not found");
        }
    }
    for (int e = 0; e < kNumE; ++e) u->fn[d][m][e] = f[e];
    for (int e = 0; e < kNumMcE; ++e) u->mc[d][m][e] = f[kNumE + e];
    u->mod[d][m] = mod;
    return REACH_OK;
}

}  // namespace

extern "C" {

reach_status reach_user_create(reach_ctx* c, const char* source, reach_user** out) {
    if (!c || !source || !out) return REACH_E_INVAL;
    *out = nullptr;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, rt::ctx_device(c)) != hipSuccess)
        return rt::set_error(c, REACH_E_DEVICE, "hipGetDeviceProperties failed");
    reach_user* u = new reach_user;
    u->device = rt::ctx_device(c);
    u->arch = std::string("--offload-arch=") + prop.gcnArchName;
    u->arch = u->arch.substr(0, u->arch.find(':'));
    u->text = kPrelude;
    u->text += "struct UserPass { " REACH_STR(REACH_USER_PASS_FIELDS) " };\n";
    u->text += "struct UserMcPass { " REACH_STR(REACH_USER_MC_FIELDS) " };\n";
    u->text += "namespace reach_user_f64 {\ntypedef double real;\n";
    u->text += source;
    u->text += "\n}\nnamespace reach_user_f32 {\ntypedef float real;\n";
    u->text += source;
    u->text += "\n}\n";
    u->text += kKernel;
    // FP64 with no or scalar inputs now (this also rejects text that does not
    // compile); the other precision and per-cell inputs on first use
    const reach_status st = compile_set(c, u, 0, 0);
    if (st != REACH_OK) {
        delete u;
        return st;
    }
    *out = u;
    return REACH_OK;
}

void reach_user_destroy(reach_user* u) {
    if (!u) return;
    hipSetDevice(u->device);
    for (int d = 0; d < 2; ++d)
        for (int m = 0; m < 2; ++m)
            if (u->mod[d][m]) hipModuleUnload(u->mod[d][m]);
    delete u;
}

reach_status reach_embed_rk4_user(reach_ctx* c, reach_user* u, const reach_system* s,
                                  reach_dtype dtype, const void* x_lo, const void* x_hi,
                                  const void* p_lo, const void* p_hi, double t0, double dt,
                                  int64_t nsteps, void* r_lo, void* r_hi, void* ws,
                                  size_t ws_bytes, void* stream) {
    if (!c) return REACH_E_INVAL;
    if (!u) return rt::set_error(c, REACH_E_INVAL, "user system is NULL");
    reach_status st = rt::validate_user(c, s, dtype);
    if (st != REACH_OK) return st;
    if (u->device != rt::ctx_device(c))
        return rt::set_error(c, REACH_E_INVAL, "user system compiled for another device");
    if (!x_lo || !x_hi || !r_lo || !r_hi) return rt::set_error(c, REACH_E_INVAL, "NULL state pointer");
    if (s->n_in > 0 && (!p_lo || !p_hi)) return rt::set_error(c, REACH_E_INVAL, "NULL input pointer");
    if (!(std::isfinite(dt) && dt > 0.0)) return rt::set_error(c, REACH_E_INVAL, "dt must be finite and > 0");
    if (!std::isfinite(t0)) return rt::set_error(c, REACH_E_INVAL, "t0 must be finite");
    if (nsteps < 0) return rt::set_error(c, REACH_E_INVAL, "nsteps < 0");
    if (hipSetDevice(u->device) != hipSuccess) return rt::set_error(c, REACH_E_DEVICE, "hipSetDevice failed");
    hipStream_t hs = (hipStream_t)stream;
    const size_t bytes = (size_t)s->n * (dtype == REACH_F64 ? 8 : 4);
    if (nsteps == 0) {
        if (r_lo != x_lo && hipMemcpyAsync(r_lo, x_lo, bytes, hipMemcpyDeviceToDevice, hs) != hipSuccess)
            return rt::set_error(c, REACH_E_DEVICE, "copy failed");
        if (r_hi != x_hi && hipMemcpyAsync(r_hi, x_hi, bytes, hipMemcpyDeviceToDevice, hs) != hipSuccess)
            return rt::set_error(c, REACH_E_DEVICE, "copy failed");
        return REACH_OK;
    }
    // plan: the smallest tile that holds the chain, else E = 8 with K steps per
    // pass (K = 12 by default: within a few per cent of the best K for a cheap
    // d, whose passes are bandwidth-heavy, and for a transcendental one)
    const int64_t n = s->n;
    const int di = dtype == REACH_F64 ? 0 : 1;
    int E = (int)rt::option(c, "user.E");
    int K = (int)rt::option(c, "user.K");
    int ei = -1;
    if (E) {
        for (int j = 0; j < kNumE; ++j) if (kUserE[j] == E) ei = j;
        if (ei < 0) return rt::set_error(c, REACH_E_INVAL, "user.E must be 1, 2, 4 or 8");
    } else {
        for (int j = 0; j < kNumE && ei < 0; ++j) if ((int64_t)64 * kUserE[j] >= n) ei = j;
        if (ei < 0) ei = kNumE - 1;
        E = kUserE[ei];
    }
    const int64_t span = (int64_t)64 * E;
    UserPass a{};
    int64_t passes;
    if (n <= span && !K) {
        K = (int)std::min<int64_t>(nsteps, 1 << 30);
        a.W = 1; a.OUT = 0; a.H = 0;
        passes = (nsteps + K - 1) / K;
    } else {
        if (!K) K = (int)std::max<int64_t>(1, std::min<int64_t>(12, (span - 1) / 8));
        if ((int64_t)8 * K >= span)
            return rt::set_error(c, REACH_E_INVAL, "user.K too large for the tile width");
        a.H = 4 * K;
        a.OUT = span - 2 * a.H;
        a.W = (n <= span) ? 1 : 1 + (n - span + a.OUT - 1) / a.OUT;
        passes = (nsteps + K - 1) / K;
    }
    const bool alias = (r_lo == x_lo) || (r_hi == x_hi) || (r_lo == x_hi) || (r_hi == x_lo);
    const bool inplace_ok = (a.W == 1);
    const bool need_ws = !inplace_ok && (passes >= 2 || alias);
    void *w_lo = nullptr, *w_hi = nullptr;
    if (need_ws) {
        if (!ws || ws_bytes < 2 * bytes)
            return rt::set_error(c, REACH_E_INVAL, "workspace of " + std::to_string(2 * bytes) +
                                                       " bytes needed");
        w_lo = ws;
        w_hi = (char*)ws + bytes;
    }
    std::vector<std::pair<int, int>> io;
    bool final_copy = false;
    rt::pass_buffers(passes, inplace_ok, alias, &io, &final_copy);
    const void* lo_of[3] = {x_lo, r_lo, w_lo};
    const void* hi_of[3] = {x_hi, r_hi, w_hi};
    a.p_lo = s->n_in ? p_lo : nullptr;
    a.p_hi = s->n_in ? p_hi : nullptr;
    a.in_mode = s->n_in == 0 ? 0 : (s->n_in == 1 ? 1 : 2);
    a.n = n;
    a.per_xcd = (int)((a.W + 7) / 8);
    for (int j = 0; j < 8; ++j) a.prm[j] = s->prm[j];
    a.h2 = dt / 2.0; a.dt = dt; a.dt6 = dt / 6.0;
    a.status = rt::ctx_status(c);
    const int mode = a.in_mode == 2 ? 1 : 0;
    st = compile_set(c, u, di, mode);
    if (st != REACH_OK) return st;
    hipFunction_t fn = u->fn[di][mode][ei];
    const unsigned grid = (unsigned)(8 * (int64_t)a.per_xcd);
    int64_t done = 0;
    for (int64_t p = 0; p < passes; ++p) {
        a.src_lo = lo_of[io[p].first];
        a.src_hi = hi_of[io[p].first];
        a.dst_lo = (void*)lo_of[io[p].second];
        a.dst_hi = (void*)hi_of[io[p].second];
        a.ksteps = std::min<int64_t>(K, nsteps - done);
        a.check = (p == passes - 1) ? 1 : 0;
        void* args[] = {&a};
        if (hipModuleLaunchKernel(fn, grid, 1, 1, 64, 1, 1, 0, hs, args, nullptr) != hipSuccess)
            return rt::set_error(c, REACH_E_DEVICE, "user kernel launch failed");
        done += a.ksteps;
    }
    if (final_copy) {
        if (hipMemcpyAsync(r_lo, w_lo, bytes, hipMemcpyDeviceToDevice, hs) != hipSuccess ||
            hipMemcpyAsync(r_hi, w_hi, bytes, hipMemcpyDeviceToDevice, hs) != hipSuccess)
            return rt::set_error(c, REACH_E_DEVICE, "copy failed");
    }
    return REACH_OK;
}

// Monte Carlo plan: tile width holding the whole chain, resident waves.
static int user_mc_E(int64_t n) {
    for (int j = 0; j < kNumMcE; ++j)
        if ((int64_t)64 * kUserE[j] >= n) return j;
    return -1;
}

static int64_t user_mc_waves(const reach_ctx* c, int64_t m) {
    int64_t w = rt::option(c, "mc.waves");
    if (w <= 0) w = (int64_t)rt::ctx_cus(c) * 8;
    return std::max<int64_t>(1, std::min<int64_t>(std::min(w, kMcMaxWaves), m));
}

size_t reach_user_workspace_bytes(reach_ctx* c, const reach_system* s, reach_dtype dtype,
                                  int64_t m) {
    if (!c || rt::validate_user(c, s, dtype) != REACH_OK || m < 0) return (size_t)-1;
    const size_t el = dtype == REACH_F64 ? 8 : 4;
    if (m == 0) return 2 * (size_t)s->n * el;
    const int ei = user_mc_E(s->n);
    if (ei < 0) return (size_t)-1;
    return 2 * (size_t)user_mc_waves(c, m) * 64 * (size_t)kUserE[ei] * el;
}

reach_status reach_montecarlo_user(reach_ctx* c, reach_user* u, const reach_system* s,
                                   reach_dtype dtype, const void* x_lo, const void* x_hi,
                                   const void* p_lo, const void* p_hi, double t0, double dt,
                                   int64_t nsteps, int64_t s0, int64_t m, uint64_t seed,
                                   void* r_min, void* r_max, void* ws, size_t ws_bytes,
                                   void* stream) {
    if (!c) return REACH_E_INVAL;
    if (!u) return rt::set_error(c, REACH_E_INVAL, "user system is NULL");
    reach_status st = rt::validate_user(c, s, dtype);
    if (st != REACH_OK) return st;
    if (u->device != rt::ctx_device(c))
        return rt::set_error(c, REACH_E_INVAL, "user system compiled for another device");
    if (!x_lo || !x_hi || !r_min || !r_max) return rt::set_error(c, REACH_E_INVAL, "NULL pointer");
    if (s->n_in > 0 && (!p_lo || !p_hi)) return rt::set_error(c, REACH_E_INVAL, "NULL input pointer");
    if (!(std::isfinite(dt) && dt > 0.0)) return rt::set_error(c, REACH_E_INVAL, "dt must be finite and > 0");
    if (!std::isfinite(t0)) return rt::set_error(c, REACH_E_INVAL, "t0 must be finite");
    if (nsteps < 0) return rt::set_error(c, REACH_E_INVAL, "nsteps < 0");
    if (m < 1) return rt::set_error(c, REACH_E_INVAL, "m must be >= 1");
    if (s0 < 0) return rt::set_error(c, REACH_E_INVAL, "s0 must be >= 0");
    const int ei = user_mc_E(s->n);
    if (ei < 0)
        return rt::set_error(c, REACH_E_UNSUPPORTED, "Monte Carlo holds a sample in one wave: n <= 512");
    const size_t need = reach_user_workspace_bytes(c, s, dtype, m);
    if (!ws || ws_bytes < need)
        return rt::set_error(c, REACH_E_INVAL, "workspace of " + std::to_string(need) + " bytes needed");
    if (hipSetDevice(u->device) != hipSuccess) return rt::set_error(c, REACH_E_DEVICE, "hipSetDevice failed");
    hipStream_t hs = (hipStream_t)stream;
    UserMcPass a{};
    a.x_lo = x_lo; a.x_hi = x_hi;
    a.p_lo = s->n_in ? p_lo : nullptr;
    a.p_hi = s->n_in ? p_hi : nullptr;
    a.part_min = ws;
    a.part_max = (char*)ws + need / 2;
    a.n = s->n; a.nsteps = nsteps; a.s0 = s0; a.m = m;
    a.nw = user_mc_waves(c, m);
    a.seed = seed;
    a.in_mode = s->n_in == 0 ? 0 : (s->n_in == 1 ? 1 : 2);
    for (int j = 0; j < 8; ++j) a.prm[j] = s->prm[j];
    a.h2 = dt / 2.0; a.dt = dt; a.dt6 = dt / 6.0;
    const int d = dtype == REACH_F64 ? 0 : 1;
    void* args[] = {&a};
    const int mode = a.in_mode == 2 ? 1 : 0;
    const reach_status cs = compile_set(c, u, d, mode);
    if (cs != REACH_OK) return cs;
    if (hipModuleLaunchKernel(u->mc[d][mode][ei], (unsigned)a.nw, 1, 1, 64, 1, 1, 0, hs, args,
                              nullptr) != hipSuccess)
        return rt::set_error(c, REACH_E_DEVICE, "user Monte Carlo launch failed");
    if (launch_mc_reduce(d, kUserE[ei], a.part_min, a.part_max, a.nw, 1, s->n, r_min, r_max,
                         rt::ctx_status(c), hs) != hipSuccess)
        return rt::set_error(c, REACH_E_DEVICE, "Monte Carlo reduction launch failed");
    return REACH_OK;
}

}  // extern "C"
