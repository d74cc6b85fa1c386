// Host-only driver for the batch planner (reach_plan_batch, no device call):
// random query sets, NULL context (so large plans run on host threads); checks
// that every query is scheduled exactly once, that packs keep to 64 lanes and
// the balanced layout of their width, and that a bad query fails the plan.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <random>
#include <algorithm>
#include "reach.h"

static int check(int64_t nq, uint64_t seed, bool plant_bad) {
    std::mt19937_64 g(seed);
    std::vector<reach_query> q((size_t)nq);
    static double dummy[4];
    for (int64_t i = 0; i < nq; ++i) {
        reach_query& x = q[(size_t)i];
        std::memset(&x, 0, sizeof x);
        const bool ctm = g() & 1;
        x.sys.kind = ctm ? REACH_CTM : REACH_RD;
        x.sys.n = 4 + (int64_t)(g() % 509);
        if (g() % 2) x.sys.n = 4 + (int64_t)(g() % 29);      // many short ones
        x.sys.n_in = ctm ? 0 : 1;
        if (ctm) { x.sys.prm[0] = 0.5; x.sys.prm[1] = 1.0 / 6; x.sys.prm[2] = 40; x.sys.prm[3] = 20; }
        else { x.sys.prm[0] = 1.0; }
        if (g() % 4 == 0) x.sys.prm[0] += 0.25 * (double)(g() % 20);   // several classes
        x.dtype = REACH_F64;
        x.x_lo = x.x_hi = x.r_lo = x.r_hi = dummy;
        x.p_lo = x.p_hi = dummy;
        x.dt = (g() % 3) ? 0.01 : 0.1;
        x.nsteps = 10 + (int64_t)(g() % 991);
        if (g() % 50 == 0) x.nsteps = 0;
    }
    if (plant_bad && nq > 3) q[(size_t)(nq * 2 / 3)].dt = -1.0;
    std::vector<int64_t> start((size_t)nq), member((size_t)nq);
    std::vector<int32_t> count((size_t)nq), width((size_t)nq);
    int64_t ni = -1;
    const reach_status st = reach_plan_batch(nullptr, q.data(), nq, start.data(), count.data(),
                                             width.data(), member.data(), &ni);
    if (plant_bad && nq > 3) {
        if (st == REACH_OK) { std::printf("FAIL: bad query accepted\n"); return 1; }
        return 0;
    }
    if (st != REACH_OK) { std::printf("FAIL: status %d\n", (int)st); return 1; }
    std::vector<int> seen((size_t)nq, 0);
    int64_t covered = 0;
    for (int64_t k = 0; k < ni; ++k) {
        const int32_t E = width[(size_t)k];
        if (count[(size_t)k] < 1 || count[(size_t)k] > 64 || (E == 0 && count[(size_t)k] != 1) ||
            (E != 0 && E != 2 && E != 4 && E != 8 && E != 16)) { std::printf("FAIL: count/width\n"); return 1; }
        int64_t lanes = 0;
        for (int32_t j = 0; j < count[(size_t)k]; ++j) {
            const int64_t p = start[(size_t)k] + j;
            if (p < 0 || p >= nq) { std::printf("FAIL: start\n"); return 1; }
            const int64_t m = member[(size_t)p];
            if (m < 0 || m >= nq) { std::printf("FAIL: member\n"); return 1; }
            ++seen[(size_t)m];
            if (E) {
                const int64_t n = q[(size_t)m].sys.n, L = (n + E - 1) / E;
                if (n < (int64_t)(E - 1) * L) { std::printf("FAIL: layout\n"); return 1; }
                lanes += L;
            }
        }
        if (lanes > 64) { std::printf("FAIL: pack lanes\n"); return 1; }
        covered += count[(size_t)k];
    }
    if (covered != nq) { std::printf("FAIL: covered %lld of %lld\n", (long long)covered, (long long)nq); return 1; }
    for (int64_t i = 0; i < nq; ++i)
        if (seen[(size_t)i] != 1) { std::printf("FAIL: query %lld seen %d\n", (long long)i, seen[(size_t)i]); return 1; }
    std::printf("nq=%lld items=%lld ok\n", (long long)nq, (long long)ni);
    return 0;
}

int main() {
    int bad = 0;
    for (int64_t nq : {1, 2, 100, 16383, 16384, 20000, 100000, 250000})
        for (uint64_t s : {1u, 2u}) {
            bad |= check(nq, s, false);
            bad |= check(nq, s + 10, true);
        }
    std::printf(bad ? "FAILED\n" : "ALL OK\n");
    return bad;
}
