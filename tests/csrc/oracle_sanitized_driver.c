/* Drives every function of the C oracle over small seeded inputs and edge
 * cases (one body, no massive body, all massive, a pair list longer than its
 * capacity), for a build with AddressSanitizer and UndefinedBehaviorSanitizer:
 * an out-of-bounds access or undefined operation aborts the run.  Also checks
 * a few facts the functions state of one another (the fused call agrees with
 * the separate ones; the pair-list predicate agrees with the pair list). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/symba_oracle.h"

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;

static double uniform(double lo, double hi) {  /* splitmix64 */
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return lo + (hi - lo) * ((double)(z >> 11) * 0x1p-53);
}

#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            exit(1);                                                     \
        }                                                                \
    } while (0)

static int run(int64_t n, int64_t n_m, double spread, int64_t cap) {
    double *v[14];
    for (int k = 0; k < 14; ++k) v[k] = calloc((size_t)n, sizeof(double));
    double *x = v[0], *y = v[1], *z = v[2], *vx = v[3], *vy = v[4], *vz = v[5], *m = v[6], *rh = v[7];
    double *ax = v[8], *ay = v[9], *az = v[10], *hx = v[11], *hy = v[12], *hz = v[13];
    int64_t nmass = n_m >= n - 1 ? n : n_m;
    for (int64_t k = 0; k < n; ++k) {
        x[k] = uniform(-spread, spread) + 6.0;
        y[k] = uniform(-spread, spread);
        z[k] = uniform(-spread, spread);
        vx[k] = uniform(-0.1, 0.1);
        vy[k] = uniform(-0.1, 0.1);
        vz[k] = uniform(-0.1, 0.1);
        m[k] = k < nmass ? uniform(1e-9, 1e-7) : 0.0;
        rh[k] = k < nmass ? uniform(0.01, 0.2) : 0.0;
    }
    const double dt = 0.7, f = 3.0;
    int32_t *pi = calloc((size_t)(cap > 0 ? cap : 1), sizeof(int32_t));
    int32_t *pj = calloc((size_t)(cap > 0 ? cap : 1), sizeof(int32_t));
    int32_t *gid = calloc((size_t)n, sizeof(int32_t));
    int32_t *partner = calloc((size_t)n, sizeof(int32_t));
    CHECK(oracle_accel(n, n_m, x, y, z, m, ax, ay, az) == 0);
    double one[3];
    CHECK(oracle_accel_body(n - 1, n, n_m, x, y, z, m, one) == 0);
    CHECK(oracle_helio(n, n_m, x, y, z, m, ax, ay, az, hx, hy, hz) == 0);
    int64_t count = oracle_pairs(n, n_m, x, y, z, vx, vy, vz, rh, dt, f, pi, pj, cap);
    CHECK(count >= 0);
    int64_t stored = count < cap ? count : cap;
    for (int64_t k = 0; k < stored; ++k) CHECK(pi[k] < pj[k] && pj[k] < n);
    uint8_t *flag = calloc((size_t)(stored > 0 ? stored : 1), 1);
    CHECK(oracle_encounter_list(n, x, y, z, vx, vy, vz, rh, dt, f, stored, pi, pj, flag) == 0);
    for (int64_t k = 0; k < stored; ++k) CHECK(flag[k] == 1);
    if (count <= cap) {
        int64_t groups = oracle_groups(n, count, pi, pj, gid);
        CHECK(groups >= 0);
        for (int64_t k = 0; k < n; ++k) CHECK(gid[k] >= 0 && gid[k] <= k);
    }
    int64_t np = oracle_partners(0, n, n_m, x, y, z, vx, vy, vz, rh, dt, f, partner, n);
    CHECK(np >= 0 && np < n);
    int64_t ng = 0;
    int64_t fused = oracle_kick_encounter(n, n_m, x, y, z, vx, vy, vz, m, rh, dt, f, hx, hy, hz, pi, pj, cap,
                                          gid, &ng);
    CHECK(fused == count);
    CHECK(count <= cap ? ng >= 0 : ng == -1);
    for (int64_t k = 0; k < n; ++k) CHECK(hx[k] == ax[k] && hy[k] == ay[k] && hz[k] == az[k]);
    /* invalid arguments are refused, not read */
    CHECK(oracle_pairs(n, n + 1, x, y, z, vx, vy, vz, rh, dt, f, pi, pj, cap) == -1);
    int32_t bad_i = (int32_t)n, zero = 0;
    CHECK(oracle_encounter_list(n, x, y, z, vx, vy, vz, rh, dt, f, 1, &bad_i, &zero, flag) == -1);
    free(flag);
    free(pi);
    free(pj);
    free(gid);
    free(partner);
    for (int k = 0; k < 14; ++k) free(v[k]);
    return (int)count;
}

int main(void) {
    static const struct { int64_t n, n_m; double spread; int64_t cap; } cases[] = {
        {1, 0, 1.0, 4}, {1, 1, 1.0, 4},   {2, 1, 0.1, 4},    {3, 0, 0.3, 4},      {17, 16, 0.3, 2},
        {40, 12, 0.5, 1000}, {64, 64, 0.4, 5}, {200, 199, 1.0, 100000}, {300, 30, 0.6, 8}, {257, 256, 0.5, 3},
    };
    for (size_t c = 0; c < sizeof cases / sizeof cases[0]; ++c) {
        int count = run(cases[c].n, cases[c].n_m, cases[c].spread, cases[c].cap);
        printf("n=%lld n_m=%lld pairs=%d\n", (long long)cases[c].n, (long long)cases[c].n_m, count);
    }
    printf("ok\n");
    return 0;
}
