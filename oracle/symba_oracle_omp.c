/*
 * All-core build of the oracle's kick/encounter step -- TEST INFRASTRUCTURE
 * ONLY (the benchmark's CPU-baseline leg times it for context; the tests
 * check it against the single-thread oracle).  The GPU library never links,
 * loads or calls it.
 *
 * The loop body is the single-thread oracle's, operation for operation; the
 * work is shared out the way the paper's Sec. 2 describes for its OpenMP
 * code:
 *   * the triangle of rows is mapped onto a rectangle: row i is paired with
 *     row rows-1-i, so every folded row holds the same number of pairs and a
 *     static schedule gives every thread the same work;
 *   * each thread accumulates into private acceleration arrays, and the
 *     private arrays are summed into the result in thread order, a fixed
 *     order for a fixed thread count (the paper's alternative to a critical
 *     section around the shared arrays);
 *   * each thread collects its own flagged pairs; they are put in
 *     lexicographic order afterwards, and the groups are formed from them as
 *     in the single-thread oracle.
 * Accelerations therefore differ from the single-thread oracle's only by the
 * order of the additions; pairs and groups are identical.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "symba_oracle.h"

static int64_t rows_of(int64_t n, int64_t n_m) { return n_m < n - 1 ? n_m : n - 1; }
static int64_t massive_of(int64_t n, int64_t n_m) { return n_m >= n - 1 ? n : n_m; }

/* The single-thread oracle's encounter test (the same expression). */
static int encounter_test(double dx, double dy, double dz, double wx, double wy, double wz,
                          double rc_i, double rc_j, double dt)
{
    double rc = rc_i + rc_j;
    double rc2 = rc * rc;
    double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    double v2 = fma(wz, wz, fma(wy, wy, wx * wx));
    double vr = fma(dz, wz, fma(dy, wy, dx * wx));
    if (r2 < rc2)
        return 1;
    double end2 = fma(v2, dt * dt, fma(vr, 2.0 * dt, r2));
    if (end2 < rc2)
        return 1;
    if (vr < 0.0 && -vr < v2 * dt) {
        double cross2 = fma(-vr, vr, r2 * v2);
        if (cross2 < rc2 * v2)
            return 1;
    }
    return 0;
}

typedef struct {
    int32_t *i, *j;
    int64_t n, cap;
} pair_buf;

static int push_pair(pair_buf *b, int64_t i, int64_t j)
{
    if (b->n == b->cap) {
        int64_t cap = b->cap ? 2 * b->cap : 1024;
        int32_t *ni = realloc(b->i, sizeof(int32_t) * cap), *nj = NULL;
        if (!ni)
            return -1;
        b->i = ni;
        nj = realloc(b->j, sizeof(int32_t) * cap);
        if (!nj)
            return -1;
        b->j = nj;
        b->cap = cap;
    }
    b->i[b->n] = (int32_t)i;
    b->j[b->n] = (int32_t)j;
    ++b->n;
    return 0;
}

static int cmp_pair(const void *a, const void *b)
{
    const int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Row i of the trapezoid: the pair loop of the single-thread oracle. */
static int one_row(int64_t i, int64_t n, int64_t nmass,
                   const double *x, const double *y, const double *z,
                   const double *vx, const double *vy, const double *vz,
                   const double *m, const double *rh, double dt, double f,
                   double *ax, double *ay, double *az, pair_buf *pb)
{
    for (int64_t j = i + 1; j < n; ++j) {
        double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
        double r2 = dx * dx + dy * dy + dz * dz;
        double q = 1.0 / (r2 * sqrt(r2));
        if (j < nmass) {
            ax[i] += m[j] * q * dx;
            ay[i] += m[j] * q * dy;
            az[i] += m[j] * q * dz;
        }
        ax[j] -= m[i] * q * dx;
        ay[j] -= m[i] * q * dy;
        az[j] -= m[i] * q * dz;
        if (encounter_test(dx, dy, dz, vx[j] - vx[i], vy[j] - vy[i], vz[j] - vz[i], f * rh[i], f * rh[j], dt) &&
            push_pair(pb, i, j) != 0)
            return -1;
    }
    return 0;
}

int64_t oracle_kick_encounter_omp(int64_t n, int64_t n_m,
                                  const double *x, const double *y, const double *z,
                                  const double *vx, const double *vy, const double *vz,
                                  const double *m, const double *rh, double dt, double rcrit_factor,
                                  double *ax, double *ay, double *az,
                                  int32_t *pair_i, int32_t *pair_j, int64_t cap,
                                  int32_t *group_id, int64_t *n_groups, int32_t *threads_used)
{
    if (n < 1 || n_m < 0 || n_m > n || !(dt >= 0.0) || !(rcrit_factor > 0.0) || cap < 0)
        return -1;
    const int64_t rows = rows_of(n, n_m), nmass = massive_of(n, n_m);
    const int64_t folded = (rows + 1) / 2; /* row i with row rows-1-i */
    const int T = omp_get_max_threads();
    double *priv = calloc((size_t)T * 3 * (size_t)n, sizeof(double));
    pair_buf *pbs = calloc((size_t)T, sizeof(pair_buf));
    int failed = 0;
    if (!priv || !pbs) {
        free(priv);
        free(pbs);
        return -2;
    }
#pragma omp parallel num_threads(T) reduction(| : failed)
    {
        const int t = omp_get_thread_num();
        double *px = priv + (size_t)t * 3 * n, *py = px + n, *pz = py + n;
#pragma omp for schedule(static)
        for (int64_t r = 0; r < folded; ++r) {
            failed |= one_row(r, n, nmass, x, y, z, vx, vy, vz, m, rh, dt, rcrit_factor, px, py, pz, &pbs[t]);
            if (rows - 1 - r != r)
                failed |= one_row(rows - 1 - r, n, nmass, x, y, z, vx, vy, vz, m, rh, dt, rcrit_factor, px, py, pz,
                                  &pbs[t]);
        }
    }
    /* private accumulators summed in thread order */
    for (int64_t k = 0; k < n; ++k) {
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int t = 0; t < T; ++t) {
            const double *px = priv + (size_t)t * 3 * n;
            sx += px[k];
            sy += px[n + k];
            sz += px[2 * n + k];
        }
        ax[k] = sx;
        ay[k] = sy;
        az[k] = sz;
    }
    int64_t count = 0;
    for (int t = 0; t < T; ++t)
        count += pbs[t].n;
    int64_t *keys = failed ? NULL : malloc(sizeof(int64_t) * (size_t)(count > 0 ? count : 1));
    if (keys) {
        int64_t c = 0;
        for (int t = 0; t < T; ++t)
            for (int64_t e = 0; e < pbs[t].n; ++e)
                keys[c++] = ((int64_t)pbs[t].i[e] << 32) | (int64_t)(uint32_t)pbs[t].j[e];
        qsort(keys, (size_t)count, sizeof(int64_t), cmp_pair);
        for (int64_t e = 0; e < count && e < cap; ++e) {
            pair_i[e] = (int32_t)(keys[e] >> 32);
            pair_j[e] = (int32_t)(keys[e] & 0xffffffff);
        }
    }
    for (int t = 0; t < T; ++t) {
        free(pbs[t].i);
        free(pbs[t].j);
    }
    free(pbs);
    free(priv);
    if (!keys)
        return -2;
    free(keys);
    if (threads_used)
        *threads_used = T;
    if (count > cap) {
        *n_groups = -1;
        return count;
    }
    *n_groups = oracle_groups(n, count, pair_i, pair_j, group_id);
    return count;
}
