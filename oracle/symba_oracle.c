/*
 * Oracle for the SyMBA kick/encounter step -- TEST INFRASTRUCTURE ONLY.
 * Only tests, the smoke check and the benchmark's CPU-baseline leg use it;
 * the GPU library never links, loads or calls it.
 *
 * Plain FP64 loops, one thread, written to be read against the paper
 * (Lau & Lee, Sec. 2 and 3).  Build: gcc -O2 -ffp-contract=off -mfma
 * (no -ffast-math): every a*b+c below is two roundings unless it is an
 * explicit fma(), which is one.
 *
 * Readings of the paper used here (it gives the loop structure but no
 * formulas for the force convention or the encounter test):
 *   * force: Newtonian pair force with G = 1, heliocentric positions, the
 *     Sun excluded (its terms belong to the Kepler and Sun drifts);
 *   * encounter test: relative motion of the pair is taken as straight over
 *     the step [0, dt]; the pair is flagged when its separation at the start,
 *     at the end, or at an interior closest approach is below
 *     rc = f*R_H,i + f*R_H,j, evaluated by the fixed sequence of correctly
 *     rounded operations in encounter_test();
 *   * groups: connected components of the flagged-pair graph, labelled by the
 *     smallest body index.
 */
#include "symba_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static int64_t rows_of(int64_t n, int64_t n_m) { return n_m < n - 1 ? n_m : n - 1; }
static int64_t massive_of(int64_t n, int64_t n_m) { return n_m >= n - 1 ? n : n_m; }

static int bad_args(int64_t n, int64_t n_m) { return n < 1 || n_m < 0 || n_m > n; }

/* The encounter test on one pair, from the pair's relative position d and
 * relative velocity w (either orientation gives the same bits: negating both
 * d and w leaves every product below unchanged).
 * Minimum of |d + w t|^2 over t in [0, dt] is below rc^2 iff one of
 *   (1) |d|^2 < rc^2                                   (start of step),
 *   (2) |d + w dt|^2 = |d|^2 + 2 (d.w) dt + |w|^2 dt^2 < rc^2   (end of step),
 *   (3) d.w < 0, t* = -(d.w)/|w|^2 < dt and
 *       |d|^2 |w|^2 - (d.w)^2 < rc^2 |w|^2            (interior closest approach,
 *                                                       multiplied through by |w|^2 > 0). */
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

int oracle_encounter(double xi, double yi, double zi, double vxi, double vyi, double vzi, double rhi,
                     double xj, double yj, double zj, double vxj, double vyj, double vzj, double rhj,
                     double dt, double rcrit_factor)
{
    return encounter_test(xj - xi, yj - yi, zj - zi, vxj - vxi, vyj - vyi, vzj - vzi,
                          rcrit_factor * rhi, rcrit_factor * rhj, dt);
}

int oracle_accel(int64_t n, int64_t n_m,
                 const double *x, const double *y, const double *z, const double *m,
                 double *ax, double *ay, double *az)
{
    if (bad_args(n, n_m))
        return -1;
    int64_t rows = rows_of(n, n_m), nmass = massive_of(n, n_m);
    for (int64_t k = 0; k < n; ++k)
        ax[k] = ay[k] = az[k] = 0.0;
    for (int64_t i = 0; i < rows; ++i) {
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
        }
    }
    return 0;
}

int oracle_accel_body(int64_t k, int64_t n, int64_t n_m,
                      const double *x, const double *y, const double *z, const double *m,
                      double out[3])
{
    if (bad_args(n, n_m) || k < 0 || k >= n)
        return -1;
    int64_t nmass = massive_of(n, n_m);
    double sx = 0.0, sy = 0.0, sz = 0.0;
    if (rows_of(n, n_m) > 0) {
        for (int64_t j = 0; j < nmass; ++j) {
            if (j == k)
                continue;
            double dx = x[j] - x[k], dy = y[j] - y[k], dz = z[j] - z[k];
            double r2 = dx * dx + dy * dy + dz * dz;
            double q = 1.0 / (r2 * sqrt(r2));
            sx += m[j] * q * dx;
            sy += m[j] * q * dy;
            sz += m[j] * q * dz;
        }
    }
    out[0] = sx;
    out[1] = sy;
    out[2] = sz;
    return 0;
}

int64_t oracle_pairs(int64_t n, int64_t n_m,
                     const double *x, const double *y, const double *z,
                     const double *vx, const double *vy, const double *vz, const double *rh,
                     double dt, double rcrit_factor,
                     int32_t *pair_i, int32_t *pair_j, int64_t cap)
{
    if (bad_args(n, n_m) || !(dt >= 0.0) || !(rcrit_factor > 0.0))
        return -1;
    int64_t rows = rows_of(n, n_m), count = 0;
    for (int64_t i = 0; i < rows; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            if (oracle_encounter(x[i], y[i], z[i], vx[i], vy[i], vz[i], rh[i],
                                 x[j], y[j], z[j], vx[j], vy[j], vz[j], rh[j], dt, rcrit_factor)) {
                if (count < cap) {
                    pair_i[count] = (int32_t)i;
                    pair_j[count] = (int32_t)j;
                }
                ++count;
            }
        }
    }
    return count;
}

int oracle_encounter_list(int64_t n, const double *x, const double *y, const double *z,
                          const double *vx, const double *vy, const double *vz, const double *rh,
                          double dt, double rcrit_factor, int64_t n_pairs,
                          const int32_t *pair_i, const int32_t *pair_j, uint8_t *flag)
{
    if (n < 1 || n_pairs < 0 || !(dt >= 0.0) || !(rcrit_factor > 0.0))
        return -1;
    for (int64_t k = 0; k < n_pairs; ++k) {
        int64_t i = pair_i[k], j = pair_j[k];
        if (i < 0 || i >= n || j < 0 || j >= n)
            return -1;
        flag[k] = (uint8_t)oracle_encounter(x[i], y[i], z[i], vx[i], vy[i], vz[i], rh[i],
                                            x[j], y[j], z[j], vx[j], vy[j], vz[j], rh[j], dt, rcrit_factor);
    }
    return 0;
}

int64_t oracle_partners(int64_t i, int64_t n, int64_t n_m,
                        const double *x, const double *y, const double *z,
                        const double *vx, const double *vy, const double *vz, const double *rh,
                        double dt, double rcrit_factor, int32_t *partner, int64_t cap)
{
    if (bad_args(n, n_m) || i < 0 || i >= n || !(dt >= 0.0) || !(rcrit_factor > 0.0))
        return -1;
    int64_t rows = rows_of(n, n_m), count = 0;
    for (int64_t j = 0; j < n; ++j) {
        int64_t lo = j < i ? j : i;
        if (j == i || lo >= rows)
            continue;
        if (oracle_encounter(x[i], y[i], z[i], vx[i], vy[i], vz[i], rh[i],
                             x[j], y[j], z[j], vx[j], vy[j], vz[j], rh[j], dt, rcrit_factor)) {
            if (count < cap)
                partner[count] = (int32_t)j;
            ++count;
        }
    }
    return count;
}

int64_t oracle_groups(int64_t n, int64_t n_pairs, const int32_t *pair_i, const int32_t *pair_j,
                      int32_t *group_id)
{
    if (n < 1 || n_pairs < 0)
        return -1;
    for (int64_t p = 0; p < n_pairs; ++p)
        if (pair_i[p] < 0 || pair_i[p] >= n || pair_j[p] < 0 || pair_j[p] >= n)
            return -1;
    /* adjacency lists in compressed rows */
    int64_t *start = calloc((size_t)n + 1, sizeof *start);
    int32_t *adj = malloc(sizeof *adj * (size_t)(2 * n_pairs + 1));
    int64_t *fill = malloc(sizeof *fill * (size_t)(n + 1));
    int32_t *queue = malloc(sizeof *queue * (size_t)n);
    if (!start || !adj || !fill || !queue) {
        free(start); free(adj); free(fill); free(queue);
        return -1;
    }
    for (int64_t p = 0; p < n_pairs; ++p) {
        start[pair_i[p] + 1]++;
        start[pair_j[p] + 1]++;
    }
    for (int64_t k = 0; k < n; ++k)
        start[k + 1] += start[k];
    memcpy(fill, start, sizeof *fill * (size_t)(n + 1));
    for (int64_t p = 0; p < n_pairs; ++p) {
        adj[fill[pair_i[p]]++] = pair_j[p];
        adj[fill[pair_j[p]]++] = pair_i[p];
    }
    for (int64_t k = 0; k < n; ++k)
        group_id[k] = -1;
    int64_t groups = 0;
    /* visiting seeds in increasing order makes every seed its component's minimum */
    for (int64_t s = 0; s < n; ++s) {
        if (group_id[s] >= 0)
            continue;
        int64_t head = 0, tail = 0;
        queue[tail++] = (int32_t)s;
        group_id[s] = (int32_t)s;
        while (head < tail) {
            int32_t v = queue[head++];
            for (int64_t e = start[v]; e < start[v + 1]; ++e) {
                int32_t u = adj[e];
                if (group_id[u] < 0) {
                    group_id[u] = (int32_t)s;
                    queue[tail++] = u;
                }
            }
        }
        if (tail >= 2)
            ++groups;
    }
    free(start); free(adj); free(fill); free(queue);
    return groups;
}

int64_t oracle_kick_encounter(int64_t n, int64_t n_m,
                              const double *x, const double *y, const double *z,
                              const double *vx, const double *vy, const double *vz,
                              const double *m, const double *rh, double dt, double rcrit_factor,
                              double *ax, double *ay, double *az,
                              int32_t *pair_i, int32_t *pair_j, int64_t cap,
                              int32_t *group_id, int64_t *n_groups)
{
    if (bad_args(n, n_m) || !(dt >= 0.0) || !(rcrit_factor > 0.0) || cap < 0)
        return -1;
    int64_t rows = rows_of(n, n_m), nmass = massive_of(n, n_m), count = 0;
    for (int64_t k = 0; k < n; ++k)
        ax[k] = ay[k] = az[k] = 0.0;
    for (int64_t i = 0; i < rows; ++i) {
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
            if (encounter_test(dx, dy, dz, vx[j] - vx[i], vy[j] - vy[i], vz[j] - vz[i],
                               rcrit_factor * rh[i], rcrit_factor * rh[j], dt)) {
                if (count < cap) {
                    pair_i[count] = (int32_t)i;
                    pair_j[count] = (int32_t)j;
                }
                ++count;
            }
        }
    }
    if (count > cap) {
        *n_groups = -1;
        return count;
    }
    *n_groups = oracle_groups(n, count, pair_i, pair_j, group_id);
    return count;
}

int oracle_helio(int64_t n, int64_t n_m,
                 const double *x, const double *y, const double *z, const double *m,
                 const double *ax, const double *ay, const double *az,
                 double *hx, double *hy, double *hz)
{
    if (bad_args(n, n_m))
        return -1;
    int64_t nmass = massive_of(n, n_m);
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int64_t j = 0; j < nmass; ++j) {
        double r2 = x[j] * x[j] + y[j] * y[j] + z[j] * z[j];
        double q = 1.0 / (r2 * sqrt(r2));
        sx += m[j] * q * x[j];
        sy += m[j] * q * y[j];
        sz += m[j] * q * z[j];
    }
    for (int64_t k = 0; k < n; ++k) {
        double r2 = x[k] * x[k] + y[k] * y[k] + z[k] * z[k];
        double q = 1.0 / (r2 * sqrt(r2));
        hx[k] = ax[k] - q * x[k] - sx;
        hy[k] = ay[k] - q * y[k] - sy;
        hz[k] = az[k] - q * z[k] - sz;
    }
    return 0;
}
