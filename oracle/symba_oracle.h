/*
 * Oracle for the SyMBA kick/encounter step (test infrastructure only).
 *
 * A plain, slow, single-threaded FP64 CPU implementation of what the GPU
 * library computes, written from the paper (Lau & Lee, "Parallelization of
 * the Symplectic Massive Body Algorithm (SyMBA) N-body Code"):
 *   - Sec. 2: the pair loop over the right-angled trapezoid
 *     {(i, j): 0 <= i < N_m, i < j < N}, with N_m = N - 1 when every body is
 *     massive; massive bodies interact with all bodies, field particles only
 *     feel the massive ones;
 *   - Sec. 2: the close-encounter check over the same pairs, and the grouping
 *     of encounter pairs into independent groups.
 *
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  It shares no source with the GPU library.  All pointers are
 * host pointers, all arrays are length-N structure-of-arrays, indices are
 * 0-based, G = 1 and the Sun (mass 1) is implicit and excluded from N.
 *
 * Return codes: >= 0 success (a count where documented); -1 invalid argument.
 */
#ifndef SYMBA_ORACLE_H
#define SYMBA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Interaction acceleration over the trapezoid (Sec. 2):
 * a_i += m_j (x_j - x_i)/|x_j - x_i|^3 for massive j, a_j -= m_i (...)/|..|^3.
 * Field particles (index >= N_m when N_m < N - 1) exert no force. */
int oracle_accel(int64_t n, int64_t n_m,
                 const double *x, const double *y, const double *z, const double *m,
                 double *ax, double *ay, double *az);

/* Acceleration of one body k, summed over every massive j != k in increasing j
 * (the same quantity as oracle_accel, computed body by body). */
int oracle_accel_body(int64_t k, int64_t n, int64_t n_m,
                      const double *x, const double *y, const double *z, const double *m,
                      double out[3]);

/* The encounter predicate on one pair (1 = flagged, 0 = not). */
int oracle_encounter(double xi, double yi, double zi, double vxi, double vyi, double vzi, double rhi,
                     double xj, double yj, double zj, double vxj, double vyj, double vzj, double rhj,
                     double dt, double rcrit_factor);

/* The encounter predicate on each listed pair (pair_i[k], pair_j[k]) of a
 * state, body i taken first as in oracle_pairs: flag[k] = 1 if flagged, else
 * 0.  Returns 0, or -1 for invalid arguments or an index outside [0, n). */
int oracle_encounter_list(int64_t n, const double *x, const double *y, const double *z,
                          const double *vx, const double *vy, const double *vz, const double *rh,
                          double dt, double rcrit_factor, int64_t n_pairs,
                          const int32_t *pair_i, const int32_t *pair_j, uint8_t *flag);

/* Flagged pairs of the trapezoid in lexicographic (i, j) order, i < j.
 * Stores at most `cap` pairs; returns the true count (may exceed cap). */
int64_t oracle_pairs(int64_t n, int64_t n_m,
                     const double *x, const double *y, const double *z,
                     const double *vx, const double *vy, const double *vz, const double *rh,
                     double dt, double rcrit_factor,
                     int32_t *pair_i, int32_t *pair_j, int64_t cap);

/* Flagged partners j of one body i (any j != i whose pair is in the trapezoid),
 * in increasing j.  Stores at most `cap`; returns the true count. */
int64_t oracle_partners(int64_t i, int64_t n, int64_t n_m,
                        const double *x, const double *y, const double *z,
                        const double *vx, const double *vy, const double *vz, const double *rh,
                        double dt, double rcrit_factor, int32_t *partner, int64_t cap);

/* Connected components of the graph (V = [0, N), E = pairs) by breadth-first
 * search; group_id[k] = smallest vertex of k's component (k when isolated).
 * Returns the number of components with at least two vertices. */
int64_t oracle_groups(int64_t n, int64_t n_pairs, const int32_t *pair_i, const int32_t *pair_j,
                      int32_t *group_id);

/* Whole step in one trapezoid loop nest: accelerations, flagged pairs (at most
 * `cap` stored), groups.  Returns the true pair count; if it exceeds cap the
 * groups are not computed and *n_groups is set to -1. */
int64_t oracle_kick_encounter(int64_t n, int64_t n_m,
                              const double *x, const double *y, const double *z,
                              const double *vx, const double *vy, const double *vz,
                              const double *m, const double *rh, double dt, double rcrit_factor,
                              double *ax, double *ay, double *az,
                              int32_t *pair_i, int32_t *pair_j, int64_t cap,
                              int32_t *group_id, int64_t *n_groups);

/* Full heliocentric acceleration from the interaction part:
 * a_hel_k = a_k - x_k/|x_k|^3 - sum_{massive j} m_j x_j/|x_j|^3. */
int oracle_helio(int64_t n, int64_t n_m,
                 const double *x, const double *y, const double *z, const double *m,
                 const double *ax, const double *ay, const double *az,
                 double *hx, double *hy, double *hz);

/* All-core build (symba_oracle_omp.c, OpenMP; the benchmark's CPU context):
 * oracle_kick_encounter computed with the paper's Sec. 2 scheme -- rows
 * folded so that every thread gets the same number of pairs, thread-private
 * accumulators summed in thread order.  Pairs and groups equal the
 * single-thread oracle's; accelerations differ by the order of additions.
 * *threads_used = the OpenMP thread count.  Returns as
 * oracle_kick_encounter, or -2 when host memory runs out. */
int64_t oracle_kick_encounter_omp(int64_t n, int64_t n_m,
                                  const double *x, const double *y, const double *z,
                                  const double *vx, const double *vy, const double *vz,
                                  const double *m, const double *rh, double dt, double rcrit_factor,
                                  double *ax, double *ay, double *az,
                                  int32_t *pair_i, int32_t *pair_j, int64_t cap,
                                  int32_t *group_id, int64_t *n_groups, int32_t *threads_used);

#ifdef __cplusplus
}
#endif

#endif
