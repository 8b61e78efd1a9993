/*
 * libsymba -- SyMBA's per-step pair-interaction and close-encounter path on
 * AMD Instinct MI355X (gfx950), behind a plain C ABI.
 *
 * The operation (Lau & Lee, "Parallelization of the Symplectic Massive Body
 * Algorithm (SyMBA) N-body Code", Sec. 2):
 *   - every pair of the right-angled trapezoid {(i, j): 0 <= i < R, i < j < N},
 *     R = min(N_m, N - 1), interacts once; massive bodies attract everything,
 *     field particles (indices >= N_m when N_m < N - 1) feel the massive bodies
 *     but attract nothing, and field-field pairs are never formed;
 *   - the same pairs go through the close-encounter check;
 *   - flagged pairs are grouped into independent encounter groups as they are
 *     found (connected components of the flagged-pair graph).
 *
 * Units: G = 1; the Sun (mass 1) is implicit and excluded from N; positions
 * are heliocentric.  Indices are 0-based.
 *
 * Outputs:
 *   acc      the interaction acceleration a_k = sum over massive j != k whose
 *            pair is in the trapezoid of m_j (x_j - x_k)/|x_j - x_k|^3;
 *   pairs    flagged pairs (i < j) in lexicographic order;
 *   group_id the smallest body index in k's encounter group (k if it has none);
 *   n_groups the number of groups with at least two bodies.
 *
 * Encounter test on a pair (the paper names the check but gives no formula;
 * this is the library's reading, evaluated bit-for-bit as written):
 *   d = x_j - x_i, w = v_j - v_i componentwise;  rc_k = f * rh_k;
 *   rc = rc_i + rc_j;  rc2 = rc * rc;
 *   r2 = fma(dz,dz, fma(dy,dy, dx*dx));  v2 likewise from w;
 *   vr = fma(dz,wz, fma(dy,wy, dx*wx));
 *   flagged iff  r2 < rc2
 *            or  fma(v2, dt*dt, fma(vr, 2*dt, r2)) < rc2
 *            or  (vr < 0  and  -vr < v2*dt  and  fma(-vr, vr, r2*v2) < rc2*v2),
 * i.e. the straight relative path over [0, dt] comes within rc at the start,
 * at the end, or at an interior closest approach.  Every operation is a
 * correctly rounded IEEE-754 binary64 operation, so any conforming
 * implementation of the expression reproduces the flags exactly.
 *
 * Thread safety: a context serves one stream at a time.  Calls on different
 * contexts are independent.
 */
#ifndef SYMBA_H
#define SYMBA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return and status codes. */
#define SYMBA_OK 0
#define SYMBA_EINVAL 1     /* null pointer, N < 1, N_m outside [0, N], dt < 0, rcrit_factor <= 0, NaN scalar */
#define SYMBA_ENOMEM 2     /* device allocation failed */
#define SYMBA_EDEVICE 3    /* a HIP runtime call failed */
#define SYMBA_ETOOBIG 4    /* N above the context's max_n */

/* Bits of the device-side status word (symba_out.status). */
#define SYMBA_STATUS_CAPACITY 1   /* more flagged pairs than fit; *n_pairs holds the true count */
#define SYMBA_STATUS_NONFINITE 2  /* an acceleration is Inf or NaN (e.g. coincident bodies) */
#define SYMBA_STATUS_ENC_SKIPPED 4  /* symba_step_enc / symba_enc_prepare: some flagged pairs were not
                                       resolved through the shells (more than SYMBA_ENC_MAX_PAIRS flagged
                                       pairs, a group of more than SYMBA_ENC_MAX_GROUP_PAIRS pairs, or a
                                       pair list that did not fit pair_cap): their bodies took the plain
                                       step's Kepler drift and unweighted forces */

/* Context options (symba_set_option). */
#define SYMBA_OPT_TILE_ROWS 1   /* bodies per lane in triangle tiles: 1, 2 or 4 (0 = automatic) */
#define SYMBA_OPT_FIELD_ROWS 2  /* field bodies per lane in massive x field tiles: 1 or 2 (0 = automatic) */
#define SYMBA_OPT_SCREEN 4      /* pair screen precision: SYMBA_SCREEN_* below.  Both screens are
                                   conservative and every candidate gets the exact FP64 test, so the
                                   pair list, groups and accelerations are the same bits either way */
#define SYMBA_OPT_TIMING 5      /* 1 = record HIP events around the kernels of every call (symba_read_timing) */
#define SYMBA_OPT_BIN 6         /* spatial binning: 0 = by problem size, 1 = never, 2 = always */
#define SYMBA_OPT_ACC 7         /* what symba_kick_encounter(_batch) writes to ax, ay, az: SYMBA_ACC_* below.
                                   symba_step and symba_step_batch ignore it: their kicks and the
                                   accelerations they leave are the interaction term */
#define SYMBA_OPT_SPLIT 8       /* split diagonals of the folded triangle (R = 2 or 4): their block pairs run
                                   as single tile pairs at the end of the tile kernel.  -1 = automatic
                                   (the autotuner's choice, else a rule by launch depth), 0..8 = that many
                                   (clamped to what the fold has) */
#define SYMBA_OPT_ENC_FUSE 9    /* symba_step_enc / symba_enc_prepare on problems of at most 256 bodies:
                                   1 (default) = the work around the evaluation in two fused launches,
                                   0 = the general launches (the same results, bit for bit) */
#define SYMBA_OPT_ENC_REGS 10   /* symba_step_enc, encounter groups of at most 64 bodies and 64 pairs:
                                   1 (default) = integrated through the shells with bodies and pairs in
                                   registers (lane per body, lane per pair), 0 = by the routines for groups of
                                   any size, which keep them in LDS (the same results, bit for bit) */

/* Values of SYMBA_OPT_ACC.  The paper's loop (Sec. 2) sums the pair
 * interactions, the kick term of the democratic heliocentric splitting
 * (Duncan, Levison & Lee 1998, cited in Sec. 1); the Sun's terms belong to
 * the drifts of that splitting and are added here only on request. */
#define SYMBA_ACC_INTERACTION 0  /* the pair interaction sum only (default): what the kick of the
                                    democratic heliocentric map applies */
#define SYMBA_ACC_HELIO 1        /* the full heliocentric acceleration (Sun's mass 1, G = 1):
                                    a_i - x_i / |x_i|^3 - sum_j m_j x_j / |x_j|^3, the sum over
                                    the massive bodies (the Sun's pull and the indirect term of
                                    the accelerated heliocentric frame) */

/* Values of SYMBA_OPT_SCREEN. */
#define SYMBA_SCREEN_AUTO 0  /* the library's choice: the FP32 screen */
#define SYMBA_SCREEN_FP32 1  /* screen data rounded to FP32, margins proven to cover the rounding */
#define SYMBA_SCREEN_FP64 2  /* the FP64 screen */

typedef struct symba_ctx symba_ctx;

/* Input state: N-element device arrays of binary64 (structure of arrays).
 * x, y, z heliocentric positions; vx, vy, vz velocities; m masses (masses of
 * field particles are never read); rh Hill radii (field particles normally 0).
 * Preconditions: every value finite, |positions| < 2^200 and |velocities| <
 * 2^200 (the kernels park padding slots at 2^300). */
typedef struct {
    const double *x, *y, *z;
    const double *vx, *vy, *vz;
    const double *m;
    const double *rh;
} symba_state;

/* Outputs: device pointers, allocated and owned by the caller.
 * ax, ay, az    [N]          interaction accelerations.
 * pair_i/j      [pair_cap]   flagged pairs, lexicographic; written only when
 *                            the count fits both pair_cap and the context's max_pairs.
 * n_pairs       scalar       true number of flagged pairs (even when it does not fit).
 * group_id      [N]          encounter-group label (smallest index in the group).
 * n_groups      scalar       groups with at least two bodies.
 * status        scalar       0 or an OR of SYMBA_STATUS_* bits.
 * The scalars are written by the device; read them after the stream has
 * completed.  With SYMBA_STATUS_CAPACITY set, acc, group_id and n_groups are
 * still valid; only the pair arrays are not written. */
typedef struct {
    double *ax, *ay, *az;
    int32_t *pair_i, *pair_j;
    int64_t pair_cap;
    int64_t *n_pairs;
    int32_t *group_id;
    int32_t *n_groups;
    int32_t *status;
} symba_out;

/* State of symba_step: positions and velocities are updated in place. */
typedef struct {
    double *x, *y, *z;
    double *vx, *vy, *vz;
    const double *m;
    const double *rh;
} symba_mstate;

/* One simulation of a step batch (symba_step_batch). */
typedef struct {
    symba_mstate state;
    int64_t n, n_m;
    double h, rcrit_factor;
    symba_out out;
} symba_step_problem;

/* One independent problem of a batch. */
typedef struct {
    symba_state state;
    int64_t n, n_m;
    double dt, rcrit_factor;
    symba_out out;
} symba_problem;

/* Create a context on HIP device `device` able to take N <= max_n and store up
 * to max_pairs flagged pairs (0 picks max(4*max_n, 4096)).  The context owns
 * its device scratch; flags are reserved (pass 0).  Returns SYMBA_OK and sets
 * *ctx, or an error code and leaves *ctx NULL. */
int symba_ctx_create(symba_ctx **ctx, int device, int64_t max_n, int64_t max_pairs, uint32_t flags);

/* Free the context and its scratch (after all work on it has completed). */
int symba_ctx_destroy(symba_ctx *ctx);

/* Set an option (SYMBA_OPT_*).  Returns SYMBA_EINVAL for an unknown option
 * or value.  SYMBA_OPT_ACC chooses what the accelerations hold; the other
 * options change speed only: pairs, groups and status are unaffected, and the
 * tile sizes change the order in which the accelerations are summed, so
 * their bits (not their tolerance) depend on them. */
int symba_set_option(symba_ctx *ctx, int option, int value);

/* One kick/encounter evaluation (Sec. 2 of the paper): accelerations over the
 * trapezoid, encounter flags over the same pairs, encounter groups.
 * s: device input arrays of length n; n_m: massive-body count (n_m = n - 1
 * and n_m = n both mean "all massive"); dt >= 0 the step; rcrit_factor > 0
 * the critical radius in Hill radii; out: caller-owned device outputs;
 * stream: a hipStream_t (NULL = default stream).  Enqueues the work and
 * returns without waiting; host-checkable faults return an error before
 * anything is enqueued.  Graph capture is allowed (see "Graph capture"
 * below). */
int symba_kick_encounter(symba_ctx *ctx, const symba_state *s, int64_t n, int64_t n_m,
                         double dt, double rcrit_factor, const symba_out *out, void *stream);

/* Many independent problems in one set of launches (the paper's
 * parameter-space scans run many simulations; Sec. 1).  Each problem's
 * outputs are those of symba_kick_encounter on it.  The total of the n's must
 * not exceed the context's max_n and the total pair storage is the context's
 * max_pairs, shared in problem order.  problems: host array of n_problems.
 * Graph capture is allowed (see "Graph capture" below).
 *
 * Graph capture.  symba_kick_encounter, symba_kick_encounter_batch,
 * symba_step and symba_step_batch may be captured into a HIP graph.  A
 * captured call allocates nothing, synchronises nothing and records no memset
 * node; the per-problem descriptors of a captured batch are copied into a
 * capture arena of the context that is only ever appended to, so later calls
 * on the context, captured or not, never change what a graph replays.  The
 * context's partial-sum buffer is never freed while a captured call may use
 * it.  Limits: (1) a captured call that needs a larger partial-sum buffer
 * than the context holds returns SYMBA_EINVAL (run the same problem sizes
 * once outside capture first); (2) the capture arena holds 8 MiB of
 * descriptors (about 13,000 problems over all captured batches of the
 * context's life); a capture beyond it returns SYMBA_ENOMEM; (3) graphs and
 * calls on one context share its scratch, so their executions must not
 * overlap (replay them on the stream the context serves, or order them);
 * (4) symba_autotune, symba_read_timing and symba_read_stats synchronise and
 * must not be captured, and SYMBA_OPT_TIMING records nothing under capture. */
int symba_kick_encounter_batch(symba_ctx *ctx, const symba_problem *problems, int32_t n_problems,
                               void *stream);

/* Kernel time of the calls made since the last read while SYMBA_OPT_TIMING
 * was 1, from HIP events recorded on each call's stream: *tiles_ms sums the
 * tile kernel (pair forces, encounter screen and test, grouping), *finalize_ms
 * the two finalize kernels, *calls the number of calls timed (at most 4096 are
 * kept).  Waits for the recorded events, then starts a new accumulation.
 * Any output pointer may be NULL.  Do not enable timing under graph capture. */
int symba_read_timing(symba_ctx *ctx, double *tiles_ms, double *finalize_ms, int64_t *calls);

/* Static text for a code. */
const char *symba_strerror(int code);

/* symba_kick_encounter for callers that cannot allocate device memory: code
 * under HIP graph capture where allocation is forbidden, tight serving loops,
 * harnesses that forbid hipMalloc.  No context: the scratch is a fixed
 * region of the library's own device memory, SYMBA_NOALLOC_SCRATCH_BYTES per
 * GPU, loaded with the library and held until the process ends.  Limits:
 * n <= SYMBA_NOALLOC_MAX_N (else SYMBA_ETOOBIG, before anything is enqueued)
 * and at most SYMBA_NOALLOC_MAX_PAIRS flagged pairs stored (more set
 * SYMBA_STATUS_CAPACITY, as with a context's max_pairs); the default options
 * (FP32 screen, built-in tile sizes, no binning, the interaction term).
 * Arguments, outputs, errors and asynchrony as symba_kick_encounter; the
 * same plan runs the same kernels, so the outputs are the same bits as a
 * default context's.  Every call on one GPU uses that GPU's one region:
 * calls that overlap on a GPU (two streams, two host threads) race and give
 * wrong results; order them.  The device is the current HIP device. */
#define SYMBA_NOALLOC_MAX_N 8192
#define SYMBA_NOALLOC_MAX_PAIRS 65536
#define SYMBA_NOALLOC_SCRATCH_BYTES 17434880
int symba_kick_encounter_noalloc(const symba_state *s, int64_t n, int64_t n_m, double dt,
                                 double rcrit_factor, const symba_out *out, void *stream);

/* One step of length h of the democratic heliocentric map that SyMBA is
 * built on (the paper's Sec. 1: Duncan, Levison & Lee 1998), outside close
 * encounters: with heliocentric positions, barycentric velocities, G = 1 and
 * the Sun's mass 1,
 *   v += (h/2) a;  x += (h/2) P;  Kepler drift of every body about the Sun
 *   for h;  x += (h/2) P;  a = the evaluation of symba_kick_encounter at the
 *   new positions;  v += (h/2) a,
 * P = sum of m v over the massive bodies (taken before and after the Kepler
 * drift).  Every pair gets its full force: the partition-weighted kick of
 * pairs inside the critical radius and the recursive sub-steps of encounter
 * groups are not part of this step.
 * s: positions and velocities, updated in place; out->ax/ay/az: on entry
 * the accelerations at the current positions (from symba_kick_encounter or
 * the previous step), on return those at the new positions, with the
 * encounter pairs (screened |h| ahead), groups and status of the new state
 * as symba_kick_encounter writes them.  h may be negative (the map is time
 * reversible).  Errors and asynchrony as symba_kick_encounter. */
int symba_step(symba_ctx *ctx, const symba_mstate *s, int64_t n, int64_t n_m, double h,
               double rcrit_factor, const symba_out *out, void *stream);

/* The encounter step: symba_step with the close encounters resolved (the
 * paper's Sec. 2, last paragraph: the encounter groups integrated in
 * parallel, the pairs of a group one after the other; Sec. 3: SyMBA's
 * M = 4 substeps per level, shell radius ratio 2.08, partition function f_l
 * with l = 3, read as the degree-7 polynomial 35x^4 - 84x^5 + 70x^6 - 20x^7).
 * A pair's shells have radii R_0 = rcrit_factor (rh_i + rh_j) and R_k =
 * R_{k-1} / 2.08 (k <= 8); the pair potential is split over the levels by
 * the partition function and every kick applies the exact gradient of its
 * level's part.  The step is
 *   v += (h/2) a0;  x += (h/2) P;  bodies in no flagged pair: Kepler drift
 *   for h; each encounter group: 4 substeps of level 1, where a level-k
 *   substep of length t kicks with the level's forces for t/2, tests its
 *   pairs with radius R_k over t, drifts the bodies of unflagged pairs for t,
 *   takes 4 substeps of level k + 1 for the flagged ones and kicks again;
 *   x += (h/2) P;  evaluation at the new positions (symba_kick_encounter with
 *   dt = |h|);  a0 reweighted to level 0;  v += (h/2) a0,
 * where a0, the level-0 acceleration, weights each pair inside R_0 by the
 * partition function.  The flagged pairs and groups of a step are those on
 * entry in out (written by the previous step or by symba_enc_prepare).
 * One workgroup integrates each group; a step takes at most
 * SYMBA_ENC_MAX_PAIRS flagged pairs and SYMBA_ENC_MAX_GROUP_PAIRS pairs per
 * group (beyond these SYMBA_STATUS_ENC_SKIPPED is set and those bodies take
 * the plain step).  Mergers are not modelled.
 * s: positions and velocities, updated in place.  out on entry: the level-0
 * accelerations, pairs (lexicographic), groups and status of the current
 * state; on return the same for the new state.  h may be negative.  Errors
 * and asynchrony as symba_step; the step makes no host synchronisation, so
 * it may be captured into a graph. */
#define SYMBA_ENC_MAX_PAIRS 8192
#define SYMBA_ENC_MAX_GROUP_PAIRS 255
int symba_step_enc(symba_ctx *ctx, const symba_mstate *s, int64_t n, int64_t n_m, double h,
                   double rcrit_factor, const symba_out *out, void *stream);

/* What symba_step_enc expects in out for state s: the evaluation of
 * symba_kick_encounter (dt = |h|) with the accelerations of flagged pairs
 * inside R_0 reweighted to level 0.  s is not changed.  Errors as
 * symba_step_enc. */
int symba_enc_prepare(symba_ctx *ctx, const symba_mstate *s, int64_t n, int64_t n_m, double h,
                      double rcrit_factor, const symba_out *out, void *stream);

/* symba_step for many independent simulations in one set of launches, each
 * with its own h; every simulation's state and outputs are the same bits as
 * its own symba_step call would give.  Graph capture is allowed (see "Graph
 * capture" above). */
int symba_step_batch(symba_ctx *ctx, const symba_step_problem *steps, int32_t n_problems, void *stream);

/* Host-only helper (no device work): the task list of the folded trapezoid
 * for n, n_m and a tile size of 64*rows bodies, in the order a single call
 * launches them (field tasks first, then the folded triangle's whole block
 * pairs, row by row, then the 64 x 64 tile pairs of the block pairs that are
 * split so that the launch ends with short tasks).  Writes up to cap tasks as
 * (kind, a, b) triples into tasks[3*k..3*k+2] (kind 0: triangle block pair
 * (a, b) in units of 64*rows; kind 1: field block a (64*field_rows field
 * bodies) against segment b of the massive rows, rows [192 b, 192 b + 192);
 * kind 2: triangle tile pair (a, b) in units of 64 bodies) and returns the
 * task count, or -1 on invalid arguments. */
int64_t symba_plan_tasks(int64_t n, int64_t n_m, int32_t rows, int32_t field_rows,
                         int64_t *tasks, int64_t cap);

/* Screen statistics accumulated over the context's calls since the last
 * read: pairs the conservative screen passed to the exact encounter test,
 * pairs the test flagged (the false-positive rate of the screen is
 * 1 - flagged/candidates; it has no false negatives by construction) and
 * problems evaluated.  Waits for the device, then starts a new accumulation.
 * Any output pointer may be NULL. */
int symba_read_stats(symba_ctx *ctx, int64_t *candidates, int64_t *flagged, int64_t *problems);

/* Autotuner of the tile size and the fold schedule: runs the problem
 * (arguments as symba_kick_encounter) with every tile size (64, 128 and 256
 * massive bodies per block row) and, for 128 and 256, with 0 to 3 split
 * diagonals of the folded triangle (SYMBA_OPT_SPLIT), times the calls with
 * HIP events, and keeps the fastest pair in the context for every later
 * problem of the same size class (the same power of two of n_tri = N if
 * N_m >= N - 1, else N_m), in single and batched calls alike, unless
 * SYMBA_OPT_TILE_ROWS or SYMBA_OPT_SPLIT forces a choice.  Results stay
 * within the same tolerance whichever plan runs (pairs and groups are
 * exact); accelerations are bit-reproducible for a given plan.  Writes the
 * outputs of a final call with the chosen plan, *chosen_rows (may be NULL)
 * = bodies per lane (1, 2 or 4); symba_plan_for reports the split.
 * Synchronizes the stream; do not call it under graph capture. */
int symba_autotune(symba_ctx *ctx, const symba_state *s, int64_t n, int64_t n_m, double dt,
                   double rcrit_factor, const symba_out *out, void *stream, int32_t *chosen_rows);

/* Host-only helper (no device work): device scratch, in bytes, that one
 * problem of n bodies (n_m massive) with an output pair capacity of
 * pair_cap takes from the context in a call with the context's current
 * options: the per-task partial sums (which grow the context's buffer on
 * demand) plus the per-body and per-pair scratch.  Lets a caller that keeps
 * many problems resident budget device memory before it batches them.
 * Returns -1 on invalid arguments. */
int64_t symba_scratch_bytes(const symba_ctx *ctx, int64_t n, int64_t n_m, int64_t pair_cap);

/* The plan a call on a problem of n bodies, n_m massive, would use now (the
 * options and the autotuner's table as they stand): *rows = bodies per lane
 * of the triangle tiles (1, 2 or 4), *split = split diagonals of the folded
 * triangle (Sec. 2: the triangle mapped onto a rectangle; the tile pairs of
 * the split diagonals run last).  Host only, no device work; either pointer
 * may be NULL.  Returns SYMBA_EINVAL for a null context or invalid sizes. */
int symba_plan_for(const symba_ctx *ctx, int64_t n, int64_t n_m, int32_t *rows, int32_t *split);

#ifdef __cplusplus
}
#endif

#endif
