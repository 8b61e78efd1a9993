// Internal declarations shared by the kernels and the C-ABI layer of libsymba.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace symba {

constexpr int kWave = 64;          // wavefront width on gfx950
constexpr int kFinalizeThreads = 256;
constexpr int kFinBodies = 32;     // bodies per finalize block
constexpr int kFinSplit = kFinalizeThreads / kFinBodies;  // threads per body in the slot sums
constexpr int kMaxBuckets = 4096;  // index buckets of the canonical pair order
constexpr int kFieldSegRows = 192; // massive rows per field task (its segment of the rows; 3 tiles of 64)
constexpr int kBoxDoubles = 16;    // tile box record: pos lo[3] hi[3], vel lo[3] hi[3], qmax, pad
constexpr int kGatherWaves = 4;    // tiles per block of the tile-box kernel
constexpr int kBinTempInts = 2 * 2048 + 2 * 2048 + 2 * 2049;  // cell counts, fills, starts

// Per-problem device counters (zero between calls).
constexpr int kCtrPairs = 0;   // flagged pairs found (appended to by the tile kernel)
constexpr int kCtrFound = 1;   // the final count, published by the final kernel for the closing kernel
                               // (written every call, never reset: see close_block)
constexpr int kCtrStatus = 3;  // status bits (slot 2 is unused)
constexpr int kCtrSlots = 4;

// Context-wide statistics accumulated over calls (read by symba_read_stats).
constexpr int kStatFlagged = 1;     // pairs flagged by the exact test
constexpr int kStatCalls = 2;       // problems evaluated
constexpr int kStatCandidates = 4;  // pairs passed by the screen to the exact test, spread over
constexpr int kStatCandLanes = 64;  // this many counters (one atomic per drain would serialise on one)
constexpr int kStatSlots = kStatCandidates + kStatCandLanes;

// Per-problem view handed to the kernels: inputs, outputs, plan and scratch slices.
struct Desc {
    // inputs (device, length n)
    const double *x, *y, *z, *vx, *vy, *vz, *m, *rh;
    // the same inputs as the tile kernel reads them: the binned copies when
    // the problem is binned (positions in the binned order), else the inputs
    const double *bx, *by, *bz, *bvx, *bvy, *bvz, *bm, *brh;
    const int32_t *bidx;  // [n] caller's index of each binned position, null when not binned
    const double *tbox;   // [n_boxes][kBoxDoubles] tile boxes, null when not binned
    // caller outputs (device)
    double *ax, *ay, *az;
    int32_t *pair_i, *pair_j;
    int64_t pair_cap;
    int64_t *n_pairs_out;
    int32_t *group_id;
    int32_t *n_groups_out;
    int32_t *status_out;
    // problem
    int64_t n;       // bodies
    int64_t n_rows;  // rows of the trapezoid: min(N_m, N - 1)
    int64_t n_tri;   // bodies that carry mass: N if N_m >= N - 1, else N_m
    double dt, f;
    double k15, k1875;    // 1.5 and 1.875 (series coefficients of r^-3)
    double screen_dt2;    // 2 (1 + 2^-20) dt^2, the screen's velocity term
    // plan
    int64_t B;            // triangle blocks of 64*rows bodies
    int64_t n_split;      // split diagonals D of the folded triangle
    int64_t n_whole;      // whole block pairs of the folded triangle (launched first)
    int64_t n_slots;      // partial-sum slots per body: B + 2 D (rows - 1), D split diagonals
    int64_t n_tri_tasks;  // whole block pairs + tile pairs of the split diagonals
    int64_t n_tasks;      // triangle + field tasks
    int64_t task_base;    // first global task of this problem
    int64_t n_blk;        // body blocks of this problem's final kernel (kFinBodies bodies each)
    int64_t fin_base;     // first global final-kernel block of this problem
    int64_t n_tboxes;     // 64-body tiles of the massive segment [0, n_tri)
    int64_t n_boxes;      // all tiles (massive, then field [n_tri, n))
    int64_t field_block;  // field bodies per field task (64*field_rows)
    // scratch slices (context-owned)
    double *partial;      // [n_slots][3][n_tri] per-slot partial sums
    double *fpartial;     // [n_fslots][3][n - n_tri] field bodies' partial sums, one slot per segment
    int64_t n_fslots;     // segments of kFieldSegRows massive rows (0 without field tasks)
    int64_t n_fblocks;    // field blocks (64 field_rows field bodies each)
    int32_t *parent;      // [n] union-find forest as offsets to the parent (0 = root), zero between calls
    int32_t *touched;     // [n] body appears in a flagged pair, zero between calls
    int32_t *blk_groups;  // [n_blk] encounter groups rooted in each final-kernel body block
    int2 *pairs;          // [pair_scratch_cap] flagged pairs as found, (min, max)
    int64_t pair_scratch_cap;
    int4 *sorted;         // [pair_scratch_cap] flagged pairs grouped by bucket, with the bucket's range
    int32_t *bcnt;        // [nb] flagged pairs per bucket, zero between calls
    int32_t *bfill;       // [nb] bucket fill counters, zero between calls
    int32_t nb;           // buckets: min(n, kMaxBuckets)
    unsigned long long *ctr;  // [kCtrSlots] counters, zero between calls (kCtrFound excepted)
    unsigned long long *stats;  // [kStatSlots] context-wide statistics
    // binning scratch (written by the binning kernels); null when not binned
    int32_t *bin_key;     // [n] grid cell of each body
    int32_t *bin_tmp;     // [n] bodies grouped by cell
    int32_t *bin_idx;     // [n] binned order (the array bidx points at)
    double *binned;       // [8][n] inputs in the binned order (bx.. point into it)
    double *tbox_w;       // [n_boxes][kBoxDoubles] (the array tbox points at)
    unsigned long long *bin_bbox;  // [2][6] segment boxes (atomic max of ordered keys), zero between calls
    int32_t *bin_hist;    // [2][2048] bodies per cell, zero between calls
    int32_t *bin_fill;    // [2][2048] cell fill counters, zero between calls
    int32_t *bin_start;   // [2][2049] cell starts
    // step epilogue: v += kick_h a for every body once its acceleration is
    // final (null outside symba_step)
    double *kvx, *kvy, *kvz;
    double kick_h;
    // full heliocentric output (SYMBA_ACC_HELIO): per-block partial sums of
    // m x / |x|^3 over the massive bodies, written by k_indirect before the
    // final kernel; null for the interaction term alone
    double *ind;          // [n_ind][3]
    int64_t n_ind;        // k_indirect blocks of this problem (kIndBodies massive bodies each)
    int64_t ind_base;     // first global k_indirect block of this problem
};

// The drifts of a step (symba_step) before the evaluation at the new positions.
struct StepDesc {
    double *x, *y, *z, *vx, *vy, *vz;  // updated in place
    const double *m;
    const double *ax, *ay, *az;         // accelerations of the first kick
    int64_t n, n_tri;                   // bodies; massive bodies [0, n_tri)
    double kick_h, sun_h, kepler_h;     // h/2, h/2, h
    double *mom0, *mom1;                // [launch blocks][3] momentum partial sums (indexed by launch block)
    int64_t blk_base, nblk;             // this problem's blocks [blk_base, blk_base + nblk) of the launch
    const int32_t *skip;                // [n] nonzero: no Kepler drift here (the encounter step), or null
};

// The encounter step (symba_step_enc): a table of the encounter groups built
// from a pair list, the groups' integration through the shells, the level-0
// reweighting of flagged pairs inside the critical radius and the closing
// kick.  Limits: kEncMaxPairs flagged pairs per step, kEncGroupMaxPairs pairs
// (so at most kEncGroupMaxPairs + 1 bodies) per group.
constexpr int kEncMaxPairs = 8192;
constexpr int kEncGroupMaxPairs = 255;
constexpr int kEncGroupBodies = kEncGroupMaxPairs + 1;
constexpr int kEncMaxLevel = 8;       // deepest level
constexpr int kEncSub = 4;            // substeps per level
constexpr double kEncShellRatio = 2.08;
constexpr int kEncCtlGroups = 0;      // ctl[]: groups of the current table
constexpr int kEncCtlSkipped = 1;     // ctl[]: nonzero when pairs went unresolved this step
constexpr int kEncCtlClaim = 2;       // ctl[]: groups the group launch's workgroups have taken so far
constexpr int kEncCtlInts = 4;

struct EncDesc {
    double *x, *y, *z, *vx, *vy, *vz;   // state (device, n), updated in place
    const double *m, *rh;
    double *ax, *ay, *az;               // accelerations (the caller's outputs)
    int64_t n, n_tri;                   // bodies; massive bodies [0, n_tri)
    double f;                           // critical-radius factor: R_0 = f (rh_i + rh_j)
    double h;                           // the step
    double kick_h;                      // the closing kick (0: none)
    // the pair list the table is built from (the caller's outputs)
    const int32_t *pair_i, *pair_j;
    const int64_t *n_pairs;
    int32_t *status;
    const int32_t *group_id;
    int64_t pair_cap;
    // scratch (context-owned)
    int32_t *gp;      // [kEncMaxPairs] pair indices grouped by group, each group's in the pairs' order
    int32_t *gstart;  // [kEncMaxPairs + 1] first entry of each group in gp
    int32_t *gskip;   // [kEncMaxPairs] 1: the group is larger than the limit (not resolved)
    int32_t *ctl;     // [kEncCtlInts]
    int32_t *ingroup; // [n] 1 for bodies of resolved groups while the step runs, zero between calls
    int mark;         // 1: the table marks ingroup (the table at the step's start)
    int regs;         // 1: groups of at most one wave's bodies and pairs integrated in registers
};

// Encounter-step launches (csrc/symba_enc.hip) and the drifts of the
// encounter step around them (csrc/symba_step.hip): first kick, table of the
// step's groups, Sun drift and Kepler drift of the other bodies, the groups'
// integration, momentum, Sun drift.
hipError_t launch_enc_table(const EncDesc &e, hipStream_t stream);
hipError_t launch_enc_groups(const EncDesc &e, hipStream_t stream);
hipError_t launch_enc_level0(const EncDesc &e, hipStream_t stream);
hipError_t launch_enc_kick(const EncDesc &e, hipStream_t stream);
hipError_t launch_drifts_enc(const StepDesc &one, const EncDesc &enc, hipStream_t stream);
// The same for a problem of one block (n <= 256): everything before the
// evaluation in one launch, and the table, reweighting and kick after it in
// another.
hipError_t launch_enc_drifts_block(const StepDesc &one, const EncDesc &enc, hipStream_t stream);
hipError_t launch_enc_post_block(const EncDesc &e, hipStream_t stream);

// Blocks of the drift kernels for n bodies, and their launch (first kick,
// Sun drift, Kepler drift, Sun drift): one problem (`one`, list null) or the
// n_list problems of a device array whose blocks tile [0, total_blocks).
int64_t step_blocks(int64_t n);
hipError_t launch_drifts(const StepDesc &one, const StepDesc *list, int n_list, int64_t total_blocks,
                         hipStream_t stream);

// Problems [p0, p1) of a launch that share a tile size and binning: their tasks are
// [task_begin, task_begin + n_tasks) of the launch's task numbering.
struct TileGroup {
    int rows;        // 1, 2 or 4
    int field_rows;  // 1 or 2
    int binned;      // 1: the problems are binned
    int screen32;    // 1: the pair screen runs in FP32 (SYMBA_OPT_SCREEN 1)
    int p0, p1;
    int64_t task_begin, n_tasks;
};

struct LaunchCfg {
    int scatter_blocks_per_problem;  // pair-scatter blocks per problem (final kernel)
    int close_blocks_per_problem;    // closing-kernel blocks per problem
    int64_t ind_blocks;              // k_indirect blocks of all problems (0: interaction term only)
};

constexpr int kIndBodies = 256;  // massive bodies per k_indirect block (one per thread)

// Folded triangle: block pair (I, J) with J = I + k (mod B) for offsets
// k = 0 .. K - 1, K = (B - 1) / 2 + 1, plus, when B is even, the pairs
// (I, I + B / 2) for I < B / 2: every unordered block pair, diagonal
// included, appears once and every block row gets the same number of tasks
// (the triangle mapped onto a rectangle).
__host__ __device__ inline int64_t fold_offsets(int64_t B) { return (B - 1) / 2 + 1; }

__host__ __device__ inline int64_t fold_count(int64_t B) {
    if (B <= 0) return 0;
    return B * fold_offsets(B) + ((B % 2 == 0) ? B / 2 : 0);
}

// Tail split.  The block pairs of offsets 1 .. D (D split diagonals, at most
// K - 1) are not run whole: each is cut into its R x R tile pairs (stationary
// tile r of block I against tile q of block J), run as separate small tasks
// after all whole block pairs, so that the end of the launch is made of short
// tasks that even out the finishing times of the workgroups.  A body's
// partial sums then come from more tasks than there are blocks: tile pair
// (r, q) of the split pair at offset k writes the sums of its stationary
// bodies to slot J when q = 0, else to extra slot B + (k - 1) 2 (R - 1) + q - 1,
// and those of its streamed bodies to slot I when r = 0, else to extra slot
// B + (k - 1) 2 (R - 1) + (R - 1) + r - 1.  On a split diagonal every block is
// the stationary block of one pair and the streamed block of another, so every
// body receives every one of the B + 2 D (R - 1) slots exactly once.
__host__ __device__ inline int64_t split_diagonals(int64_t B, int R, int64_t want) {
    if (R < 2 || B < 3) return 0;
    const int64_t most = fold_offsets(B) - 1;
    return want < most ? want : most;
}

__host__ __device__ inline int64_t partial_slots(int64_t B, int R, int64_t D) { return B + 2 * D * (R - 1); }

// Whole block pairs of a folded triangle with D split diagonals.
__host__ __device__ inline int64_t whole_count(int64_t B, int64_t D) { return fold_count(B) - D * B; }

// Whole task t (t < whole_count) -> block pair (I, J): offset 0, then the
// offsets past the split ones, then the even-B extra pairs.
__host__ __device__ inline void whole_decode(int64_t B, int64_t D, int64_t t, int64_t &I, int64_t &J) {
    const int64_t K = fold_offsets(B) - D;
    const int64_t main_tasks = B * K;
    if (t < main_tasks) {
        I = t / K;
        const int64_t kk = t % K;
        J = I + (kk == 0 ? 0 : kk + D);
        if (J >= B) J -= B;
    } else {
        I = t - main_tasks;
        J = I + B / 2;
    }
}

// Split task s (s < D B R^2) -> block pair (I, J) at offset k, stationary tile
// r of I, streamed tile q of J, and the partial slots of the two sides.
struct SplitTask {
    int64_t I, J, k;
    int r, q;
    int64_t slot_i, slot_j;
};

__host__ __device__ inline SplitTask split_decode(int64_t B, int R, int64_t s) {
    SplitTask t;
    const int64_t pair = s / (R * R);
    const int sub = (int)(s % (R * R));
    t.r = sub / R;
    t.q = sub % R;
    t.k = pair / B + 1;
    t.I = pair % B;
    t.J = t.I + t.k;
    if (t.J >= B) t.J -= B;
    const int64_t extra = B + (t.k - 1) * 2 * (R - 1);
    t.slot_i = t.q == 0 ? t.J : extra + t.q - 1;
    t.slot_j = t.r == 0 ? t.I : extra + (R - 1) + t.r - 1;
    return t;
}

// Field task f (f < n_fblocks n_fslots) -> (field block, segment).  The
// segments of a field block are 8 task indices apart: the dispatcher deals
// consecutive workgroups to MI355X's 8 XCDs in turn, so a block's segments
// run on one XCD and read its field bodies through one L2.  Groups of 8
// blocks take 8 S consecutive tasks (the last group fewer blocks).
constexpr int kXcds = 8;
__host__ __device__ inline void field_decode(int64_t n_fblocks, int64_t n_fslots, int64_t f, int64_t &fb,
                                             int64_t &sg) {
    const int64_t g = f / (kXcds * n_fslots), r = f % (kXcds * n_fslots);
    const int64_t rest = n_fblocks - g * kXcds;
    const int64_t cnt = rest < kXcds ? rest : kXcds;
    fb = g * kXcds + r % cnt;
    sg = r / cnt;
}

// Order in which a single problem's tasks are launched (position f of the
// launch order -> task index): the field tasks, which are the longest when
// there are many massive rows, first; then the folded triangle.
__host__ __device__ inline int64_t task_in_order(int64_t n_tri_tasks, int64_t n_tasks, int64_t f) {
    const int64_t n_field = n_tasks - n_tri_tasks;
    return f < n_field ? n_tri_tasks + f : f - n_field;
}

// Final-kernel blocks of a problem of n bodies: one body block per kFinBodies
// bodies, then the pair-scatter blocks.
inline int64_t final_blocks(int64_t n, int scatter_blocks) {
    return (n + kFinBodies - 1) / kFinBodies + scatter_blocks;
}

inline int32_t bucket_count(int64_t n) { return (int32_t)(n < kMaxBuckets ? n : kMaxBuckets); }

// Zeroes `bytes` (a multiple of 4) of device memory with a kernel on
// `stream` (no memset node, so it may be captured).
hipError_t launch_zero(void *p, size_t bytes, hipStream_t stream);

// Launch the kernels of one step over n_desc problems: binning (n_binned
// problems use it), the tile kernel (once per group of
// problems sharing a tile size), the final kernel (body
// sums and labels, pairs into index buckets) and the closing kernel
// (canonical pair order, outputs, scratch reset).
// descs_dev is a device copy of descs (may be null when n_desc == 1).  ev,
// when not null, holds three events recorded before the tile kernel, after
// it, and after the closing kernel.
hipError_t launch_step(const Desc *descs_host, const Desc *descs_dev, int n_desc, const TileGroup *groups,
                       int n_groups, int n_binned, int64_t n_fin_total, const LaunchCfg &cfg, hipStream_t stream,
                       hipEvent_t *ev);

}  // namespace symba
