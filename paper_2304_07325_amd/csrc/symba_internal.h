// Internal declarations shared by the kernels and the C-ABI layer of libsymba.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace symba {

constexpr int kWave = 64;          // wavefront width on gfx950
constexpr int kFinalizeThreads = 256;
constexpr int kFinBodies = 32;     // bodies per finalize block
constexpr int kFinSplit = kFinalizeThreads / kFinBodies;  // threads per body in the slot sums
constexpr int kRankTile = 256;     // pairs per rank tile side

// Per-problem view handed to the kernels: inputs, outputs, plan and scratch slices.
struct Desc {
    // inputs (device, length n)
    const double *x, *y, *z, *vx, *vy, *vz, *m, *rh;
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
    int64_t n_tri_tasks;  // folded block pairs
    int64_t n_tasks;      // triangle + field tasks
    int64_t task_base;    // first global task of this problem
    int64_t blk_base;     // first global finalize block of this problem
    int64_t n_blk;        // finalize blocks of this problem (kFinBodies bodies each)
    int64_t field_block;  // field bodies per field task (64*field_rows)
    // scratch slices (context-owned)
    double *partial;      // [B][3][n_tri] per-slot partial sums
    int32_t *parent;      // [n] union-find forest as offsets to the parent (0 = root), zero between calls
    int32_t *touched;     // [n] body appears in a flagged pair, zero between calls
    int2 *pairs;          // [pair_scratch_cap] flagged pairs as found, (min, max)
    int64_t pair_scratch_cap;
    int32_t *rank;        // [pair_scratch_cap] output position, zero between calls
    unsigned long long *ctr;  // [4]: found pairs, screen candidates, groups, status bits; zero between calls
};

struct LaunchCfg {
    int rows;        // 1, 2 or 4
    int field_rows;  // 1 or 2
    int rotate;      // 0 DPP, 1 ds_bpermute
    int screen;      // 0 FP64 reach screen, 1 FP32 pre-screen
    int rank_blocks_per_problem;
};

// Folded triangle: task t of B blocks -> block pair (I, J); every unordered
// block pair, diagonal included, appears once and every block row gets the
// same number of tasks (the triangle mapped onto a rectangle).
__host__ __device__ inline void fold_decode(int64_t B, int64_t t, int64_t &I, int64_t &J) {
    const int64_t K = (B - 1) / 2 + 1;
    const int64_t main_tasks = B * K;
    if (t < main_tasks) {
        I = t / K;
        J = I + t % K;
        if (J >= B) J -= B;
    } else {
        I = t - main_tasks;
        J = I + B / 2;
    }
}

__host__ __device__ inline int64_t fold_count(int64_t B) {
    if (B <= 0) return 0;
    return B * ((B - 1) / 2 + 1) + ((B % 2 == 0) ? B / 2 : 0);
}

// Launch the three kernels of one step over n_desc problems.  descs_dev is a
// device copy of descs (may be null when n_desc == 1).
// device copy of descs (may be null when n_desc == 1).  ev, when not null,
// holds three events recorded before the tile kernel, after it, and after the
// finalize kernels.
hipError_t launch_step(const Desc *descs_host, const Desc *descs_dev, int n_desc,
                       int64_t n_tasks_total, int64_t n_blk_total, const LaunchCfg &cfg,
                       hipStream_t stream, hipEvent_t *ev);

}  // namespace symba
