// HIP kernels of the SyMBA kick/encounter step for gfx950 (CDNA4).
//
// One step (the paper's Sec. 2: trapezoid pair loop, close-encounter check,
// grouping of encounter pairs) runs as three launches:
//   k_tiles     the folded trapezoid in 64-lane tasks: FP64 pair forces, a
//               conservative per-pair screen whose candidates are queued in
//               LDS, the exact FP64 encounter test on the candidates, and the
//               union of every flagged pair into a lock-free union-find;
//   k_finalize  per body: fixed-order sum of the per-task partial
//               accelerations, group label = root of the union-find;
//               per pair: canonical (lexicographic) position by counting;
//   k_scatter   pairs to their canonical slots, scalar outputs, and the
//               scratch returned to its between-calls state.
//
// Triangle tasks (massive x massive) are symmetric: each lane of a wave owns
// `R` stationary bodies in registers; a 64-body j tile sits in LDS (stored
// twice so that lane l reads entry l + t at step t without wrapping), and the
// j-side sum of each pair travels with its j body by rotating the three
// accumulators one lane per step, so that after 64 steps every j-side sum is
// back in the lane that staged its body and no cross-lane reduction is
// needed.  Field tasks (massive x field) are one-sided: the massive body is
// broadcast from LDS to lanes that own field bodies.
#include "symba_internal.h"

#include <float.h>
#include <math.h>

namespace symba {
namespace {

constexpr double kPadPos = 0x1p300;          // padding slots sit far away with zero mass
constexpr double kReachMargin = 1.0 + 0x1p-20;
constexpr int kQMask = kQueueCap - 1;
// fewer than 64 outstanding after a step plus one step's pushes (4 slots x 64)
static_assert(kQueueCap >= kWave * 5 && (kQueueCap & kQMask) == 0, "candidate queue too small");
constexpr unsigned long long kStatusCapacity = 1;
constexpr unsigned long long kStatusNonfinite = 2;

struct __align__(16) TileLds {
    double x[2 * kWave], y[2 * kWave], z[2 * kWave], m[2 * kWave], reach[2 * kWave];
    uint2 queue[kQueueCap];
};

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// Set bits of `mask` below this lane.
__device__ __forceinline__ int prefix_count(unsigned long long mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// r2^(-3/2): the hardware reciprocal-square-root estimate y (relative error
// near 2^-23) corrected by the binomial series of (1 - e)^(-3/2), e = 1 - r2 y^2,
// to second order: q = y^3 (1 + 3e/2 + 15e^2/8), truncation ~ (35/16) e^3.
// k15 = 1.5 and k1875 = 1.875 arrive as kernel arguments so that they sit in
// scalar registers (gfx950's VOP3 FMA takes no literal operand).
__device__ __forceinline__ double inv_r3(double r2, double k15, double k1875) {
    const double y = __builtin_amdgcn_rsq(r2);
    const double y2 = y * y;
    const double e = __builtin_fma(-r2, y2, 1.0);
    const double y3 = y2 * y;
    const double a = e * y3;
    return __builtin_fma(a * e, k1875, __builtin_fma(a, k15, y3));
}

// Upper bound on how close a body's pairs can come within one step:
// (|f rh| + |v| dt)(1 + 2^-20).  A pair whose separation is at least the sum
// of the two bodies' reaches cannot be flagged by the encounter test; the
// margin dominates every rounding error of both the bound and the test.
__device__ __forceinline__ double reach_of(double vx, double vy, double vz, double rh, double f,
                                           double dt) {
    const double sp = sqrt(__builtin_fma(vz, vz, __builtin_fma(vy, vy, vx * vx)));
    const double r = (fabs(f * rh) + sp * dt) * kReachMargin;
    return (r <= DBL_MAX) ? r : INFINITY;  // NaN or Inf: every pair becomes a candidate
}

// The library's encounter test, operation for operation as documented in
// symba.h; both orientations of a pair give the same bits.
__device__ __forceinline__ bool encounter_test(double dx, double dy, double dz, double wx,
                                               double wy, double wz, double rh_i, double rh_j,
                                               double f, double dt) {
#pragma clang fp contract(off)
    const double rc = f * rh_i + f * rh_j;
    const double rc2 = rc * rc;
    const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
    const double v2 = __builtin_fma(wz, wz, __builtin_fma(wy, wy, wx * wx));
    const double vr = __builtin_fma(dz, wz, __builtin_fma(dy, wy, dx * wx));
    const bool start = r2 < rc2;
    const double end2 = __builtin_fma(v2, dt * dt, __builtin_fma(vr, 2.0 * dt, r2));
    const bool end = end2 < rc2;
    const bool inner = (vr < 0.0) && (-vr < v2 * dt) && (__builtin_fma(-vr, vr, r2 * v2) < rc2 * v2);
    return start || end || inner;
}

__device__ __forceinline__ int uf_load(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x.  Parents only ever decrease (parent[v] <= v), so every value
// read is an ancestor and the walk ends at a root.
__device__ __forceinline__ int uf_find(int32_t *parent, int x) {
    int p = uf_load(parent + x);
    while (p != x) {
        x = p;
        p = uf_load(parent + x);
    }
    return x;
}

// Lock-free union: hook the larger root under the smaller one with a CAS and
// retry if another lane or wave re-hooked it first.  Each root stays the
// minimum of its tree, so the final roots are the component minima whatever
// the interleaving.
__device__ __forceinline__ void uf_unite(int32_t *parent, int a, int b) {
    while (true) {
        a = uf_find(parent, a);
        b = uf_find(parent, b);
        if (a == b) return;
        if (a > b) {
            const int t = a;
            a = b;
            b = t;
        }
        int expected = b;
        if (__hip_atomic_compare_exchange_strong(parent + b, &expected, a, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
    }
}

// Exact test of up to 64 queued candidates, one per lane; flagged pairs are
// appended (wave ballot + prefix, one atomic per wave) and grouped at once.
__device__ __forceinline__ void drain(const Desc &d, const TileLds &L, int head, int count) {
    const int l = lane();
    bool flag = false;
    int a = 0, b = 0;
    if (l < count) {
        const uint2 c = L.queue[(head + l) & kQMask];
        const int i = (int)c.x, j = (int)c.y;
        if (i < d.n && j < d.n)
            flag = encounter_test(d.x[j] - d.x[i], d.y[j] - d.y[i], d.z[j] - d.z[i],
                              d.vx[j] - d.vx[i], d.vy[j] - d.vy[i], d.vz[j] - d.vz[i],
                              d.rh[i], d.rh[j], d.f, d.dt);
        a = i < j ? i : j;
        b = i < j ? j : i;
    }
    const unsigned long long fm = __ballot(flag);
    if (l == 0) atomicAdd(d.ctr + 1, (unsigned long long)count);
    if (fm == 0) return;
    const int leader = __ffsll((long long)fm) - 1;
    unsigned long long base = 0;
    if (l == leader) base = atomicAdd(d.ctr, (unsigned long long)__popcll(fm));
    base = __shfl(base, leader);
    if (flag) {
        const unsigned long long pos = base + (unsigned long long)prefix_count(fm);
        if (pos < (unsigned long long)d.pair_scratch_cap) d.pairs[pos] = make_int2(a, b);
        d.touched[a] = 1;
        d.touched[b] = 1;
        uf_unite(d.parent, a, b);
    }
}

// Append this lane's candidate (i, j) if `c`; the mask is the wave's ballot of c.
__device__ __forceinline__ void push(TileLds &L, int &tail, unsigned long long mask, bool c,
                                     int64_t i, int64_t j) {
    if (c) L.queue[(tail + prefix_count(mask)) & kQMask] = make_uint2((unsigned)i, (unsigned)j);
    tail += __popcll(mask);
}

// Keeps fewer than 64 candidates outstanding after every step, so one step's
// pushes (at most 64 per slot) always fit the queue.
__device__ __forceinline__ void maybe_drain(const Desc &d, TileLds &L, int &head, int tail) {
    if (tail - head >= kWave) {
        __syncthreads();
        do {
            drain(d, L, head, kWave);
            head += kWave;
        } while (tail - head >= kWave);
        __syncthreads();
    }
}

__device__ __forceinline__ void drain_rest(const Desc &d, TileLds &L, int &head, int tail) {
    __syncthreads();
    while (tail - head > 0) {
        const int c = (tail - head) < kWave ? (tail - head) : kWave;
        drain(d, L, head, c);
        head += c;
    }
}

// Stage bodies [j0, j0 + 64) (entries past `limit` become padding) into the
// LDS tile, each stored at l and l + 64.
__device__ __forceinline__ void stage(const Desc &d, TileLds &L, int64_t j0, int64_t limit) {
    const int l = lane();
    const int64_t j = j0 + l;
    double x = kPadPos, y = 0.0, z = 0.0, m = 0.0, r = 0.0;
    if (j < limit) {
        x = d.x[j];
        y = d.y[j];
        z = d.z[j];
        m = d.m[j];
        r = reach_of(d.vx[j], d.vy[j], d.vz[j], d.rh[j], d.f, d.dt);
    }
    __syncthreads();
    L.x[l] = x; L.x[l + kWave] = x;
    L.y[l] = y; L.y[l + kWave] = y;
    L.z[l] = z; L.z[l + kWave] = z;
    L.m[l] = m; L.m[l + kWave] = m;
    L.reach[l] = r; L.reach[l + kWave] = r;
    __syncthreads();
}

__device__ __forceinline__ void load_body(const Desc &d, int64_t k, int64_t limit, double &x,
                                          double &y, double &z, double &m, double &r) {
    if (k < limit) {
        x = d.x[k];
        y = d.y[k];
        z = d.z[k];
        m = d.m[k];
        r = reach_of(d.vx[k], d.vy[k], d.vz[k], d.rh[k], d.f, d.dt);
    } else {
        x = kPadPos;
        y = z = m = r = 0.0;
    }
}

__device__ __forceinline__ double rotate_dpp(double v) {
    // lane l receives the value of lane (l + 1) mod 64 (DPP wave_rol:1); every
    // lane has a source, so no "old" value is needed
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x134, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x134, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double rotate_bperm(double v, int addr) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_ds_bpermute(addr, lo);
    hi = __builtin_amdgcn_ds_bpermute(addr, hi);
    return __hiloint2double(hi, lo);
}

template <int R>
struct Slots {
    double x[R], y[R], z[R], m[R], r[R];
    double ax[R], ay[R], az[R];
};

__device__ __forceinline__ void write_partial(const Desc &d, int64_t slot, int64_t k, double ax,
                                              double ay, double az) {
    if (k < d.n_tri) {
        double *p = d.partial + slot * 3 * d.n_tri + k;
        p[0] = ax;
        p[d.n_tri] = ay;
        p[2 * d.n_tri] = az;
    }
}

// 64 rotation steps of one staged j tile against the first NACT slots: both
// sides of every pair are accumulated; returns the j-side sums home.
template <int R, int NACT, int ROT>
__device__ __forceinline__ void rotation_pass(const Desc &d, TileLds &L, Slots<R> &S, int64_t ib, int64_t js,
                              int &head, int &tail, double &ajx, double &ajy, double &ajz) {
    const int l = lane();
    const int baddr = ((l + 1) & (kWave - 1)) << 2;
    ajx = ajy = ajz = 0.0;
#pragma unroll 2
    for (int t = 0; t < kWave; ++t) {
        const int idx = l + t;
        const double xj = L.x[idx], yj = L.y[idx], zj = L.z[idx], mj = L.m[idx], rj = L.reach[idx];
        bool cand[R];
        unsigned long long mask[R];
        unsigned long long any = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            cand[r] = false;
            mask[r] = 0;
            if (r < NACT) {
                const double dx = xj - S.x[r], dy = yj - S.y[r], dz = zj - S.z[r];
                const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                const double q = inv_r3(r2, d.k15, d.k1875);
                const double fi = mj * q, fj = S.m[r] * q;
                S.ax[r] = __builtin_fma(fi, dx, S.ax[r]);
                S.ay[r] = __builtin_fma(fi, dy, S.ay[r]);
                S.az[r] = __builtin_fma(fi, dz, S.az[r]);
                ajx = __builtin_fma(-fj, dx, ajx);
                ajy = __builtin_fma(-fj, dy, ajy);
                ajz = __builtin_fma(-fj, dz, ajz);
                const double rs = S.r[r] + rj;
                cand[r] = r2 < rs * rs;
                mask[r] = __ballot(cand[r]);
                any |= mask[r];
            }
        }
        if (any) {
            const int64_t j = js + ((l + t) & (kWave - 1));
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (r < NACT && mask[r]) push(L, tail, mask[r], cand[r], ib + r * kWave + l, j);
            maybe_drain(d, L, head, tail);
        }
        if (ROT == 0) {
            ajx = rotate_dpp(ajx);
            ajy = rotate_dpp(ajy);
            ajz = rotate_dpp(ajz);
        } else {
            ajx = rotate_bperm(ajx, baddr);
            ajy = rotate_bperm(ajy, baddr);
            ajz = rotate_bperm(ajz, baddr);
        }
    }
}

// Slot Q against its own 64-body tile (a diagonal sub-block): each unordered
// pair is met from both ends, only the stationary side is accumulated, and the
// pair is screened once (from the lane whose partner is 1..31 steps ahead, or
// 32 steps ahead for the lower half of the wave).
template <int R, int Q>
__device__ __forceinline__ void diagonal_pass(const Desc &d, TileLds &L, Slots<R> &S, int64_t ib, int &head,
                              int &tail) {
    const int l = lane();
    for (int t = 1; t < kWave; ++t) {
        const int idx = l + t;
        const double xj = L.x[idx], yj = L.y[idx], zj = L.z[idx], mj = L.m[idx], rj = L.reach[idx];
        const double dx = xj - S.x[Q], dy = yj - S.y[Q], dz = zj - S.z[Q];
        const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
        const double fi = mj * inv_r3(r2, d.k15, d.k1875);
        S.ax[Q] = __builtin_fma(fi, dx, S.ax[Q]);
        S.ay[Q] = __builtin_fma(fi, dy, S.ay[Q]);
        S.az[Q] = __builtin_fma(fi, dz, S.az[Q]);
        const double rs = S.r[Q] + rj;
        const bool owner = (t < kWave / 2) || (t == kWave / 2 && l < kWave / 2);
        const bool c = owner && (r2 < rs * rs);
        const unsigned long long mask = __ballot(c);
        if (mask) {
            push(L, tail, mask, c, ib + Q * kWave + l, ib + Q * kWave + ((l + t) & (kWave - 1)));
            maybe_drain(d, L, head, tail);
        }
    }
}

template <int R, int ROT, int Q>
__device__ __forceinline__ void diagonal_subtiles(const Desc &d, TileLds &L, Slots<R> &S, int64_t ib, int &head,
                                  int &tail) {
    if constexpr (Q < R) {
        stage(d, L, ib + Q * kWave, d.n_tri);
        if constexpr (Q > 0) {
            double ajx, ajy, ajz;
            rotation_pass<R, Q, ROT>(d, L, S, ib, ib + Q * kWave, head, tail, ajx, ajy, ajz);
            S.ax[Q] += ajx;
            S.ay[Q] += ajy;
            S.az[Q] += ajz;
        }
        diagonal_pass<R, Q>(d, L, S, ib, head, tail);
        diagonal_subtiles<R, ROT, Q + 1>(d, L, S, ib, head, tail);
    }
}

// Block pair (I, J) of the folded triangle.  Partial sums land in slot J for
// the stationary bodies of block I and in slot I for the bodies of block J.
template <int R, int ROT>
__device__ __forceinline__ void triangle_task(const Desc &d, TileLds &L, int64_t I, int64_t J) {
    const int l = lane();
    const int64_t ib = I * R * kWave, jb = J * R * kWave;
    Slots<R> S;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        load_body(d, ib + r * kWave + l, d.n_tri, S.x[r], S.y[r], S.z[r], S.m[r], S.r[r]);
        S.ax[r] = S.ay[r] = S.az[r] = 0.0;
    }
    int head = 0, tail = 0;
    if (I != J) {
        for (int q = 0; q < R; ++q) {
            const int64_t js = jb + q * kWave;
            stage(d, L, js, d.n_tri);
            double ajx, ajy, ajz;
            rotation_pass<R, R, ROT>(d, L, S, ib, js, head, tail, ajx, ajy, ajz);
            write_partial(d, I, js + l, ajx, ajy, ajz);
        }
    } else {
        diagonal_subtiles<R, ROT, 0>(d, L, S, ib, head, tail);
    }
    drain_rest(d, L, head, tail);
#pragma unroll
    for (int r = 0; r < R; ++r) write_partial(d, J, ib + r * kWave + l, S.ax[r], S.ay[r], S.az[r]);
}

// Field block fb against every massive row: one-sided pairs; the field
// bodies' accelerations are complete at the end and written directly.
template <int RF>
__device__ __forceinline__ void field_task(const Desc &d, TileLds &L, int64_t fb) {
    const int l = lane();
    const int64_t f0 = d.n_tri + fb * RF * kWave;
    double xf[RF], yf[RF], zf[RF], rf[RF], ax[RF], ay[RF], az[RF];
#pragma unroll
    for (int r = 0; r < RF; ++r) {
        double m;
        load_body(d, f0 + r * kWave + l, d.n, xf[r], yf[r], zf[r], m, rf[r]);
        ax[r] = ay[r] = az[r] = 0.0;
    }
    int head = 0, tail = 0;
    for (int64_t s0 = 0; s0 < d.n_rows; s0 += kWave) {
        stage(d, L, s0, d.n_rows);
        const int nv = (d.n_rows - s0) < kWave ? (int)(d.n_rows - s0) : kWave;
        for (int t = 0; t < nv; ++t) {
            const double xi = L.x[t], yi = L.y[t], zi = L.z[t], mi = L.m[t], ri = L.reach[t];
            bool cand[RF];
            unsigned long long mask[RF];
            unsigned long long any = 0;
#pragma unroll
            for (int r = 0; r < RF; ++r) {
                const double dx = xf[r] - xi, dy = yf[r] - yi, dz = zf[r] - zi;
                const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                const double fj = mi * inv_r3(r2, d.k15, d.k1875);
                ax[r] = __builtin_fma(-fj, dx, ax[r]);
                ay[r] = __builtin_fma(-fj, dy, ay[r]);
                az[r] = __builtin_fma(-fj, dz, az[r]);
                const double rs = rf[r] + ri;
                cand[r] = r2 < rs * rs;
                mask[r] = __ballot(cand[r]);
                any |= mask[r];
            }
            if (any) {
#pragma unroll
                for (int r = 0; r < RF; ++r)
                    if (mask[r]) push(L, tail, mask[r], cand[r], s0 + t, f0 + r * kWave + l);
                maybe_drain(d, L, head, tail);
            }
        }
    }
    drain_rest(d, L, head, tail);
#pragma unroll
    for (int r = 0; r < RF; ++r) {
        const int64_t k = f0 + r * kWave + l;
        if (k < d.n) {
            d.ax[k] = ax[r];
            d.ay[k] = ay[r];
            d.az[k] = az[r];
        }
    }
}

__device__ inline int problem_of(const Desc *descs, int n_desc, int64_t key, bool by_task) {
    int lo = 0, hi = n_desc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t base = by_task ? descs[mid].task_base : descs[mid].blk_base;
        if (base <= key)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <int R, int RF, int ROT>
__global__ __launch_bounds__(kWave) void k_tiles(Desc inl, const Desc *descs, int n_desc) {
    __shared__ TileLds L;
    const int64_t t = blockIdx.x;
    const Desc d = descs ? descs[problem_of(descs, n_desc, t, true)] : inl;
    const int64_t lt = t - d.task_base;
    if (lt < d.n_tri_tasks) {
        int64_t I, J;
        fold_decode(d.B, lt, I, J);
        triangle_task<R, ROT>(d, L, I, J);
    } else {
        field_task<RF>(d, L, lt - d.n_tri_tasks);
    }
}

__global__ __launch_bounds__(kFinalizeThreads) void k_finalize(Desc inl, const Desc *descs,
                                                                int n_desc, int64_t n_blk_total,
                                                                int rank_per_problem) {
    __shared__ unsigned long long keys[kRankTile];
    const int64_t b = blockIdx.x;
    const int tid = threadIdx.x;
    if (b < n_blk_total) {
        const Desc &d = descs ? descs[problem_of(descs, n_desc, b, false)] : inl;
        const int64_t lb = b - d.blk_base;
        const int64_t k = lb * kFinalizeThreads + tid;
        bool root_of_group = false, nonfinite = false;
        if (k < d.n) {
            double sx = 0.0, sy = 0.0, sz = 0.0;
            if (k < d.n_tri || d.n_rows == 0) {
                const double *p = d.partial + k;
                for (int64_t c = 0; c < d.B; ++c) {
                    sx += p[(3 * c) * d.n_tri];
                    sy += p[(3 * c + 1) * d.n_tri];
                    sz += p[(3 * c + 2) * d.n_tri];
                }
                d.ax[k] = sx;
                d.ay[k] = sy;
                d.az[k] = sz;
            } else {
                sx = d.ax[k];
                sy = d.ay[k];
                sz = d.az[k];
            }
            nonfinite = !(isfinite(sx) && isfinite(sy) && isfinite(sz));
            const int g = uf_find(d.parent, (int)k);
            d.group_id[k] = g;
            root_of_group = d.touched[k] && g == (int)k;
            d.touched[k] = 0;
        }
        const int groups = __syncthreads_count(root_of_group);
        const int bad = __syncthreads_or(nonfinite);
        if (tid == 0) {
            if (groups) atomicAdd(d.ctr + 2, (unsigned long long)groups);
            if (bad) atomicOr(d.ctr + 3, kStatusNonfinite);
            if (lb == 0) *d.n_pairs_out = (int64_t)d.ctr[0];
        }
        return;
    }
    // canonical order of the stored pairs: rank = number of smaller keys
    const int64_t rb = b - n_blk_total;
    const int p = (int)(rb / rank_per_problem);
    if (p >= n_desc) return;
    const int r = (int)(rb % rank_per_problem);
    const Desc &d = descs ? descs[p] : inl;
    const unsigned long long found = d.ctr[0];
    const int64_t ns = (int64_t)found < d.pair_scratch_cap ? (int64_t)found : d.pair_scratch_cap;
    const int64_t side = (ns + kRankTile - 1) / kRankTile;
    for (int64_t t = r; t < side * side; t += rank_per_problem) {
        const int64_t pc = t / side, kc = t % side;
        const int64_t kq = kc * kRankTile + tid;
        __syncthreads();
        if (kq < ns) {
            const int2 e = d.pairs[kq];
            keys[tid] = ((unsigned long long)(unsigned)e.x << 32) | (unsigned)e.y;
        }
        __syncthreads();
        const int64_t me = pc * kRankTile + tid;
        const int nk = (ns - kc * kRankTile) < kRankTile ? (int)(ns - kc * kRankTile) : kRankTile;
        if (me < ns) {
            const int2 e = d.pairs[me];
            const unsigned long long mine = ((unsigned long long)(unsigned)e.x << 32) | (unsigned)e.y;
            int less = 0;
            for (int q = 0; q < nk; ++q) less += keys[q] < mine;
            if (less) atomicAdd(d.rank + me, less);
        }
    }
}

__global__ __launch_bounds__(kFinalizeThreads) void k_scatter(Desc inl, const Desc *descs,
                                                               int n_desc) {
    const int64_t b = blockIdx.x;
    const int tid = threadIdx.x;
    const Desc &d = descs ? descs[problem_of(descs, n_desc, b, false)] : inl;
    const int64_t lb = b - d.blk_base;
    const int64_t stride = d.n_blk * kFinalizeThreads;
    const int64_t found = *d.n_pairs_out;
    const int64_t ns = found < d.pair_scratch_cap ? found : d.pair_scratch_cap;
    const int64_t cap = d.pair_cap < d.pair_scratch_cap ? d.pair_cap : d.pair_scratch_cap;
    const bool fits = found <= cap;
    for (int64_t p = lb * kFinalizeThreads + tid; p < ns; p += stride) {
        const int r = d.rank[p];
        d.rank[p] = 0;
        if (fits) {
            const int2 e = d.pairs[p];
            d.pair_i[r] = e.x;
            d.pair_j[r] = e.y;
        }
    }
    for (int64_t k = lb * kFinalizeThreads + tid; k < d.n; k += stride) d.parent[k] = (int32_t)k;
    if (lb == 0 && tid == 0) {
        *d.n_groups_out = (int32_t)d.ctr[2];
        *d.status_out = (int32_t)(d.ctr[3] | (fits ? 0ull : kStatusCapacity));
        d.ctr[0] = d.ctr[1] = d.ctr[2] = d.ctr[3] = 0;
    }
}

__global__ void k_identity(int32_t *parent, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) parent[k] = (int32_t)k;
}

template <int R, int RF, int ROT>
void launch_tiles(int64_t n_tasks, const Desc &inl, const Desc *descs, int n_desc,
                  hipStream_t stream) {
    hipLaunchKernelGGL((k_tiles<R, RF, ROT>), dim3((unsigned)n_tasks), dim3(kWave), 0, stream,
                       inl, descs, n_desc);
}

template <int R>
void launch_tiles_r(int rf, int rot, int64_t n_tasks, const Desc &inl, const Desc *descs,
                    int n_desc, hipStream_t stream) {
    if (rf == 2) {
        if (rot) launch_tiles<R, 2, 1>(n_tasks, inl, descs, n_desc, stream);
        else launch_tiles<R, 2, 0>(n_tasks, inl, descs, n_desc, stream);
    } else {
        if (rot) launch_tiles<R, 1, 1>(n_tasks, inl, descs, n_desc, stream);
        else launch_tiles<R, 1, 0>(n_tasks, inl, descs, n_desc, stream);
    }
}

}  // namespace

hipError_t launch_step(const Desc *descs_host, const Desc *descs_dev, int n_desc,
                       int64_t n_tasks_total, int64_t n_blk_total, const LaunchCfg &cfg,
                       hipStream_t stream, hipEvent_t *ev) {
    const Desc &inl = descs_host[0];
    const Desc *dd = n_desc == 1 ? nullptr : descs_dev;
    if (ev && hipEventRecord(ev[0], stream) != hipSuccess) return hipErrorUnknown;
    if (n_tasks_total > 0) {
        switch (cfg.rows) {
            case 1: launch_tiles_r<1>(cfg.field_rows, cfg.rotate, n_tasks_total, inl, dd, n_desc, stream); break;
            case 2: launch_tiles_r<2>(cfg.field_rows, cfg.rotate, n_tasks_total, inl, dd, n_desc, stream); break;
            default: launch_tiles_r<4>(cfg.field_rows, cfg.rotate, n_tasks_total, inl, dd, n_desc, stream); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (ev && hipEventRecord(ev[1], stream) != hipSuccess) return hipErrorUnknown;
    const int64_t rank_blocks = (int64_t)cfg.rank_blocks_per_problem * n_desc;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)(n_blk_total + rank_blocks)), dim3(kFinalizeThreads),
                       0, stream, inl, dd, n_desc, n_blk_total, cfg.rank_blocks_per_problem);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)n_blk_total), dim3(kFinalizeThreads), 0, stream, inl,
                       dd, n_desc);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev && hipEventRecord(ev[2], stream) != hipSuccess) return hipErrorUnknown;
    return hipSuccess;
}

hipError_t launch_init_scratch(int32_t *parent, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_identity, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, parent, n);
    return hipGetLastError();
}

}  // namespace symba
