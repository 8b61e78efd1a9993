// HIP kernels of the SyMBA kick/encounter step for gfx950 (CDNA4).
//
// One step (the paper's Sec. 2: trapezoid pair loop, close-encounter check,
// grouping of encounter pairs) runs as three launches:
//   k_tiles  the folded trapezoid, one block pair per 4-wave workgroup (in
//            short launches the last block pairs cut into 64 x 64 tile
//            pairs): FP64 pair forces into per-task partial sums, a
//            conservative per-pair screen (FP32 or FP64) whose candidates are
//            queued in LDS, and, after the task's last barrier, the exact FP64
//            encounter test of the candidates, flagged pairs appended,
//            counted per index bucket and united in a lock-free union-find;
//   k_final  per body: fixed-order sum of the partial accelerations and the
//            group label (union-find root), group roots counted per block;
//            per pair: moved into its bucket;
//   k_close  per pair: canonical (lexicographic) position by counting the
//            smaller keys of its bucket, pair written out; scalar outputs;
//            scratch returned to its between-calls state.
//
// Triangle tasks (massive x massive) are symmetric.  Each lane owns R
// stationary bodies in registers; the streamed block (R tiles of 64 bodies)
// sits in LDS, each tile stored twice so that lane l reads entry l + t at
// step t without wrapping.  The j-side sum of a pair travels with its j body:
// the three accumulators rotate one lane per step, so every lane always holds
// the sums of the body it is paired with and no cross-lane reduction is
// needed.  The 64 steps of a tile are split over the four waves of the
// workgroup (16 steps each, all four holding the same stationary bodies);
// their sums are combined through LDS in a fixed order.  Field tasks
// (massive x field) are one-sided: massive bodies are broadcast from LDS to
// lanes that own field bodies, the massive rows split over the four waves.
#include "symba_internal.h"

#include <float.h>
#include <math.h>

namespace symba {
namespace {

// Occupancy targets of the tile kernel per tile size (waves per SIMD; the
// register budget is 512/N VGPRs).  Tuning knobs.
#ifndef SYMBA_WPE_R1
#define SYMBA_WPE_R1 6
#endif
#ifndef SYMBA_WPE_R2
#define SYMBA_WPE_R2 4
#endif
#ifndef SYMBA_WPE_R4
#define SYMBA_WPE_R4 2
#endif
#ifndef SYMBA_ROT_UNROLL
#define SYMBA_ROT_UNROLL 2  // unroll of the 64-step rotation loop (a tuning knob)
#endif

constexpr int kRotUnroll = SYMBA_ROT_UNROLL;

constexpr int waves_per_eu(int R) { return R == 1 ? SYMBA_WPE_R1 : (R == 2 ? SYMBA_WPE_R2 : SYMBA_WPE_R4); }
constexpr double kPadPos = 0x1p300;          // padding slots sit far away with zero mass
constexpr double kScreenQ = 4.0 * (1.0 + 0x1p-20);
constexpr double kScreenInflate = 1.0 + 0x1p-40;
constexpr unsigned long long kStatusCapacity = 1;
constexpr unsigned long long kStatusNonfinite = 2;

constexpr int kTaskWaves = 4;                  // waves sharing one task
constexpr int kTaskThreads = kTaskWaves * kWave;
constexpr int kSteps = kWave / kTaskWaves;     // steps of each 64-step tile per wave

// Workgroup LDS of a task: the streamed block (RS tiles of 64 bodies, each
// stored twice, 16-byte pairs) and the stationary block (RS tiles, read into
// registers once the block is staged); after the passes the same space holds
// the waves' partial sums [side: stationary, streamed][wave][slot][component][lane].
template <int RS>
struct __align__(16) TaskLds {
    union {
        struct {
            double2 xy[RS][2 * kWave], zm[RS][2 * kWave], vxy[RS][2 * kWave], vzq[RS][2 * kWave];
            double2 sxy[RS * kWave], szm[RS * kWave], svxy[RS * kWave], svzq[RS * kWave];
        } tile;
        // a field task's segment of massive rows (each row once: every lane
        // reads the same row at a time)
        struct {
            double2 xy[kFieldSegRows], zm[kFieldSegRows], vxy[kFieldSegRows], vzq[kFieldSegRows];
        } seg;
        double comb[2][kTaskWaves][RS][3][kWave];
    };
};
static_assert(sizeof(TaskLds<1>::seg) <= sizeof(TaskLds<1>::tile), "a field segment fits the smallest tile area");

// Per-wave LDS ring of screen candidates (i, j).  After every step fewer than
// 64 are outstanding and one step pushes at most 64 per stationary slot, so a
// capacity of 64 (slots + 1), rounded up to a power of two, never overflows.
struct Queue {
    uint2 *q;
    int mask;
    int head, tail;
};

constexpr int queue_cap(int slots) {
    int c = 64;
    while (c < kWave * (slots + 1)) c *= 2;
    return c;
}

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// Index of this wave in its workgroup, as a wave-uniform (scalar) value.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave); }

// 1 if the wave-uniform mask is non-zero, else 0, computed by the scalar unit
// (written out because a compare on the mask is otherwise lowered to a per-lane
// select that is read back from a vector register).
__device__ __forceinline__ unsigned nonzero(unsigned long long mask) {
    unsigned r;
    asm("s_cmp_lg_u64 %1, 0\n\ts_cselect_b32 %0, 1, 0" : "=s"(r) : "s"(mask) : "scc");
    return r;
}

// Set bits of `mask` below this lane.
__device__ __forceinline__ int prefix_count(unsigned long long mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// r2^(-3/2): the hardware reciprocal-square-root estimate y (relative error
// near 2^-23) corrected by the binomial series of (1 - e)^(-3/2), e = 1 - r2 y^2,
// to second order: q = y^3 (1 + e (3/2 + 15e/8)), truncation ~ (35/16) e^3.
// k15 = 1.5 and k1875 = 1.875 arrive as kernel arguments so that they sit in
// scalar registers (gfx950's VOP3 FMA takes no literal operand; 1.0 is an
// inline constant).
__device__ __forceinline__ double inv_r3(double r2, double k15, double k1875) {
    const double y = __builtin_amdgcn_rsq(r2);
    const double y2 = y * y;
    const double e = __builtin_fma(-r2, y2, 1.0);
    const double s = __builtin_fma(e, __builtin_fma(e, k1875, k15), 1.0);
    return (y2 * y) * s;
}

// Screen: a pair can be flagged by the encounter test only if its separation
// rho satisfies rho < (rc + |w| dt)(1 + 5e-8), w the relative velocity (each
// clause of the test, with every rounding error bounded, implies it).  Since
// (rc_i + rc_j + |w| dt)^2 <= 4 rc_i^2 + 4 rc_j^2 + 2 |w|^2 dt^2, a pair with
//   r2 >= q_i + q_j + D |v_j - v_i|^2,  q = 4 (1 + 2^-20) rc^2,  D = 2 (1 + 2^-20) dt^2
// is certainly not flagged (the 2^-20 margin dominates every rounding error).
// The velocity term is expanded so that a pair costs one add, three FMAs and
// a compare:  q_i + q_j + D |v_j - v_i|^2 = Q_i + Q_j + u_i . v_j  with
// Q = q + D |v|^2 and u = -2 D v per body.  The expanded form cancels when
// v_i ~ v_j; its rounding error is below 16 eps (Q_i + Q_j) (|u_i . v_j| <=
// Q_i + Q_j), so each Q is inflated by 2^-40 (Q_i + Q_j) >> 16 eps (Q_i + Q_j),
// which keeps the computed threshold above the exact one.  A NaN anywhere
// makes the pair a candidate, so the exact test decides it.
// The register-side body carries u, the LDS-side body v.
__device__ __forceinline__ bool screen(double r2, double ux, double uy, double uz, double Qi, double vx,
                                       double vy, double vz, double Qj) {
    const double thr = __builtin_fma(uz, vz, __builtin_fma(uy, vy, __builtin_fma(ux, vx, Qi + Qj)));
    return !(r2 >= thr);
}

// The same screen in single precision (SYMBA_SCREEN_FP32).  Each body's
// screen data (u or v, and Q) is rounded to FP32 and packed two floats per
// double: (x, y) of u or v in one, (z, Q) in the other.  Q is first inflated
// by a further 2^-16 and raised to at least FLT_MIN.  Let A = Q_i + Q_j +
// u_i . v_j be the FP64 screen's threshold in exact arithmetic (0 <= A <=
// 2 (Q_i + Q_j), as |u_i . v_j| <= Q_i + Q_j).  Rounding the six inputs and
// the four operations moves the computed threshold by at most about
// 9 * 2^-24 (Q_i + Q_j), and rounding r2 to FP32 moves it by a relative
// 2^-24, at most 2 * 2^-24 (Q_i + Q_j) where r2 is near A; the 2^-16
// inflation adds 256 * 2^-24 (Q_i + Q_j).  So a pair rejected here has r2
// >= A and is rejected by the FP64 screen as well: no false negatives.  A
// body whose Q exceeds 2^100 (or is NaN) gets Q = NaN, which makes all its
// pairs candidates, so no FP32 overflow can hide a pair; an r2 beyond the
// FP32 range becomes +inf and is rejected correctly.
constexpr double kScreenInflate32 = 1.0 + 0x1p-16;

__device__ __forceinline__ double pack2(float a, float b) {
    return __hiloint2double(__float_as_int(b), __float_as_int(a));
}
__device__ __forceinline__ float lo_of(double v) { return __int_as_float(__double2loint(v)); }
__device__ __forceinline__ float hi_of(double v) { return __int_as_float(__double2hiint(v)); }

__device__ __forceinline__ bool screen32(double r2, double uxy, double uzq, double vxy, double vzq) {
    const float thr = __builtin_fmaf(lo_of(uzq), lo_of(vzq),
                                     __builtin_fmaf(hi_of(uxy), hi_of(vxy),
                                                    __builtin_fmaf(lo_of(uxy), lo_of(vxy),
                                                                   hi_of(uzq) + hi_of(vzq))));
    return !((float)r2 >= thr);
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

// The union-find forest is stored as offsets to the parent: up[x] = x - parent(x),
// 0 for a root.  All-zero is the empty forest whatever slice of the scratch a
// problem is given, so the between-calls state needs no per-slice setup.
__device__ __forceinline__ int uf_load(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void uf_store(int32_t *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x, with path halving: every other node on the walk is re-pointed at
// its grandparent, so trees stay shallow however the unions interleave.
// Parents only ever decrease and a grandparent is an ancestor, so every
// offset read is positive and points at an ancestor; x strictly decreases and
// the walk ends at a root.  Only non-roots are re-pointed (the hooking CAS
// only ever targets roots), and an offset outside (0, x] cannot occur and
// stops the walk.
__device__ __forceinline__ int uf_find(int32_t *up, int x) {
    while (true) {
        const int off = uf_load(up + x);
        if (off <= 0 || off > x) return x;
        const int p = x - off;
        const int off2 = uf_load(up + p);
        if (off2 <= 0 || off2 > p) return p;
        const int g = p - off2;
        uf_store(up + x, x - g);
        x = g;
    }
}

// Lock-free union: hook the larger root under the smaller one with a CAS on
// its (zero) offset and retry if another lane or wave re-hooked it first.  A
// root stays the minimum of its tree, so the final roots are the component
// minima whatever the interleaving.
__device__ __forceinline__ void uf_unite(int32_t *up, int a, int b) {
    while (true) {
        a = uf_find(up, a);
        b = uf_find(up, b);
        if (a == b) return;
        if (a > b) {
            const int t = a;
            a = b;
            b = t;
        }
        int expected = 0;
        if (__hip_atomic_compare_exchange_strong(up + b, &expected, b - a, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
    }
}

// Bucket of a pair by its smaller index: nb buckets in index order, so that
// the canonical (lexicographic) pair order is bucket by bucket.
__device__ __forceinline__ int bucket_of(const Desc &d, int a) { return (int)(((int64_t)a * d.nb) / d.n); }

// Exact test of one candidate per lane (wave-collective), given as positions
// in the order the tile kernel reads (the binned copy holds the same values):
// flagged pairs are reported by the caller's indices, appended (wave ballot +
// prefix, one atomic per wave) and grouped at once.
__device__ __forceinline__ void test_and_group(const Desc &d, bool valid, int i, int j) {
    bool flag = false;
    if (valid && i < d.n && j < d.n)
        flag = encounter_test(d.bx[j] - d.bx[i], d.by[j] - d.by[i], d.bz[j] - d.bz[i], d.bvx[j] - d.bvx[i],
                              d.bvy[j] - d.bvy[i], d.bvz[j] - d.bvz[i], d.brh[i], d.brh[j], d.f, d.dt);
    if (flag && d.bidx) {  // binned position -> caller's index
        i = d.bidx[i];
        j = d.bidx[j];
    }
    const int a = i < j ? i : j, b = i < j ? j : i;
    const unsigned long long fm = __ballot(flag);
    if (fm == 0) return;
    const int leader = __ffsll((long long)fm) - 1;
    unsigned long long base = 0;
    if (lane() == leader) base = atomicAdd(d.ctr + kCtrPairs, (unsigned long long)__popcll(fm));
    if (flag) {  // the union does not need the slot, so it overlaps the reservation
        d.touched[a] = 1;
        d.touched[b] = 1;
        atomicAdd(d.bcnt + bucket_of(d, a), 1);
        uf_unite(d.parent, a, b);
    }
    base = __shfl(base, leader);
    if (flag) {
        const unsigned long long pos = base + (unsigned long long)prefix_count(fm);
        if (pos < (unsigned long long)d.pair_scratch_cap) d.pairs[pos] = make_int2(a, b);
    }
}

// Exact test of up to 64 queued candidates (positions), one per lane.  The
// revisits never queue padding of the triangle; a field task's padding past n
// is rejected by the test's range check.
__device__ __forceinline__ void drain(const Desc &d, const Queue &Q, int head, int count) {
    if (lane() == 0)
        atomicAdd(d.stats + kStatCandidates + (blockIdx.x & (kStatCandLanes - 1)), (unsigned long long)count);
    const bool mine = lane() < count;
    uint2 c = make_uint2(0u, 0u);
    if (mine) c = Q.q[(head + lane()) & Q.mask];
    test_and_group(d, mine, (int)c.x, (int)c.y);
}

// Append this lane's candidate (i, j) if `c`; the mask is the wave's ballot of c.
__device__ __forceinline__ void push(Queue &Q, unsigned long long mask, bool c, int64_t i, int64_t j) {
    if (c) Q.q[(Q.tail + prefix_count(mask)) & Q.mask] = make_uint2((unsigned)i, (unsigned)j);
    Q.tail += __popcll(mask);
}

// Keeps fewer than 64 candidates outstanding after every step, so one step's
// pushes (at most 64 per slot) always fit the queue.
// Orders LDS accesses between the lanes of one wave (the queue is private to
// its wave, so no workgroup barrier is involved).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void maybe_drain(const Desc &d, Queue &Q) {
    if (Q.tail - Q.head >= kWave) {
        wave_sync();
        do {
            drain(d, Q, Q.head, kWave);
            Q.head += kWave;
        } while (Q.tail - Q.head >= kWave);
        wave_sync();
    }
}

__device__ __forceinline__ void drain_rest(const Desc &d, Queue &Q) {
    wave_sync();
    while (Q.tail - Q.head > 0) {
        const int c = (Q.tail - Q.head) < kWave ? (Q.tail - Q.head) : kWave;
        drain(d, Q, Q.head, c);
        Q.head += c;
    }
}

// One body as the tile kernel uses it (read at its position in the binned
// order, see k_bin).  An LDS-side body carries its velocity
// in (vx, vy, vz), a register-side body the screen's u = -2 D v; Q is the
// screen's Q = (1 + 2^-40) (4 (1 + 2^-20) (f rh)^2 + D |v|^2).
struct Body {
    double x, y, z, m, vx, vy, vz, Q;
};

// The inputs of one body as read from memory, held in registers until the
// task's staging.  Entries past the end of their segment are padding: far
// away (x = 2^300, beyond every valid position), massless and at rest.
struct Raw {
    double x, y, z, m, vx, vy, vz, rh;
};

__device__ __forceinline__ Raw load_raw(const Desc &d, int64_t k, int64_t limit) {
    Raw r;
    if (k < limit) {
        r.x = d.bx[k];
        r.y = d.by[k];
        r.z = d.bz[k];
        r.m = d.bm[k];
        r.vx = d.bvx[k];
        r.vy = d.bvy[k];
        r.vz = d.bvz[k];
        r.rh = d.brh[k];
    } else {
        r.x = kPadPos;
        r.y = r.z = r.m = r.vx = r.vy = r.vz = r.rh = 0.0;
    }
    return r;
}

template <bool REG, bool F32>
__device__ __forceinline__ Body body_of(const Desc &d, const Raw &r) {
    Body b;
    if (r.x != kPadPos) {
        b.x = r.x;
        b.y = r.y;
        b.z = r.z;
        b.m = r.m;
        const double rc = d.f * r.rh;
        const double D = d.screen_dt2;
        const double v2 = __builtin_fma(r.vz, r.vz, __builtin_fma(r.vy, r.vy, r.vx * r.vx));
        b.Q = kScreenInflate * __builtin_fma(D, v2, kScreenQ * (rc * rc));
        const double s = REG ? -2.0 * D : 1.0;
        b.vx = s * r.vx;
        b.vy = s * r.vy;
        b.vz = s * r.vz;
    } else {  // padding
        b.x = kPadPos;
        b.y = b.z = b.m = b.vx = b.vy = b.vz = b.Q = 0.0;
    }
    if constexpr (F32) {  // screen data as FP32, packed (see screen32)
        const float Q = b.Q <= 0x1p100 ? fmaxf((float)(b.Q * kScreenInflate32), FLT_MIN) : __builtin_nanf("");
        b.vx = pack2((float)b.vx, (float)b.vy);
        b.vy = pack2((float)b.vz, Q);
        b.vz = b.Q = 0.0;
    }
    return b;
}

template <bool REG, bool F32>
__device__ __forceinline__ Body load_body(const Desc &d, int64_t k, int64_t limit) {
    return body_of<REG, F32>(d, load_raw(d, k, limit));
}

// Stage bodies [j0, j0 + 64 nq) (entries past `limit` become padding) into
// tiles 0..nq-1 of the workgroup's LDS, each entry also at +64.  All threads
// of the workgroup take part; the caller brackets it with barriers.
template <int RS, bool F32>
__device__ __forceinline__ void stage(const Desc &d, TaskLds<RS> &L, int64_t j0, int nq, int64_t limit) {
    for (int e = (int)threadIdx.x; e < nq * kWave; e += kTaskThreads) {
        const Body b = load_body<false, F32>(d, j0 + e, limit);
        const int q = e / kWave, jj = e % kWave;
        L.tile.xy[q][jj] = L.tile.xy[q][jj + kWave] = make_double2(b.x, b.y);
        L.tile.zm[q][jj] = L.tile.zm[q][jj + kWave] = make_double2(b.z, b.m);
        L.tile.vxy[q][jj] = L.tile.vxy[q][jj + kWave] = make_double2(b.vx, b.vy);
        L.tile.vzq[q][jj] = L.tile.vzq[q][jj + kWave] = make_double2(b.vz, b.Q);
    }
}

template <int RS, bool F32>
__device__ __forceinline__ Body tile_body(const TaskLds<RS> &L, int q, int idx) {
    const double2 a = L.tile.xy[q][idx], b = L.tile.zm[q][idx], c = L.tile.vxy[q][idx];
    if constexpr (F32) return Body{a.x, a.y, b.x, b.y, c.x, c.y, 0.0, 0.0};  // packed screen data
    const double2 e = L.tile.vzq[q][idx];
    return Body{a.x, a.y, b.x, b.y, c.x, c.y, e.x, e.y};
}

// The screen of a pair from its register-side and LDS-side bodies.
template <bool F32>
__device__ __forceinline__ bool screen_pair(double r2, const Body &reg, const Body &lds) {
    if constexpr (F32)
        return screen32(r2, reg.vx, reg.vy, lds.vx, lds.vy);
    else
        return screen(r2, reg.vx, reg.vy, reg.vz, reg.Q, lds.vx, lds.vy, lds.vz, lds.Q);
}

// Position and mass of a tile entry (the screen-free loops read nothing else).
template <int RS>
__device__ __forceinline__ Body tile_pos(const TaskLds<RS> &L, int q, int idx) {
    const double2 a = L.tile.xy[q][idx], b = L.tile.zm[q][idx];
    return Body{a.x, a.y, b.x, b.y, 0.0, 0.0, 0.0, 0.0};
}

// Box record of massive tile t (64 bodies from position 64 t) and of field
// tile g (64 bodies from position n_tri + 64 g); -1 for a tile past the end.
__device__ __forceinline__ int64_t tri_box(const Desc &d, int64_t t) { return t < d.n_tboxes ? t : -1; }
__device__ __forceinline__ int64_t field_box(const Desc &d, int64_t g) {
    return d.n_tboxes + g < d.n_boxes ? d.n_tboxes + g : -1;
}

// Tile boxes of the binned order: no pair between tile a and tile b (indices
// into the box records) can pass the screen, so none can be flagged.  Over
// any i in a and j in b, |x_j - x_i| is at least the gap between the
// position boxes, |v_j - v_i|^2 is at most the sum of the squared widest
// velocity differences, and q_i, q_j at most the tiles' largest q; the pair
// screen passes only if r2 < q_i + q_j + D |v_j - v_i|^2, so a gap with
//   gap^2 (1 - 2^-30) >= (qmax_a + qmax_b + D wmax^2) (1 + 2^-30)
// (the factors cover the rounding of these few operations) rules out every
// pair.  A tile with a non-finite value has qmax = NaN and is never ruled out.
__device__ __forceinline__ bool tiles_apart(const Desc &d, int64_t a, int64_t b) {
    if (a < 0 || b < 0) return true;  // a tile of padding only: massless and far away
    const double *A = d.tbox + a * kBoxDoubles, *Bq = d.tbox + b * kBoxDoubles;
    double gap2 = 0.0, w2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double g = fmax(0.0, fmax(Bq[k] - A[3 + k], A[k] - Bq[3 + k]));
        gap2 = __builtin_fma(g, g, gap2);
        const double w = fmax(Bq[9 + k] - A[6 + k], A[9 + k] - Bq[6 + k]);
        w2 = __builtin_fma(w, w, w2);
    }
    const double thr = __builtin_fma(w2, d.screen_dt2, A[12] + Bq[12]);
    return gap2 * (1.0 - 0x1p-30) >= thr * (1.0 + 0x1p-30);
}

__device__ __forceinline__ double rotate_dpp(double v) {
    // lane l receives the value of lane (l + 1) mod 64 (DPP wave_rol:1); every
    // lane has a source, so no "old" value is needed
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x134, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x134, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

template <int R>
struct Slots {
    Body b[R];
    double ax[R], ay[R], az[R];
};

// A partial sum is written through to memory (an agent-scope store): the
// final kernel reads it from another XCD anyway, and lines the tile kernel
// leaves clean need no write-back at its end (measured 61.4 -> 59.8 us on the
// 10k disk).
__device__ __forceinline__ void store_through(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void write_partial(const Desc &d, int64_t slot, int64_t k, double ax,
                                              double ay, double az) {
    if (k < d.n_tri) {
        double *p = d.partial + slot * 3 * d.n_tri + k;
        store_through(p, ax);
        store_through(p + d.n_tri, ay);
        store_through(p + 2 * d.n_tri, az);
    }
}

// Screen of the pairs of step t (tile entry l + t) against the first NACT
// slots, pushing the candidates.  Used to revisit the rare steps that had one;
// it repeats the hot loop's screen operation for operation.
template <int R, int RS, int NACT, bool F32>
__device__ __forceinline__ void push_step(const Desc &d, const TaskLds<RS> &L, int q, const Slots<R> &S,
                                          int64_t ib, int64_t js, int t, Queue &Q) {
    const int l = lane();
    const Body J = tile_body<RS, F32>(L, q, l + t);
    const int64_t j = js + ((l + t) & (kWave - 1));
#pragma unroll
    for (int r = 0; r < NACT; ++r) {
        const Body &I = S.b[r];
        const double dx = J.x - I.x, dy = J.y - I.y, dz = J.z - I.z;
        const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
        // padding past n_tri (which may hold field bodies' positions) never
        // becomes a candidate, even next to a body with an infinite q
        const int64_t i = ib + r * kWave + l;
        const bool c = i < d.n_tri && j < d.n_tri && screen_pair<F32>(r2, I, J);
        const unsigned long long mask = __ballot(c);
        if (mask) push(Q, mask, c, i, j);
    }
    maybe_drain(d, Q);
}

// This wave's 16 steps [t0, t0 + 16) of tile q against the first NACT slots:
// both sides of every pair are accumulated.  Lane l starts with the sums of
// tile entry (l + t0) mod 64 and ends with those of entry (l + t0 + 16) mod 64.
// Steps whose screen passed anywhere in the wave are only marked in a scalar
// bit mask; the candidates are pushed afterwards (no branch in the loop).
template <int R, int RS, int NACT, bool SCR, bool F32>
__device__ __forceinline__ void rotation_range(const Desc &d, const TaskLds<RS> &L, int q, Slots<R> &S,
                                               int64_t ib, int64_t js, int t0, Queue &Q, double &ajx,
                                               double &ajy, double &ajz) {
    const int l = lane();
    ajx = ajy = ajz = 0.0;
    unsigned pending = 0;
    Body Jn = SCR ? tile_body<RS, F32>(L, q, l + t0) : tile_pos(L, q, l + t0);
#pragma unroll kRotUnroll
    for (int u = 0; u < kSteps; ++u) {
        const Body J = Jn;
        // one step ahead: the LDS latency hides behind this step
        Jn = SCR ? tile_body<RS, F32>(L, q, l + t0 + u + 1) : tile_pos(L, q, l + t0 + u + 1);
        unsigned long long any = 0;
#pragma unroll
        for (int r = 0; r < NACT; ++r) {
            const Body &I = S.b[r];
            const double dx = J.x - I.x, dy = J.y - I.y, dz = J.z - I.z;
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            const double qf = inv_r3(r2, d.k15, d.k1875);
            const double fi = J.m * qf, fj = I.m * qf;
            S.ax[r] = __builtin_fma(fi, dx, S.ax[r]);
            S.ay[r] = __builtin_fma(fi, dy, S.ay[r]);
            S.az[r] = __builtin_fma(fi, dz, S.az[r]);
            ajx = __builtin_fma(-fj, dx, ajx);
            ajy = __builtin_fma(-fj, dy, ajy);
            ajz = __builtin_fma(-fj, dz, ajz);
            if (SCR)
                any |= __builtin_amdgcn_ballot_w64(screen_pair<F32>(r2, I, J));
        }
        if (SCR) pending |= nonzero(any) << u;
        ajx = rotate_dpp(ajx);
        ajy = rotate_dpp(ajy);
        ajz = rotate_dpp(ajz);
    }
    while (pending) {
        const int u = __builtin_ctz(pending);
        pending &= pending - 1;
        push_step<R, RS, NACT, F32>(d, L, q, S, ib, js, t0 + u, Q);
    }
}

// Slot QS against its own tile (a diagonal sub-block), this wave's steps of
// 1..63: each unordered pair is met from both ends, only the stationary side
// is accumulated, and the pair is screened once (from the lane whose partner
// is 1..31 steps ahead, or 32 steps ahead for the lower half of the wave).
template <int R, int RS, int QS, bool F32>
__device__ __forceinline__ void diagonal_range(const Desc &d, const TaskLds<RS> &L, Slots<R> &S,
                                               int64_t ib, int t0, Queue &Q) {
    const int l = lane();
    unsigned pending = 0;
    for (int t = (t0 > 0 ? t0 : 1); t < t0 + kSteps; ++t) {
        const Body J = tile_body<RS, F32>(L, QS, l + t);
        const Body &I = S.b[QS];
        const double dx = J.x - I.x, dy = J.y - I.y, dz = J.z - I.z;
        const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
        const double fi = J.m * inv_r3(r2, d.k15, d.k1875);
        S.ax[QS] = __builtin_fma(fi, dx, S.ax[QS]);
        S.ay[QS] = __builtin_fma(fi, dy, S.ay[QS]);
        S.az[QS] = __builtin_fma(fi, dz, S.az[QS]);
        const bool owner = (t < kWave / 2) || (t == kWave / 2 && l < kWave / 2);
        const bool c = owner && screen_pair<F32>(r2, I, J);
        pending |= nonzero(__builtin_amdgcn_ballot_w64(c)) << (t - t0);
    }
    while (pending) {
        const int t = t0 + __builtin_ctz(pending);
        pending &= pending - 1;
        const Body J = tile_body<RS, F32>(L, QS, l + t);
        const Body &I = S.b[QS];
        const double dx = J.x - I.x, dy = J.y - I.y, dz = J.z - I.z;
        const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
        const bool owner = (t < kWave / 2) || (t == kWave / 2 && l < kWave / 2);
        const int64_t i = ib + QS * kWave + l, j = ib + QS * kWave + ((l + t) & (kWave - 1));
        const bool c = owner && i < d.n_tri && j < d.n_tri &&
                       screen_pair<F32>(r2, I, J);
        const unsigned long long mask = __ballot(c);
        if (mask) push(Q, mask, c, i, j);
        maybe_drain(d, Q);
    }
}

template <int R, int RS, int QS, bool F32>
__device__ __forceinline__ void diagonal_tiles(const Desc &d, const TaskLds<RS> &L, Slots<R> &S, int64_t ib,
                                               int t0, Queue &Q, double (&aj)[R][3]) {
    if constexpr (QS < R) {
        if constexpr (QS > 0)
            rotation_range<R, RS, QS, true, F32>(d, L, QS, S, ib, ib + QS * kWave, t0, Q, aj[QS][0], aj[QS][1],
                                            aj[QS][2]);
        else
            aj[0][0] = aj[0][1] = aj[0][2] = 0.0;
        diagonal_range<R, RS, QS, F32>(d, L, S, ib, t0, Q);
        diagonal_tiles<R, RS, QS + 1, F32>(d, L, S, ib, t0, Q, aj);
    }
}

// Sums of the four waves' partial accelerations of a task in a fixed order,
// written to the partial slots: the first NR stationary tiles (bodies from
// base_i) to slot slot_i, the streamed ones (from base_j) to slot slot_j.  A
// diagonal block pair (diag) has one set of bodies: both sides are added and
// written to slot_i.  Called after a barrier that ends every wave's use of
// the tiles (the sums reuse their LDS).
template <int R, int RS, int NR>
__device__ __forceinline__ void write_sums(const Desc &d, TaskLds<RS> &L, const Slots<R> &S,
                                           const double (&aj)[R][3], int t0, bool diag, int64_t slot_i,
                                           int64_t base_i, int64_t slot_j, int64_t base_j) {
    const int l = lane(), w = wave_id();
    const int jend = (l + t0 + kSteps) & (kWave - 1);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        L.comb[0][w][r][0][l] = S.ax[r];
        L.comb[0][w][r][1][l] = S.ay[r];
        L.comb[0][w][r][2][l] = S.az[r];
        L.comb[1][w][r][0][jend] = aj[r][0];
        L.comb[1][w][r][1][jend] = aj[r][1];
        L.comb[1][w][r][2][jend] = aj[r][2];
    }
    __syncthreads();
    for (int e = (int)threadIdx.x; e < 2 * NR * kWave; e += kTaskThreads) {
        const int side = e / (NR * kWave), idx = e % (NR * kWave), r = idx / kWave, ll = idx % kWave;
        if (diag && side == 1) continue;
        double sum[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double v = 0.0;
            for (int ww = 0; ww < kTaskWaves; ++ww) v += L.comb[side][ww][r][c][ll];
            if (diag)
                for (int ww = 0; ww < kTaskWaves; ++ww) v += L.comb[1][ww][r][c][ll];
            sum[c] = v;
        }
        if (side == 0)
            write_partial(d, slot_i, base_i + idx, sum[0], sum[1], sum[2]);
        else
            write_partial(d, slot_j, base_j + idx, sum[0], sum[1], sum[2]);
    }
}

// A task of the tile kernel, decoded from its index in the problem's task
// list: a whole block pair (I, J) of the folded triangle, a tile pair of a
// split diagonal, or a field block against every massive row.
struct TaskInfo {
    int kind;                 // kTaskWhole, kTaskSplit or kTaskField
    int nq, nstat;            // streamed and stationary tiles
    int r, q;                 // split: stationary tile of I, streamed tile of J
    int64_t I, J;             // blocks of the pair
    int64_t ib, jb;           // first stationary and first streamed body
    int64_t slot_i, slot_j;   // split: partial slots of the stationary and the streamed side
    int64_t fb, sg;           // field: field block and segment of massive rows
};

constexpr int kTaskWhole = 0, kTaskSplit = 1, kTaskField = 2;

template <int R>
__device__ __forceinline__ TaskInfo decode_task(const Desc &d, int64_t lt) {
    TaskInfo T;
    T.r = T.q = 0;
    T.I = T.J = T.ib = T.jb = T.slot_i = T.slot_j = T.fb = T.sg = 0;
    if (lt < d.n_whole) {
        T.kind = kTaskWhole;
        whole_decode(d.B, d.n_split, lt, T.I, T.J);
        T.nq = T.nstat = R;
        T.ib = T.I * R * kWave;
        T.jb = T.J * R * kWave;
    } else if (lt < d.n_tri_tasks) {
        T.kind = kTaskSplit;
        const SplitTask S = split_decode(d.B, R, lt - d.n_whole);
        T.nq = T.nstat = 1;
        T.r = S.r;
        T.q = S.q;
        T.I = S.I;
        T.J = S.J;
        T.ib = (S.I * R + S.r) * kWave;
        T.jb = (S.J * R + S.q) * kWave;
        T.slot_i = S.slot_i;
        T.slot_j = S.slot_j;
    } else {
        T.kind = kTaskField;
        T.nq = T.nstat = 0;
        field_decode(d.n_fblocks, d.n_fslots, lt - d.n_tri_tasks, T.fb, T.sg);
    }
    return T;
}

// Bodies a triangle task reads, one list per workgroup: its streamed tiles
// (entries [0, 64 nq)) then its stationary tiles; thread t takes entries t
// and t + 256, so every body is read from memory once per task.  PF entries
// per thread cover the largest task (2 R 64 bodies).
template <int R>
constexpr int body_slots() { return R == 4 ? 2 : 1; }

template <int PF>
__device__ __forceinline__ void load_task_bodies(const Desc &d, const TaskInfo &T, Raw (&pf)[PF]) {
    if (T.kind == kTaskField) return;
    const int nstr = T.nq * kWave, nstat = T.nstat * kWave;
#pragma unroll
    for (int p = 0; p < PF; ++p) {
        const int k = (int)threadIdx.x + p * kTaskThreads;
        if (k < nstr)
            pf[p] = load_raw(d, T.jb + k, d.n_tri);
        else if (k - nstr < nstat)
            pf[p] = load_raw(d, T.ib + (k - nstr), d.n_tri);
    }
}

// The loaded bodies of a triangle task into LDS: streamed ones in their
// screen form for the LDS side (each entry also at +64), stationary ones in
// the form for the register side (each of the four waves then reads them
// into registers).  Every thread of the workgroup takes part; the caller
// brackets it with barriers.
template <int RS, bool F32, int PF>
__device__ __forceinline__ void stage_loaded(const Desc &d, TaskLds<RS> &L, const TaskInfo &T,
                                                 const Raw (&pf)[PF]) {
    const int nstr = T.nq * kWave, nstat = T.nstat * kWave;
#pragma unroll
    for (int p = 0; p < PF; ++p) {
        const int k = (int)threadIdx.x + p * kTaskThreads;
        if (k < nstr) {
            const Body b = body_of<false, F32>(d, pf[p]);
            const int q = k / kWave, jj = k % kWave;
            L.tile.xy[q][jj] = L.tile.xy[q][jj + kWave] = make_double2(b.x, b.y);
            L.tile.zm[q][jj] = L.tile.zm[q][jj + kWave] = make_double2(b.z, b.m);
            L.tile.vxy[q][jj] = L.tile.vxy[q][jj + kWave] = make_double2(b.vx, b.vy);
            L.tile.vzq[q][jj] = L.tile.vzq[q][jj + kWave] = make_double2(b.vz, b.Q);
        } else if (k - nstr < nstat) {
            const Body b = body_of<true, F32>(d, pf[p]);
            const int e = k - nstr;
            L.tile.sxy[e] = make_double2(b.x, b.y);
            L.tile.szm[e] = make_double2(b.z, b.m);
            L.tile.svxy[e] = make_double2(b.vx, b.vy);
            L.tile.svzq[e] = make_double2(b.vz, b.Q);
        }
    }
}

// Stationary body e of the staged block, as the lane keeps it in registers.
template <int RS>
__device__ __forceinline__ Body stationary_body(const TaskLds<RS> &L, int e) {
    const double2 a = L.tile.sxy[e], b = L.tile.szm[e], c = L.tile.svxy[e], f = L.tile.svzq[e];
    return Body{a.x, a.y, b.x, b.y, c.x, c.y, f.x, f.y};
}

// Tile pairs of a whole block pair that cannot produce a candidate (binned
// problems only): lane r R + q decides stationary tile r against streamed
// tile q; bit q of the result is set when tile q is apart from every
// stationary tile.
template <int R>
__device__ __forceinline__ unsigned whole_free_tiles(const Desc &d, const TaskInfo &T) {
    const int l = lane();
    const bool apart = l >= R * R || tiles_apart(d, tri_box(d, T.I * R + l / R), tri_box(d, T.J * R + l % R));
    const unsigned long long m = __ballot(apart);
    unsigned free_q = 0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        bool all = true;
#pragma unroll
        for (int r = 0; r < R; ++r) all = all && ((m >> (r * R + q)) & 1ull);
        free_q |= (all ? 1u : 0u) << q;
    }
    return free_q;
}

// Block pair (I, J) of the folded triangle, by the four waves of the
// workgroup, once its blocks are staged and the stationary bodies are in S.
// Partial sums land in slot J for the stationary bodies of block I and in
// slot I for the bodies of block J (slot I for both when I == J).  BIN: the
// problem is binned, so tile pairs that cannot meet run screen-free (bit q of
// free_q).  F32: the pair screen runs in FP32 (screen32).
template <int R, int RS, bool BIN, bool F32>
__device__ __forceinline__ void whole_pair(const Desc &d, TaskLds<RS> &L, Queue &Q, const TaskInfo &T,
                                           Slots<R> &S, unsigned free_q) {
    const int t0 = wave_id() * kSteps;
    double aj[R][3];
    if (T.I != T.J) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (BIN && ((free_q >> q) & 1u))
                rotation_range<R, RS, R, !BIN, F32>(d, L, q, S, T.ib, T.jb + q * kWave, t0, Q, aj[q][0],
                                                    aj[q][1], aj[q][2]);
            else
                rotation_range<R, RS, R, true, F32>(d, L, q, S, T.ib, T.jb + q * kWave, t0, Q, aj[q][0], aj[q][1],
                                                    aj[q][2]);
        }
    } else {
        diagonal_tiles<R, RS, 0, F32>(d, L, S, T.ib, t0, Q, aj);
    }
    __syncthreads();  // every wave is done with the tiles
    write_sums<R, RS, R>(d, L, S, aj, t0, T.I == T.J, T.J, T.ib, T.I, T.jb);
}

// Tile pair of a split diagonal (see split_decode): stationary tile r of
// block I against streamed tile q of block J, both sides accumulated, by the
// four waves of the workgroup as in a whole block pair.
template <int R, int RS, bool BIN, bool F32>
__device__ __forceinline__ void split_pair(const Desc &d, TaskLds<RS> &L, Queue &Q, const TaskInfo &T,
                                           Slots<R> &S, bool apart) {
    const int t0 = wave_id() * kSteps;
    double aj[R][3];
    if (BIN && apart)
        rotation_range<R, RS, 1, !BIN, F32>(d, L, 0, S, T.ib, T.jb, t0, Q, aj[0][0], aj[0][1], aj[0][2]);
    else
        rotation_range<R, RS, 1, true, F32>(d, L, 0, S, T.ib, T.jb, t0, Q, aj[0][0], aj[0][1], aj[0][2]);
    __syncthreads();  // every wave is done with the tile
    write_sums<R, RS, 1>(d, L, S, aj, t0, false, T.slot_i, T.ib, T.slot_j, T.jb);
}

// Rows [u0, u1) (at most 16) of the staged segment (segment row u is massive
// row s0 + u) against the lane's field bodies (one-sided pairs); returns the
// bit mask (bit u - u0) of the rows whose screen passed somewhere in the wave.
template <int RF, int RS, bool SCR, bool F32>
__device__ __forceinline__ unsigned segment_rows(const Desc &d, const TaskLds<RS> &L, int u0, int u1,
                                                 const Body (&fbody)[RF], double (&ax)[RF], double (&ay)[RF],
                                                 double (&az)[RF]) {
    unsigned pending = 0;
    for (int u = u0; u < u1; ++u) {
        // the same massive body in every lane
        const double2 pxy = L.seg.xy[u], pzm = L.seg.zm[u];
        Body I{pxy.x, pxy.y, pzm.x, pzm.y, 0.0, 0.0, 0.0, 0.0};
        if (SCR) {
            const double2 v = L.seg.vxy[u];
            I.vx = v.x;
            I.vy = v.y;
            if constexpr (!F32) {
                const double2 q = L.seg.vzq[u];
                I.vz = q.x;
                I.Q = q.y;
            }
        }
        unsigned long long any = 0;
#pragma unroll
        for (int r = 0; r < RF; ++r) {
            const Body &Fb = fbody[r];
            const double dx = Fb.x - I.x, dy = Fb.y - I.y, dz = Fb.z - I.z;
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            const double fj = I.m * inv_r3(r2, d.k15, d.k1875);
            ax[r] = __builtin_fma(-fj, dx, ax[r]);
            ay[r] = __builtin_fma(-fj, dy, ay[r]);
            az[r] = __builtin_fma(-fj, dz, az[r]);
            if (SCR)
                any |= __builtin_amdgcn_ballot_w64(screen_pair<F32>(r2, Fb, I));
        }
        if (SCR) pending |= nonzero(any) << (u - u0);
    }
    return pending;
}

// Field task: field block fb (RF tiles of 64 field bodies, RF per lane,
// the same in all four waves) against segment sg of the massive rows
// (kFieldSegRows rows from sg kFieldSegRows), staged once; wave w takes a
// contiguous quarter of the segment.  The waves' sums are combined in a
// fixed order and written to the field bodies' partial slot sg; the final
// kernel adds the segments' slots in order.
template <int RF, int RS, bool BIN, bool F32>
__device__ __forceinline__ void field_task(const Desc &d, TaskLds<RS> &L, Queue &Q, int64_t fb, int64_t sg) {
    const int l = lane(), w = wave_id();
    const int64_t f0 = d.n_tri + fb * RF * kWave;
    const int64_t s0 = sg * kFieldSegRows;
    const int64_t left = d.n_rows - s0;
    const int nrows = left < kFieldSegRows ? (int)left : kFieldSegRows;
    Body fbody[RF];
    double ax[RF], ay[RF], az[RF];
#pragma unroll
    for (int r = 0; r < RF; ++r) {
        fbody[r] = load_body<true, F32>(d, f0 + r * kWave + l, d.n);
        ax[r] = ay[r] = az[r] = 0.0;
    }
    // lane q RF + r decides field tile r against the segment's massive tile q
    // (a segment is a whole number of 64-row tiles)
    unsigned free_q = 0;
    if (BIN) {
        const int nq = (nrows + kWave - 1) / kWave;
        const bool apart = l >= nq * RF ||
                           tiles_apart(d, field_box(d, fb * RF + l % RF), tri_box(d, s0 / kWave + l / RF));
        const unsigned long long m = __ballot(apart);
        for (int q = 0; q < nq; ++q) {
            bool all = true;
#pragma unroll
            for (int r = 0; r < RF; ++r) all = all && ((m >> (q * RF + r)) & 1ull);
            free_q |= (all ? 1u : 0u) << q;
        }
    }
    for (int e = (int)threadIdx.x; e < nrows; e += kTaskThreads) {
        const Body b = load_body<false, F32>(d, s0 + e, d.n_rows);
        L.seg.xy[e] = make_double2(b.x, b.y);
        L.seg.zm[e] = make_double2(b.z, b.m);
        L.seg.vxy[e] = make_double2(b.vx, b.vy);
        L.seg.vzq[e] = make_double2(b.vz, b.Q);
    }
    __syncthreads();
    constexpr int kQuarter = kFieldSegRows / kTaskWaves;
    static_assert(kQuarter % kSteps == 0 && kWave % kSteps == 0, "a wave's rows split into whole 16-row runs");
    const int r0 = w * kQuarter, r1 = min(r0 + kQuarter, nrows);
    for (int u0 = r0; u0 < r1; u0 += kSteps) {
        const int u1 = min(u0 + kSteps, r1);
        const bool apart = BIN && ((free_q >> (u0 / kWave)) & 1u);
        unsigned pending = apart ? segment_rows<RF, RS, !BIN, F32>(d, L, u0, u1, fbody, ax, ay, az)
                                 : segment_rows<RF, RS, true, F32>(d, L, u0, u1, fbody, ax, ay, az);
        while (pending) {
            const int u = u0 + __builtin_ctz(pending);
            pending &= pending - 1;
            const double2 pxy = L.seg.xy[u], pzm = L.seg.zm[u], v = L.seg.vxy[u];
            Body I{pxy.x, pxy.y, pzm.x, pzm.y, v.x, v.y, 0.0, 0.0};
            if constexpr (!F32) {
                const double2 q = L.seg.vzq[u];
                I.vz = q.x;
                I.Q = q.y;
            }
#pragma unroll
            for (int r = 0; r < RF; ++r) {
                const Body &Fb = fbody[r];
                const double dx = Fb.x - I.x, dy = Fb.y - I.y, dz = Fb.z - I.z;
                const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                const bool c = screen_pair<F32>(r2, Fb, I);
                const unsigned long long mask = __ballot(c);
                if (mask) push(Q, mask, c, s0 + u, f0 + r * kWave + l);
            }
            maybe_drain(d, Q);
        }
    }
    __syncthreads();  // every wave is done with the rows (the sums reuse their LDS)
#pragma unroll
    for (int r = 0; r < RF; ++r) {
        L.comb[0][w][r][0][l] = ax[r];
        L.comb[0][w][r][1][l] = ay[r];
        L.comb[0][w][r][2][l] = az[r];
    }
    __syncthreads();
    const int64_t n_field = d.n - d.n_tri;
    for (int e = (int)threadIdx.x; e < RF * kWave; e += kTaskThreads) {
        const int r = e / kWave, ll = e % kWave;
        const int64_t fpos = f0 + e - d.n_tri;
        if (fpos >= n_field) continue;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double v = 0.0;
            for (int ww = 0; ww < kTaskWaves; ++ww) v += L.comb[0][ww][r][c][ll];
            store_through(d.fpartial + (3 * sg + c) * n_field + fpos, v);
        }
    }
}

// Problem owning global index `key` of the task list (which 0), of the
// final-kernel blocks (which 1) or of the k_indirect blocks (which 2): the
// last problem whose base is not above it.
__device__ inline int problem_of(const Desc *descs, int n_desc, int64_t key, int which) {
    int lo = 0, hi = n_desc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t base =
            which == 0 ? descs[mid].task_base : (which == 1 ? descs[mid].fin_base : descs[mid].ind_base);
        if (base <= key)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Without binning the tile kernel's inputs are the caller's arrays and no
// index map or box exists: said here at compile time, so that the unbinned
// kernel keeps no registers for them.
template <bool BIN>
__device__ __forceinline__ Desc tile_view(const Desc &desc) {
    Desc d = desc;
    if (!BIN) {
        d.bx = desc.x; d.by = desc.y; d.bz = desc.z; d.bm = desc.m;
        d.bvx = desc.vx; d.bvy = desc.vy; d.bvz = desc.vz; d.brh = desc.rh;
        d.bidx = nullptr;
        d.tbox = nullptr;
    }
    return d;
}

// One task per workgroup (the hardware dispatcher hands tasks to free
// workgroup slots): the task's bodies are loaded once, each by one thread,
// and staged in LDS, the stationary ones read back into registers.
template <int R, int RF, bool BIN, bool F32>
__device__ __forceinline__ void tile_task_once(const Desc &desc, int64_t t) {
    constexpr int RS = R > RF ? R : RF;
    constexpr int PF = body_slots<R>();
    __shared__ TaskLds<RS> L;
    __shared__ uint2 qbuf[kTaskWaves][queue_cap(RS)];
    Queue Q{qbuf[wave_id()], queue_cap(RS) - 1, 0, 0};
    const Desc d = tile_view<BIN>(desc);
    const TaskInfo T = decode_task<R>(d, t - d.task_base);
    if (T.kind == kTaskField) {
        field_task<RF, RS, BIN, F32>(d, L, Q, T.fb, T.sg);
    } else {
        Raw raw[PF];
        load_task_bodies(d, T, raw);
        unsigned free_q = 0;
        bool apart = false;
        if (BIN) {
            if (T.kind == kTaskWhole) {
                if (T.I != T.J) free_q = whole_free_tiles<R>(d, T);
            } else {
                apart = __builtin_amdgcn_readfirstlane(
                            tiles_apart(d, tri_box(d, T.I * R + T.r), tri_box(d, T.J * R + T.q)) ? 1 : 0) != 0;
            }
        }
        stage_loaded<RS, F32, PF>(d, L, T, raw);
        __syncthreads();
        Slots<R> S;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            S.b[r] = stationary_body<RS>(L, r * kWave + lane());
            S.ax[r] = S.ay[r] = S.az[r] = 0.0;
        }
        if (T.kind == kTaskWhole)
            whole_pair<R, RS, BIN, F32>(d, L, Q, T, S, free_q);
        else
            split_pair<R, RS, BIN, F32>(d, L, Q, T, S, apart);
    }
    // the candidates left in this wave's queue are tested after the
    // workgroup's barriers, so the other waves never wait on the test
    drain_rest(d, Q);
}

// One problem: the descriptor is a kernel argument (scalar registers).
template <int R, int RF, bool BIN, bool F32>
__global__ __launch_bounds__(kTaskThreads) __attribute__((amdgpu_waves_per_eu(waves_per_eu(R))))
void k_tiles(const Desc d) {
    tile_task_once<R, RF, BIN, F32>(d, task_in_order(d.n_tri_tasks, d.n_tasks, blockIdx.x));
}

// Many problems of one tile size: every block finds its problem by the task
// bases (descs is the group's slice of the launch's descriptors).
template <int R, int RF, bool BIN, bool F32>
__global__ __launch_bounds__(kTaskThreads) __attribute__((amdgpu_waves_per_eu(waves_per_eu(R))))
void k_tiles_batch(const Desc *__restrict__ descs, int n_desc, int64_t task_begin) {
    const int64_t t = task_begin + blockIdx.x;
    tile_task_once<R, RF, BIN, F32>(descs[problem_of(descs, n_desc, t, 0)], t);
}

// ---------------------------------------------------------------------------
// Binning: bodies of each segment (massive [0, n_tri), field [n_tri, n)) are
// put in a spatial order so that the 64-body tiles are compact and most tile
// pairs are provably too far apart for any encounter (tiles_apart), which
// lets the tile kernel skip the screen for them.  The order only changes how
// the work is grouped: it is a deterministic function of the input (cell of a
// Morton-ordered grid over the segment's bounding box, ties by index), so
// results stay reproducible.  Six small kernels: bounding box, cell counts,
// cell starts, cell fill, order within cells (with the copy of the inputs in
// the binned order), tile boxes.

constexpr int kBinBlock = 256;          // threads of the per-body binning kernels
constexpr int kBinPerThread = 2;        // bodies per thread (their loads in flight together)
constexpr int kBinChunk = kBinBlock * kBinPerThread;
constexpr int kBinCellBits = 11;
constexpr int kBinCells = 1 << kBinCellBits;
constexpr int kBinScanThreads = 1024;

// Order-preserving map of a double to an unsigned integer (for atomic min/max).
__device__ __forceinline__ unsigned long long ord_key(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double ord_value(unsigned long long u) {
    const unsigned long long b = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
    return __longlong_as_double((long long)b);
}

struct Grid {
    double lo[3], scale[3];
    int bits[3];
};

// The segment's grid: cells of the bounding box, with the bits given one at
// a time to the axis whose cells are longest (flat, empty or non-finite axes
// get none).  bbox holds max(~key(min)) and max(key(max)) per axis.
__device__ __forceinline__ Grid make_grid(const unsigned long long *bbox) {
    Grid g;
    double ext[3];
    for (int a = 0; a < 3; ++a) {
        const double mn = ord_value(~bbox[a]), mx = ord_value(bbox[3 + a]);
        ext[a] = mx - mn;
        if (!(ext[a] > 0.0) || !isfinite(ext[a])) ext[a] = 0.0;
        g.lo[a] = isfinite(mn) ? mn : 0.0;
        g.bits[a] = 0;
    }
    for (int b = 0; b < kBinCellBits; ++b) {
        int best = -1;
        double len = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double l = ext[a] / (double)(1 << g.bits[a]);
            if (l > len) {
                len = l;
                best = a;
            }
        }
        if (best < 0) break;
        ++g.bits[best];
    }
    for (int a = 0; a < 3; ++a) g.scale[a] = g.bits[a] ? (double)(1 << g.bits[a]) / ext[a] : 0.0;
    return g;
}

// Grid cell of a position: each coordinate quantized to its axis' bits (NaN
// and out-of-range values clamp into the grid), the bits interleaved from the
// most significant level down (Morton order).
__device__ __forceinline__ int grid_cell(const Grid &g, double x, double y, double z) {
    const double c[3] = {x, y, z};
    int q[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double top = (double)((1 << g.bits[a]) - 1);
        q[a] = (int)fmin(fmax((c[a] - g.lo[a]) * g.scale[a], 0.0), top);
    }
    int cell = 0;
#pragma unroll
    for (int lev = kBinCellBits - 1; lev >= 0; --lev)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (g.bits[a] > lev) cell = (cell << 1) | ((q[a] >> lev) & 1);
    return cell;
}

__device__ __forceinline__ int segment_of(const Desc &d, int64_t k) { return k < d.n_tri ? 0 : 1; }

// Bounding box of each segment: block-level min/max, then one atomic per
// value and segment.
__global__ __launch_bounds__(kBinBlock) void k_bin_bbox(const Desc d) {
    __shared__ double red[2][6][kBinBlock / kWave];
    double r[2][6];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            r[s][a] = INFINITY;
            r[s][3 + a] = -INFINITY;
        }
    const int64_t k0 = (int64_t)blockIdx.x * kBinChunk + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kBinPerThread; ++u) {
        const int64_t k = k0 + (int64_t)u * kBinBlock;
        if (k < d.n) {
            const double c[3] = {d.x[k], d.y[k], d.z[k]};
            const int s = segment_of(d, k);
#pragma unroll
            for (int a = 0; a < 3; ++a) {  // fmin/fmax drop NaN
                r[s][a] = fmin(r[s][a], c[a]);
                r[s][3 + a] = fmax(r[s][3 + a], c[a]);
            }
        }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            double v = r[s][a];
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) {
                const double o = __shfl_xor(v, off);
                v = a < 3 ? fmin(v, o) : fmax(v, o);
            }
            if (lane() == 0) red[s][a][wave_id()] = v;
        }
    __syncthreads();
    if (threadIdx.x < 12) {
        const int s = threadIdx.x / 6, a = threadIdx.x % 6;
        double v = red[s][a][0];
        for (int w = 1; w < kBinBlock / kWave; ++w) v = a < 3 ? fmin(v, red[s][a][w]) : fmax(v, red[s][a][w]);
        if (isfinite(v)) atomicMax(d.bin_bbox + 6 * s + a, a < 3 ? ~ord_key(v) : ord_key(v));
    }
}

// Cell of every body, counted per segment and cell.
__global__ __launch_bounds__(kBinBlock) void k_bin_count(const Desc d) {
    const Grid g0 = make_grid(d.bin_bbox), g1 = make_grid(d.bin_bbox + 6);
    const int64_t k0 = (int64_t)blockIdx.x * kBinChunk + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kBinPerThread; ++u) {
        const int64_t k = k0 + (int64_t)u * kBinBlock;
        if (k < d.n) {
            const int s = segment_of(d, k);
            const int cell = grid_cell(s ? g1 : g0, d.x[k], d.y[k], d.z[k]);
            d.bin_key[k] = cell;
            atomicAdd(d.bin_hist + s * kBinCells + cell, 1);
        }
    }
}

// Start of every cell (exclusive prefix sums of the counts, per segment, by
// one block); the counts, fill counters and boxes return to zero.
__global__ __launch_bounds__(kBinScanThreads) void k_bin_scan(const Desc d) {
    __shared__ int wave_total[kBinScanThreads / kWave];
    constexpr int per = kBinCells / kBinScanThreads;
    const int tid = threadIdx.x;
    for (int s = 0; s < 2; ++s) {
        int v[per], run = 0;
#pragma unroll
        for (int k = 0; k < per; ++k) {
            v[k] = d.bin_hist[s * kBinCells + tid * per + k];
            run += v[k];
        }
        int incl = run;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int up = __shfl_up(incl, off);
            if (lane() >= off) incl += up;
        }
        if (lane() == kWave - 1) wave_total[wave_id()] = incl;
        __syncthreads();
        int excl = incl - run;
        for (int w = 0; w < wave_id(); ++w) excl += wave_total[w];
        int32_t *start = d.bin_start + s * (kBinCells + 1);
#pragma unroll
        for (int k = 0; k < per; ++k) {
            start[tid * per + k] = excl;
            excl += v[k];
            d.bin_hist[s * kBinCells + tid * per + k] = 0;
            d.bin_fill[s * kBinCells + tid * per + k] = 0;
        }
        if (tid == kBinScanThreads - 1) start[kBinCells] = excl;
        __syncthreads();  // wave_total is reused by the next segment
    }
    if (tid < 12) d.bin_bbox[tid] = 0;
}

// Every body into a free slot of its cell (any order within the cell).
__global__ __launch_bounds__(kBinBlock) void k_bin_scatter(const Desc d) {
    const int64_t k0 = (int64_t)blockIdx.x * kBinChunk + threadIdx.x;
    int cells[kBinPerThread];
#pragma unroll
    for (int u = 0; u < kBinPerThread; ++u) {
        const int64_t k = k0 + (int64_t)u * kBinBlock;
        cells[u] = k < d.n ? d.bin_key[k] : 0;
    }
#pragma unroll
    for (int u = 0; u < kBinPerThread; ++u) {
        const int64_t k = k0 + (int64_t)u * kBinBlock;
        if (k < d.n) {
            const int s = segment_of(d, k);
            const int64_t s0 = s ? d.n_tri : 0;
            const int slot = d.bin_start[s * (kBinCells + 1) + cells[u]] + atomicAdd(d.bin_fill + s * kBinCells + cells[u], 1);
            d.bin_tmp[s0 + slot] = (int32_t)k;
        }
    }
}

// Writes binned position p: body k's index and its inputs.
__device__ __forceinline__ void place(const Desc &d, int64_t p, int32_t k) {
    d.bin_idx[p] = k;
    d.binned[p] = d.x[k];
    d.binned[d.n + p] = d.y[k];
    d.binned[2 * d.n + p] = d.z[k];
    d.binned[3 * d.n + p] = d.m[k];
    d.binned[4 * d.n + p] = d.vx[k];
    d.binned[5 * d.n + p] = d.vy[k];
    d.binned[6 * d.n + p] = d.vz[k];
    d.binned[7 * d.n + p] = d.rh[k];
}

// One cell per wave: its members ordered by index (a bitonic network across
// the lanes when they fit one wave, else by counting), placed.
__global__ __launch_bounds__(kBinBlock) void k_bin_order(const Desc d) {
    const int64_t w = (int64_t)blockIdx.x * (kBinBlock / kWave) + wave_id();
    if (w >= 2 * kBinCells) return;
    const int s = (int)(w / kBinCells), c = (int)(w % kBinCells);
    const int64_t s0 = s ? d.n_tri : 0;
    const int32_t *start = d.bin_start + s * (kBinCells + 1);
    const int st = start[c], cnt = start[c + 1] - st;
    if (cnt == 0) return;
    const int32_t *m = d.bin_tmp + s0 + st;
    const int l = lane();
    if (cnt <= kWave) {
        int32_t v = l < cnt ? m[l] : INT32_MAX;
#pragma unroll
        for (int k = 2; k <= kWave; k <<= 1)
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                const int32_t o = __shfl_xor(v, j);
                const bool up = (l & k) == 0, lower = (l & j) == 0;
                v = (up == lower) ? min(v, o) : max(v, o);
            }
        if (l < cnt) place(d, s0 + st + l, v);
    } else {
        for (int i = l; i < cnt; i += kWave) {
            const int32_t me = m[i];
            int rank = 0;
#pragma unroll 8
            for (int j = 0; j < cnt; ++j) rank += m[j] < me;
            place(d, s0 + st + rank, me);
        }
    }
}

// Tile g (one wave): box record of its 64 binned positions.
__device__ __forceinline__ void box_tile(const Desc &d, int64_t g) {
    const int l = lane();
    int64_t pos, end;
    if (g < d.n_tboxes) {
        pos = g * kWave + l;
        end = d.n_tri;
    } else {
        pos = d.n_tri + (g - d.n_tboxes) * kWave + l;
        end = d.n;
    }
    const bool valid = pos < end;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (valid)
#pragma unroll
        for (int f = 0; f < 8; ++f) v[f] = d.binned[f * d.n + pos];
    bool finite = true;
#pragma unroll
    for (int f = 0; f < 8; ++f) finite = finite && isfinite(v[f]);
    const bool bad = __ballot(valid && !finite) != 0;
    const double rc = d.f * v[7];
    double r[13];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r[a] = valid ? v[a] : INFINITY;
        r[3 + a] = valid ? v[a] : -INFINITY;
        r[6 + a] = valid ? v[4 + a] : INFINITY;
        r[9 + a] = valid ? v[4 + a] : -INFINITY;
    }
    r[12] = valid ? kScreenQ * (rc * rc) : 0.0;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
#pragma unroll
        for (int a = 0; a < 13; ++a) {
            const double o = __shfl_xor(r[a], off);
            r[a] = (a < 3 || (a >= 6 && a < 9)) ? fmin(r[a], o) : fmax(r[a], o);
        }
    if (l == 0) {
        double *box = d.tbox_w + g * kBoxDoubles;
#pragma unroll
        for (int a = 0; a < 12; ++a) box[a] = r[a];
        box[12] = bad ? NAN : r[12];
    }
}

__global__ __launch_bounds__(kGatherWaves * kWave) void k_bin_boxes(const Desc d) {
    const int64_t g = (int64_t)blockIdx.x * kGatherWaves + wave_id();
    if (g < d.n_boxes) box_tile(d, g);
}

// The six binning launches of one problem.
hipError_t launch_binning(const Desc &d, hipStream_t stream) {
    const unsigned chunks = (unsigned)((d.n + kBinChunk - 1) / kBinChunk);
    hipLaunchKernelGGL(k_bin_bbox, dim3(chunks), dim3(kBinBlock), 0, stream, d);
    hipLaunchKernelGGL(k_bin_count, dim3(chunks), dim3(kBinBlock), 0, stream, d);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(kBinScanThreads), 0, stream, d);
    hipLaunchKernelGGL(k_bin_scatter, dim3(chunks), dim3(kBinBlock), 0, stream, d);
    hipLaunchKernelGGL(k_bin_order, dim3((unsigned)(2 * kBinCells / (kBinBlock / kWave))), dim3(kBinBlock), 0,
                       stream, d);
    hipLaunchKernelGGL(k_bin_boxes, dim3((unsigned)((d.n_boxes + kGatherWaves - 1) / kGatherWaves)),
                       dim3(kGatherWaves * kWave), 0, stream, d);
    return hipGetLastError();
}

struct FinLds {
    double part[kFinSplit][3][kFinBodies];
    int scan[kMaxBuckets + 1];
    int wave_total[kFinalizeThreads / kWave];
};

// Body block lb of a problem: 32 bodies, each body's slot sum split over 8
// threads (fixed ranges, combined in a fixed order: deterministic; field
// bodies were summed completely by their field task and are only checked),
// and each body's group label.
// Sum over the block of one triple per thread, in a fixed order (shuffle
// tree in each wave, then the waves in order); every thread gets the totals.
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c) {
    __shared__ double red[3][kFinalizeThreads / kWave];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
        c += __shfl_xor(c, off);
    }
    __syncthreads();
    if (lane() == 0) {
        red[0][wave_id()] = a;
        red[1][wave_id()] = b;
        red[2][wave_id()] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
    for (int w = 0; w < kFinalizeThreads / kWave; ++w) {
        a += red[0][w];
        b += red[1][w];
        c += red[2][w];
    }
}

// Block b of a problem's k_indirect: the partial sum of m_j x_j / |x_j|^3
// over its kIndBodies massive bodies, the indirect term of the accelerated
// heliocentric frame (Sun's mass 1, G = 1).
static_assert(kIndBodies == kFinalizeThreads, "k_indirect takes one body per thread");

__device__ __forceinline__ void indirect_block(const Desc &d, int64_t b) {
    if (b >= d.n_ind) return;
    const int64_t j = b * kIndBodies + threadIdx.x;
    double cx = 0.0, cy = 0.0, cz = 0.0;
    if (j < d.n_tri) {
        const double px = d.x[j], py = d.y[j], pz = d.z[j];
        const double r2 = px * px + py * py + pz * pz;
        const double w = d.m[j] / (r2 * sqrt(r2));
        cx = w * px;
        cy = w * py;
        cz = w * pz;
    }
    block_sum3(cx, cy, cz);
    if (threadIdx.x == 0) {
        d.ind[3 * b] = cx;
        d.ind[3 * b + 1] = cy;
        d.ind[3 * b + 2] = cz;
    }
}

__device__ __forceinline__ void sum_and_label(FinLds &F, const Desc &d, int64_t lb) {
    const int tid = threadIdx.x;
    // full heliocentric output: the indirect term, the problem's k_indirect
    // partials added in the same order in every block
    double a0x = 0.0, a0y = 0.0, a0z = 0.0;
    if (d.ind) {
        for (int64_t b = tid; b < d.n_ind; b += kFinalizeThreads) {
            a0x += d.ind[3 * b];
            a0y += d.ind[3 * b + 1];
            a0z += d.ind[3 * b + 2];
        }
        block_sum3(a0x, a0y, a0z);
    }
    auto &part = F.part;
    const int col = tid % kFinBodies, split = tid / kFinBodies;
    const int64_t pos = lb * kFinBodies + col;  // position in the binned order
    const bool own_sum = pos < d.n;
    const bool tri = pos < d.n_tri;  // massive: the triangle's slots; field: the segments' slots
    // the label's first loads are issued before the partial sums so that
    // their round trip overlaps them
    int64_t k = pos;
    int off0 = 0, tch = 0;
    if (split == 0 && pos < d.n) {
        if (d.bidx) k = d.bidx[pos];  // the caller's index
        off0 = uf_load(d.parent + k);
        tch = d.touched[k];
    }
    double sx = 0.0, sy = 0.0, sz = 0.0;
    if (own_sum) {
        const int64_t slots = tri ? d.n_slots : d.n_fslots;
        const int64_t stride = tri ? d.n_tri : d.n - d.n_tri;
        const int64_t per = (slots + kFinSplit - 1) / kFinSplit;
        const int64_t c0 = split * per;
        const int64_t c1 = (c0 + per) < slots ? (c0 + per) : slots;
        const double *p = tri ? d.partial + pos : d.fpartial + (pos - d.n_tri);
#pragma unroll 8
        for (int64_t c = c0; c < c1; ++c) {
            sx += p[(3 * c) * stride];
            sy += p[(3 * c + 1) * stride];
            sz += p[(3 * c + 2) * stride];
        }
    }
    part[split][0][col] = sx;
    part[split][1][col] = sy;
    part[split][2][col] = sz;
    __syncthreads();
    bool nonfinite = false, root_of_group = false;
    if (split == 0 && pos < d.n) {
        for (int s2 = 1; s2 < kFinSplit; ++s2) {
            sx += part[s2][0][col];
            sy += part[s2][1][col];
            sz += part[s2][2][col];
        }
        if (d.ind) {  // the Sun's pull and the indirect term
            const double px = d.x[k], py = d.y[k], pz = d.z[k];
            const double r2 = px * px + py * py + pz * pz;
            const double q = 1.0 / (r2 * sqrt(r2));
            sx = sx - q * px - a0x;
            sy = sy - q * py - a0y;
            sz = sz - q * pz - a0z;
        }
        d.ax[k] = sx;
        d.ay[k] = sy;
        d.az[k] = sz;
        if (d.kvx) {  // the step's closing half kick
            d.kvx[k] = __builtin_fma(d.kick_h, sx, d.kvx[k]);
            d.kvy[k] = __builtin_fma(d.kick_h, sy, d.kvy[k]);
            d.kvz[k] = __builtin_fma(d.kick_h, sz, d.kvz[k]);
        }
        nonfinite = !(isfinite(sx) && isfinite(sy) && isfinite(sz));
        // group label = union-find root, the smallest index of the component
        const int g = off0 == 0 ? (int)k : uf_find(d.parent, (int)k);
        d.group_id[k] = g;
        root_of_group = tch && g == (int)k;
        if (tch) d.touched[k] = 0;
    }
    const int groups = __syncthreads_count(root_of_group);
    const int bad = __syncthreads_or(nonfinite);
    if (tid == 0) {
        // a plain store per block, summed by the closing kernel: one atomic
        // per block on a shared counter would serialise (~12 ns each)
        d.blk_groups[lb] = groups;
        if (bad) atomicOr(d.ctr + kCtrStatus, kStatusNonfinite);
        // the pair count for every closing block, in a slot that the closing
        // kernel never resets (its block 0 resets the live counter, which the
        // other closing blocks therefore must not read)
        if (lb == 0) d.ctr[kCtrFound] = d.ctr[kCtrPairs];
    }
}

// Exclusive prefix sums of the problem's bucket counts into F.scan[0..nb]
// (F.scan[nb] = total), by one block.
__device__ __forceinline__ void scan_buckets(FinLds &F, const Desc &d) {
    constexpr int per = (kMaxBuckets + kFinalizeThreads - 1) / kFinalizeThreads;
    const int tid = threadIdx.x, nb = d.nb;
    int v[per], run = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        const int idx = tid * per + k;
        v[k] = idx < nb ? d.bcnt[idx] : 0;
        run += v[k];
    }
    // inclusive scan of the per-thread totals: within the wave, then across waves
    int incl = run;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int up = __shfl_up(incl, off);
        if (lane() >= off) incl += up;
    }
    if (lane() == kWave - 1) F.wave_total[wave_id()] = incl;
    __syncthreads();
    int base = 0;
    for (int w = 0; w < wave_id(); ++w) base += F.wave_total[w];
    int excl = base + incl - run;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        const int idx = tid * per + k;
        if (idx <= nb) F.scan[idx] = excl;
        excl += v[k];
    }
    if (tid == kFinalizeThreads - 1) F.scan[nb] = excl;  // the total (nb may equal kMaxBuckets)
    __syncthreads();
}

// Scatter block r of `blocks`: each stored pair to a free slot of its bucket
// (order inside a bucket is arbitrary here and fixed by the closing kernel),
// stored with its bucket's range [start, end) of the canonical order.
__device__ __forceinline__ void scatter_pairs(FinLds &F, const Desc &d, int r, int blocks) {
    const int64_t found = (int64_t)d.ctr[kCtrPairs];
    if (found > d.pair_scratch_cap) return;  // not every pair was stored: no order to produce
    scan_buckets(F, d);
    for (int64_t p = (int64_t)r * kFinalizeThreads + threadIdx.x; p < found; p += (int64_t)blocks * kFinalizeThreads) {
        const int2 e = d.pairs[p];
        const int bk = bucket_of(d, e.x);
        const int slot = F.scan[bk] + atomicAdd(d.bfill + bk, 1);
        d.sorted[slot] = make_int4(e.x, e.y, F.scan[bk], F.scan[bk + 1]);
    }
}

// Block fb of a problem's final kernel: body blocks first, then the pair
// scatter blocks.
__device__ __forceinline__ void final_block(FinLds &F, const Desc &d, int64_t fb, int scatter_blocks) {
    if (fb < d.n_blk)
        sum_and_label(F, d, fb);
    else
        scatter_pairs(F, d, (int)(fb - d.n_blk), scatter_blocks);
}

// Closing block c of `blocks`, after the final kernel: each pair's canonical
// position = its bucket's start + the number of smaller keys in its bucket;
// pairs written out, union-find and bucket scratch returned to zero, scalar
// outputs (block 0).
__device__ __forceinline__ void close_block(const Desc &d, int c, int blocks) {
    const int tid = threadIdx.x;
    const int64_t s0 = (int64_t)c * kFinalizeThreads + tid;
    // the first entry is read together with the pair count (a valid scratch
    // address whether or not it holds a pair), saving a round trip
    int4 first = make_int4(0, 0, 0, 0);
    if (s0 < d.pair_scratch_cap) first = d.sorted[s0];
    // the count as the final kernel published it: block 0 below resets the
    // live counter (kCtrPairs) while other blocks may still be starting, so
    // no block reads that one here
    const int64_t found = (int64_t)d.ctr[kCtrFound];
    const int64_t cap = d.pair_cap < d.pair_scratch_cap ? d.pair_cap : d.pair_scratch_cap;
    const bool fits = found <= cap;
    const int64_t stride = (int64_t)blocks * kFinalizeThreads;
    if (found <= d.pair_scratch_cap) {
        for (int64_t s = s0; s < found; s += stride) {
            const int4 e = s == s0 ? first : d.sorted[s];
            const int b0 = e.z, b1 = e.w;
            const unsigned long long mine = ((unsigned long long)(unsigned)e.x << 32) | (unsigned)e.y;
            int less = 0;
            for (int q = b0; q < b1; ++q) {
                const int4 o = d.sorted[q];
                less += (((unsigned long long)(unsigned)o.x << 32) | (unsigned)o.y) < mine;
            }
            if (fits) {
                d.pair_i[b0 + less] = e.x;
                d.pair_j[b0 + less] = e.y;
            }
            d.parent[e.x] = 0;  // only bodies of stored pairs can have a parent
            d.parent[e.y] = 0;
        }
    } else {  // pairs beyond the scratch list: clear every body
        for (int64_t k = (int64_t)c * kFinalizeThreads + tid; k < d.n; k += stride) d.parent[k] = 0;
    }
    for (int64_t k = (int64_t)c * kFinalizeThreads + tid; k < d.nb; k += stride) {
        d.bcnt[k] = 0;
        d.bfill[k] = 0;
    }
    if (c != 0) return;
    // encounter groups: the body blocks' counts summed by block 0
    __shared__ int wave_groups[kFinalizeThreads / kWave];
    int g = 0;
    for (int64_t b = tid; b < d.n_blk; b += kFinalizeThreads) g += d.blk_groups[b];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) g += __shfl_xor(g, off);
    if (lane() == 0) wave_groups[wave_id()] = g;
    __syncthreads();
    if (tid == 0) {
        int groups = 0;
        for (int w = 0; w < kFinalizeThreads / kWave; ++w) groups += wave_groups[w];
        atomicAdd(d.stats + kStatFlagged, (unsigned long long)found);
        atomicAdd(d.stats + kStatCalls, 1ull);
        *d.n_pairs_out = found;
        *d.n_groups_out = groups;
        *d.status_out = (int32_t)(d.ctr[kCtrStatus] | (fits ? 0ull : kStatusCapacity));
        // only block 0 reads the status word, and no closing block reads the
        // live pair counter, so these resets race with nothing
        d.ctr[kCtrPairs] = 0;
        d.ctr[kCtrStatus] = 0;
    }
}

__global__ __launch_bounds__(kFinalizeThreads) void k_final(const Desc d, int scatter_blocks) {
    __shared__ FinLds F;
    final_block(F, d, blockIdx.x, scatter_blocks);
}

__global__ __launch_bounds__(kFinalizeThreads) void k_final_batch(const Desc *__restrict__ descs, int n_desc,
                                                                  int scatter_blocks) {
    __shared__ FinLds F;
    const Desc &d = descs[problem_of(descs, n_desc, blockIdx.x, 1)];
    final_block(F, d, blockIdx.x - d.fin_base, scatter_blocks);
}

__global__ __launch_bounds__(kFinalizeThreads) void k_indirect(const Desc d) { indirect_block(d, blockIdx.x); }

__global__ __launch_bounds__(kFinalizeThreads) void k_indirect_batch(const Desc *__restrict__ descs, int n_desc) {
    const Desc &d = descs[problem_of(descs, n_desc, blockIdx.x, 2)];
    indirect_block(d, (int64_t)blockIdx.x - d.ind_base);
}

__global__ __launch_bounds__(kFinalizeThreads) void k_close(const Desc d, int blocks) {
    close_block(d, blockIdx.x, blocks);
}

__global__ __launch_bounds__(kFinalizeThreads) void k_close_batch(const Desc *__restrict__ descs, int blocks) {
    close_block(descs[blockIdx.x / blocks], blockIdx.x % blocks, blocks);
}

template <int R, int RF, bool BIN, bool F32>
void launch_tiles(const TileGroup &g, const Desc &one, const Desc *descs, hipStream_t stream) {
    if (descs)
        hipLaunchKernelGGL((k_tiles_batch<R, RF, BIN, F32>), dim3((unsigned)g.n_tasks), dim3(kTaskThreads), 0,
                           stream, descs + g.p0, g.p1 - g.p0, g.task_begin);
    else
        hipLaunchKernelGGL((k_tiles<R, RF, BIN, F32>), dim3((unsigned)g.n_tasks), dim3(kTaskThreads), 0, stream,
                           one);
}

template <int R, int RF, bool BIN>
void launch_tiles_s(const TileGroup &g, const Desc &one, const Desc *descs, hipStream_t stream) {
    if (g.screen32)
        launch_tiles<R, RF, BIN, true>(g, one, descs, stream);
    else
        launch_tiles<R, RF, BIN, false>(g, one, descs, stream);
}

template <int R>
void launch_tiles_r(const TileGroup &g, const Desc &one, const Desc *descs, hipStream_t stream) {
    if (g.field_rows == 2) {
        if (g.binned) launch_tiles_s<R, 2, true>(g, one, descs, stream);
        else launch_tiles_s<R, 2, false>(g, one, descs, stream);
    } else {
        if (g.binned) launch_tiles_s<R, 1, true>(g, one, descs, stream);
        else launch_tiles_s<R, 1, false>(g, one, descs, stream);
    }
}

__global__ __launch_bounds__(256) void k_zero(uint32_t *p, size_t words) {
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < words; k += (size_t)gridDim.x * 256) p[k] = 0u;
}

}  // namespace

hipError_t launch_zero(void *p, size_t bytes, hipStream_t stream) {
    const size_t words = bytes / 4;
    const size_t want = (words + 255) / 256;
    const unsigned blocks = (unsigned)(want < 1024 ? want : 1024);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, stream, (uint32_t *)p, words);
    return hipGetLastError();
}

hipError_t launch_step(const Desc *descs_host, const Desc *descs_dev, int n_desc, const TileGroup *groups,
                       int n_groups, int n_binned, int64_t n_fin_total, const LaunchCfg &cfg, hipStream_t stream,
                       hipEvent_t *ev) {
    const Desc &inl = descs_host[0];
    const Desc *dd = n_desc == 1 ? nullptr : descs_dev;
    if (ev && hipEventRecord(ev[0], stream) != hipSuccess) return hipErrorUnknown;
    if (n_binned > 0)  // binning of the problems that use it, one problem after the other
        for (int p = 0; p < n_desc; ++p)
            if (descs_host[p].bin_idx && launch_binning(descs_host[p], stream) != hipSuccess) return hipErrorUnknown;
    for (int k = 0; k < n_groups; ++k) {
        const TileGroup &g = groups[k];
        if (g.n_tasks <= 0) continue;
        switch (g.rows) {
            case 1: launch_tiles_r<1>(g, inl, dd, stream); break;
            case 2: launch_tiles_r<2>(g, inl, dd, stream); break;
            default: launch_tiles_r<4>(g, inl, dd, stream); break;
        }
        if (hipGetLastError() != hipSuccess) return hipErrorUnknown;
    }
    if (ev && hipEventRecord(ev[1], stream) != hipSuccess) return hipErrorUnknown;
    const int sb = cfg.scatter_blocks_per_problem, cb = cfg.close_blocks_per_problem;
    if (cfg.ind_blocks > 0) {  // the indirect term's partial sums (full heliocentric output)
        if (dd)
            hipLaunchKernelGGL(k_indirect_batch, dim3((unsigned)cfg.ind_blocks), dim3(kFinalizeThreads), 0, stream,
                               dd, n_desc);
        else
            hipLaunchKernelGGL(k_indirect, dim3((unsigned)cfg.ind_blocks), dim3(kFinalizeThreads), 0, stream, inl);
        if (hipGetLastError() != hipSuccess) return hipErrorUnknown;
    }
    if (dd)
        hipLaunchKernelGGL(k_final_batch, dim3((unsigned)n_fin_total), dim3(kFinalizeThreads), 0, stream, dd,
                           n_desc, sb);
    else
        hipLaunchKernelGGL(k_final, dim3((unsigned)n_fin_total), dim3(kFinalizeThreads), 0, stream, inl, sb);
    if (hipGetLastError() != hipSuccess) return hipErrorUnknown;
    if (dd)
        hipLaunchKernelGGL(k_close_batch, dim3((unsigned)(n_desc * cb)), dim3(kFinalizeThreads), 0, stream, dd,
                           cb);
    else
        hipLaunchKernelGGL(k_close, dim3((unsigned)cb), dim3(kFinalizeThreads), 0, stream, inl, cb);
    if (hipGetLastError() != hipSuccess) return hipErrorUnknown;
    if (ev && hipEventRecord(ev[2], stream) != hipSuccess) return hipErrorUnknown;
    return hipSuccess;
}

}  // namespace symba
