// Encounter groups through SyMBA's shells (the paper's Sec. 2, last
// paragraph, and Sec. 3: M = 4 substeps per level, shell radius ratio 2.08,
// the partition function f_l with l = 3).  The groups are integrated in
// parallel, one workgroup each; inside a group the work is sequential in the
// levels, parallel over bodies and pairs.
//
// Shells: a pair's critical radius R_0 = f (rh_i + rh_j) and R_k = R_{k-1} /
// 2.08.  Partition: f_3(x) = 35 x^4 - 84 x^5 + 70 x^6 - 20 x^7 (from 0 to 1
// with three vanishing derivatives at both ends); F_k(r) = f_3((r - R_{k+1}) /
// (R_k - R_{k+1})) clipped to [0, 1], F_{-1} = 0.  Level weights W_k = F_k -
// F_{k-1} (W_L = 1 - F_{L-1} at the deepest level L = 8) split each pair's
// potential exactly; a level's force on body i is m_j (W - r W') (x_j - x_i) /
// r^3, the exact gradient.
//
// A group's drift over the step h is M substeps of level 1.  A level-k
// substep of length tau: kick with the level-k forces of the level's pairs for
// tau / 2; the close-encounter test with radius R_k over tau on those pairs
// (the flagged ones make up level k + 1); the level's bodies in no flagged
// pair drift on their Kepler orbits for tau, the others take M substeps of
// level k + 1; kick for tau / 2.  Level L tests nothing and drifts its
// bodies.  The recursion runs as a loop over (level, substep) with the
// pairs' levels in LDS.
#include "symba_drift.h"
#include "symba_internal.h"
#include "symba_kepler.h"

#include <math.h>

namespace symba {
namespace {

constexpr int kTableThreads = 1024;
constexpr int kGroupThreads = 64;         // one wave per group
constexpr int kGroupBlocks = 1024;        // most workgroups of a group launch (each takes groups g, g + grid, ...)
constexpr int kEnds = 2 * kEncGroupBodies;  // pair endpoints of a group, padded to a power of two
constexpr int kStatusEncSkipped = 4;      // SYMBA_STATUS_ENC_SKIPPED
constexpr int kStatusCapacityBit = 1;     // SYMBA_STATUS_CAPACITY

static_assert((kEnds & (kEnds - 1)) == 0, "the endpoint sort needs a power of two");
static_assert(kEncSub == 4 && 2 * (kEncMaxLevel + 1) <= 32, "substep counters: two bits per level");
static_assert((kEncMaxPairs & (kEncMaxPairs - 1)) == 0, "the table sort needs a power of two");

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// A group is worked on by one wave: its LDS is ordered among the wave's
// lanes by a wave barrier (several waves of a block may run different groups).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The arithmetic of the group integration spells out every fused
// multiply-add (no contraction left to the compiler), so that a value does
// not depend on where the compiler inlined it: the routines for groups of any
// size and the register path for one pair give the same bits.

// f_3 and its derivative at x clipped to [0, 1] (f_3 = 1 and f_3' = 0 exactly
// at x = 1, 0 and 0 at x = 0).
__device__ __forceinline__ void partition(double x, double &f, double &df) {
#pragma clang fp contract(off)
    x = x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x);
    const double x2 = x * x, x3 = x2 * x, u = 1.0 - x;
    // 35 - 84 x + 70 x^2 - 20 x^3 in Horner form
    const double p = __builtin_fma(__builtin_fma(__builtin_fma(-20.0, x, 70.0), x, -84.0), x, 35.0);
    f = x3 * x * p;
    df = 140.0 * x3 * (u * u * u);
}

// F(r) and dF/dr of the changeover between the shells hi = R_k and lo =
// R_{k+1} (F_k of the pair).  At r <= lo the argument rounds to at most 0
// and at r >= hi to at least 1, where the clipped f_3 gives exactly 0 and 0,
// or 1 and 0: those values directly, without the divisions (same bits).
__device__ __forceinline__ void changeover(double r, double hi, double lo, double &F, double &dF) {
#pragma clang fp contract(off)
    if (r <= lo) {
        F = 0.0;
        dF = 0.0;
        return;
    }
    if (r >= hi) {
        F = 1.0;
        dF = 0.0;
        return;
    }
    const double w = hi - lo;
    double f, df;
    partition((r - lo) / w, f, df);
    F = f;
    dF = df / w;
}

// W - r W' of level k for a pair at separation r whose shell radii are rm =
// R_{k-1} (read for k >= 1), rk = R_k and rp = R_{k+1} (read for k < L);
// F_{-1} = 0.
__device__ __forceinline__ double force_factor(int k, double r, double rm, double rk, double rp) {
#pragma clang fp contract(off)
    double w, dw;
    if (k == kEncMaxLevel) {
        double F, dF;
        changeover(r, rm, rk, F, dF);
        w = 1.0 - F;
        dw = -dF;
    } else {
        double Fa, dFa, Fb = 0.0, dFb = 0.0;
        changeover(r, rk, rp, Fa, dFa);
        if (k > 0) changeover(r, rm, rk, Fb, dFb);
        w = Fa - Fb;
        dw = dFa - dFb;
    }
    return __builtin_fma(-r, dw, w);
}

// A pair's separation r and 1/r^3 from r^2 inside the substeps' serial
// chain: the reciprocal-square-root estimate corrected to second order in its
// relative error e (truncation ~ (5/16) e^3, so a few ulp), without the
// square root's and the division's longer sequences.
__device__ __forceinline__ void pair_r(double r2, double &r, double &ir3) {
#pragma clang fp contract(off)
    const double y0 = __builtin_amdgcn_rsq(r2);
    const double e = __builtin_fma(-r2, y0 * y0, 1.0);
    const double ir = y0 * __builtin_fma(e, __builtin_fma(e, 0.375, 0.5), 1.0);
    r = r2 * ir;
    ir3 = ir * ir * ir;
}

// The close-encounter test with radius `radius` over an interval tau (for tau
// < 0 on the reversed motion): inside now, inside at the linearly
// extrapolated end, or a closest approach inside the interval.
__device__ __forceinline__ bool encounter(double dx, double dy, double dz, double wx, double wy, double wz,
                                          double radius, double tau) {
#pragma clang fp contract(off)
    if (tau < 0.0) {
        wx = -wx;
        wy = -wy;
        wz = -wz;
        tau = -tau;
    }
    const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
    const double v2 = __builtin_fma(wz, wz, __builtin_fma(wy, wy, wx * wx));
    const double vr = __builtin_fma(dz, wz, __builtin_fma(dy, wy, dx * wx));
    const double rc2 = radius * radius;
    if (r2 < rc2) return true;
    if (__builtin_fma(v2 * tau, tau, __builtin_fma(2.0 * vr, tau, r2)) < rc2) return true;
    if (vr < 0.0 && -vr < v2 * tau) return __builtin_fma(-vr, vr, r2 * v2) < rc2 * v2;
    return false;
}

// ---------------------------------------------------------------------------
// Table of the groups of a pair list, by one workgroup: the pairs sorted by
// (group label, pair index), so each group's pairs are contiguous and in the
// pairs' order and the groups are in the order of their labels.

template <int THREADS>
__device__ void build_table(const EncDesc &e, unsigned long long *key) {
    __shared__ int wave_sum[THREADS / kWave];
    const int tid = threadIdx.x;
    const int64_t np64 = *e.n_pairs;
    const int st = *e.status;
    if ((st & kStatusCapacityBit) || np64 > e.pair_cap || np64 > kEncMaxPairs || np64 <= 0) {
        if (tid == 0) {
            e.ctl[kEncCtlGroups] = 0;
            e.ctl[kEncCtlClaim] = 0;
            if (np64 > 0) e.ctl[kEncCtlSkipped] = 1;
        }
        return;
    }
    const int np = (int)np64;
    int P2 = 1;
    while (P2 < np) P2 <<= 1;
    for (int t = tid; t < P2; t += THREADS)
        key[t] = t < np ? ((unsigned long long)(unsigned)e.group_id[e.pair_i[t]] << 32) | (unsigned)t : ~0ull;
    __syncthreads();
    for (int k = 2; k <= P2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < P2; i += THREADS) {
                const int o = i ^ j;
                if (o > i) {
                    const unsigned long long a = key[i], b = key[o];
                    if ((a > b) == ((i & k) == 0)) {
                        key[i] = b;
                        key[o] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    // group starts in this thread's chunk (at most 32 entries), then their
    // exclusive prefix over the threads
    const int chunk = (np + THREADS - 1) / THREADS;
    const int c0 = tid * chunk, c1 = min(c0 + chunk, np);
    unsigned starts = 0;
    int count = 0;
    for (int t = c0; t < c1; ++t) {
        const bool s = t == 0 || (key[t] >> 32) != (key[t - 1] >> 32);
        starts |= (s ? 1u : 0u) << (t - c0);
        count += s;
    }
    int incl = count;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int up = __shfl_up(incl, off);
        if (lane() >= off) incl += up;
    }
    if (lane() == kWave - 1) wave_sum[tid / kWave] = incl;
    __syncthreads();
    int base = 0, total = 0;
    for (int w = 0; w < THREADS / kWave; ++w) {
        if (w < tid / kWave) base += wave_sum[w];
        total += wave_sum[w];
    }
    int g = base + incl - count - 1;
    for (int t = c0; t < c1; ++t) {
        if ((starts >> (t - c0)) & 1u) {
            ++g;
            e.gstart[g] = t;
        }
        e.gp[t] = (int)(key[t] & 0xffffffffull);
        key[t] = ((unsigned long long)(unsigned)g << 32) | (key[t] & 0xffffffffull);
    }
    if (tid == 0) {
        e.gstart[total] = np;
        e.ctl[kEncCtlGroups] = total;
        e.ctl[kEncCtlClaim] = 0;
    }
    __syncthreads();
    // groups over the limit are left out (and reported); the others' bodies
    // are marked for the drift kernels when asked
    int over = 0;
    for (int gg = tid; gg < total; gg += THREADS) {
        const int big = (e.gstart[gg + 1] - e.gstart[gg]) > kEncGroupMaxPairs;
        e.gskip[gg] = big;
        over |= big;
    }
    if (__syncthreads_or(over) && tid == 0) e.ctl[kEncCtlSkipped] = 1;
    if (e.mark) {
        for (int t = tid; t < np; t += THREADS) {
            const int gg = (int)(key[t] >> 32);
            if (e.gstart[gg + 1] - e.gstart[gg] > kEncGroupMaxPairs) continue;
            const int p = (int)(key[t] & 0xffffffffull);
            e.ingroup[e.pair_i[p]] = 1;
            e.ingroup[e.pair_j[p]] = 1;
        }
    }
}

__global__ __launch_bounds__(kTableThreads) void k_enc_table(const EncDesc e) {
    __shared__ unsigned long long key[kEncMaxPairs];
    build_table<kTableThreads>(e, key);
}

// ---------------------------------------------------------------------------
// One group in LDS, worked on by one wave: its bodies (ascending global
// index) and its pairs (the pairs' order) as local indices.

struct GroupLds {
    double x[kEncGroupBodies], y[kEncGroupBodies], z[kEncGroupBodies];
    double vx[kEncGroupBodies], vy[kEncGroupBodies], vz[kEncGroupBodies];
    double m[kEncGroupBodies], rc[kEncGroupBodies];
    int body[kEncGroupBodies];       // global index of each local body
    int pa[kEncGroupMaxPairs], pb[kEncGroupMaxPairs];  // local bodies of each pair (pa < pb globally)
    int depth[kEncGroupMaxPairs];    // deepest level the pair is in
    int bdepth[kEncGroupBodies];     // deepest level of each body's pairs
    double ax[kEncGroupBodies], ay[kEncGroupBodies], az[kEncGroupBodies];  // the last kick's accelerations
    int akick[kEncGroupBodies];      // whether the last kick touched the body
    // R_q of each pair, q = 0 .. L + 1: R_0 = rc_i + rc_j, then successive
    // divisions by the shell ratio, once per step instead of in every kick
    double rk[kEncMaxLevel + 2][kEncGroupMaxPairs];
    int ends[kEnds];
    int nb, np;
};

// Loads group g: pair endpoints sorted and made unique (the bodies), pairs
// mapped to local bodies, the bodies' state (positions when `full` is 0).
// False (nothing loaded) when the pairs hold more bodies than fit, which a
// pair list whose groups are its connected components never does.
__device__ bool load_group(const EncDesc &e, GroupLds &G, int g, bool full) {
    const int l = lane();
    const int p0 = e.gstart[g], np = e.gstart[g + 1] - p0;
    // the endpoints, padded to a power of two no larger than needed (every
    // pass of the sort is a round of dependent LDS accesses and a barrier)
    int ends = 2;
    while (ends < 2 * np) ends <<= 1;
    for (int t = l; t < ends / 2; t += kGroupThreads) {
        int a = INT_MAX, b = INT_MAX;
        if (t < np) {
            const int p = e.gp[p0 + t];
            a = e.pair_i[p];
            b = e.pair_j[p];
        }
        G.ends[2 * t] = a;
        G.ends[2 * t + 1] = b;
    }
    wave_sync();
    for (int k = 2; k <= ends; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = l; i < ends; i += kGroupThreads) {
                const int o = i ^ j;
                if (o > i) {
                    const int a = G.ends[i], b = G.ends[o];
                    if ((a > b) == ((i & k) == 0)) {
                        G.ends[i] = b;
                        G.ends[o] = a;
                    }
                }
            }
            wave_sync();
        }
    }
    int nb = 0;
    for (int base = 0; base < 2 * np; base += kGroupThreads) {
        const int t = base + l;
        const bool first = t < 2 * np && (t == 0 || G.ends[t] != G.ends[t - 1]);
        const unsigned long long mask = __ballot(first);
        const int pos = nb + __popcll(mask & ((1ull << l) - 1ull));
        if (first && pos < kEncGroupBodies) G.body[pos] = G.ends[t];
        nb += __popcll(mask);
    }
    wave_sync();
    if (nb > kEncGroupBodies) {  // report it, and unmark the bodies the table marked
        if (l == 0) e.ctl[kEncCtlSkipped] = 1;
        if (full)
            for (int t = l; t < np; t += kGroupThreads) {
                const int p = e.gp[p0 + t];
                e.ingroup[e.pair_i[p]] = 0;
                e.ingroup[e.pair_j[p]] = 0;
            }
        wave_sync();
        return false;
    }
    for (int t = l; t < np; t += kGroupThreads) {
        const int p = e.gp[p0 + t];
        const int gi = e.pair_i[p], gj = e.pair_j[p];
        int lo = 0, hi = nb - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (G.body[mid] < gi) lo = mid + 1; else hi = mid;
        }
        G.pa[t] = lo;
        lo = 0;
        hi = nb - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (G.body[mid] < gj) lo = mid + 1; else hi = mid;
        }
        G.pb[t] = lo;
        G.depth[t] = 1;  // every pair of the group is flagged at level 0
    }
    for (int b = l; b < nb; b += kGroupThreads) {
        const int k = G.body[b];
        G.x[b] = e.x[k];
        G.y[b] = e.y[k];
        G.z[b] = e.z[k];
        if (full) {
            G.vx[b] = e.vx[k];
            G.vy[b] = e.vy[k];
            G.vz[b] = e.vz[k];
        }
        G.m[b] = k < e.n_tri ? e.m[k] : 0.0;
        G.rc[b] = e.f * e.rh[k];
    }
    if (l == 0) {
        G.nb = nb;
        G.np = np;
    }
    wave_sync();
    if (full) {  // the shells of the recursion, and every body at level 1
        for (int t = l; t < np; t += kGroupThreads) {
            double r = G.rc[G.pa[t]] + G.rc[G.pb[t]];
            G.rk[0][t] = r;
            for (int q = 1; q < kEncMaxLevel + 2; ++q) {
                r = r / kEncShellRatio;
                G.rk[q][t] = r;
            }
        }
        for (int b = l; b < nb; b += kGroupThreads) G.bdepth[b] = 1;
        wave_sync();
    }
    return true;
}

// Kick of level k for dt: each body's level-k acceleration (its level-k pair
// forces summed in the pairs' order) times dt added to its velocity; bodies
// in no level-k pair are not touched.  The accelerations are kept in LDS:
// with `reuse` those of the previous kick are applied again, which the
// caller passes only when no body has moved and no pair has changed level
// since, so they are the values a new evaluation would give.  A pair at r
// >= R_{k-1}, or at r <= R_{k+1} below the deepest level, has W_k = 0 and
// W_k' = 0 exactly (both changeovers clip to the same end), so its force is
// an exact zero and is not evaluated.
__device__ __forceinline__ void kick(GroupLds &G, int k, double dt, bool reuse) {
#pragma clang fp contract(off)
    const int nb = G.nb, np = G.np;
    for (int b = lane(); b < nb; b += kGroupThreads) {
        double ax = 0.0, ay = 0.0, az = 0.0;
        bool any = false;
        if (reuse) {
            ax = G.ax[b];
            ay = G.ay[b];
            az = G.az[b];
            any = G.akick[b] != 0;
        } else {
            for (int t = 0; t < np; ++t) {
                if (G.depth[t] < k) continue;
                const int i = G.pa[t], j = G.pb[t];
                if (i != b && j != b) continue;
                any = true;
                const double dx = G.x[j] - G.x[i], dy = G.y[j] - G.y[i], dz = G.z[j] - G.z[i];
                double r, ir3;
                pair_r(__builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx)), r, ir3);
                const double rm = G.rk[k - 1][t], rk = G.rk[k][t], rp = G.rk[k + 1][t];
                const bool ordered = rp < rk && rk < rm;
                if (ordered && (r >= rm || (k < kEncMaxLevel && r <= rp))) continue;
                const double g = force_factor(k, r, rm, rk, rp) * ir3;
                if (b == i) {
                    const double s = G.m[j] * g;
                    ax = __builtin_fma(s, dx, ax);
                    ay = __builtin_fma(s, dy, ay);
                    az = __builtin_fma(s, dz, az);
                } else {
                    const double s = G.m[i] * g;
                    ax = __builtin_fma(-s, dx, ax);
                    ay = __builtin_fma(-s, dy, ay);
                    az = __builtin_fma(-s, dz, az);
                }
            }
            G.ax[b] = ax;
            G.ay[b] = ay;
            G.az[b] = az;
            G.akick[b] = any;
        }
        if (any) {
            G.vx[b] = __builtin_fma(dt, ax, G.vx[b]);
            G.vy[b] = __builtin_fma(dt, ay, G.vy[b]);
            G.vz[b] = __builtin_fma(dt, az, G.vz[b]);
        }
    }
    wave_sync();
}

// The test of level k over tau on the level's pairs: flagged pairs go to
// level k + 1, the others stay at k.  Returns whether any was flagged.
__device__ __forceinline__ bool check(GroupLds &G, int k, double tau) {
    bool any = false;
    for (int t = lane(); t < G.np; t += kGroupThreads) {
        if (G.depth[t] < k) continue;
        const int i = G.pa[t], j = G.pb[t];
        const bool fl = encounter(G.x[j] - G.x[i], G.y[j] - G.y[i], G.z[j] - G.z[i], G.vx[j] - G.vx[i],
                                  G.vy[j] - G.vy[i], G.vz[j] - G.vz[i], G.rk[k][t], tau);
        G.depth[t] = fl ? k + 1 : k;
        any = any || fl;
    }
    // each body's deepest level, for the drift
    for (int b = lane(); b < G.nb; b += kGroupThreads) G.bdepth[b] = 0;
    wave_sync();
    for (int t = lane(); t < G.np; t += kGroupThreads) {
        atomicMax(&G.bdepth[G.pa[t]], G.depth[t]);
        atomicMax(&G.bdepth[G.pb[t]], G.depth[t]);
    }
    wave_sync();
    return __ballot(any) != 0;
}

// Kepler drift for tau of the bodies whose deepest pair is at level k
// (exactly k, or at least k when `at_least`).
__device__ __forceinline__ void drift(GroupLds &G, int k, double tau, bool at_least) {
    const int nb = G.nb;
    for (int b = lane(); b < nb; b += kGroupThreads) {
        const int d = G.bdepth[b];
        if (at_least ? d < k : d != k) continue;
        double x = G.x[b], y = G.y[b], z = G.z[b], vx = G.vx[b], vy = G.vy[b], vz = G.vz[b];
        kepler::kepler_drift(x, y, z, vx, vy, vz, tau);
        G.x[b] = x;
        G.y[b] = y;
        G.z[b] = z;
        G.vx[b] = vx;
        G.vy[b] = vy;
        G.vz[b] = vz;
    }
    wave_sync();
}

// The group's drift over h: M substeps of level 1, each recursing as deep as
// its pairs need.  The loop visits (level, substep) in the order of the
// recursion; every wave reaches its end after at most sum_k M^k substeps.
__device__ __forceinline__ void integrate(GroupLds &G, double h) {
    unsigned subs = 0;  // substeps done at each level, two bits per level (M = 4)
    int k = 1;
    bool enter = true;
    // the level whose accelerations the last kick left in LDS, while no body
    // has drifted since: a substep's closing kick and the next substep's
    // opening kick at the same level see the same positions and pairs
    int cached = -1;
    while (true) {
        const double tau = ldexp(h, -2 * k);  // h / M^k, M = 4
        if (enter) {
            kick(G, k, 0.5 * tau, cached == k);
            cached = -1;  // a drift follows
            if (k == kEncMaxLevel) {
                drift(G, k, tau, true);
                enter = false;
            } else if (check(G, k, tau)) {
                drift(G, k, tau, false);
                ++k;
                subs &= ~(3u << (2 * k));
            } else {
                drift(G, k, tau, false);
                enter = false;
            }
        } else {
            kick(G, k, 0.5 * tau, false);
            cached = k;
            const unsigned done = ((subs >> (2 * k)) & 3u) + 1u;
            subs = (subs & ~(3u << (2 * k))) | ((done & 3u) << (2 * k));
            if (done < (unsigned)kEncSub) {
                enter = true;
            } else if (k == 1) {
                break;
            } else {
                --k;
            }
        }
    }
}

// Level-0 reweighting of a group's accelerations: for each pair inside R_0,
// m (F_0 - r F_0' - 1) (x_j - x_i) / r^3 on i and its opposite on j, summed
// per body in the pairs' order and added to the Newtonian sums.  One wave.
__device__ void level0_group(const EncDesc &e, GroupLds &G, int g) {
#pragma clang fp contract(off)
    if (e.gskip[g] || !load_group(e, G, g, false)) return;
    for (int b = lane(); b < G.nb; b += kGroupThreads) {
        double ax = 0.0, ay = 0.0, az = 0.0;
        bool any = false;
        for (int t = 0; t < G.np; ++t) {
            const int i = G.pa[t], j = G.pb[t];
            if (i != b && j != b) continue;
            const double dx = G.x[j] - G.x[i], dy = G.y[j] - G.y[i], dz = G.z[j] - G.z[i];
            const double r = sqrt(__builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx)));
            const double r0 = G.rc[i] + G.rc[j];
            if (r >= r0) continue;
            any = true;
            const double gf = (force_factor(0, r, 0.0, r0, r0 / kEncShellRatio) - 1.0) / (r * r * r);
            if (b == i) {
                const double s = G.m[j] * gf;
                ax = __builtin_fma(s, dx, ax);
                ay = __builtin_fma(s, dy, ay);
                az = __builtin_fma(s, dz, az);
            } else {
                const double s = G.m[i] * gf;
                ax = __builtin_fma(-s, dx, ax);
                ay = __builtin_fma(-s, dy, ay);
                az = __builtin_fma(-s, dz, az);
            }
        }
        if (any) {
            const int k = G.body[b];
            e.ax[k] += ax;
            e.ay[k] += ay;
            e.az[k] += az;
        }
    }
    wave_sync();
}

// Lane-uniform reads of another lane's value (the lane index is uniform).
__device__ __forceinline__ int lane_int(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ double lane_dbl(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// The value of lane l ^ 1 (DPP quad_perm [1, 0, 3, 2]: lanes 0 and 1 swap).
__device__ __forceinline__ double swap_pair(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0xb1, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0xb1, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

// A group of one pair, the common case of the deep recursions: integrate()
// with the two bodies in registers, body i of the pair in the even lanes and
// body j in the odd ones (every lane pair holds the same two), each lane
// reading its partner through a lane swap instead of LDS.  The same
// operations on the same values as the LDS routines (kick, check, drift with
// a single pair), so the same bits.
__device__ __forceinline__ void drift_pair(const EncDesc &e, int g) {
#pragma clang fp contract(off)
    const int p = e.gp[e.gstart[g]];
    const bool first = (lane() & 1) == 0;
    const int b = first ? e.pair_i[p] : e.pair_j[p];
    double x = e.x[b], y = e.y[b], z = e.z[b], vx = e.vx[b], vy = e.vy[b], vz = e.vz[b];
    const double m_other = swap_pair(b < e.n_tri ? e.m[b] : 0.0);
    // the pair's shells, as load_group computes them: R_0 = rc_i + rc_j of
    // the rounded products, R_q = R_{q-1} / ratio.  Lane q keeps R_q (a
    // register array indexed by the level would live in scratch memory);
    // going one level deeper divides again, which gives the same bits
    double Rl = 0.0, rm, rk, rp;  // R_{k-1}, R_k, R_{k+1}, moved along with k
    {
        const double rc = e.f * e.rh[b];
        const double rc_other = swap_pair(rc);
        double r = first ? rc + rc_other : rc_other + rc;
        rm = rk = rp = r;
#pragma unroll
        for (int q = 0; q < kEncMaxLevel + 2; ++q) {
            if (q > 0) r = r / kEncShellRatio;
            if (lane() == q) Rl = r;
            if (q == 1) rk = r;
            if (q == 2) rp = r;
        }
    }
    const double h = e.h;
    int depth = 1;  // the pair's deepest level
    double cax = 0.0, cay = 0.0, caz = 0.0;  // the last kick's acceleration
    bool cany = false;
    unsigned subs = 0;  // substeps done at each level, two bits per level
    int k = 1;
    bool enter = true;
    int cached = -1;
    while (true) {
        const double tau = ldexp(h, -2 * k);
        // kick of level k for tau / 2 (the pair's force at level k, nothing
        // below it), the accelerations of the last kick again when no body
        // has drifted since it at this level
        if (!(enter && cached == k)) {
            cax = cay = caz = 0.0;
            cany = depth >= k;
            if (cany) {
                // the partner's position minus this lane's: x_j - x_i on
                // body i, and on body j its exact negative, so the squares
                // are those of x_j - x_i and s (x_i - x_j) = -s (x_j - x_i)
                // gives body j's term without a branch
                const double dx = swap_pair(x) - x, dy = swap_pair(y) - y, dz = swap_pair(z) - z;
                double r, ir3;
                pair_r(__builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx)), r, ir3);
                const bool ordered = rp < rk && rk < rm;
                if (!(ordered && (r >= rm || (k < kEncMaxLevel && r <= rp)))) {
                    const double gf = force_factor(k, r, rm, rk, rp) * ir3;
                    const double s = m_other * gf;
                    cax = __builtin_fma(s, dx, cax);
                    cay = __builtin_fma(s, dy, cay);
                    caz = __builtin_fma(s, dz, caz);
                }
            }
        }
        if (cany) {
            const double dt = 0.5 * tau;
            vx = __builtin_fma(dt, cax, vx);
            vy = __builtin_fma(dt, cay, vy);
            vz = __builtin_fma(dt, caz, vz);
        }
        if (enter) {
            cached = -1;
            if (k == kEncMaxLevel) {
                if (depth >= k) kepler::kepler_drift(x, y, z, vx, vy, vz, tau);
                enter = false;
            } else {
                // the level-k test over tau: the pair goes to level k + 1 or
                // stays at k.  On body j both differences are the exact
                // negatives of body i's, which the test's products do not
                // see, so every lane decides the same; lane 0's decision is
                // taken for the wave
                const bool fl = encounter(swap_pair(x) - x, swap_pair(y) - y, swap_pair(z) - z, swap_pair(vx) - vx,
                                          swap_pair(vy) - vy, swap_pair(vz) - vz, rk, tau);
                depth = __builtin_amdgcn_readfirstlane(fl ? k + 1 : k);
                if (depth > k) {
                    ++k;
                    subs &= ~(3u << (2 * k));
                    rm = rk;
                    rk = rp;
                    rp = rk / kEncShellRatio;
                } else {
                    kepler::kepler_drift(x, y, z, vx, vy, vz, tau);
                    enter = false;
                }
            }
        } else {
            cached = k;
            const unsigned done = ((subs >> (2 * k)) & 3u) + 1u;
            subs = (subs & ~(3u << (2 * k))) | ((done & 3u) << (2 * k));
            if (done < (unsigned)kEncSub) {
                enter = true;
            } else if (k == 1) {
                break;
            } else {
                --k;
                rp = rk;
                rk = rm;
                rm = lane_dbl(Rl, k - 1);
            }
        }
    }
    if (lane() < 2) {
        e.x[b] = x;
        e.y[b] = y;
        e.z[b] = z;
        e.vx[b] = vx;
        e.vy[b] = vy;
        e.vz[b] = vz;
        e.ingroup[b] = 0;
    }
}

// A group of at most one wave's bodies and pairs, loaded by load_group, then
// integrated like integrate() with lane b holding body b and lane t pair t in
// registers: a kick evaluates every pair's force at once (lane t) and each
// body adds its pairs' terms in the pairs' order, fetching each from its
// pair's lane (a walk over the body's own pairs); the test runs on every pair
// at once; the drifts on every body at once.  While a single pair is at the
// current level or deeper, its two bodies are read with lane-uniform reads
// and only they can change level.  The same operations on the same values as
// the LDS routines, so the same bits.
__device__ __forceinline__ void integrate_small(const EncDesc &e, GroupLds &G) {
#pragma clang fp contract(off)
    const int l = lane(), nb = G.nb, np = G.np;
    const bool isb = l < nb, isp = l < np;
    double x = 0.0, y = 0.0, z = 0.0, vx = 0.0, vy = 0.0, vz = 0.0, m = 0.0;
    if (isb) {
        x = G.x[l]; y = G.y[l]; z = G.z[l];
        vx = G.vx[l]; vy = G.vy[l]; vz = G.vz[l];
        m = G.m[l];
    }
    int pa = 0, pb = 0, depth = 0;  // pair l's bodies and level (0: no pair in this lane)
    // pair lane's R_{k-1}, R_k, R_{k+1}, moved along with k: one level deeper
    // divides again (how load_group made them, so the same bits), one level
    // up reads the shell back from LDS
    double rm = 0.0, rk = 0.0, rp = 0.0;
    if (isp) {
        pa = G.pa[l];
        pb = G.pb[l];
        depth = 1;
        rm = G.rk[0][l];
        rk = G.rk[1][l];
        rp = G.rk[2][l];
    }
    int bd = isb ? 1 : 0;  // body l's deepest level
    // body l's pairs (bit t: pair t), those where it is body i, and on pair
    // lane t the masses of its bodies, all fixed for the step
    unsigned long long mine = 0ull, firstm = 0ull;
    for (int t = 0; t < np; ++t) {
        const int ia = lane_int(pa, t), ib = lane_int(pb, t);
        if (l == ia) firstm |= 1ull << t;
        if (l == ia || l == ib) mine |= 1ull << t;
    }
    const double ma = __shfl(m, pa), mb = __shfl(m, pb);
    const double h = e.h;
    double cax = 0.0, cay = 0.0, caz = 0.0;
    bool cany = false;
    unsigned subs = 0;
    int k = 1;
    bool enter = true;
    int cached = -1;
    while (true) {
        const double tau = ldexp(h, -2 * k);
        const bool reuse = enter && cached == k;
        // the pairs at level k or deeper.  With one of them (the common case
        // deep in a recursion, the group's other pairs waiting at shallower
        // levels) its bodies ia1 and ib1 are read with lane-uniform reads
        // instead of the fetches over the whole group; same values, so the
        // same bits
        const unsigned long long act_mask = __ballot(depth >= k);
        const bool one = __popcll(act_mask) == 1;
        int t1 = 0, ia1 = 0, ib1 = 0;
        if (one) {
            t1 = __builtin_ctzll(act_mask);
            ia1 = lane_int(pa, t1);
            ib1 = lane_int(pb, t1);
        }
        // lane t: pair t's x_j - x_i, for a new kick and for the test (with
        // one pair at level k or deeper, every lane holds that pair's)
        double dx = 0.0, dy = 0.0, dz = 0.0;
        if (!reuse || (enter && k < kEncMaxLevel)) {
            if (one) {
                dx = lane_dbl(x, ib1) - lane_dbl(x, ia1);
                dy = lane_dbl(y, ib1) - lane_dbl(y, ia1);
                dz = lane_dbl(z, ib1) - lane_dbl(z, ia1);
            } else {
                dx = __shfl(x, pb) - __shfl(x, pa);
                dy = __shfl(y, pb) - __shfl(y, pa);
                dz = __shfl(z, pb) - __shfl(z, pa);
            }
        }
        if (!reuse) {
            // lane t: pair t's level-k factor g (flagged `zero` outside the band)
            const bool act = depth >= k;
            bool zero = true;
            double gf = 0.0;
            if (act) {
                double r, ir3;
                pair_r(__builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx)), r, ir3);
                const bool ordered = rp < rk && rk < rm;
                zero = ordered && (r >= rm || (k < kEncMaxLevel && r <= rp));
                if (!zero) gf = force_factor(k, r, rm, rk, rp) * ir3;
            }
            const unsigned long long zero_mask = __ballot(act && zero);
            // body i adds m_j g (x_j - x_i), body j adds -m_i g (x_j - x_i)
            const double si = mb * gf, sj = -(ma * gf);
            cax = cay = caz = 0.0;
            unsigned long long rest = mine & act_mask;
            cany = rest != 0ull;
            rest &= ~zero_mask;
            if (one) {
                // the single term of bodies ia1 and ib1, from lane t1
                const double sgl = l == ia1 ? lane_dbl(si, t1) : lane_dbl(sj, t1);
                if (rest != 0ull) {
                    cax = __builtin_fma(sgl, dx, cax);
                    cay = __builtin_fma(sgl, dy, cay);
                    caz = __builtin_fma(sgl, dz, caz);
                }
                rest = 0ull;
            }
            // lane b: its nonzero level-k terms in the pairs' order, each
            // fetched from its pair's lane (every lane takes part in the
            // fetches; a lane with no term left fetches from itself)
            while (__ballot(rest != 0ull)) {
                const bool have = rest != 0ull;
                const int t = have ? __builtin_ctzll(rest) : l;
                rest &= rest - 1ull;
                const double dxt = __shfl(dx, t), dyt = __shfl(dy, t), dzt = __shfl(dz, t);
                const double sit = __shfl(si, t), sjt = __shfl(sj, t);
                const double sgl = (firstm >> t) & 1ull ? sit : sjt;
                if (have) {
                    cax = __builtin_fma(sgl, dxt, cax);
                    cay = __builtin_fma(sgl, dyt, cay);
                    caz = __builtin_fma(sgl, dzt, caz);
                }
            }
        }
        if (cany) {
            const double dt = 0.5 * tau;
            vx = __builtin_fma(dt, cax, vx);
            vy = __builtin_fma(dt, cay, vy);
            vz = __builtin_fma(dt, caz, vz);
        }
        if (enter) {
            cached = -1;
            bool deeper = false;
            if (k < kEncMaxLevel) {
                // the level-k test of every pair at level k or deeper
                double dvx, dvy, dvz;
                if (one) {
                    dvx = lane_dbl(vx, ib1) - lane_dbl(vx, ia1);
                    dvy = lane_dbl(vy, ib1) - lane_dbl(vy, ia1);
                    dvz = lane_dbl(vz, ib1) - lane_dbl(vz, ia1);
                } else {
                    dvx = __shfl(vx, pb) - __shfl(vx, pa);
                    dvy = __shfl(vy, pb) - __shfl(vy, pa);
                    dvz = __shfl(vz, pb) - __shfl(vz, pa);
                }
                bool fl = false;
                if (depth >= k) {
                    fl = encounter(dx, dy, dz, dvx, dvy, dvz, rk, tau);
                    depth = fl ? k + 1 : k;
                }
                deeper = __ballot(fl) != 0;
                // each body's deepest level, over its pairs.  With one pair
                // tested, only its bodies can change: every other pair is
                // shallower than k, so theirs is that pair's new level
                unsigned long long rest = mine;
                if (one) {
                    if (l == ia1 || l == ib1) bd = lane_int(depth, t1);
                    rest = 0ull;
                } else {
                    bd = 0;
                }
                while (__ballot(rest != 0ull)) {
                    const bool have = rest != 0ull;
                    const int t = have ? __builtin_ctzll(rest) : l;
                    rest &= rest - 1ull;
                    const int dt_ = __shfl(depth, t);
                    if (have) bd = max(bd, dt_);
                }
            }
            // the bodies whose deepest pair is at level k (at least k at the
            // deepest level) drift for tau
            if (isb && (k == kEncMaxLevel ? bd >= k : bd == k)) kepler::kepler_drift(x, y, z, vx, vy, vz, tau);
            if (deeper) {
                ++k;
                subs &= ~(3u << (2 * k));
                rm = rk;
                rk = rp;
                rp = rk / kEncShellRatio;
            } else {
                enter = false;
            }
        } else {
            cached = k;
            const unsigned done = ((subs >> (2 * k)) & 3u) + 1u;
            subs = (subs & ~(3u << (2 * k))) | ((done & 3u) << (2 * k));
            if (done < (unsigned)kEncSub) {
                enter = true;
            } else if (k == 1) {
                break;
            } else {
                --k;
                rp = rk;
                rk = rm;
                rm = G.rk[k - 1][l];
            }
        }
    }
    if (isb) {
        const int b = G.body[l];
        e.x[b] = x;
        e.y[b] = y;
        e.z[b] = z;
        e.vx[b] = vx;
        e.vy[b] = vy;
        e.vz[b] = vz;
        e.ingroup[b] = 0;
    }
    wave_sync();
}

// The two register forms as functions of their own, for the group kernel:
// each gets its own register allocation and schedule (inlined together, a
// change to one moved the other's substep time by 4%).  A call gives the
// kernel a stack in scratch memory, which costs its launch about 1.5 us; the
// one-block kernel of small problems, launched every step, inlines them.
__device__ __noinline__ void drift_pair_call(const EncDesc &e, int g) { drift_pair(e, g); }
__device__ __noinline__ void integrate_small_call(const EncDesc &e, GroupLds &G) { integrate_small(e, G); }

// One group's drift over the step, from its bodies in memory back to them
// (the table marked them, so the drift kernels left them alone).  One wave.
// Every form and both ways of calling them give the same bits.
template <bool kCall>
__device__ void drift_group(const EncDesc &e, GroupLds &G, int g) {
    if (e.gskip[g]) return;
    if (e.regs && e.gstart[g + 1] - e.gstart[g] == 1) {
        if (kCall) drift_pair_call(e, g); else drift_pair(e, g);
        return;
    }
    if (!load_group(e, G, g, true)) return;
    if (e.regs && G.nb <= kGroupThreads && G.np <= kGroupThreads) {
        if (kCall) integrate_small_call(e, G); else integrate_small(e, G);
        return;
    }
    integrate(G, e.h);
    for (int b = lane(); b < G.nb; b += kGroupThreads) {
        const int k = G.body[b];
        e.x[k] = G.x[b];
        e.y[k] = G.y[b];
        e.z[k] = G.z[b];
        e.vx[k] = G.vx[b];
        e.vy[k] = G.vy[b];
        e.vz[k] = G.vz[b];
        e.ingroup[k] = 0;
    }
    wave_sync();
}

// Each workgroup takes the next group from a counter when it is free: a
// group's cost varies by orders of magnitude (the depth of its recursion), so
// a fixed deal could give two deep groups to one workgroup.  Groups are
// independent, so which workgroup integrates which changes no bit.
__global__ __launch_bounds__(kGroupThreads) void k_enc_groups(const EncDesc e) {
    __shared__ GroupLds G;
    const int ng = e.ctl[kEncCtlGroups];
    while (true) {
        int g = 0;
        if (lane() == 0) g = atomicAdd(e.ctl + kEncCtlClaim, 1);
        g = __shfl(g, 0);
        if (g >= ng) break;
        drift_group<true>(e, G, g);
    }
}

__global__ __launch_bounds__(kGroupThreads) void k_enc_level0(const EncDesc e) {
    __shared__ GroupLds G;
    const int ng = e.ctl[kEncCtlGroups];
    for (int g = blockIdx.x; g < ng; g += gridDim.x) level0_group(e, G, g);
}

// The closing kick v += kick_h a of every body (when kick_h is not 0), and
// the step's unresolved-pairs report ORed into the status.
__global__ __launch_bounds__(256) void k_enc_kick(const EncDesc e) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e.kick_h != 0.0 && k < e.n) {
        e.vx[k] = __builtin_fma(e.kick_h, e.ax[k], e.vx[k]);
        e.vy[k] = __builtin_fma(e.kick_h, e.ay[k], e.vy[k]);
        e.vz[k] = __builtin_fma(e.kick_h, e.az[k], e.vz[k]);
    }
    if (k == 0 && e.ctl[kEncCtlSkipped]) {
        *e.status |= kStatusEncSkipped;
        e.ctl[kEncCtlSkipped] = 0;
    }
}

// A problem of one block (n <= 256 bodies): the step's work before the
// evaluation in one launch.  The first kick with the momentum's block sum,
// the table (bodies of resolved groups marked), the Sun drift of every body
// and the Kepler drift of the unmarked ones, the groups (wave w < 3 takes
// groups w, w + 3, ...), then the momentum and the second Sun drift: the operations
// of the separate launches in the same order, on the same values.
constexpr int kFusedThreads = 256;
constexpr int kFusedGroups = 3;  // waves that take groups (three groups' LDS fit beside the rest)
union FusedLds {
    unsigned long long key[kEncMaxPairs];
    GroupLds G[kFusedGroups];
};

__global__ __launch_bounds__(kFusedThreads) void k_enc_drifts_block(const StepDesc one, const EncDesc e) {
    __shared__ FusedLds U;
    double px, py, pz;
    drift::kick_momentum(one, px, py, pz);
    build_table<kFusedThreads>(e, U.key);
    __syncthreads();  // the marks and the table are in place; the keys' LDS is free
    drift::sun_kepler(one, px, py, pz);
    __syncthreads();  // every body's Sun drift (and Kepler drift) is in memory
    const int w = threadIdx.x / kWave;
    const int ng = e.ctl[kEncCtlGroups];
    if (w < kFusedGroups)
        for (int g = w; g < ng; g += kFusedGroups) drift_group<false>(e, U.G[w], g);
    __syncthreads();  // the groups' bodies are back in memory
    const int64_t k = drift::body_of(one);
    double vx = 0.0, vy = 0.0, vz = 0.0;
    if (k < one.n) {
        vx = one.vx[k];
        vy = one.vy[k];
        vz = one.vz[k];
    }
    drift::write_momentum(one, one.mom1, k, vx, vy, vz, px, py, pz);
    drift::sun(one, px, py, pz);
}

// A problem of one block: the step's work after the evaluation in one
// launch: the table of the new pairs, the level-0 reweighting (wave w < 3
// takes groups w, w + 3, ...), the closing kick and the status.
__global__ __launch_bounds__(kFusedThreads) void k_enc_post_block(const EncDesc e) {
    __shared__ FusedLds U;
    build_table<kFusedThreads>(e, U.key);
    __syncthreads();
    const int w = threadIdx.x / kWave;
    const int ng = e.ctl[kEncCtlGroups];
    if (w < kFusedGroups)
        for (int g = w; g < ng; g += kFusedGroups) level0_group(e, U.G[w], g);
    __syncthreads();
    const int64_t k = threadIdx.x;
    if (e.kick_h != 0.0 && k < e.n) {
        e.vx[k] = __builtin_fma(e.kick_h, e.ax[k], e.vx[k]);
        e.vy[k] = __builtin_fma(e.kick_h, e.ay[k], e.vy[k]);
        e.vz[k] = __builtin_fma(e.kick_h, e.az[k], e.vz[k]);
    }
    if (k == 0 && e.ctl[kEncCtlSkipped]) {
        *e.status |= kStatusEncSkipped;
        e.ctl[kEncCtlSkipped] = 0;
    }
}

}  // namespace

hipError_t launch_enc_drifts_block(const StepDesc &one, const EncDesc &e, hipStream_t stream) {
    hipLaunchKernelGGL(k_enc_drifts_block, dim3(1), dim3(kFusedThreads), 0, stream, one, e);
    return hipGetLastError();
}

hipError_t launch_enc_post_block(const EncDesc &e, hipStream_t stream) {
    hipLaunchKernelGGL(k_enc_post_block, dim3(1), dim3(kFusedThreads), 0, stream, e);
    return hipGetLastError();
}

hipError_t launch_enc_table(const EncDesc &e, hipStream_t stream) {
    hipLaunchKernelGGL(k_enc_table, dim3(1), dim3(kTableThreads), 0, stream, e);
    return hipGetLastError();
}

// Workgroups of a group launch: a problem of n bodies has at most n / 2
// groups, and the dispatcher hands out about 200 workgroups per microsecond,
// so a small problem gets a small grid (the launch is mostly empty).
static unsigned group_blocks(int64_t n) {
    const int64_t b = n / 8;
    return (unsigned)(b < 64 ? 64 : (b > kGroupBlocks ? kGroupBlocks : b));
}

hipError_t launch_enc_groups(const EncDesc &e, hipStream_t stream) {
    hipLaunchKernelGGL(k_enc_groups, dim3(group_blocks(e.n)), dim3(kGroupThreads), 0, stream, e);
    return hipGetLastError();
}

hipError_t launch_enc_level0(const EncDesc &e, hipStream_t stream) {
    hipLaunchKernelGGL(k_enc_level0, dim3(group_blocks(e.n)), dim3(kGroupThreads), 0, stream, e);
    return hipGetLastError();
}

hipError_t launch_enc_kick(const EncDesc &e, hipStream_t stream) {
    const unsigned blocks = (unsigned)((e.n + 255) / 256);
    hipLaunchKernelGGL(k_enc_kick, dim3(blocks), dim3(256), 0, stream, e);
    return hipGetLastError();
}

}  // namespace symba
