// HIP kernels of the drifts around the kick/encounter evaluation: one step
// of the democratic heliocentric map that SyMBA is built on (the paper's
// Sec. 1: Duncan, Levison & Lee 1998, a variant of the Wisdom-Holman map),
// outside close encounters.  With heliocentric positions x, barycentric
// velocities v, G = 1 and the Sun's mass 1, a step of length h is
//   kick(h/2) . Sun drift(h/2) . Kepler drift(h) . Sun drift(h/2) . kick(h/2):
//   kick        v_i += (h/2) a_i, a_i the trapezoid's interaction acceleration;
//   Sun drift   x_i += (h/2) P, P = sum over massive bodies of m_i v_i;
//   Kepler      each body on its two-body orbit about the Sun for h.
// Three launches do the first kick and the drifts (k_kick_momentum,
// k_sun_kepler, k_sun), for one problem or a batch (each problem owning a
// range of the launch's blocks), or one launch (k_drifts_block) for a single
// problem of one block.  The evaluation at the new positions follows, and
// the final kick is an epilogue of its final kernel.  P is summed in a fixed
// order (per-block partial sums, then every block adds the partials in the
// same order), so every block sees the same bits and the step is
// reproducible.
#include "symba_internal.h"

#include <math.h>

namespace symba {
namespace {

constexpr int kStepThreads = 256;
constexpr int kStepWaves = kStepThreads / kWave;

// Fixed-order block sum of one value per thread (shuffle tree in each wave,
// then the waves in order); every thread gets the total.
__device__ __forceinline__ double block_sum(double v, double *lds) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) lds[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < kStepWaves; ++k) t += lds[k];
    return t;
}

// This block's share of P = sum m_i v_i over the massive bodies [0, n_tri),
// written to the launch's partials and returned to every thread.
__device__ __forceinline__ void write_momentum(const StepDesc &s, double *part, int64_t k, double vx, double vy,
                                               double vz, double &px, double &py, double &pz) {
    __shared__ double red[kStepWaves];
    const double m = k < s.n_tri ? s.m[k] : 0.0;
    px = block_sum(m * vx, red);
    py = block_sum(m * vy, red);
    pz = block_sum(m * vz, red);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = px;
        part[3 * blockIdx.x + 1] = py;
        part[3 * blockIdx.x + 2] = pz;
    }
}

// P from the problem's blocks' partial sums, in the same order in every block.
__device__ __forceinline__ void read_momentum(const StepDesc &s, const double *part, double &px, double &py,
                                              double &pz) {
    __shared__ double red[kStepWaves];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t k = s.blk_base + threadIdx.x; k < s.blk_base + s.nblk; k += kStepThreads) {
        a += part[3 * k];
        b += part[3 * k + 1];
        c += part[3 * k + 2];
    }
    px = block_sum(a, red);
    py = block_sum(b, red);
    pz = block_sum(c, red);
}

// Coefficients of the Stumpff series: 1/(2k+2)! and 1/(2k+3)!, k = 0 ..
// kStumpffTerms - 1, computed at compile time.  For |x| < 1 the first
// omitted terms, 1/24! and 1/25!, are below 2^-53 of c2 and c3.
constexpr int kStumpffTerms = 11;
struct StumpffCoeffs {
    double c2[kStumpffTerms], c3[kStumpffTerms];
};
constexpr StumpffCoeffs make_stumpff_coeffs() {
    StumpffCoeffs t{};
    double f = 2.0;  // (2k+2)!
    for (int k = 0; k < kStumpffTerms; ++k) {
        t.c2[k] = 1.0 / f;
        f *= 2.0 * k + 3.0;
        t.c3[k] = 1.0 / f;
        f *= 2.0 * k + 4.0;
    }
    return t;
}
constexpr StumpffCoeffs kStumpff = make_stumpff_coeffs();

// Stumpff functions c0..c3 of x (Danby, Fundamentals of Celestial Mechanics,
// Sec. 6.9): c0 = cos sqrt x, c1 = sin sqrt x / sqrt x, c2 = (1 - cos sqrt x) / x,
// c3 = (sqrt x - sin sqrt x) / sqrt(x)^3, continued through x <= 0.  Near 0
// the series of c2 and c3 (terms (-x)^k / (2k+2)! and (-x)^k / (2k+3)!) in
// Horner form, one FMA per term with no division on the solver's critical
// path, then c0 = 1 - x c2 and c1 = 1 - x c3.
__device__ __forceinline__ void stumpff(double x, double &c0, double &c1, double &c2, double &c3) {
    if (fabs(x) < 1.0) {
        const double y = -x;
        double s2 = kStumpff.c2[kStumpffTerms - 1], s3 = kStumpff.c3[kStumpffTerms - 1];
#pragma unroll
        for (int k = kStumpffTerms - 2; k >= 0; --k) {
            s2 = __builtin_fma(s2, y, kStumpff.c2[k]);
            s3 = __builtin_fma(s3, y, kStumpff.c3[k]);
        }
        c2 = s2;
        c3 = s3;
        c0 = 1.0 - x * c2;
        c1 = 1.0 - x * c3;
    } else if (x > 0.0) {
        const double q = sqrt(x), sn = sin(q), cs = cos(q);
        c0 = cs;
        c1 = sn / q;
        c2 = (1.0 - cs) / x;
        c3 = (q - sn) / (x * q);
    } else {
        const double q = sqrt(-x), sn = sinh(q), cs = cosh(q);
        c0 = cs;
        c1 = sn / q;
        c2 = (cs - 1.0) / -x;
        c3 = (sn - q) / (-x * q);
    }
}

// Two-body drift about a centre of gravitational parameter 1 for time h, in
// Danby's universal variable s: r0 s c1 + eta s^2 c2 + s^3 c3 = h with
// beta = 2 / r0 - |v|^2, eta = x . v and the c's at beta s^2, solved by the
// Laguerre-Conway iteration (Conway 1986), then the f and g functions
// f = 1 - s^2 c2 / r0, g = h - s^3 c3, fdot = -s c1 / (r r0), gdot = 1 - s^2 c2 / r.
__device__ __forceinline__ void kepler_drift(double &x, double &y, double &z, double &vx, double &vy, double &vz,
                                             double h) {
    const double r0 = sqrt(x * x + y * y + z * z);
    const double beta = 2.0 / r0 - (vx * vx + vy * vy + vz * vz);
    const double eta = x * vx + y * vy + z * vz;
    const double zeta = 1.0 - beta * r0;
    // first guess: h / r0 for short arcs and ellipses; on a hyperbola the
    // variable grows like log(v_inf t) / v_inf (r ~ v_inf t far out)
    double s = h / r0, c0, c1, c2, c3;
    if (beta < 0.0) {
        const double vinf = sqrt(-beta);
        s = copysign(log1p(vinf * fabs(h) / r0) / vinf, h);
    }
    for (int it = 0; it < 40; ++it) {
        stumpff(beta * s * s, c0, c1, c2, c3);
        const double F = s * (r0 * c1 + s * (eta * c2 + s * c3)) - h;
        const double dF = r0 * c0 + s * (eta * c1 + s * c2);
        const double ddF = eta * c0 + zeta * s * c1;
        const double root = sqrt(fabs(16.0 * dF * dF - 20.0 * F * ddF));
        const double ds = -5.0 * F / (dF + (dF >= 0.0 ? root : -root));
        s += ds;
        if (!(fabs(ds) > 1e-15 * fabs(s))) break;  // converged (or NaN input)
    }
    stumpff(beta * s * s, c0, c1, c2, c3);
    const double r = r0 * c0 + s * (eta * c1 + s * c2);
    const double inv_r0 = 1.0 / r0, inv_r = 1.0 / r;
    const double f = 1.0 - s * s * c2 * inv_r0, g = h - s * s * s * c3;
    const double fd = -s * c1 * inv_r0 * inv_r, gd = 1.0 - s * s * c2 * inv_r;
    const double nx = f * x + g * vx, ny = f * y + g * vy, nz = f * z + g * vz;
    vx = fd * x + gd * vx;
    vy = fd * y + gd * vy;
    vz = fd * z + gd * vz;
    x = nx;
    y = ny;
    z = nz;
}

// The problem of launch block b: `one`, or the last of the list whose first
// block is not above b.
template <bool LIST>
__device__ __forceinline__ const StepDesc &problem(const StepDesc &one, const StepDesc *list, int n_list) {
    if (!LIST) return one;
    int lo = 0, hi = n_list - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (list[mid].blk_base <= (int64_t)blockIdx.x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return list[lo];
}

__device__ __forceinline__ int64_t body_of(const StepDesc &s) {
    return ((int64_t)blockIdx.x - s.blk_base) * kStepThreads + threadIdx.x;
}

// v += kick_h a, then this block's momentum partial sum (returned in p*).
__device__ __forceinline__ void kick_momentum(const StepDesc &s, double &px, double &py, double &pz) {
    const int64_t k = body_of(s);
    double vx = 0.0, vy = 0.0, vz = 0.0;
    if (k < s.n) {
        vx = s.vx[k] + s.kick_h * s.ax[k];
        vy = s.vy[k] + s.kick_h * s.ay[k];
        vz = s.vz[k] + s.kick_h * s.az[k];
        s.vx[k] = vx;
        s.vy[k] = vy;
        s.vz[k] = vz;
    }
    write_momentum(s, s.mom0, k, vx, vy, vz, px, py, pz);
}

// x += sun_h P (P = p* on entry), Kepler drift for kepler_h, then the new
// momentum partial sum (returned in p*).
__device__ __forceinline__ void sun_kepler(const StepDesc &s, double &px, double &py, double &pz) {
    const int64_t k = body_of(s);
    double vx = 0.0, vy = 0.0, vz = 0.0;
    if (k < s.n) {
        double x = s.x[k] + s.sun_h * px, y = s.y[k] + s.sun_h * py, z = s.z[k] + s.sun_h * pz;
        vx = s.vx[k];
        vy = s.vy[k];
        vz = s.vz[k];
        kepler_drift(x, y, z, vx, vy, vz, s.kepler_h);
        s.x[k] = x;
        s.y[k] = y;
        s.z[k] = z;
        s.vx[k] = vx;
        s.vy[k] = vy;
        s.vz[k] = vz;
    }
    write_momentum(s, s.mom1, k, vx, vy, vz, px, py, pz);
}

// x += sun_h P with the momentum after the Kepler drift.
__device__ __forceinline__ void sun(const StepDesc &s, double px, double py, double pz) {
    const int64_t k = body_of(s);
    if (k < s.n) {
        s.x[k] += s.sun_h * px;
        s.y[k] += s.sun_h * py;
        s.z[k] += s.sun_h * pz;
    }
}

template <bool LIST>
__global__ __launch_bounds__(kStepThreads) void k_kick_momentum(const StepDesc one, const StepDesc *list,
                                                                int n_list) {
    double px, py, pz;
    kick_momentum(problem<LIST>(one, list, n_list), px, py, pz);
}

template <bool LIST>
__global__ __launch_bounds__(kStepThreads) void k_sun_kepler(const StepDesc one, const StepDesc *list,
                                                             int n_list) {
    const StepDesc &s = problem<LIST>(one, list, n_list);
    double px, py, pz;
    read_momentum(s, s.mom0, px, py, pz);
    sun_kepler(s, px, py, pz);
}

template <bool LIST>
__global__ __launch_bounds__(kStepThreads) void k_sun(const StepDesc one, const StepDesc *list, int n_list) {
    const StepDesc &s = problem<LIST>(one, list, n_list);
    double px, py, pz;
    read_momentum(s, s.mom1, px, py, pz);
    sun(s, px, py, pz);
}

// All three for a problem of one block (n <= kStepThreads), in one launch:
// each thread reads back only its own body, and the momentum is the block's
// own sum, which is exactly what reading back the one partial would give
// (that sum plus zeros), so the bits are those of the three launches.
__global__ __launch_bounds__(kStepThreads) void k_drifts_block(const StepDesc one) {
    double px, py, pz;
    kick_momentum(one, px, py, pz);
    sun_kepler(one, px, py, pz);
    sun(one, px, py, pz);
}

}  // namespace

int64_t step_blocks(int64_t n) { return (n + kStepThreads - 1) / kStepThreads; }

hipError_t launch_drifts(const StepDesc &one, const StepDesc *list, int n_list, int64_t total_blocks,
                         hipStream_t stream) {
    const unsigned blocks = (unsigned)(list ? total_blocks : one.nblk);
    if (list) {
        hipLaunchKernelGGL(k_kick_momentum<true>, dim3(blocks), dim3(kStepThreads), 0, stream, one, list, n_list);
        hipLaunchKernelGGL(k_sun_kepler<true>, dim3(blocks), dim3(kStepThreads), 0, stream, one, list, n_list);
        hipLaunchKernelGGL(k_sun<true>, dim3(blocks), dim3(kStepThreads), 0, stream, one, list, n_list);
    } else if (blocks == 1) {  // launch latency dominates a problem this small
        hipLaunchKernelGGL(k_drifts_block, dim3(1), dim3(kStepThreads), 0, stream, one);
    } else {
        hipLaunchKernelGGL(k_kick_momentum<false>, dim3(blocks), dim3(kStepThreads), 0, stream, one, list, 0);
        hipLaunchKernelGGL(k_sun_kepler<false>, dim3(blocks), dim3(kStepThreads), 0, stream, one, list, 0);
        hipLaunchKernelGGL(k_sun<false>, dim3(blocks), dim3(kStepThreads), 0, stream, one, list, 0);
    }
    return hipGetLastError();
}

}  // namespace symba
