// Device pieces of the step's drifts (the first kick with the momentum's
// partial sums, the Sun and Kepler drifts), shared by the step kernels and
// the encounter step's fused kernels for one-block problems, so both run the
// same operations in the same order.
#pragma once

#include "symba_internal.h"
#include "symba_kepler.h"

namespace symba {
namespace drift {

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

// x += sun_h P (P = p* on entry), Kepler drift for kepler_h (not for the
// bodies that `skip` marks: the encounter-group integrator moves them), then
// the new momentum partial sum (returned in p*).
__device__ __forceinline__ void sun_kepler(const StepDesc &s, double &px, double &py, double &pz) {
    const int64_t k = body_of(s);
    double vx = 0.0, vy = 0.0, vz = 0.0;
    if (k < s.n) {
        double x = s.x[k] + s.sun_h * px, y = s.y[k] + s.sun_h * py, z = s.z[k] + s.sun_h * pz;
        vx = s.vx[k];
        vy = s.vy[k];
        vz = s.vz[k];
        if (!s.skip || !s.skip[k]) kepler::kepler_drift(x, y, z, vx, vy, vz, s.kepler_h);
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

}  // namespace drift
}  // namespace symba
