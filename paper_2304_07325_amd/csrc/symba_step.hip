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
#include "symba_drift.h"
#include "symba_kepler.h"

#include <math.h>

namespace symba {
namespace {

using namespace drift;

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

// The momentum partial sums after the drifts, from the velocities in memory
// (the encounter step: its group integrator moves some bodies after
// k_sun_kepler).  The same sums, in the same order, as k_sun_kepler's.
__global__ __launch_bounds__(kStepThreads) void k_momentum(const StepDesc one) {
    const int64_t k = body_of(one);
    double vx = 0.0, vy = 0.0, vz = 0.0, px, py, pz;
    if (k < one.n) {
        vx = one.vx[k];
        vy = one.vy[k];
        vz = one.vz[k];
    }
    write_momentum(one, one.mom1, k, vx, vy, vz, px, py, pz);
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

hipError_t launch_drifts_enc(const StepDesc &one, const EncDesc &enc, hipStream_t stream) {
    const unsigned blocks = (unsigned)one.nblk;
    hipLaunchKernelGGL(k_kick_momentum<false>, dim3(blocks), dim3(kStepThreads), 0, stream, one, nullptr, 0);
    if (launch_enc_table(enc, stream) != hipSuccess) return hipErrorUnknown;
    hipLaunchKernelGGL(k_sun_kepler<false>, dim3(blocks), dim3(kStepThreads), 0, stream, one, nullptr, 0);
    if (launch_enc_groups(enc, stream) != hipSuccess) return hipErrorUnknown;
    hipLaunchKernelGGL(k_momentum, dim3(blocks), dim3(kStepThreads), 0, stream, one);
    hipLaunchKernelGGL(k_sun<false>, dim3(blocks), dim3(kStepThreads), 0, stream, one, nullptr, 0);
    return hipGetLastError();
}

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
