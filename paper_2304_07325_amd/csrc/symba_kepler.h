// Two-body (Kepler) drift about the Sun for the device code of the step
// kernels and the encounter-group integrator (one solver, so a body drifts
// the same way in both).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace symba {
namespace kepler {

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
        // converged (or NaN input).  Near the root the iteration is cubic: a
        // correction below 1e-7 |s| leaves an error of order 1e-21 |s|, so a
        // short arc (the encounter substeps, the accuracy disk's steps) stops
        // after one iteration instead of a second that would only confirm it
        if (!(fabs(ds) > 1e-7 * fabs(s))) break;
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

}  // namespace kepler
}  // namespace symba
