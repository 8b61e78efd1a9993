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
#pragma clang fp contract(off)
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
        c0 = __builtin_fma(-x, c2, 1.0);
        c1 = __builtin_fma(-x, c3, 1.0);
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

// Short arcs (the substeps of deep encounter levels): the Lagrange f and g
// series in the time, x(h) = f x + g v and v(h) = f' x + g' v, through h^6.
// With u = 1/r^3, p = (x . v)/r^2, q = |v|^2/r^2 - u, the terms of order n are
// polynomials in a = u h^2, b = p h and c = q h^2 of degree n/2; it is taken
// when a, |c| and b^2 are at most 1e-6, where the first omitted terms are
// below 1e-18 of the result (checked against the iterative solution to 2e-16
// over eccentric orbits of both time signs).  No division and no iteration.
// Returns false (nothing changed) for longer arcs; the test needs no square
// root, so the solver's own path costs a few multiplications more.
__device__ __forceinline__ bool short_arc(double &x, double &y, double &z, double &vx, double &vy, double &vz,
                                          double h, double r2, double v2, double eta) {
#pragma clang fp contract(off)
    const double h2 = h * h, lim = 1e-6;
    // a <= lim <=> h^4 <= lim^2 r^6; b^2 <= lim; h^2 |v|^2 / r^2 <= lim, which
    // with a <= lim bounds |c| = |h^2 |v|^2 / r^2 - a| by lim
    if (!(h2 * h2 <= lim * lim * (r2 * r2 * r2) && h2 * (eta * eta) <= lim * (r2 * r2) && h2 * v2 <= lim * r2))
        return false;
    // 1/r: the reciprocal-square-root estimate corrected to second order in
    // its relative error e (truncation ~ (5/16) e^3)
    const double y0 = __builtin_amdgcn_rsq(r2);
    const double e = __builtin_fma(-r2, y0 * y0, 1.0);
    const double ir = y0 * __builtin_fma(e, __builtin_fma(e, 0.375, 0.5), 1.0);
    const double ir2 = ir * ir;
    const double u = ir2 * ir, p = eta * ir2, q = __builtin_fma(v2, ir2, -u);
    const double a = u * h2, b = p * h, c = q * h2, b2 = b * b;
    const double t4 = __builtin_fma(3.0, c, __builtin_fma(-15.0, b2, a));      // 3c - 15b^2 + a
    const double t5 = __builtin_fma(7.0, b2, __builtin_fma(-3.0, c, -a));      // 7b^2 - 3c - a
    const double f6 = -(1.0 / 720.0) *
                      __builtin_fma(b2, __builtin_fma(945.0, b2, __builtin_fma(-630.0, c, -210.0 * a)),
                                    __builtin_fma(c, __builtin_fma(45.0, c, 24.0 * a), a * a));
    const double s5 = __builtin_fma(9.0, c, __builtin_fma(-45.0, b2, a));      // 9c - 45b^2 + a
    const double s6 = __builtin_fma(14.0, b2, __builtin_fma(-6.0, c, -a));     // 14b^2 - 6c - a
    const double bt5 = b * t5, bs6 = b * s6;
    // f - 1, g / h - 1, h f' / a and g' - 1, small terms first
    const double fs = a * (__builtin_fma(0.5, b, -0.5) + __builtin_fma(t4, 1.0 / 24.0, __builtin_fma(bt5, 0.125, f6)));
    const double gs = a * (__builtin_fma(0.25, b, -1.0 / 6.0) +
                           __builtin_fma(s5, 1.0 / 120.0, bs6 * (1.0 / 24.0)));
    const double fk = __builtin_fma(1.5, b, -1.0) + __builtin_fma(t4, 1.0 / 6.0, __builtin_fma(bt5, 0.625, 6.0 * f6));
    const double gds = a * ((b - 0.5) + __builtin_fma(s5, 1.0 / 24.0, bs6 * 0.25));
    const double f = 1.0 + fs, g = __builtin_fma(h, gs, h);
    const double fd = (u * h) * fk, gd = 1.0 + gds;
    const double nx = __builtin_fma(f, x, g * vx), ny = __builtin_fma(f, y, g * vy), nz = __builtin_fma(f, z, g * vz);
    vx = __builtin_fma(fd, x, gd * vx);
    vy = __builtin_fma(fd, y, gd * vy);
    vz = __builtin_fma(fd, z, gd * vz);
    x = nx;
    y = ny;
    z = nz;
    return true;
}

// Two-body drift about a centre of gravitational parameter 1 for time h, in
// Danby's universal variable s: r0 s c1 + eta s^2 c2 + s^3 c3 = h with
// beta = 2 / r0 - |v|^2, eta = x . v and the c's at beta s^2, solved by the
// Laguerre-Conway iteration (Conway 1986), then the f and g functions
// f = 1 - s^2 c2 / r0, g = h - s^3 c3, fdot = -s c1 / (r r0), gdot = 1 - s^2 c2 / r.
__device__ __forceinline__ void kepler_drift(double &x, double &y, double &z, double &vx, double &vy, double &vz,
                                             double h) {
    // every fused multiply-add spelled out, so the drift of a body gives the
    // same bits wherever the compiler inlines it
#pragma clang fp contract(off)
    const double r2 = __builtin_fma(z, z, __builtin_fma(y, y, x * x));
    const double v2 = __builtin_fma(vz, vz, __builtin_fma(vy, vy, vx * vx));
    const double eta = __builtin_fma(z, vz, __builtin_fma(y, vy, x * vx));
    if (short_arc(x, y, z, vx, vy, vz, h, r2, v2, eta)) return;
    const double r0 = sqrt(r2);
    const double beta = 2.0 / r0 - v2;
    const double zeta = __builtin_fma(-beta, r0, 1.0);
    // first guess: h / r0 for short arcs and ellipses; on a hyperbola the
    // variable grows like log(v_inf t) / v_inf (r ~ v_inf t far out)
    double s = h / r0, c0, c1, c2, c3;
    if (beta < 0.0) {
        const double vinf = sqrt(-beta);
        s = copysign(log1p(vinf * fabs(h) / r0) / vinf, h);
    }
    for (int it = 0; it < 40; ++it) {
        stumpff(beta * s * s, c0, c1, c2, c3);
        const double F = __builtin_fma(s, __builtin_fma(s, __builtin_fma(s, c3, eta * c2), r0 * c1), -h);
        const double dF = __builtin_fma(s, __builtin_fma(s, c2, eta * c1), r0 * c0);
        const double ddF = __builtin_fma(zeta * s, c1, eta * c0);
        const double root = sqrt(fabs(__builtin_fma(16.0 * dF, dF, -20.0 * F * ddF)));
        const double ds = -5.0 * F / (dF + (dF >= 0.0 ? root : -root));
        s += ds;
        // converged (or NaN input).  Near the root the iteration is cubic: a
        // correction below 1e-7 |s| leaves an error of order 1e-21 |s|, so a
        // short arc (the encounter substeps, the accuracy disk's steps) stops
        // after one iteration instead of a second that would only confirm it
        if (!(fabs(ds) > 1e-7 * fabs(s))) break;
    }
    stumpff(beta * s * s, c0, c1, c2, c3);
    const double r = __builtin_fma(s, __builtin_fma(s, c2, eta * c1), r0 * c0);
    const double inv_r0 = 1.0 / r0, inv_r = 1.0 / r;
    const double s2c2 = s * s * c2;
    const double f = __builtin_fma(-s2c2, inv_r0, 1.0), g = __builtin_fma(-(s * s * s), c3, h);
    const double fd = -s * c1 * inv_r0 * inv_r, gd = __builtin_fma(-s2c2, inv_r, 1.0);
    const double nx = __builtin_fma(f, x, g * vx), ny = __builtin_fma(f, y, g * vy),
                 nz = __builtin_fma(f, z, g * vz);
    vx = __builtin_fma(fd, x, gd * vx);
    vy = __builtin_fma(fd, y, gd * vy);
    vz = __builtin_fma(fd, z, gd * vz);
    x = nx;
    y = ny;
    z = nz;
}

}  // namespace kepler
}  // namespace symba
