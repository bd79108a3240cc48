// Double-double (~106-bit) arithmetic for the exact geometric predicates of
// the tree build: HEALPix keys near pixel edges and MAC tests near their
// thresholds.  Dekker/Knuth error-free transformations (two-sum, two-product
// with a fused multiply-add), a Taylor series for sin (cos from it by a
// square root), one Newton step for atan2.  Every routine disables FMA contraction locally: the error-free
// transformations are only exact when each operation rounds separately.
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>

namespace sfmm {

struct dd {
    double hi, lo;
};

#define SFMM_HD __host__ __device__ __forceinline__

SFMM_HD dd dd_from(double a) { return {a, 0.0}; }

SFMM_HD dd two_sum(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    const double bb = s - a;
    const double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

SFMM_HD dd quick_two_sum(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    const double e = b - (s - a);
    return {s, e};
}

SFMM_HD dd two_prod(double a, double b) {
#pragma clang fp contract(off)
    const double p = a * b;
    const double e = fma(a, b, -p);
    return {p, e};
}

SFMM_HD dd dd_add(dd a, dd b) {
#pragma clang fp contract(off)
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}

// a - b when |b| is well below |a| (no cancellation): one two-sum of the
// high parts, the low parts added in double.  The relative error stays near
// 2^-104 because |a - b| is close to |a|.
SFMM_HD dd dd_sub_small(dd a, dd b) {
#pragma clang fp contract(off)
    dd s = two_sum(a.hi, -b.hi);
    s.lo += a.lo - b.lo;
    return quick_two_sum(s.hi, s.lo);
}

SFMM_HD dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
SFMM_HD dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

SFMM_HD dd dd_mul(dd a, dd b) {
#pragma clang fp contract(off)
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}

SFMM_HD dd dd_mul_d(dd a, double b) {
#pragma clang fp contract(off)
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return quick_two_sum(p.hi, p.lo);
}

SFMM_HD dd dd_div(dd a, dd b) {
#pragma clang fp contract(off)
    const double q1 = a.hi / b.hi;
    dd r = dd_sub(a, dd_mul_d(b, q1));
    const double q2 = r.hi / b.hi;
    r = dd_sub(r, dd_mul_d(b, q2));
    const double q3 = r.hi / b.hi;
    dd q = quick_two_sum(q1, q2);
    return dd_add(q, dd_from(q3));
}

SFMM_HD dd dd_sqrt(dd a) {
#pragma clang fp contract(off)
    if (a.hi <= 0.0) return {0.0, 0.0};
    const double x = sqrt(a.hi);
    // x + (a - x^2) / (2x)
    const dd r = dd_sub(a, two_prod(x, x));
    return quick_two_sum(x, r.hi / (2.0 * x));
}

SFMM_HD bool dd_lt(dd a, dd b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }

// pi/2 and 2/pi to double-double precision
SFMM_HD dd dd_half_pi() { return {1.5707963267948966192, 6.123233995736766036e-17}; }
SFMM_HD dd dd_two_over_pi() { return {0.63661977236758138243, -3.9357353350364971764e-17}; }
SFMM_HD dd dd_quarter_pi() { return {0.78539816339744830962, 3.0616169978683830179e-17}; }

// 1/n! to double-double precision, n = 0..31: hi is 1/n! rounded to the
// nearest double and lo the nearest double to the remainder.
SFMM_HD dd inv_factorial(int n) {
    constexpr double t[32][2] = {
        {0x1.0000000000000p+0, 0x0.0p+0},
        {0x1.0000000000000p+0, 0x0.0p+0},
        {0x1.0000000000000p-1, 0x0.0p+0},
        {0x1.5555555555555p-3, 0x1.5555555555555p-57},
        {0x1.5555555555555p-5, 0x1.5555555555555p-59},
        {0x1.1111111111111p-7, 0x1.1111111111111p-63},
        {0x1.6c16c16c16c17p-10, -0x1.f49f49f49f49fp-65},
        {0x1.a01a01a01a01ap-13, 0x1.a01a01a01a01ap-73},
        {0x1.a01a01a01a01ap-16, 0x1.a01a01a01a01ap-76},
        {0x1.71de3a556c734p-19, -0x1.c154f8ddc6c00p-73},
        {0x1.27e4fb7789f5cp-22, 0x1.cbbc05b4fa99ap-76},
        {0x1.ae64567f544e4p-26, -0x1.c062e06d1f209p-80},
        {0x1.1eed8eff8d898p-29, -0x1.2aec959e14c06p-83},
        {0x1.6124613a86d09p-33, 0x1.f28e0cc748ebep-87},
        {0x1.93974a8c07c9dp-37, 0x1.05d6f8a2efd1fp-92},
        {0x1.ae7f3e733b81fp-41, 0x1.1d8656b0ee8cbp-97},
        {0x1.ae7f3e733b81fp-45, 0x1.1d8656b0ee8cbp-101},
        {0x1.952c77030ad4ap-49, 0x1.ac981465ddc6cp-103},
        {0x1.6827863b97d97p-53, 0x1.eec01221a8b0bp-107},
        {0x1.2f49b46814157p-57, 0x1.2650f61dbdcb4p-112},
        {0x1.e542ba4020225p-62, 0x1.ea72b4afe3c2fp-120},
        {0x1.71b8ef6dcf572p-66, -0x1.d043ae40c4647p-120},
        {0x1.0ce396db7f853p-70, -0x1.aebcdbd20331cp-124},
        {0x1.761b41316381ap-75, -0x1.3423c7d91404fp-130},
        {0x1.f2cf01972f578p-80, -0x1.9ada5fcc1ab14p-135},
        {0x1.3f3ccdd165fa9p-84, -0x1.58ddadf344487p-139},
        {0x1.88e85fc6a4e5ap-89, -0x1.71c37ebd16540p-143},
        {0x1.d1ab1c2dccea3p-94, 0x1.054d0c78aea14p-149},
        {0x1.0a18a2635085dp-98, 0x1.b9e2e28e1aa54p-153},
        {0x1.259f98b4358adp-103, 0x1.eaf8c39dd9bc5p-157},
        {0x1.3932c5047d60ep-108, 0x1.832b7b530a627p-162},
        {0x1.434d2e783f5bcp-113, 0x1.0b87b91be9affp-167},
    };
    return {t[n][0], t[n][1]};
}

// sin and cos of a double-double angle: reduction by multiples of pi/2 to
// |r| <= pi/4, the Taylor series of sin r in r^2 by Horner's rule with the
// tabulated 1/n! (terms through r^31/31!, whose successor is below 1e-33 on
// that range), and cos r = sqrt(1 - sin^2 r), well conditioned there since
// cos r >= 0.7.
SFMM_HD void dd_sincos(dd x, dd* s_out, dd* c_out) {
#pragma clang fp contract(off)
    const double kf = nearbyint(x.hi * 0.63661977236758138243);
    const int k = (int)kf;
    // r = x - k pi/2 ; pi/2 carried to a third word for the reduction
    dd r = dd_sub(x, dd_mul_d(dd_half_pi(), kf));
    r = dd_sub(r, dd_from(kf * -1.4973849048591698e-33));
    const dd r2 = dd_mul(r, r);
    // s = sum_j (-1)^j r^2j / (2j+1)!, c = sum_j (-1)^j r^2j / (2j)!
    dd s = inv_factorial(31);
#pragma unroll
    // each step subtracts at most a tenth of the term (r^2 / ((2j+2)(2j+3)) < 0.1)
    for (int j = 14; j >= 0; --j) s = dd_sub_small(inv_factorial(2 * j + 1), dd_mul(r2, s));
    s = dd_mul(s, r);
    // cos r = sqrt(1 - sin^2 r), well conditioned for |r| <= pi/4 (cos >= 0.7)
    const dd c = dd_sqrt(dd_sub(dd_from(1.0), dd_mul(s, s)));
    dd so, co;
    switch (k & 3) {
        case 0: so = s; co = c; break;
        case 1: so = c; co = dd_neg(s); break;
        case 2: so = dd_neg(s); co = dd_neg(c); break;
        default: so = dd_neg(c); co = s; break;
    }
    *s_out = so;
    *c_out = co;
}

// atan2 of double-double arguments: FP64 estimate, then one Newton step on
// f(t) = y cos t - x sin t, which doubles the number of correct digits.
SFMM_HD dd dd_atan2(dd y, dd x) {
    const double t0 = atan2(y.hi, x.hi);
    dd s, c;
    dd_sincos(dd_from(t0), &s, &c);
    const dd num = dd_sub(dd_mul(y, c), dd_mul(x, s));
    const dd den = dd_add(dd_mul(x, c), dd_mul(y, s));
    return dd_add(dd_from(t0), dd_div(num, den));
}

// floor with values within 1e-20 of an integer taken as that integer: the
// exact value of such a configuration is the integer itself (a point on a
// pixel edge, an azimuth on a face boundary).
SFMM_HD long long dd_floor_snap(dd v) {
#pragma clang fp contract(off)
    const double r = nearbyint(v.hi);
    const dd diff = dd_sub(v, dd_from(r));
    if (fabs(diff.hi) < 1e-20) return (long long)r;
    double f = floor(v.hi);
    if (f == v.hi && v.lo < 0.0) f -= 1.0;
    return (long long)f;
}

}  // namespace sfmm
