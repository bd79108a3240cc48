// Double-double (~106-bit) arithmetic for the exact geometric predicates of
// the tree build: HEALPix keys near pixel edges and MAC tests near their
// thresholds.  Dekker/Knuth error-free transformations (two-sum, two-product
// with a fused multiply-add), Taylor series for sin/cos, one Newton step for
// atan2.  Every routine disables FMA contraction locally: the error-free
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

// sin and cos of a double-double argument: reduce by multiples of pi/2 to
// |r| <= pi/4, then Taylor series to the 29th power (|r|^31/31! < 1e-34).
SFMM_HD void dd_sincos(dd x, dd* s_out, dd* c_out) {
#pragma clang fp contract(off)
    const double kf = nearbyint(x.hi * 0.63661977236758138243);
    const int k = (int)kf;
    // r = x - k pi/2 ; pi/2 carried to a third word for the reduction
    dd r = dd_sub(x, dd_mul_d(dd_half_pi(), kf));
    r = dd_sub(r, dd_from(kf * -1.4973849048591698e-33));
    const dd r2 = dd_mul(r, r);
    // sin r = r (1 - r^2/(2*3) (1 - r^2/(4*5) (1 - ...)))  Horner from the top
    dd s = dd_from(1.0), c = dd_from(1.0);
    for (int n = 30; n >= 2; n -= 2) {
        // sin: factor r^2 / ((n)(n+1)) with n even -> terms r^{n+1}/(n+1)!
        s = dd_sub(dd_from(1.0), dd_mul(s, dd_div(r2, dd_from((double)(n * (n + 1))))));
        c = dd_sub(dd_from(1.0), dd_mul(c, dd_div(r2, dd_from((double)((n - 1) * n)))));
    }
    s = dd_mul(s, r);
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
