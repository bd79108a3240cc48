// Host build of the library's device math (the same headers, compiled for
// the CPU) for tests/test_host_math.py.  Modes:
//   sincos : reads "hi lo" pairs (hex floats), prints dd sin and cos
//   atan2  : reads "yhi ylo xhi xlo" (hex floats), prints dd_atan2 as hi lo
//   log    : reads x (hex float), prints the pair loop's table log of x
//            (log_recip_tab) and 1/x
//   mac    : random pairs of unit vectors and radii around the thresholds;
//            counts decisions of the angle-free FP64 MAC filter that
//            contradict the angle computed in long double, and how many it
//            leaves undecided; the undecided ones go to the double-double
//            sine-form test, checked against the double-double angle test
//            and against long double where that settles the sign
//   pool   : reads "dev stream has_event event_done alloc_stream alloc_dev"
//            rows (integers; streams as small handles), prints the memory
//            pool's reuse decision (1 = the cached block may be handed out)
#include "../paper_2210_07021_amd/csrc/common.hpp"
#include "../paper_2210_07021_amd/csrc/expand.hpp"
#include "../paper_2210_07021_amd/csrc/geom.hpp"
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>

using namespace sfmm;

static long double angle_ld(const double* a, const double* b) {
    const long double cx = (long double)a[1] * b[2] - (long double)a[2] * b[1];
    const long double cy = (long double)a[2] * b[0] - (long double)a[0] * b[2];
    const long double cz = (long double)a[0] * b[1] - (long double)a[1] * b[0];
    const long double c = (long double)a[0] * b[0] + (long double)a[1] * b[1] + (long double)a[2] * b[2];
    return atan2l(sqrtl(cx * cx + cy * cy + cz * cz), c);
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    if (!strcmp(argv[1], "pool")) {
        long d, st, he, ed, as, ad;
        while (scanf("%ld %ld %ld %ld %ld %ld", &d, &st, &he, &ed, &as, &ad) == 6) {
            PoolBlockState b{(int)d, (hipStream_t)(intptr_t)st, he != 0, ed != 0};
            printf("%d\n", pool_reusable(b, (hipStream_t)(intptr_t)as, (int)ad) ? 1 : 0);
        }
        return 0;
    }
    if (!strcmp(argv[1], "sincos")) {
        double hi, lo;
        while (scanf("%lf %lf", &hi, &lo) == 2) {
            dd s, c;
            dd_sincos(dd{hi, lo}, &s, &c);
            printf("%a %a %a %a\n", s.hi, s.lo, c.hi, c.lo);
        }
        return 0;
    }
    if (!strcmp(argv[1], "atan2")) {
        double a, b, c, d;
        while (scanf("%lf %lf %lf %lf", &a, &b, &c, &d) == 4) {
            const dd t = dd_atan2(dd{a, b}, dd{c, d});
            printf("%a %a\n", t.hi, t.lo);
        }
        return 0;
    }
    if (!strcmp(argv[1], "log")) {
        double2 tab[kLogTab];
        for (int j = 0; j < kLogTab; ++j) tab[j] = log_tab_entry(j);
        double x;
        while (scanf("%lf", &x) == 1) {
            double l, i;
            log_recip_tab(x, tab, kLogPoly, &l, &i);
            printf("%a %a\n", l, i);
        }
        return 0;
    }
    if (!strcmp(argv[1], "mac")) {
        std::mt19937_64 rng(20221007);
        std::uniform_real_distribution<double> U(-1.0, 1.0), E(-14.0, 0.45);
        const double cst[3][2] = {{2.0, 0.5}, {1.5, 0.7}, {3.0, 0.25}};
        long long n = 0, decided = 0, wrong = 0, undecided = 0, tie_wrong = 0, tie_disagree = 0, tie_checked = 0;
        for (int it = 0; it < 1000000; ++it) {
            double a[3], p[3], b[3];
            for (;;) {
                for (double& x : a) x = U(rng);
                const double r = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
                if (r > 0.1 && r < 1.0) {
                    for (double& x : a) x /= r;
                    break;
                }
            }
            for (;;) {
                for (double& x : p) x = U(rng);
                const double dt = p[0] * a[0] + p[1] * a[1] + p[2] * a[2];
                for (int k = 0; k < 3; ++k) p[k] -= dt * a[k];
                const double r = std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
                if (r > 0.1) {
                    for (double& x : p) x /= r;
                    break;
                }
            }
            const double dist = std::pow(10.0, E(rng));
            for (int k = 0; k < 3; ++k) b[k] = std::cos(dist) * a[k] + std::sin(dist) * p[k];
            const double c_s = cst[it % 3][0], c_t = cst[it % 3][1];
            double rs, rt;
            switch (it % 4) {
                case 0: rs = 0.5 * std::pow(10.0, E(rng)); rt = 0.5 * std::pow(10.0, E(rng)); break;
                case 1: rt = dist * c_t * (1.0 + 1e-12 * U(rng)); rs = std::fabs(U(rng)) * (dist - rt) / c_s; break;
                case 2: rs = std::fabs(U(rng)) * dist / c_s; rt = (dist - c_s * rs) * (1.0 + 1e-12 * U(rng)); break;
                default: rs = dist * std::fabs(U(rng)); rt = dist * std::fabs(U(rng)); break;
            }
            if (!(rs > 0.0) || !(rt > 0.0)) continue;
            const double2 st = make_double2(std::cos(c_s * rs), std::sin(c_s * rs));
            const double4 tt = make_double4(std::cos(rt), std::sin(rt), std::cos(rt / c_t), std::sin(rt / c_t));
            const int f = mac_far_filter_trig(a[0], a[1], a[2], b[0], b[1], b[2], rs, rt, st, tt, c_s, c_t);
            const long double d = angle_ld(a, b);
            const long double m1 = d - rt - (long double)c_s * rs, m2 = (long double)c_t * d - rt;
            ++n;
            if (f == 0) {
                ++undecided;
                const dd cs[3] = {dd_from(a[0]), dd_from(a[1]), dd_from(a[2])};
                const dd ct[3] = {dd_from(b[0]), dd_from(b[1]), dd_from(b[2])};
                dd ts[2], tt2[4];
                dd_sincos(dd_mul_d(dd_from(rs), c_s), &ts[1], &ts[0]);  // cos before sin
                dd_sincos(dd_from(rt), &tt2[1], &tt2[0]);
                dd_sincos(dd_div(dd_from(rt), dd_from(c_t)), &tt2[3], &tt2[2]);
                const bool far = mac_far_dd_trig(cs, ct, dd_from(rs), dd_from(rt), ts, tt2, c_s, c_t);
                // the two double-double tests place their 1e-20 guards
                // differently (absolute, relative to d): compare them where
                // the margins exceed both
                if (std::fabs((double)m1) > 1e-18 && std::fabs((double)m2) > 1e-18 &&
                    far != mac_far_dd(cs, ct, dd_from(rs), dd_from(rt), c_s, c_t))
                    ++tie_disagree;
                if (std::fabs((double)m1) > 1e-16 && std::fabs((double)m2) > 1e-16) {
                    ++tie_checked;
                    if (far != (m1 > 0 && m2 > 0)) ++tie_wrong;
                }
                continue;
            }
            ++decided;
            // a decision is checked where long double settles the sign
            if (std::fabs((double)m1) > 1e-15 && std::fabs((double)m2) > 1e-15) {
                const bool far = m1 > 0 && m2 > 0;
                if ((f > 0) != far) ++wrong;
            } else if (m1 < -1e-15 || m2 < -1e-15) {
                if (f > 0) ++wrong;
            }
        }
        printf("%lld %lld %lld %lld %lld %lld %lld\n", n, decided, undecided, wrong, tie_checked, tie_wrong, tie_disagree);
        return 0;
    }
    return 2;
}
