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
//   hess   : random local and multipole expansions (order 12) in random
//            frames; prints the largest difference, relative to the largest
//            entry, between the Hessian of l2p_eval_hess / m2p_eval_hess and
//            central differences of their deflection along great circles
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
    if (!strcmp(argv[1], "hess")) {
        std::mt19937_64 g(11);
        std::normal_distribution<double> nd(0.0, 1.0);
        std::uniform_real_distribution<double> ud(0.0, 1.0);
        auto unit = [&](double* v) {
            const double r = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            for (int d = 0; d < 3; ++d) v[d] /= r;
        };
        constexpr int P = 12;
        double worst[2] = {0, 0};
        for (int trial = 0; trial < 200; ++trial) {
            double c[3] = {nd(g), nd(g), nd(g)};
            unit(c);
            const Frame f = make_frame(c[0], c[1], c[2]);
            const double rho = 0.05 + 0.2 * ud(g);
            double e[2 * P + 2];
            for (int k = 0; k < 2 * P + 2; ++k) e[k] = nd(g);
            for (int kind = 0; kind < 2; ++kind) {
                // a target at stereographic radius 0.8 rho (local) or 2.5 rho
                // (multipole) from the centre, in a random direction
                const double rr = (kind == 0 ? 0.8 : 2.5) * rho * (kind == 0 ? ud(g) : 1.0 + ud(g));
                const double ang = 6.283185307179586 * ud(g);
                const double u = rr * std::cos(ang), v = rr * std::sin(ang);
                // inverse stereographic map in the frame: n = ((2u, 2v, 1 - |w|^2) / (1 + |w|^2))
                const double w2 = u * u + v * v, den = 1.0 / (1.0 + w2);
                double n[3];
                for (int d = 0; d < 3; ++d)
                    n[d] = (2.0 * u * f.et[d] + 2.0 * v * f.ep[d] + (1.0 - w2) * f.c[d]) * den;
                double et[3], ep[3];
                target_basis(n[0], n[1], n[2], et, ep);
                double ps, a0, a1, a2, h[3];
                if (kind == 0) l2p_eval_hess<P>(e, f, rho, n[0], n[1], n[2], et, ep, &ps, &a0, &a1, &a2, h);
                else m2p_eval_hess<P>(e, f, rho, n[0], n[1], n[2], et, ep, &ps, &a0, &a1, &a2, h);
                const double H[2][2] = {{h[0], h[1]}, {h[1], h[2]}};
                const double* E[2] = {et, ep};
                const double hs = 1e-5;
                double err = 0, big = 0;
                for (int a = 0; a < 2; ++a) {
                    double al[2][3];
                    for (int sgn = 0; sgn < 2; ++sgn) {
                        const double sg = sgn == 0 ? 1.0 : -1.0;
                        double m[3];
                        for (int d = 0; d < 3; ++d) m[d] = n[d] * std::cos(hs) + sg * E[a][d] * std::sin(hs);
                        if (kind == 0) l2p_eval<P>(e, f, rho, m[0], m[1], m[2], &ps, &al[sgn][0], &al[sgn][1], &al[sgn][2]);
                        else m2p_eval<P>(e, f, rho, m[0], m[1], m[2], &ps, &al[sgn][0], &al[sgn][1], &al[sgn][2]);
                    }
                    for (int b = 0; b < 2; ++b) {
                        double fd = 0;
                        for (int d = 0; d < 3; ++d) fd += E[b][d] * (al[0][d] - al[1][d]) / (2 * hs);
                        err = std::max(err, std::fabs(fd - H[a][b]));
                        big = std::max(big, std::fabs(H[a][b]));
                    }
                }
                worst[kind] = std::max(worst[kind], err / big);
            }
        }
        printf("%.3e %.3e\n", worst[0], worst[1]);
        return 0;
    }
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
