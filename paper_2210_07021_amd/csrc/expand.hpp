// Expansion arithmetic of the sFMM (Sec. 3.1-3.3, 3.6) for one box or one box
// pair, written for one GPU lane with the order P fixed at compile time so
// the coefficients live in registers.
//
// Frames.  A box centre c carries the system K_c whose zenith is c and whose
// azimuth reference is e_theta(c) (Sec. 3.1).  The base function
// z = tan(theta/2) e^{i phi} is the stereographic projection from -c,
// w = ((n - c).e_theta + i (n - c).e_phi) / (1 + n.c), with 1 + n.c computed
// as |n + c|^2 / 2 so that neither near nor antipodal points cancel.
//
// Scaled coefficients.  A box of radius R has scale rho = tan(R/2), the
// largest |w| of a point inside it.  Multipole coefficients are stored as
// A_l / rho^l and local ones as A_l rho^l, so every stored number is bounded
// by the box's mass and nothing over- or underflows down to depth 29.
//
// Translations.  Lemmas 2, 3 and 4 share one shape,
//   A'_l = ph2^l [ -(Q/l) x^l + sum_l' T_ll'(x) ph1^l' A_l' ],
//   T_ll'(x) = sum_n C(l-1,n-1) C(l',n) x^{l+l'-2n} (1+x^2)^n,
// and with the scalings folded in, T_ll' s_T^l s_S^l' factors as
//   sum_n [C(l-1,n-1) a^{l-n}] g^n [C(l',n) b^{l'-n}],
//   a = x s_T, b = x s_S, g = s_T s_S (1+x^2),
// i.e. a Taylor shift by b (right factor), a diagonal g^n, and a transposed
// Taylor shift by a (left factor).  Both shifts run in place with P(P+1)/2
// complex*real FMAs and no binomial table; a, b, g are all below ~1 for every
// pair the MACs accept, so nothing overflows.  The kernels (the FP64 M2L and
// M2M ones from order 30 up) apply the diagonal first, on the input phases
// ((g ph1)^l'), and then the shift by b/g: every
// elementary step a_j += b a_{j+1} of the shift turns into g^j a_j +=
// (b/g) g^{j+1} a_{j+1}, so D(g) T_b = T_{b/g} D(g) exactly and each
// intermediate is the old one times g^j (no new range, one multiply per
// coefficient fewer).  The n = 0 entry of the first shift is
// sum_l' b^l' ph1^l' A_l', the series part of C'.
#pragma once
#include "dd.hpp"

namespace sfmm {

constexpr double kInv4Pi = 0.079577471545947667884;  // 1 / (4 pi)
constexpr double kInv2Pi = 0.15915494309189533577;   // 1 / (2 pi)
constexpr double kLog2 = 0.69314718055994530942;
constexpr double kLog4 = 1.3862943611198906188;

// 1/x for a positive normal double: the hardware estimate refined by two
// Newton steps on the GPU (full precision), a division on the host.
SFMM_HD double recip(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
#else
    return 1.0 / x;
#endif
}

// Natural log of a positive normal double, ~2 ulp: x = 2^e m with
// m in [1/sqrt2, sqrt2), s = (m - 1)/(m + 1), and
//   log m = 2 atanh s = 2 s (1 + s^2/3 + s^4/5 + ... + s^20/21),
// whose first omitted term is below 3e-17 relative since s^2 <= 0.0295
// (the reduction of fdlibm's e_log.c, here with the Taylor coefficients of
// atanh instead of its minimax polynomial).  e log 2 is added with the
// Cody-Waite two-word split of log 2 that fdlibm's e_log.c uses (Sun
// Microsystems, freely distributable): ln2_hi keeps 32 significant bits, so
// e ln2_hi is exact for every exponent of a double, and ln2_lo = log 2 -
// ln2_hi to double precision.  Written for the
// near-field inner loop, where the library log (a double-double algorithm
// of ~85 instructions) dominated the cost.
SFMM_HD double log_f64(double x) {
    int e;
    double m = frexp(x, &e);  // x = m 2^e, m in [1/2, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double f = m - 1.0;  // exact (Sterbenz)
    const double s = f * recip(2.0 + f);
    const double z = s * s;
    double poly = 1.0 / 21.0;
    poly = fma(poly, z, 1.0 / 19.0);
    poly = fma(poly, z, 1.0 / 17.0);
    poly = fma(poly, z, 1.0 / 15.0);
    poly = fma(poly, z, 1.0 / 13.0);
    poly = fma(poly, z, 1.0 / 11.0);
    poly = fma(poly, z, 1.0 / 9.0);
    poly = fma(poly, z, 1.0 / 7.0);
    poly = fma(poly, z, 1.0 / 5.0);
    poly = fma(poly, z, 1.0 / 3.0);
    // 2s + 2s z poly, the small part added last
    const double two_s = 2.0 * s;
    const double lm = fma(two_s * z, poly, two_s);
    const double de = (double)e;
    const double ln2_hi = 6.93147180369123816490e-01;  // top bits of log 2, e * ln2_hi exact
    const double ln2_lo = 1.90821492927058770002e-10;
    return fma(de, ln2_hi, fma(de, ln2_lo, lm));
}

// The pair loop's log and reciprocal with a table in place of the atanh
// series (the table-driven method of P. T. P. Tang, ACM TOMS 16 (1990)
// 378-400, with a smaller table and a longer polynomial):
// x = 2^e m, m in [1/2, 1); the top 7 fraction bits of m pick c_j =
// 1/2 + (j + 1/2)/256 and tab[j] = {1/c_j, -log(1/c_j)} (log_tab_entry), so
// that r = m/c_j - 1 (one FMA) has |r| < 2^-8 and
//   log x = e log 2 - log(1/c_j) + log(1 + r),
// log(1 + r) = r + r^2 (-1/2 + r/3 - ... + r^5/7), first omitted term below
// 2^-67.  The absolute error is a few 1e-16 (no relative bound near x = 1,
// where the terms cancel; the sums it feeds only need the absolute one).
// 1/x is the reciprocal refined by two Newton steps.
// The Horner coefficients of q(r) after its leading 1/7 (the last one, -1/2,
// is an inline constant of the FMA): kernels take them as an argument, which
// keeps them in scalar registers.
struct LogPoly {
    double c6, c5, c4, c3;  // -1/6, 1/5, -1/4, 1/3
};
constexpr LogPoly kLogPoly = {-1.0 / 6.0, 1.0 / 5.0, -0.25, 1.0 / 3.0};
constexpr int kLogTab = 128;
SFMM_HD double2 log_tab_entry(int j) {
    const double c = 0.5 + (j + 0.5) / 256.0;
    const double ci = 1.0 / c;
    return make_double2(ci, -log_f64(ci));
}

SFMM_HD void log_recip_tab(double x, const double2* tab, const LogPoly& k, double* lg, double* inv) {
    int e;
    const double m = frexp(x, &e);
    const int j = (int)((__builtin_bit_cast(unsigned long long, m) >> 45) & (kLogTab - 1));
    const double2 t = tab[j];
    const double r = fma(m, t.x, -1.0);
    double q = fma(1.0 / 7.0, r, k.c6);
    q = fma(q, r, k.c5);
    q = fma(q, r, k.c4);
    q = fma(q, r, k.c3);
    q = fma(q, r, -0.5);
    const double lp = fma(r * r, q, r);
    const double de = (double)e;
    *lg = fma(de, 6.93147180369123816490e-01, fma(de, 1.90821492927058770002e-10, t.y + lp));  // log_f64's split
    *inv = recip(x);
}

struct cplx {
    double re, im;
};
SFMM_HD cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
SFMM_HD cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
SFMM_HD cplx cconj(cplx a) { return {a.re, -a.im}; }

struct Frame {
    double c[3], et[3], ep[3];
};

// e_theta and e_phi at the centre c (never a pole for a HEALPix centre)
SFMM_HD Frame make_frame(double x, double y, double z) {
    Frame f;
    f.c[0] = x;
    f.c[1] = y;
    f.c[2] = z;
    const double rxy = sqrt(x * x + y * y);
    const double inv = 1.0 / rxy;
    f.et[0] = x * z * inv;
    f.et[1] = y * z * inv;
    f.et[2] = -rxy;
    f.ep[0] = -y * inv;
    f.ep[1] = x * inv;
    f.ep[2] = 0.0;
    return f;
}

// stereographic coordinate of n in K_c; also returns 1 + n.c
SFMM_HD cplx stereo(const Frame& f, double nx, double ny, double nz, double* one_plus_cos) {
    const double dx = nx - f.c[0], dy = ny - f.c[1], dz = nz - f.c[2];
    const double sx = nx + f.c[0], sy = ny + f.c[1], sz = nz + f.c[2];
    const double den = 0.5 * (sx * sx + sy * sy + sz * sz);
    const double inv = 1.0 / den;
    *one_plus_cos = den;
    return {(dx * f.et[0] + dy * f.et[1] + dz * f.et[2]) * inv,
            (dx * f.ep[0] + dy * f.ep[1] + dz * f.ep[2]) * inv};
}

enum TransKind { kM2M = 0, kM2L = 1, kL2L = 2 };

// Everything a translation S -> T needs besides the coefficients.
struct TransGeom {
    cplx ph1, ph2;        // phase factors applied per power on input / output
    double a, b, g;       // shift parameters of the factorised T
    double bg;            // b / g: the right shift once the diagonal g^n is applied first
    double clog;          // log cos^2(T/2) (M2M, L2L) or log sin^2(T/2) (M2L)
};

// Pair geometry from centres and scales (rho = tan(R/2)) of the source box S
// and the target box T.
template <int KIND>
SFMM_HD TransGeom trans_geom(const Frame& fs, double rho_s, const Frame& ft, double rho_t) {
    TransGeom G;
    const double dx = ft.c[0] - fs.c[0], dy = ft.c[1] - fs.c[1], dz = ft.c[2] - fs.c[2];
    const double sx = ft.c[0] + fs.c[0], sy = ft.c[1] + fs.c[1], sz = ft.c[2] + fs.c[2];
    const double dif2 = dx * dx + dy * dy + dz * dz;  // 4 sin^2(T/2)
    const double sum2 = sx * sx + sy * sy + sz * sz;  // 4 cos^2(T/2)
    // phase of T's centre seen from S, and of S's centre seen from T
    cplx e1, e2;
    if (sum2 < 1e-24) {
        // exactly antipodal centres: the geodesic leaving S along e_theta(S)
        e1 = {1.0, 0.0};
        const double u = fs.et[0] * ft.et[0] + fs.et[1] * ft.et[1] + fs.et[2] * ft.et[2];
        const double v = fs.et[0] * ft.ep[0] + fs.et[1] * ft.ep[1] + fs.et[2] * ft.ep[2];
        const double r = 1.0 / sqrt(u * u + v * v);
        e2 = {u * r, v * r};
    } else {
        const double u1 = dx * fs.et[0] + dy * fs.et[1] + dz * fs.et[2];
        const double v1 = dx * fs.ep[0] + dy * fs.ep[1] + dz * fs.ep[2];
        const double r1 = 1.0 / sqrt(u1 * u1 + v1 * v1);
        e1 = {u1 * r1, v1 * r1};
        const double u2 = -(dx * ft.et[0] + dy * ft.et[1] + dz * ft.et[2]);
        const double v2 = -(dx * ft.ep[0] + dy * ft.ep[1] + dz * ft.ep[2]);
        const double r2 = 1.0 / sqrt(u2 * u2 + v2 * v2);
        e2 = {u2 * r2, v2 * r2};
    }
    if (KIND == kM2M) {
        // Lemma 2: x = tan(T/2); s_T = 1/rho_T (multipole), s_S = rho_S
        const double t = sqrt(dif2 / sum2);
        G.ph1 = {-e1.re, e1.im};  // (-1)^l' e^{-i l' phi_T^(S)}
        G.ph2 = e2;               // e^{+i l phi_S^(T)}
        G.a = t / rho_t;
        G.b = t * rho_s;
        G.g = (rho_s / rho_t) * (1.0 + t * t);
        G.bg = t * rho_t / (1.0 + t * t);
        G.clog = log_f64(0.25 * sum2);
    } else if (KIND == kM2L) {
        // Lemma 3: x = cot(T/2); s_T = rho_T (local), s_S = rho_S
        const double c = sqrt(sum2 / dif2);
        G.ph1 = cconj(e1);  // e^{-i l' phi_T^(S)}
        G.ph2 = cconj(e2);  // e^{-i l phi_S^(T)}
        G.a = c * rho_t;
        G.b = c * rho_s;
        G.g = rho_t * rho_s * (1.0 + c * c);
        G.bg = c / (rho_t * (1.0 + c * c));
        G.clog = log_f64(0.25 * dif2);
    } else {
        // Lemma 4: x = tan(T/2); s_T = rho_T (local), s_S = 1/rho_S
        const double t = sqrt(dif2 / sum2);
        G.ph1 = e1;                  // e^{+i l' phi_T^(S)}
        G.ph2 = {-e2.re, e2.im};     // (-1)^l e^{-i l phi_S^(T)}
        G.a = t * rho_t;
        G.b = t / rho_s;
        G.g = (rho_t / rho_s) * (1.0 + t * t);
        G.bg = t / (rho_t * (1.0 + t * t));
        G.clog = log_f64(0.25 * sum2);
    }
    return G;
}

// Expansion record: e[0] = C, e[1] = Q, e[2 + 2(l-1)] = Re A_l, e[3 + 2(l-1)]
// = Im A_l (scaled).  Adds the translated expansion of `in` to acc.
template <int P>
SFMM_HD void translate_add(const double* in, const TransGeom& G, double* acc) {
    double ar[P + 1], ai[P + 1];
    const double C = in[0], Q = in[1];
    ar[0] = 0.0;
    ai[0] = 0.0;
    // diagonal g^n first, on the input phases: D(g) T_b = T_{b/g} D(g)
    const cplx pg = {G.ph1.re * G.g, G.ph1.im * G.g};
    cplx pw = pg;
#pragma unroll
    for (int l = 1; l <= P; ++l) {
        const cplx a = {in[2 * l], in[2 * l + 1]};
        const cplx v = cmul(pw, a);
        ar[l] = v.re;
        ai[l] = v.im;
        pw = cmul(pw, pg);
    }
    // right factor: Taylor shift by b/g, a[j] += (b/g) a[j+1]
#pragma unroll
    for (int i = 0; i < P; ++i) {
#pragma unroll
        for (int j = P - 1; j >= i; --j) {
            ar[j] = fma(G.bg, ar[j + 1], ar[j]);
            ai[j] = fma(G.bg, ai[j + 1], ai[j]);
        }
    }
    const double u0 = ar[0];
    // left factor: transposed Taylor shift by a on entries 1..P
#pragma unroll
    for (int i = P - 2; i >= 0; --i) {
#pragma unroll
        for (int j = i; j <= P - 2; ++j) {
            ar[j + 2] = fma(G.a, ar[j + 1], ar[j + 2]);
            ai[j + 2] = fma(G.a, ai[j + 1], ai[j + 2]);
        }
    }
    cplx pw2 = G.ph2;
    double an = G.a;
#pragma unroll
    for (int l = 1; l <= P; ++l) {
        const cplx v = {fma(-Q * (1.0 / l), an, ar[l]), ai[l]};  // 1.0 / l folds to a constant
        const cplx o = cmul(pw2, v);
        acc[2 * l] += o.re;
        acc[2 * l + 1] += o.im;
        pw2 = cmul(pw2, G.ph2);
        an *= G.a;
    }
    acc[0] += C + Q * G.clog + 2.0 * u0;
    acc[1] += Q;
}

// translate_add for one order class of a per-pair order policy: the pair's
// multipole part translated at order P, its monopole part (-(Q/l) a^l, the
// source as a point mass) completed up to the record order PO; acc holds
// 2 PO + 2 entries.
template <int P, int PO>
SFMM_HD void translate_add_po(const double* in, const TransGeom& G, double* acc) {
    translate_add<P>(in, G, acc);
    if constexpr (PO > P) {
        const double Q = in[1];
        cplx pw2 = G.ph2;
        double an = G.a;
#pragma unroll
        for (int l = 1; l <= P; ++l) {  // powers up to P
            pw2 = cmul(pw2, G.ph2);
            an *= G.a;
        }
#pragma unroll
        for (int l = P + 1; l <= PO; ++l) {
            const double v = -Q * (1.0 / l) * an;
            acc[2 * l] = fma(pw2.re, v, acc[2 * l]);
            acc[2 * l + 1] = fma(pw2.im, v, acc[2 * l + 1]);
            pw2 = cmul(pw2, G.ph2);
            an *= G.a;
        }
    }
}

// translate_add without an accumulator: in(k) gives input entry k and
// out(k, v) takes output entry k as soon as it is formed (entries 2..2P+1 in
// order, then C and Q), for kernels with one translation per lane.  Without
// the 2P + 2 accumulator registers two waves fit on a SIMD.
template <int P, class In, class Out>
SFMM_HD void translate_emit(const In& in, const TransGeom& G, const Out& out) {
    double ar[P + 1], ai[P + 1];
    const double C = in(0), Q = in(1);
    ar[0] = 0.0;
    ai[0] = 0.0;
    // from order 30 up the diagonal g^n moves in front of the right shift
    // (D(g) T_b = T_{b/g} D(g)), where it rides on the input phases: (g
    // ph1)^l.  Measured on the two-lane M2L: 3.00 -> 2.83 ms at p = 38
    // (N = 1e7); at p = 20 (N = 1e8) the folded form ran 15.5 ms against 11.2.
    constexpr bool kDiagFirst = P >= 30;
    const cplx pg = kDiagFirst ? cplx{G.ph1.re * G.g, G.ph1.im * G.g} : G.ph1;
    const double bs = kDiagFirst ? G.bg : G.b;
    cplx pw = pg;
#pragma unroll
    for (int l = 1; l <= P; ++l) {
        const cplx a = {in(2 * l), in(2 * l + 1)};
        const cplx v = cmul(pw, a);
        ar[l] = v.re;
        ai[l] = v.im;
        pw = cmul(pw, pg);
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
#pragma unroll
        for (int j = P - 1; j >= i; --j) {
            ar[j] = fma(bs, ar[j + 1], ar[j]);
            ai[j] = fma(bs, ai[j + 1], ai[j]);
        }
    }
    const double u0 = ar[0];
    if constexpr (!kDiagFirst) {
        double gn = G.g;
#pragma unroll
        for (int n = 1; n <= P; ++n) {
            ar[n] *= gn;
            ai[n] *= gn;
            gn *= G.g;
        }
    }
#pragma unroll
    for (int i = P - 2; i >= 0; --i) {
#pragma unroll
        for (int j = i; j <= P - 2; ++j) {
            ar[j + 2] = fma(G.a, ar[j + 1], ar[j + 2]);
            ai[j + 2] = fma(G.a, ai[j + 1], ai[j + 2]);
        }
    }
    cplx pw2 = G.ph2;
    double an = G.a;
#pragma unroll
    for (int l = 1; l <= P; ++l) {
        const cplx v = {fma(-Q * (1.0 / l), an, ar[l]), ai[l]};  // 1.0 / l folds to a constant
        const cplx o = cmul(pw2, v);
        out(2 * l, o.re);
        out(2 * l + 1, o.im);
        pw2 = cmul(pw2, G.ph2);
        an *= G.a;
    }
    out(0, C + Q * G.clog + 2.0 * u0);
    out(1, Q);
}

// FP32 complex numbers for the precision tier's translation (below).
struct cplxf {
    float re, im;
};
SFMM_HD cplxf cmulf(cplxf a, cplxf b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// The precision tier's Lemma 3 translation: the FP32 A-block (scaled,
// A[2l-2] = Re A_l, A[2l-1] = Im A_l) through the factorised map in FP32,
// with the pair geometry G computed in FP64 and rounded once; the results
// are added to acc[2P] in FP64, so the sum over an FMM-act list carries no
// FP32 rounding, and C and Q stay FP64 (accCQ).  With PO > P (a pair whose
// own order P is below the record order PO) the multipole part is cut at P
// and the monopole part, -(Q/l) a^l ph2^l, still runs to PO: acc[2 PO].
template <int P, int PO = P>
SFMM_HD void translate_add_f32_d(const float* __restrict__ A, double C, double Q, const TransGeom& G, double* acc,
                                 double* accCQ) {
    float ar[P + 1], ai[P + 1];
    ar[0] = 0.0f;
    ai[0] = 0.0f;
    const cplxf ph2 = {(float)G.ph2.re, (float)G.ph2.im};
    // diagonal g^n first, on the input phases: D(g) T_b = T_{b/g} D(g)
    const float a = (float)G.a, bg = (float)G.bg;
    const cplxf pg = {(float)(G.ph1.re * G.g), (float)(G.ph1.im * G.g)};
    cplxf pw = pg;
#pragma unroll
    for (int l = 1; l <= P; ++l) {
        const cplxf v = cmulf(pw, cplxf{A[2 * l - 2], A[2 * l - 1]});
        ar[l] = v.re;
        ai[l] = v.im;
        pw = cmulf(pw, pg);
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
#pragma unroll
        for (int j = P - 1; j >= i; --j) {
            ar[j] = fmaf(bg, ar[j + 1], ar[j]);
            ai[j] = fmaf(bg, ai[j + 1], ai[j]);
        }
    }
    const double u0 = (double)ar[0];
#pragma unroll
    for (int i = P - 2; i >= 0; --i) {
#pragma unroll
        for (int j = i; j <= P - 2; ++j) {
            ar[j + 2] = fmaf(a, ar[j + 1], ar[j + 2]);
            ai[j + 2] = fmaf(a, ai[j + 1], ai[j + 2]);
        }
    }
    const float qf = (float)Q;
    cplxf pw2 = ph2;
    float an = a;
#pragma unroll
    for (int l = 1; l <= P; ++l) {
        const cplxf v = {ar[l] - qf * (1.0f / l) * an, ai[l]};
        const cplxf o = cmulf(pw2, v);
        acc[2 * l - 2] += (double)o.re;
        acc[2 * l - 1] += (double)o.im;
        pw2 = cmulf(pw2, ph2);
        an *= a;
    }
#pragma unroll
    for (int l = P + 1; l <= PO; ++l) {
        const float v = -qf * (1.0f / l) * an;
        acc[2 * l - 2] += (double)(pw2.re * v);
        acc[2 * l - 1] += (double)(pw2.im * v);
        pw2 = cmulf(pw2, ph2);
        an *= a;
    }
    accCQ[0] += C + Q * G.clog + 2.0 * u0;
    accCQ[1] += Q;
}

// Lemma 1 for a set of particles about centre f with scale rho; C carries the
// zero-mean gauge's share sum q / (4 pi) (Eq. STAND_CONDITION).
template <int P>
struct P2MAcc {
    double sre[P], sim[P];
    double slog, sq;
};

template <int P>
SFMM_HD void p2m_init(P2MAcc<P>& a) {
#pragma unroll
    for (int l = 0; l < P; ++l) a.sre[l] = a.sim[l] = 0.0;
    a.slog = 0.0;
    a.sq = 0.0;
}

template <int P>
SFMM_HD void p2m_add(P2MAcc<P>& a, const Frame& f, double inv_rho, double x, double y, double z, double q) {
    double opc;
    cplx w = stereo(f, x, y, z, &opc);
    w.re *= inv_rho;
    w.im *= inv_rho;
    cplx pw = w;
#pragma unroll
    for (int l = 0; l < P; ++l) {
        a.sre[l] = fma(q, pw.re, a.sre[l]);
        a.sim[l] = fma(q, pw.im, a.sim[l]);
        pw = cmul(pw, w);
    }
    a.slog = fma(q, log_f64(0.5 * opc), a.slog);  // 2 log cos(theta/2) = log((1 + cos)/2)
    a.sq += q;
}

template <int P>
SFMM_HD void p2m_finish(const P2MAcc<P>& a, double* out) {
    const double Q = a.sq * kInv4Pi;
    out[0] = a.slog * kInv4Pi - Q * kLog2 + Q;
    out[1] = Q;
#pragma unroll
    for (int l = 1; l <= P; ++l) {
        const double s = -kInv4Pi / l;
        out[2 * l] = s * a.sre[l - 1];
        out[2 * l + 1] = s * a.sim[l - 1];
    }
}

// Local expansion at a point (Sec. 3.6), pole-free: psi_e and the tangent
// vector alpha_e = grad psi_e in global axes.  With f(w) = sum A_l w^l,
// psi_e = C + Q log(1 + cos theta) + 2 Re f and, in the orthonormal basis of
// the w-plane, alpha_u + i alpha_v = (1 + |w|^2) conj(f'(w)) - Q w.
template <int P>
SFMM_HD void l2p_eval(const double* e, const Frame& f, double rho, double nx, double ny, double nz,
                      double* psi, double* ax, double* ay, double* az) {
    double opc;
    const cplx w = stereo(f, nx, ny, nz, &opc);
    const double inv_rho = 1.0 / rho;
    const cplx zt = {w.re * inv_rho, w.im * inv_rho};
    // f = sum L_l zt^l by Horner from the top coefficient and g = f'(zt) =
    // sum l L_l zt^(l-1) by the companion recurrence d <- d zt + p
    cplx pv = {e[2 * P], e[2 * P + 1]}, gv = {0.0, 0.0};
#pragma unroll
    for (int l = P - 1; l >= 1; --l) {
        gv = {fma(gv.re, zt.re, fma(-gv.im, zt.im, pv.re)), fma(gv.re, zt.im, fma(gv.im, zt.re, pv.im))};
        pv = {fma(pv.re, zt.re, fma(-pv.im, zt.im, e[2 * l])), fma(pv.re, zt.im, fma(pv.im, zt.re, e[2 * l + 1]))};
    }
    gv = {fma(gv.re, zt.re, fma(-gv.im, zt.im, pv.re)), fma(gv.re, zt.im, fma(gv.im, zt.re, pv.im))};
    const cplx fv = cmul(pv, zt);
    const double C = e[0], Q = e[1];
    *psi = C + Q * log_f64(opc) + 2.0 * fv.re;
    // f'(w) = g / rho
    const double w2 = w.re * w.re + w.im * w.im;
    const double s = (1.0 + w2) * inv_rho;
    const double Ar = s * gv.re - Q * w.re;
    const double Ai = -s * gv.im - Q * w.im;
    const double inv = 1.0 / (1.0 + w2);
    const double u = w.re, v = w.im;
    // e_u = ((1+v^2-u^2) e_t - 2uv e_p - 2u c)/(1+|w|^2), e_v likewise
    const double eu_t = (1.0 + v * v - u * u) * inv, eu_p = -2.0 * u * v * inv, eu_c = -2.0 * u * inv;
    const double ev_t = -2.0 * u * v * inv, ev_p = (1.0 + u * u - v * v) * inv, ev_c = -2.0 * v * inv;
    const double at = Ar * eu_t + Ai * ev_t, ap = Ar * eu_p + Ai * ev_p, ac = Ar * eu_c + Ai * ev_c;
    *ax = at * f.et[0] + ap * f.ep[0] + ac * f.c[0];
    *ay = at * f.et[1] + ap * f.ep[1] + ac * f.c[1];
    *az = at * f.et[2] + ap * f.ep[2] + ac * f.c[2];
}

// Multipole expansion (Lemma 1 form) of a source box evaluated at a point n
// far from it: psi = C + Q log(1 - cos theta) + 2 Re sum A_l w^-l and its
// tangent gradient.  With zeta = rho / w, f = sum Ah_l zeta^l and
// g = sum l Ah_l zeta^l (Ah the scaled coefficients), the w-plane gradient of
// 2 Re f is -2 conj(g / w) and that of Q log(1 - cos) = Q log(2|w|^2/(1+|w|^2))
// is 2 Q w / (|w|^2 (1 + |w|^2)), so
//   alpha_u + i alpha_v = (Q - (1 + |w|^2) conj(g)) / conj(w).
template <int P>
SFMM_HD void m2p_eval(const double* __restrict__ e, const Frame& f, double rho, double nx, double ny, double nz,
                      double* psi, double* ax, double* ay, double* az) {
    double opc;
    const cplx w = stereo(f, nx, ny, nz, &opc);
    const double dx = nx - f.c[0], dy = ny - f.c[1], dz = nz - f.c[2];
    const double omc = 0.5 * (dx * dx + dy * dy + dz * dz);  // 1 - cos theta
    const double w2 = w.re * w.re + w.im * w.im;
    const double iw2 = recip(w2);
    const cplx zt = {rho * w.re * iw2, -rho * w.im * iw2};  // rho / w
    // F = h(zt) = sum_l A_l zt^l and G = zt h'(zt) = sum_l l A_l zt^l: Horner
    // for h from the top coefficient, its derivative by the companion
    // recurrence d <- d zt + p (two FMAs per real part, no l factors)
    cplx pv = {e[2 * P], e[2 * P + 1]}, dv = {0.0, 0.0};
#pragma unroll 6
    for (int l = P - 1; l >= 1; --l) {
        dv = {fma(dv.re, zt.re, fma(-dv.im, zt.im, pv.re)), fma(dv.re, zt.im, fma(dv.im, zt.re, pv.im))};
        pv = {fma(pv.re, zt.re, fma(-pv.im, zt.im, e[2 * l])), fma(pv.re, zt.im, fma(pv.im, zt.re, e[2 * l + 1]))};
    }
    dv = {fma(dv.re, zt.re, fma(-dv.im, zt.im, pv.re)), fma(dv.re, zt.im, fma(dv.im, zt.re, pv.im))};
    const cplx F = cmul(pv, zt), G = cmul(dv, zt);
    const double C = e[0], Q = e[1];
    *psi = C + Q * log_f64(omc) + 2.0 * F.re;
    // (Q - (1+|w|^2) conj(G)) / conj(w) = (Q - s conj(G)) * w / |w|^2
    const double s = 1.0 + w2;
    const cplx num = {Q - s * G.re, s * G.im};
    const cplx A = {(num.re * w.re - num.im * w.im) * iw2, (num.re * w.im + num.im * w.re) * iw2};
    const double inv = recip(s);
    const double u = w.re, v = w.im;
    const double eu_t = (1.0 + v * v - u * u) * inv, eu_p = -2.0 * u * v * inv, eu_c = -2.0 * u * inv;
    const double ev_t = -2.0 * u * v * inv, ev_p = (1.0 + u * u - v * v) * inv, ev_c = -2.0 * v * inv;
    const double at = A.re * eu_t + A.im * ev_t, ap = A.re * eu_p + A.im * ev_p, ac = A.re * eu_c + A.im * ev_c;
    *ax = at * f.et[0] + ap * f.ep[0] + ac * f.c[0];
    *ay = at * f.et[1] + ap * f.ep[1] + ac * f.c[1];
    *az = at * f.et[2] + ap * f.ep[2] + ac * f.c[2];
}


// ---------------------------------------------------------------- Hessian
// The Hessian of Sec. 2.2 (second covariant derivatives of psi in the basis
// e_theta, e_phi of the target).  In the stereographic coordinate w = u + iv
// of a box frame the sphere's metric is conformal, (2 / D)^2 |dw|^2 with
// D = 1 + |w|^2, and the covariant Hessian of psi in the orthonormal basis
// (e_u, e_v) of the w-plane is
//   H_uu + H_vv = (D^2 / 4) Laplacian_w psi,
//   H_uu - H_vv - 2i H_uv = Z = D^2 (psi_ww - 2 sigma_w psi_w),
// with psi_w = d psi / dw, sigma = log(2 / D) (so sigma_w = -conj(w) / D).
// For the local form psi = C + Q log(1 + cos) + 2 Re f(w), f = sum A_l w^l:
//   Z = D^2 f'' + 2 conj(w) D f' - Q conj(w)^2,   trace -Q;
// for the multipole form psi = C + Q log(1 - cos) + 2 Re f(w), f = sum A_l
// w^-l:
//   Z = D^2 f'' + 2 conj(w) D f' - Q / w^2,       trace -Q.
// Both are regular at w = 0 (the local form at a box centre) and need no
// angle.  The (e_u, e_v) components are then turned into the target's
// (e_theta, e_phi) ones.

// e_theta, e_phi of the target n (phi = 0 at an exact pole)
SFMM_HD void target_basis(double nx, double ny, double nz, double* et, double* ep) {
    const double rxy = sqrt(nx * nx + ny * ny);
    const double cph = rxy > 0.0 ? nx / rxy : 1.0, sph = rxy > 0.0 ? ny / rxy : 0.0;
    et[0] = nz * cph;
    et[1] = nz * sph;
    et[2] = -rxy;
    ep[0] = -sph;
    ep[1] = cph;
    ep[2] = 0.0;
}

// (H_uu, H_uv, H_vv) in the w-plane basis of frame f at w -> (H_tt, H_tp,
// H_pp) in the basis et, ep of the target
SFMM_HD void hess_to_target(const Frame& f, cplx w, double huu, double huv, double hvv, const double* et,
                            const double* ep, double* h) {
    const double u = w.re, v = w.im;
    const double inv = 1.0 / (1.0 + u * u + v * v);
    const double eu_t = (1.0 + v * v - u * u) * inv, eu_p = -2.0 * u * v * inv, eu_c = -2.0 * u * inv;
    const double ev_t = -2.0 * u * v * inv, ev_p = (1.0 + u * u - v * v) * inv, ev_c = -2.0 * v * inv;
    double eu[3], ev[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        eu[d] = eu_t * f.et[d] + eu_p * f.ep[d] + eu_c * f.c[d];
        ev[d] = ev_t * f.et[d] + ev_p * f.ep[d] + ev_c * f.c[d];
    }
    const double tu = et[0] * eu[0] + et[1] * eu[1] + et[2] * eu[2];
    const double tv = et[0] * ev[0] + et[1] * ev[1] + et[2] * ev[2];
    const double pu = ep[0] * eu[0] + ep[1] * eu[1] + ep[2] * eu[2];
    const double pv = ep[0] * ev[0] + ep[1] * ev[1] + ep[2] * ev[2];
    h[0] = tu * tu * huu + 2.0 * tu * tv * huv + tv * tv * hvv;
    h[1] = tu * pu * huu + (tu * pv + tv * pu) * huv + tv * pv * hvv;
    h[2] = pu * pu * huu + 2.0 * pu * pv * huv + pv * pv * hvv;
}

// l2p_eval and the Hessian h[3] of the local expansion at the target
// (et, ep its basis)
template <int P>
SFMM_HD void l2p_eval_hess(const double* e, const Frame& f, double rho, double nx, double ny, double nz,
                           const double* et, const double* ep, double* psi, double* ax, double* ay, double* az,
                           double* h) {
    l2p_eval<P>(e, f, rho, nx, ny, nz, psi, ax, ay, az);
    double opc;
    const cplx w = stereo(f, nx, ny, nz, &opc);
    const double inv_rho = 1.0 / rho;
    const cplx zt = {w.re * inv_rho, w.im * inv_rho};
    // Horner for q(z) = sum L_l z^(l-1) with its first derivative dv and
    // half its second ev; then g = (z q)' and k = (z q)'' = 2 (dv + z ev)
    cplx pv = {e[2 * P], e[2 * P + 1]}, dv = {0.0, 0.0}, ev = {0.0, 0.0};
#pragma unroll
    for (int l = P - 1; l >= 1; --l) {
        ev = cadd(cmul(ev, zt), dv);
        dv = cadd(cmul(dv, zt), pv);
        pv = cadd(cmul(pv, zt), cplx{e[2 * l], e[2 * l + 1]});
    }
    const cplx g = cadd(cmul(dv, zt), pv);
    const cplx k = cmul(cplx{2.0, 0.0}, cadd(dv, cmul(zt, ev)));
    const double Q = e[1];
    const double D = 1.0 + w.re * w.re + w.im * w.im;
    const cplx wc = {w.re, -w.im};
    // Z = D^2 f'' + 2 conj(w) D f' - Q conj(w)^2, f' = g / rho, f'' = k / rho^2
    const cplx t1 = cmul(cplx{D * D * inv_rho * inv_rho, 0.0}, k);
    const cplx t2 = cmul(cplx{2.0 * D * inv_rho, 0.0}, cmul(wc, g));
    const cplx wc2 = cmul(wc, wc);
    const cplx Z = {t1.re + t2.re - Q * wc2.re, t1.im + t2.im - Q * wc2.im};
    hess_to_target(f, w, 0.5 * (-Q + Z.re), -0.5 * Z.im, 0.5 * (-Q - Z.re), et, ep, h);
}

// m2p_eval and the Hessian h[3] of a source box's multipole expansion at
// the target (et, ep its basis).  With zeta = rho / w and F(zeta) = sum Ah_l
// zeta^l: f' = -G / w and f'' = K / w^2, G = sum l Ah_l zeta^l, K = sum
// l (l + 1) Ah_l zeta^l.
template <int P>
SFMM_HD void m2p_eval_hess(const double* __restrict__ e, const Frame& f, double rho, double nx, double ny,
                           double nz, const double* et, const double* ep, double* psi, double* ax, double* ay,
                           double* az, double* h) {
    m2p_eval<P>(e, f, rho, nx, ny, nz, psi, ax, ay, az);
    double opc;
    const cplx w = stereo(f, nx, ny, nz, &opc);
    const double w2 = w.re * w.re + w.im * w.im;
    const double iw2 = 1.0 / w2;
    const cplx zt = {rho * w.re * iw2, -rho * w.im * iw2};   // rho / w
    const cplx iw = {w.re * iw2, -w.im * iw2};               // 1 / w
    // Horner for q(z) = sum Ah_l z^(l-1), its derivative dv and half its
    // second ev: F = z q, F' = q + z dv, F'' = 2 (dv + z ev)
    cplx pv = {e[2 * P], e[2 * P + 1]}, dv = {0.0, 0.0}, ev = {0.0, 0.0};
#pragma unroll 4
    for (int l = P - 1; l >= 1; --l) {
        ev = cadd(cmul(ev, zt), dv);
        dv = cadd(cmul(dv, zt), pv);
        pv = cadd(cmul(pv, zt), cplx{e[2 * l], e[2 * l + 1]});
    }
    const cplx F1 = cadd(pv, cmul(zt, dv));
    const cplx F2 = cmul(cplx{2.0, 0.0}, cadd(dv, cmul(zt, ev)));
    const cplx G = cmul(zt, F1);
    const cplx z2 = cmul(zt, zt);
    const cplx K = cadd(cmul(z2, F2), cmul(cplx{2.0, 0.0}, G));
    const double Q = e[1];
    const double D = 1.0 + w2;
    const cplx wc = {w.re, -w.im};
    const cplx iw2c = cmul(iw, iw);  // 1 / w^2
    // Z = D^2 K / w^2 - 2 conj(w) D G / w - Q / w^2
    const cplx a = cmul(cplx{D * D, 0.0}, cmul(K, iw2c));
    const cplx b = cmul(cplx{2.0 * D, 0.0}, cmul(wc, cmul(G, iw)));
    const cplx Z = {a.re - b.re - Q * iw2c.re, a.im - b.im - Q * iw2c.im};
    hess_to_target(f, w, 0.5 * (-Q + Z.re), -0.5 * Z.im, 0.5 * (-Q - Z.re), et, ep, h);
}

}  // namespace sfmm
