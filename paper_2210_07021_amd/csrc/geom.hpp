// Sphere geometry of the sFMM tree (Sec. 3.1 division, Sec. 3.5 box radius
// and distance): HEALPix nested keys at order 29, pixel points, box radii,
// angular distances, and the two MAC predicates.
//
// Keys and MAC decisions are exact-arithmetic decisions: an FP64 evaluation
// settles every case whose margin exceeds a rigorous bound on its rounding
// error, and the rest (points within ~1e-5 pixel of an edge, box pairs within
// 1e-13 rad of a MAC threshold, congruent boxes of equal radius) are re-done
// in double-double.  Exact-arithmetic ties (HEALPix has many: the vertex
// shared by two diagonal neighbours is the geodesic midpoint of their
// centres) are decided "not far", as the strict inequalities say.
#pragma once
#include "dd.hpp"
#include <cstdint>

namespace sfmm {

constexpr int kOrder = 29;                 // maximum depth of Sec. 3.1
constexpr double kTieRel = 1e-20;          // relative guard of exact ties
constexpr double kMacFilter = 1e-13;       // FP64 margin that needs no recheck (rad)
constexpr double kKeyFilter = 1e-5;        // FP64 distance to a pixel edge that needs no recheck

// HEALPix face layout (Gorski et al. 2005): ring of each face's southern
// corner in units of nside, and azimuth of the face centre in units of pi/4.
SFMM_HD int face_ring(int f) { return 2 + (f >> 2); }
SFMM_HD int face_phi(int f) {
    // faces 0-3 and 8-11 sit at odd multiples of pi/4, faces 4-7 at even
    return (f >> 2) == 1 ? 2 * (f & 3) : 2 * (f & 3) + 1;
}

SFMM_HD uint64_t spread_bits(uint64_t v) {
    v &= 0x3fffffffULL;
    v = (v | (v << 16)) & 0x0000ffff0000ffffULL;
    v = (v | (v << 8)) & 0x00ff00ff00ff00ffULL;
    v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0fULL;
    v = (v | (v << 2)) & 0x3333333333333333ULL;
    v = (v | (v << 1)) & 0x5555555555555555ULL;
    return v;
}

SFMM_HD uint64_t compact_bits(uint64_t v) {
    v &= 0x5555555555555555ULL;
    v = (v | (v >> 1)) & 0x3333333333333333ULL;
    v = (v | (v >> 2)) & 0x0f0f0f0f0f0f0f0fULL;
    v = (v | (v >> 4)) & 0x00ff00ff00ff00ffULL;
    v = (v | (v >> 8)) & 0x0000ffff0000ffffULL;
    v = (v | (v >> 16)) & 0x00000000ffffffffULL;
    return v;
}

SFMM_HD uint64_t nest_index(int64_t face, int64_t ix, int64_t iy) {
    return ((uint64_t)face << (2 * kOrder)) + spread_bits((uint64_t)ix) + (spread_bits((uint64_t)iy) << 1);
}

// Order-29 nested key of the unit vector (x, y, z), double-double evaluation.
SFMM_HD uint64_t key_dd(double x, double y, double z) {
    const int64_t ns = (int64_t)1 << kOrder;
    const double za = fabs(z);
    dd tt = dd_mul(dd_atan2(dd_from(y), dd_from(x)), dd_two_over_pi());
    {
        const double r = nearbyint(tt.hi);
        if (fabs(dd_sub(tt, dd_from(r)).hi) < 1e-20) tt = dd_from(r);
    }
    if (tt.hi < 0.0) tt = dd_add(tt, dd_from(4.0));
    if (!dd_lt(tt, dd_from(4.0))) tt = dd_sub(tt, dd_from(4.0));
    int64_t face, ix, iy;
    const dd two_thirds = dd_div(dd_from(2.0), dd_from(3.0));
    if (!dd_lt(two_thirds, dd_from(za))) {
        const dd a = dd_mul_d(dd_add(dd_from(0.5), tt), (double)ns);
        const dd b = dd_mul_d(two_prod(z, 0.75), (double)ns);
        const int64_t jp = dd_floor_snap(dd_sub(a, b));
        const int64_t jm = dd_floor_snap(dd_add(a, b));
        const int64_t fp = jp >> kOrder, fm = jm >> kOrder;
        face = (fp == fm) ? (fp | 4) : (fp < fm ? fp : fm + 8);
        ix = jm & (ns - 1);
        iy = ns - (jp & (ns - 1)) - 1;
    } else {
        int ntt = (int)tt.hi;
        if (tt.hi == (double)ntt && tt.lo < 0.0) ntt -= 1;
        if (ntt > 3) ntt = 3;
        const dd tp = dd_sub(tt, dd_from((double)ntt));
        dd s;
        if (za < 0.99) {
            s = dd_sqrt(two_prod(3.0, 1.0 - za));  // 1 - za is exact for za > 1/2
        } else {
            const dd sth = dd_sqrt(dd_add(two_prod(x, x), two_prod(y, y)));
            s = dd_div(sth, dd_sqrt(dd_div(two_sum(1.0, za), dd_from(3.0))));
        }
        s = dd_mul_d(s, (double)ns);
        int64_t jp = dd_floor_snap(dd_mul(tp, s));
        int64_t jm = dd_floor_snap(dd_mul(dd_sub(dd_from(1.0), tp), s));
        if (jp > ns - 1) jp = ns - 1;
        if (jm > ns - 1) jm = ns - 1;
        if (z >= 0.0) {
            face = ntt;
            ix = ns - jm - 1;
            iy = ns - jp - 1;
        } else {
            face = ntt + 8;
            ix = jp;
            iy = jm;
        }
    }
    return nest_index(face, ix, iy);
}

SFMM_HD bool near_integer(double v, double tol) { return fabs(v - nearbyint(v)) < tol; }

// Order-29 nested key: FP64 with an exactness filter, double-double when a
// floor argument or a branch test lies within its FP64 error of a boundary.
SFMM_HD uint64_t key29(double x, double y, double z) {
    const int64_t ns = (int64_t)1 << kOrder;
    const double za = fabs(z);
    double tt = atan2(y, x) * 0.63661977236758138243;
    if (tt < 0.0) tt += 4.0;
    if (tt >= 4.0) tt -= 4.0;
    bool fragile = near_integer(tt, 1e-13) || fabs(za - 2.0 / 3.0) < 1e-14;
    int64_t face = 0, ix = 0, iy = 0;
    if (za <= 2.0 / 3.0) {
        const double a = (double)ns * (0.5 + tt);
        const double b = (double)ns * (z * 0.75);
        const double vp = a - b, vm = a + b;
        fragile |= near_integer(vp, kKeyFilter) || near_integer(vm, kKeyFilter);
        const int64_t jp = (int64_t)floor(vp), jm = (int64_t)floor(vm);
        const int64_t fp = jp >> kOrder, fm = jm >> kOrder;
        face = (fp == fm) ? (fp | 4) : (fp < fm ? fp : fm + 8);
        ix = jm & (ns - 1);
        iy = ns - (jp & (ns - 1)) - 1;
    } else {
        int ntt = (int)tt;
        if (ntt > 3) ntt = 3;
        const double tp = tt - ntt;
        double s;
        if (za < 0.99) {
            s = (double)ns * sqrt(3.0 * (1.0 - za));
        } else {
            const double sth = sqrt(x * x + y * y);
            s = (double)ns * sth / sqrt((1.0 + za) / 3.0);
        }
        const double vp = tp * s, vm = (1.0 - tp) * s;
        fragile |= near_integer(vp, kKeyFilter) || near_integer(vm, kKeyFilter);
        int64_t jp = (int64_t)floor(vp), jm = (int64_t)floor(vm);
        if (jp > ns - 1) jp = ns - 1;
        if (jm > ns - 1) jm = ns - 1;
        if (z >= 0.0) {
            face = ntt;
            ix = ns - jm - 1;
            iy = ns - jp - 1;
        } else {
            face = ntt + 8;
            ix = jp;
            iy = jm;
        }
    }
    if (fragile) return key_dd(x, y, z);
    return nest_index(face, ix, iy);
}

// Point of pixel (level, pix) at face coordinates (fx, fy) in [0,1]^2, in
// double-double: the centre is (1/2, 1/2), the vertices the corners.
SFMM_HD void pix_point_dd(int level, uint64_t pix, double fx, double fy, dd* out) {
    const double ns = (double)((int64_t)1 << level);
    const int face = (int)(pix >> (2 * level));
    const uint64_t inface = pix & ((1ULL << (2 * level)) - 1);
    // x = (ix + fx)/ns exactly in double-double (ix < 2^29, fx dyadic)
    const dd x = dd_mul_d(two_sum((double)compact_bits(inface), fx), 1.0 / ns);
    const dd y = dd_mul_d(two_sum((double)compact_bits(inface >> 1), fy), 1.0 / ns);
    const dd jr = dd_sub(dd_sub(dd_from((double)face_ring(face)), x), y);
    dd nr, z, sth;
    if (jr.hi < 1.0) {
        nr = jr;
        const dd t = dd_div(dd_mul(nr, nr), dd_from(3.0));
        z = dd_sub(dd_from(1.0), t);
        sth = dd_sqrt(dd_mul(t, dd_sub(dd_from(2.0), t)));
    } else if (jr.hi > 3.0) {
        nr = dd_sub(dd_from(4.0), jr);
        const dd t = dd_div(dd_mul(nr, nr), dd_from(3.0));
        z = dd_sub(t, dd_from(1.0));
        sth = dd_sqrt(dd_mul(t, dd_sub(dd_from(2.0), t)));
    } else {
        nr = dd_from(1.0);
        z = dd_div(dd_mul_d(dd_sub(dd_from(2.0), jr), 2.0), dd_from(3.0));
        sth = dd_sqrt(dd_mul(dd_sub(dd_from(1.0), z), dd_add(dd_from(1.0), z)));
    }
    dd u = dd_sub(dd_add(dd_mul_d(nr, (double)face_phi(face)), x), y);
    if (u.hi < 0.0) u = dd_add(u, dd_from(8.0));
    if (!dd_lt(u, dd_from(8.0))) u = dd_sub(u, dd_from(8.0));
    dd phi = dd_from(0.0);
    if (nr.hi != 0.0) phi = dd_div(dd_mul(dd_quarter_pi(), u), nr);
    dd s, c;
    dd_sincos(phi, &s, &c);
    out[0] = dd_mul(sth, c);
    out[1] = dd_mul(sth, s);
    out[2] = z;
    // a coordinate this small is an exact zero of the geometry (azimuth at a
    // multiple of pi/2); a genuine one is never below ~1e-18
    for (int k = 0; k < 3; ++k)
        if (fabs(out[k].hi) < 1e-25) out[k] = dd_from(0.0);
}

// Angular distance of two double-double unit vectors: atan2(|a x b|, a.b).
SFMM_HD dd angdist_dd(const dd* a, const dd* b) {
    const dd cx = dd_sub(dd_mul(a[1], b[2]), dd_mul(a[2], b[1]));
    const dd cy = dd_sub(dd_mul(a[2], b[0]), dd_mul(a[0], b[2]));
    const dd cz = dd_sub(dd_mul(a[0], b[1]), dd_mul(a[1], b[0]));
    const dd s = dd_sqrt(dd_add(dd_add(dd_mul(cx, cx), dd_mul(cy, cy)), dd_mul(cz, cz)));
    const dd c = dd_add(dd_add(dd_mul(a[0], b[0]), dd_mul(a[1], b[1])), dd_mul(a[2], b[2]));
    return dd_atan2(s, c);
}

SFMM_HD double angdist(double ax, double ay, double az, double bx, double by, double bz) {
    const double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
    return atan2(sqrt(cx * cx + cy * cy + cz * cz), ax * bx + ay * by + az * bz);
}

// Box geometry in double-double: centre (x,y,z) and covering radius R, the
// largest angular distance from the centre to the pixel's vertices.
struct BoxGeomDD {
    dd c[3];
    dd r;
};

SFMM_HD BoxGeomDD box_geometry(int level, uint64_t pix) {
    BoxGeomDD g;
    pix_point_dd(level, pix, 0.5, 0.5, g.c);
    // the farthest vertex is the one of largest chord |v - c| (the angle is
    // 2 asin(chord / 2), increasing in the chord); one angular distance then
    const double cf[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
    dd far[3], best = dd_from(-1.0);
    for (int k = 0; k < 4; ++k) {
        dd v[3];
        pix_point_dd(level, pix, cf[k][0], cf[k][1], v);
        dd ch = dd_from(0.0);
        for (int i = 0; i < 3; ++i) {
            const dd e = dd_sub(v[i], g.c[i]);
            ch = dd_add(ch, dd_mul(e, e));
        }
        if (dd_lt(best, ch)) {
            best = ch;
            far[0] = v[0];
            far[1] = v[1];
            far[2] = v[2];
        }
    }
    g.r = angdist_dd(g.c, far);
    return g;
}

// "B_T is far from B_S" (Sec. 3.5): d - R_T - c_s R_S > 0 and R_T < c_t d,
// each by more than the relative tie guard.  FP64 first; double-double when
// either margin is within kMacFilter of zero.
// The FP64 filter of mac_far (+1 far, -1 not far, 0 undecided: the
// double-double test decides), without an angle: for a threshold X in [0, 3), d > X
// exactly when sin(d - X) = |c_S x c_T| cos X - (c_S . c_T) sin X > 0 (d - X
// lies in (-pi, pi]), and |sin(d - X)| <= |d - X|, so a value beyond
// kMacFilter settles the sign of d - X as a margin of d would.  The two
// thresholds are X1 = R_T + c_s R_S and X2 = R_T / c_t; st = (cos, sin) of
// c_s R_S, tt = (cos, sin) of R_T and of R_T / c_t, from the FP64 radii.
// The FP64 error of either value is below 1e-14.  X >= 3 is left undecided
// (coarse boxes, few pairs) unless it exceeds pi, where the pair cannot be
// far.
SFMM_HD int mac_far_filter_trig(double csx, double csy, double csz, double ctx, double cty, double ctz, double rs,
                                double rt, double2 st, double4 tt, double c_s, double c_t) {
    const double x1 = rt + c_s * rs, x2 = rt / c_t;
    if (x1 > 3.14159265359 || x2 > 3.14159265359) return -1;  // beyond pi + 2e-12
    if (x1 >= 3.0 || x2 >= 3.0) return 0;
    const double cx = csy * ctz - csz * cty, cy = csz * ctx - csx * ctz, cz = csx * cty - csy * ctx;
    const double sn = sqrt(cx * cx + cy * cy + cz * cz), cs = csx * ctx + csy * cty + csz * ctz;
    const double cx1 = tt.x * st.x - tt.y * st.y, sx1 = tt.y * st.x + tt.x * st.y;
    const double v1 = sn * cx1 - cs * sx1;
    const double v2 = sn * tt.z - cs * tt.w;
    if (v1 < -kMacFilter || v2 < -kMacFilter) return -1;
    if (v1 > kMacFilter && v2 > kMacFilter) return 1;
    return 0;
}

// The exact decision of a near-tie: mac_far_filter_trig's test in
// double-double, v1 = sin(d - X1), v2 = sin(d - X2) from the double-double
// centres and the boxes' double-double cos / sin tables (ts: c_s R_S; tt:
// R_T, then R_T / c_t; cos before sin), far when both exceed kTieAbs.  The
// double-double errors stay below 1e-30 and a margin that is not an exact
// tie is far above 1e-20 at every depth, so exact ties come out not far, as
// the strict inequalities of the MAC say.  X >= pi: the pair cannot be far.
constexpr double kTieAbs = 1e-20;
SFMM_HD bool mac_far_dd_trig(const dd* cs, const dd* ct, dd rs, dd rt, const dd* ts, const dd* tt, double c_s,
                             double c_t) {
    const dd pi = dd_mul_d(dd_half_pi(), 2.0);
    const dd x1 = dd_add(rt, dd_mul_d(rs, c_s));
    const dd x2 = dd_div(rt, dd_from(c_t));
    if (!dd_lt(x1, pi) || !dd_lt(x2, pi)) return false;
    const dd cx = dd_sub(dd_mul(cs[1], ct[2]), dd_mul(cs[2], ct[1]));
    const dd cy = dd_sub(dd_mul(cs[2], ct[0]), dd_mul(cs[0], ct[2]));
    const dd cz = dd_sub(dd_mul(cs[0], ct[1]), dd_mul(cs[1], ct[0]));
    const dd sn = dd_sqrt(dd_add(dd_add(dd_mul(cx, cx), dd_mul(cy, cy)), dd_mul(cz, cz)));
    const dd c = dd_add(dd_add(dd_mul(cs[0], ct[0]), dd_mul(cs[1], ct[1])), dd_mul(cs[2], ct[2]));
    const dd cx1 = dd_sub(dd_mul(tt[0], ts[0]), dd_mul(tt[1], ts[1]));
    const dd sx1 = dd_add(dd_mul(tt[1], ts[0]), dd_mul(tt[0], ts[1]));
    const dd v1 = dd_sub(dd_sub(dd_mul(sn, cx1), dd_mul(c, sx1)), dd_from(kTieAbs));
    const dd v2 = dd_sub(dd_sub(dd_mul(sn, tt[2]), dd_mul(c, tt[3])), dd_from(kTieAbs));
    return v1.hi > 0.0 && v2.hi > 0.0;
}

// The double-double test of mac_far alone.
SFMM_HD bool mac_far_dd(const dd* cs_dd, const dd* ct_dd, dd rs_dd, dd rt_dd, double c_s, double c_t) {
    const dd D = angdist_dd(cs_dd, ct_dd);
    const dd guard = dd_mul_d(D, kTieRel);
    const dd M1 = dd_sub(dd_sub(dd_sub(D, rt_dd), dd_mul_d(rs_dd, c_s)), guard);
    const dd M2 = dd_sub(dd_sub(dd_mul_d(D, c_t), rt_dd), guard);
    return M1.hi > 0.0 && M2.hi > 0.0;
}

SFMM_HD bool mac_far(const double* cs, const double* ct, double rs, double rt,
                     const dd* cs_dd, const dd* ct_dd, dd rs_dd, dd rt_dd,
                     double c_s, double c_t) {
    const double d = angdist(cs[0], cs[1], cs[2], ct[0], ct[1], ct[2]);
    const double m1 = d - rt - c_s * rs;
    const double m2 = c_t * d - rt;
    if (m1 < -kMacFilter || m2 < -kMacFilter) return false;
    if (m1 > kMacFilter && m2 > kMacFilter) return true;
    const dd D = angdist_dd(cs_dd, ct_dd);
    const dd guard = dd_mul_d(D, kTieRel);
    const dd M1 = dd_sub(dd_sub(dd_sub(D, rt_dd), dd_mul_d(rs_dd, c_s)), guard);
    const dd M2 = dd_sub(dd_sub(dd_mul_d(D, c_t), rt_dd), guard);
    return M1.hi > 0.0 && M2.hi > 0.0;
}

// r(B_S) > r(B_T) of Algorithm 1, with radii equal in exact arithmetic
// (congruent boxes) counted as equal.
SFMM_HD bool radius_greater(double rs, double rt, dd rs_dd, dd rt_dd) {
    const double diff = rs - rt;
    if (fabs(diff) > 1e-13 * (rs + rt)) return diff > 0.0;
    const dd M = dd_sub(dd_sub(rs_dd, rt_dd), dd_mul_d(rt_dd, kTieRel));
    return M.hi > 0.0;
}

}  // namespace sfmm
