/*
 * Oracle: HEALPix nested pixelisation used for the sphere division of
 * Sec. 3.1 and the box geometry of Sec. 3.5.  TEST INFRASTRUCTURE ONLY.
 *
 * Restated from the published HEALPix definition (Gorski et al. 2005,
 * ApJ 622, 759): 12 base faces, each an nside x nside grid with
 * nside = 2^order; in the equatorial zone |z| <= 2/3 the pixel edges are the
 * lines nside*(1/2 + 2phi/pi -+ 3z/4) = const, in the polar caps the lines
 * through nside*sqrt(3(1-|z|)) scaled by the azimuth inside the face; the
 * nested index is face*nside^2 + Morton(ix, iy) with ix on the even bits.
 *
 * All geometry is evaluated in IEEE quad precision (__float128, 113-bit
 * significand) from the FP64 inputs, so keys, centres, radii and distances
 * are the exact-arithmetic values to ~1e-33: a floor argument within 1e-20 of
 * an integer is taken to be that integer (the exact value of such a
 * configuration is the integer itself), and FP64 outputs are the quad values
 * rounded to nearest.
 */
#include "oracle_geom.h"
#include <math.h>
#include <quadmath.h>

/* ring number (in units of nside) of each face's southern corner and the
 * azimuth of its centre in units of pi/4 */
static const int face_ring[12] = {2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4};
static const int face_phi[12] = {1, 3, 5, 7, 0, 2, 4, 6, 1, 3, 5, 7};

#define SNAP 1e-20Q

static uint64_t interleave(uint64_t v) {
    uint64_t r = 0;
    for (int b = 0; b < 31; ++b) r |= ((v >> b) & 1ULL) << (2 * b);
    return r;
}

static uint64_t deinterleave(uint64_t v) {
    uint64_t r = 0;
    for (int b = 0; b < 31; ++b) r |= ((v >> (2 * b)) & 1ULL) << b;
    return r;
}

/* floor, with values within SNAP of an integer taken as that integer */
static int64_t qfloor(__float128 v) {
    const __float128 r = roundq(v);
    if (fabsq(v - r) < SNAP) return (int64_t)r;
    return (int64_t)floorq(v);
}

int64_t oracle_key(double x, double y, double z, int order) {
    const int64_t ns = (int64_t)1 << order;
    const __float128 X = x, Y = y, Z = z;
    const __float128 za = fabsq(Z);
    __float128 tt = atan2q(Y, X) * (2.0Q / M_PIq); /* azimuth in units of pi/2 */
    if (fabsq(tt - roundq(tt)) < SNAP) tt = roundq(tt);
    if (tt < 0) tt += 4;
    if (tt >= 4) tt -= 4;
    int64_t face, ix, iy;
    if (za <= 2.0Q / 3.0Q) {
        const __float128 a = (__float128)ns * (0.5Q + tt);
        const __float128 b = (__float128)ns * (Z * 0.75Q);
        const int64_t jp = qfloor(a - b); /* ascending edge index */
        const int64_t jm = qfloor(a + b); /* descending edge index */
        const int64_t fp = jp >> order, fm = jm >> order;
        if (fp == fm)
            face = fp | 4;
        else if (fp < fm)
            face = fp;
        else
            face = fm + 8;
        ix = jm & (ns - 1);
        iy = ns - (jp & (ns - 1)) - 1;
    } else {
        int ntt = (int)tt;
        if (ntt > 3) ntt = 3;
        const __float128 tp = tt - ntt;
        __float128 s;
        if (fabs(z) < 0.99) {
            s = (__float128)ns * sqrtq(3 * (1 - za));
        } else {
            const __float128 sth = sqrtq(X * X + Y * Y);
            s = (__float128)ns * sth / sqrtq((1 + za) / 3);
        }
        int64_t jp = qfloor(tp * s);
        int64_t jm = qfloor((1 - tp) * s);
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
    return (face << (2 * order)) + (int64_t)interleave((uint64_t)ix) +
           ((int64_t)interleave((uint64_t)iy) << 1);
}

void oracle_pix_point_q(int order, int64_t pix, double fx, double fy,
                        __float128* out3) {
    const int64_t ns = (int64_t)1 << order;
    const int face = (int)(pix >> (2 * order));
    const uint64_t inface = (uint64_t)pix & (((uint64_t)1 << (2 * order)) - 1);
    const __float128 x = ((__float128)deinterleave(inface) + fx) / ns;
    const __float128 y = ((__float128)deinterleave(inface >> 1) + fy) / ns;
    const __float128 jr = face_ring[face] - x - y;
    __float128 nr, z, sth = -1;
    if (jr < 1) { /* north polar cap */
        nr = jr;
        const __float128 t = nr * nr / 3;
        z = 1 - t;
        sth = sqrtq(t * (2 - t));
    } else if (jr > 3) { /* south polar cap */
        nr = 4 - jr;
        const __float128 t = nr * nr / 3;
        z = t - 1;
        sth = sqrtq(t * (2 - t));
    } else { /* equatorial zone */
        nr = 1;
        z = (2 - jr) * 2 / 3;
        sth = sqrtq((1 - z) * (1 + z));
    }
    __float128 u = face_phi[face] * nr + x - y;
    if (u < 0) u += 8;
    if (u >= 8) u -= 8;
    const __float128 phi = (nr == 0) ? 0 : (M_PI_4q * u) / nr;
    out3[0] = sth * cosq(phi);
    out3[1] = sth * sinq(phi);
    out3[2] = z;
    /* a coordinate this small is an exact zero (azimuth at a multiple of
     * pi/2 rounded in quad); a genuine one is never below ~1e-18 */
    for (int k = 0; k < 3; ++k)
        if (fabsq(out3[k]) < 1e-25Q) out3[k] = 0;
}

void oracle_pix_point(int order, int64_t pix, double fx, double fy,
                      double* out3) {
    __float128 q[3];
    oracle_pix_point_q(order, pix, fx, fy, q);
    for (int k = 0; k < 3; ++k) out3[k] = (double)q[k];
}

__float128 oracle_angdist_q(const __float128* a, const __float128* b) {
    const __float128 cx = a[1] * b[2] - a[2] * b[1];
    const __float128 cy = a[2] * b[0] - a[0] * b[2];
    const __float128 cz = a[0] * b[1] - a[1] * b[0];
    const __float128 s = sqrtq(cx * cx + cy * cy + cz * cz);
    const __float128 c = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    return atan2q(s, c);
}

double oracle_angdist(const double* a, const double* b) {
    const __float128 A[3] = {a[0], a[1], a[2]}, B[3] = {b[0], b[1], b[2]};
    return (double)oracle_angdist_q(A, B);
}

__float128 oracle_box_radius_q(int order, int64_t pix) {
    __float128 c[3], v[3];
    oracle_pix_point_q(order, pix, 0.5, 0.5, c);
    __float128 r = 0;
    static const double corner[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
    for (int k = 0; k < 4; ++k) {
        oracle_pix_point_q(order, pix, corner[k][0], corner[k][1], v);
        const __float128 d = oracle_angdist_q(c, v);
        if (d > r) r = d;
    }
    return r;
}

double oracle_box_radius(int order, int64_t pix) {
    return (double)oracle_box_radius_q(order, pix);
}
