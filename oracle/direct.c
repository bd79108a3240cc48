/*
 * Oracle: plain FP64 direct sum of the spherical Green's function and its
 * gradient.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * What it computes, written out from the paper:
 *   psi(n)   = sum_j q_j G(n, n_j)                      Sec. 3.1 Eq. SUM
 *   G(n,n')  = (1/4pi) log((1 - n.n')/2)               Sec. 2.1 Eq. GRE_FUN
 *            = (1/4pi) log(|n - n'|^2 / 4)             (unit vectors)
 *   zero-mean gauge (Eq. STAND_CONDITION): the sphere integral of G is -1,
 *   so the gauge-fixed potential is psi + Q_tot/(4pi); per source this is
 *   the term q_j (log(|d|^2/4) + 1)/(4pi).
 *   alpha(n) = grad psi (Eq. ALP_PSI), the covariant gradient on the sphere:
 *   the ambient gradient of (q/4pi) log|d|^2 is (q/2pi) d/|d|^2, and alpha
 *   is its part tangent to the sphere at n, (q/2pi)(d - n^ (n^.d))/|d|^2
 *   with n^ = n/|n|.  For exact unit vectors n.d = |d|^2/2 and this is
 *   (q/2pi)(d/|d|^2 - n/2); FP64 inputs lie off the sphere by ~1e-16, which
 *   for very close pairs would leave a radial part of size 1e-16/|d|^2 in
 *   that second form, so the projection is written out per term.
 * Compiled with -ffp-contract=off: no fused multiply-adds, IEEE round to
 * nearest, and every accumulation is Neumaier-compensated.
 */
#include "oracle.h"
#include <math.h>
#include <omp.h>

typedef struct {
    double s, c;
} nsum_t;

static inline void nsum_add(nsum_t* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static inline double nsum_value(const nsum_t* a) { return a->s + a->c; }

void oracle_direct(const double* src, const double* q, int64_t n,
                   const double* tgt, int64_t m, int gauge, double* psi,
                   double* defl, int nthreads) {
    const double* sx = src;
    const double* sy = src + n;
    const double* sz = src + 2 * n;
    const double four_pi = 4.0 * M_PI;
    const double two_pi = 2.0 * M_PI;
    const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
    int64_t i;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
    for (i = 0; i < m; ++i) {
        const double nx = tgt[i], ny = tgt[m + i], nz = tgt[2 * m + i];
        const double inv_len = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
        const double ux = nx * inv_len, uy = ny * inv_len, uz = nz * inv_len;
        nsum_t p = {0.0, 0.0}, ax = {0.0, 0.0}, ay = {0.0, 0.0}, az = {0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            const double dx = nx - sx[j], dy = ny - sy[j], dz = nz - sz[j];
            if (dx == 0.0 && dy == 0.0 && dz == 0.0) {
                /* coincident source: no log term; in the zero-mean gauge its
                 * share q_j/(4pi) of the constant Q_tot/(4pi) remains. */
                if (gauge == ORACLE_GAUGE_ZERO_MEAN) nsum_add(&p, q[j]);
                continue;
            }
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double g = log(0.25 * r2);
            nsum_add(&p, q[j] * (gauge == ORACLE_GAUGE_ZERO_MEAN ? g + 1.0 : g));
            const double nd = ux * dx + uy * dy + uz * dz; /* radial part of d */
            nsum_add(&ax, q[j] * ((dx - ux * nd) / r2));
            nsum_add(&ay, q[j] * ((dy - uy * nd) / r2));
            nsum_add(&az, q[j] * ((dz - uz * nd) / r2));
        }
        psi[i] = nsum_value(&p) / four_pi;
        defl[i] = nsum_value(&ax) / two_pi;
        defl[m + i] = nsum_value(&ay) / two_pi;
        defl[2 * m + i] = nsum_value(&az) / two_pi;
    }
}

/*
 * Hessian of psi (Sec. 2.2): the matrix H of second covariant derivatives in
 * the normalised basis e_theta, e_phi at the target,
 *   H_11 = d^2 psi / d theta^2,
 *   H_12 = d/d theta ((1/sin theta) d psi / d phi),
 *   H_22 = (1/sin^2 theta) d^2 psi / d phi^2 + cot theta d psi / d theta,
 * summed over the sources.  Written per source through the ambient function
 * F(x) = (q/4pi) log(|x - s|^2 / 4): the covariant Hessian of its
 * restriction to the unit sphere is P D^2F P - (n.DF) P (P the tangent
 * projector: a great circle through n in direction e curves by -n), with
 *   DF = (q/2pi) d/|d|^2,  D^2F = (q/2pi) (I/|d|^2 - 2 d d^T/|d|^4),
 * so in the basis e_a, e_b:
 *   H_ab = (q/2pi) [delta_ab (1 - n.d)/|d|^2 - 2 (e_a.d)(e_b.d)/|d|^4].
 * e_theta = (cos theta cos phi, cos theta sin phi, -sin theta),
 * e_phi = (-sin phi, cos phi, 0), from the target's own coordinates; at an
 * exact pole (x = y = 0) phi = 0.  Coincident sources are left out, as in
 * oracle_direct.  hess [3][m] = (H_11, H_12, H_22).
 */
void oracle_hessian(const double* src, const double* q, int64_t n, const double* tgt, int64_t m,
                    double* hess, int nthreads) {
    const double* sx = src;
    const double* sy = src + n;
    const double* sz = src + 2 * n;
    const double two_pi = 2.0 * M_PI;
    const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
    int64_t i;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
    for (i = 0; i < m; ++i) {
        const double nx = tgt[i], ny = tgt[m + i], nz = tgt[2 * m + i];
        const double inv_len = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
        const double ux = nx * inv_len, uy = ny * inv_len, uz = nz * inv_len;
        const double rho = sqrt(ux * ux + uy * uy);
        const double cph = rho > 0.0 ? ux / rho : 1.0, sph = rho > 0.0 ? uy / rho : 0.0;
        const double cth = uz, sth = rho;
        const double et[3] = {cth * cph, cth * sph, -sth};
        const double ep[3] = {-sph, cph, 0.0};
        nsum_t h11 = {0.0, 0.0}, h12 = {0.0, 0.0}, h22 = {0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            const double dx = nx - sx[j], dy = ny - sy[j], dz = nz - sz[j];
            if (dx == 0.0 && dy == 0.0 && dz == 0.0) continue;
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double nd = ux * dx + uy * dy + uz * dz;
            const double dt = et[0] * dx + et[1] * dy + et[2] * dz;
            const double dp = ep[0] * dx + ep[1] * dy + ep[2] * dz;
            const double diag = (1.0 - nd) / r2;
            const double r4 = r2 * r2;
            nsum_add(&h11, q[j] * (diag - 2.0 * dt * dt / r4));
            nsum_add(&h12, q[j] * (-2.0 * dt * dp / r4));
            nsum_add(&h22, q[j] * (diag - 2.0 * dp * dp / r4));
        }
        hess[i] = nsum_value(&h11) / two_pi;
        hess[m + i] = nsum_value(&h12) / two_pi;
        hess[2 * m + i] = nsum_value(&h22) / two_pi;
    }
}

/*
 * Near-particle model (Sec. 3.1, NPM; Sec. 4.2 Eq. KERNEL): every source is
 * a mass distribution of the generalised Epanechnikov profile
 *   W(theta) = [1 - sin^2(theta/2) / sin^2(sigma/2)] / (2 pi sin^2(sigma/2))
 * for theta <= sigma (0 beyond), so Laplacian psi = q W - q/(4pi) (Eq.
 * POI_EQU with Eq. LAP_GRE).  With u = sin^2(theta/2) = |d|^2/4 and
 * t = sin^2(sigma/2), Gauss's law over the cap of radius theta gives
 *   d psi / du = (q/4pi) (M(u) - u) / (u (1 - u)),
 * M(u) = min(1, 2 u/t - u^2/t^2) the profile's mass fraction inside theta;
 * outside the particle this is the point mass, (q/4pi)/u, so psi is the
 * point mass's (q/4pi) log u plus a constant, and inside
 *   psi(u) = (q/4pi) log t - integral_u^t d psi/du  (+ the same constant),
 * the integral by 24-point Gauss-Legendre quadrature (the integrand is
 * smooth on [u, t]).  The constant makes psi the convolution of the
 * profile with the Green's function, whose sphere integral is -q like the
 * point mass's (Eq. GRE_FUN): with dOmega = 4 pi du,
 *   (q/4pi) c = -(q/4pi) integral_0^t (psi_in(u) - log u) du
 *            = -(q/4pi) [integral_0^t psi_in du - (t log t - t)],
 * again by Gauss-Legendre quadrature (psi_in is smooth on [0, t]); the
 * zero-mean gauge then adds q/(4pi) as for a point mass.  alpha = (d psi/du) d/2 (ambient gradient of u is d/2),
 * projected on the tangent plane, and the Hessian in e_theta, e_phi
 *   H_ab = (d^2 psi/du^2)(e_a.d)(e_b.d)/4 + (d psi/du)(1 - n.d) delta_ab / 2.
 * A source at the target itself contributes its finite central values.
 * sigma = 0 is the point-mass case of oracle_direct / oracle_hessian.
 * hess may be NULL.
 */
static const double gl24_x[12] = {0.0640568928626056260850430826247450, 0.1911188674736163091586398207570696,
                                  0.3150426796961633743867932913198102, 0.4337935076260451384870842319133497,
                                  0.5454214713888395356583756172183723, 0.6480936519369755692524957869107476,
                                  0.7401241915785543642438281030999784, 0.8200019859739029219539498726697452,
                                  0.8864155270044010342131543419821968, 0.9382745520027327585236490017087215,
                                  0.9747285559713094981983919930081691, 0.9951872199970213601799974097007368};
static const double gl24_w[12] = {0.1279381953467521569740561652246954, 0.1258374563468282961213753825111837,
                                  0.1216704729278033912044631534762625, 0.1155056680537256013533444839067835,
                                  0.1074442701159656347825773424466062, 0.0976186521041138882698806644642472,
                                  0.0861901615319532759171852029837427, 0.0733464814110803057340336152531165,
                                  0.0592985849154367807463677585001085, 0.0442774388174198061686027482113382,
                                  0.0285313886289336631813078159518782, 0.0123412297999871995468056670700372};

static double npm_dpsi(double u, double t) { /* (4pi/q) d psi / du */
    if (u >= t) return 1.0 / u;
    const double v = u / t;
    return (2.0 / t - v / t - 1.0) / (1.0 - u); /* (M - u)/(u (1 - u)) with M = 2v - v^2 */
}

static double npm_d2psi(double u, double t) { /* (4pi/q) d^2 psi / du^2 */
    if (u >= t) return -1.0 / (u * u);
    const double a = (1.0 - t) / t;
    return -(a * a) / ((1.0 - u) * (1.0 - u));
}

static double npm_psi(double u, double t) { /* (4pi/q) psi */
    if (u >= t) return log(u);
    const double h = 0.5 * (t - u), c = 0.5 * (t + u);
    double s = 0.0;
    for (int k = 0; k < 12; ++k) {
        s += gl24_w[k] * (npm_dpsi(c - h * gl24_x[k], t) + npm_dpsi(c + h * gl24_x[k], t));
    }
    return log(t) - h * s;
}

void oracle_npm(const double* src, const double* q, int64_t n, const double* tgt, int64_t m, double sigma,
                int gauge, double* psi, double* defl, double* hess, int nthreads) {
    const double* sx = src;
    const double* sy = src + n;
    const double* sz = src + 2 * n;
    const double ss = sin(0.5 * sigma);
    const double t = ss * ss;
    const double four_pi = 4.0 * M_PI;
    double chat = 0.0; /* the constant c above, 0 for point masses */
    if (t > 0.0) {
        double si = 0.0;
        for (int k = 0; k < 12; ++k)
            si += gl24_w[k] * (npm_psi(0.5 * t * (1.0 - gl24_x[k]), t) + npm_psi(0.5 * t * (1.0 + gl24_x[k]), t));
        chat = -(0.5 * t * si - (t * log(t) - t));
    }
    const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
    int64_t i;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
    for (i = 0; i < m; ++i) {
        const double nx = tgt[i], ny = tgt[m + i], nz = tgt[2 * m + i];
        const double inv_len = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
        const double ux = nx * inv_len, uy = ny * inv_len, uz = nz * inv_len;
        const double rho = sqrt(ux * ux + uy * uy);
        const double cph = rho > 0.0 ? ux / rho : 1.0, sph = rho > 0.0 ? uy / rho : 0.0;
        const double et[3] = {uz * cph, uz * sph, -rho};
        const double ep[3] = {-sph, cph, 0.0};
        nsum_t p = {0.0, 0.0}, ax = {0.0, 0.0}, ay = {0.0, 0.0}, az = {0.0, 0.0};
        nsum_t h11 = {0.0, 0.0}, h12 = {0.0, 0.0}, h22 = {0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            const double dx = nx - sx[j], dy = ny - sy[j], dz = nz - sz[j];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double u = 0.25 * r2;
            if (u == 0.0 && t == 0.0) {
                /* a point mass at the target: left out (oracle_direct) */
                if (gauge == ORACLE_GAUGE_ZERO_MEAN) nsum_add(&p, q[j]);
                continue;
            }
            const double g = npm_psi(u, t) + chat;
            nsum_add(&p, q[j] * (gauge == ORACLE_GAUGE_ZERO_MEAN ? g + 1.0 : g));
            const double d1 = npm_dpsi(u, t), d2 = npm_d2psi(u, t);
            const double nd = ux * dx + uy * dy + uz * dz;
            /* (q/4pi) d1 d/2 projected: the 1/(4pi) is applied at the end */
            nsum_add(&ax, q[j] * 0.5 * d1 * (dx - ux * nd));
            nsum_add(&ay, q[j] * 0.5 * d1 * (dy - uy * nd));
            nsum_add(&az, q[j] * 0.5 * d1 * (dz - uz * nd));
            if (hess) {
                const double dt = et[0] * dx + et[1] * dy + et[2] * dz;
                const double dp = ep[0] * dx + ep[1] * dy + ep[2] * dz;
                const double diag = 0.5 * d1 * (1.0 - nd);
                nsum_add(&h11, q[j] * (0.25 * d2 * dt * dt + diag));
                nsum_add(&h12, q[j] * (0.25 * d2 * dt * dp));
                nsum_add(&h22, q[j] * (0.25 * d2 * dp * dp + diag));
            }
        }
        psi[i] = nsum_value(&p) / four_pi;
        defl[i] = nsum_value(&ax) / four_pi;
        defl[m + i] = nsum_value(&ay) / four_pi;
        defl[2 * m + i] = nsum_value(&az) / four_pi;
        if (hess) {
            hess[i] = nsum_value(&h11) / four_pi;
            hess[m + i] = nsum_value(&h12) / four_pi;
            hess[2 * m + i] = nsum_value(&h22) / four_pi;
        }
    }
}
