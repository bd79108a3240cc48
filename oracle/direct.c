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
