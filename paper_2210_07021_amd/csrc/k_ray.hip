// Multi-plane backtracking (Sec. 2.1, Eq. DIS_PRO): one layer's step of
// every ray, theta_{i+1} = theta_i - w_i alpha_i(theta_i), taken along the
// great circle (the ray moves by |w alpha| in the direction of -alpha), and
// the distortion matrix A = d theta / d theta_0 carried with it to first
// order in the step: A <- T (I - w H) A, H the layer's Hessian (Sec. 2.2) at
// the ray and T the parallel transport of the tangent plane along the step,
// both in the e_theta, e_phi bases of the ray's positions.
#include "common.hpp"
#include "expand.hpp"

namespace sfmm {

namespace {
__global__ void k_ray_step(double* __restrict__ rays, const double* __restrict__ defl,
                           const double* __restrict__ hess, double w, int64_t m, double* __restrict__ dist) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= m) return;
    const double n[3] = {rays[k], rays[m + k], rays[2 * m + k]};
    const double v[3] = {-w * defl[k], -w * defl[m + k], -w * defl[2 * m + k]};
    const double t = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const bool moving = t > 0.0;
    const double it = moving ? 1.0 / t : 0.0;
    const double u[3] = {v[0] * it, v[1] * it, v[2] * it};
    double st, ct;
    sincos(t, &st, &ct);
    double n2[3];
    for (int d = 0; d < 3; ++d) n2[d] = moving ? n[d] * ct + u[d] * st : n[d];
    if (dist) {
        double et[3], ep[3], et2[3], ep2[3];
        target_basis(n[0], n[1], n[2], et, ep);
        target_basis(n2[0], n2[1], n2[2], et2, ep2);
        // B = (I - w H) A
        const double h11 = hess[k], h12 = hess[m + k], h22 = hess[2 * m + k];
        const double A11 = dist[k], A12 = dist[m + k], A21 = dist[2 * m + k], A22 = dist[3 * m + k];
        const double B11 = A11 - w * (h11 * A11 + h12 * A21), B12 = A12 - w * (h11 * A12 + h12 * A22);
        const double B21 = A21 - w * (h12 * A11 + h22 * A21), B22 = A22 - w * (h12 * A12 + h22 * A22);
        // transport: u -> u cos t - n sin t, b = n x u fixed
        const double b[3] = {n[1] * u[2] - n[2] * u[1], n[2] * u[0] - n[0] * u[2], n[0] * u[1] - n[1] * u[0]};
        // a ray that does not move keeps its basis: T is the identity exactly
        double T[2][2] = {{1.0, 0.0}, {0.0, 1.0}};
        const double* E[2] = {et, ep};
        for (int j = 0; moving && j < 2; ++j) {
            const double a = E[j][0] * u[0] + E[j][1] * u[1] + E[j][2] * u[2];
            const double c = E[j][0] * b[0] + E[j][1] * b[1] + E[j][2] * b[2];
            double pe[3];
            for (int d = 0; d < 3; ++d) pe[d] = a * (u[d] * ct - n[d] * st) + c * b[d];
            T[0][j] = et2[0] * pe[0] + et2[1] * pe[1] + et2[2] * pe[2];
            T[1][j] = ep2[0] * pe[0] + ep2[1] * pe[1] + ep2[2] * pe[2];
        }
        dist[k] = T[0][0] * B11 + T[0][1] * B21;
        dist[m + k] = T[0][0] * B12 + T[0][1] * B22;
        dist[2 * m + k] = T[1][0] * B11 + T[1][1] * B21;
        dist[3 * m + k] = T[1][0] * B12 + T[1][1] * B22;
    }
    rays[k] = n2[0];
    rays[m + k] = n2[1];
    rays[2 * m + k] = n2[2];
}

__global__ void k_dist_identity(double* __restrict__ dist, int64_t m) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= m) return;
    dist[k] = 1.0;
    dist[m + k] = 0.0;
    dist[2 * m + k] = 0.0;
    dist[3 * m + k] = 1.0;
}
}  // namespace

void ray_identity(double* dist, int64_t m, hipStream_t s) {
    if (m <= 0) return;
    k_dist_identity<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(dist, m);
    SFMM_LAUNCH_CHECK();
}

void ray_step(double* rays, const double* defl, const double* hess, double w, int64_t m, double* dist,
              hipStream_t s) {
    if (m <= 0) return;
    k_ray_step<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(rays, defl, hess, w, m, dist);
    SFMM_LAUNCH_CHECK();
}

}  // namespace sfmm
