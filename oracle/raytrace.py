"""Multi-plane backtracking on the sphere (test infrastructure only).

The discretised ray equation of Sec. 2.1 (Eq. DIS_PRO): a ray entering
layer i at theta_i leaves it at theta_{i+1} = theta_i - w_i alpha_i(theta_i),
w_i = f_K(r_s - r_i) / f_K(r_s), with alpha_i the deflection of layer i
(Eq. ALP_PSI; here from the oracle's direct sum over the layer's masses).
On the sphere the step is the geodesic one: the ray moves by the angle
|w_i alpha_i| along the great circle in the direction of -alpha_i
(n' = n cos t + u sin t, u the unit tangent of -alpha_i).

The distortion matrix A = d theta_n / d theta_0 (Sec. 2.2: "the Hessian can
be propagated from one to another plane") follows the same recursion to
first order in the step: A_{i+1} = T_i (I - w_i H_i) A_i, with H_i the
Hessian of layer i at theta_i (Eq. GAM_DEF, the oracle's direct sum) and
T_i the parallel transport of the tangent plane along the step, written in
the e_theta, e_phi bases of both ends.  A is stored as (A_11, A_12, A_21,
A_22): column j is the image of the initial basis vector j.
"""
import numpy as np

from . import direct, hessian


def basis(n):
    """e_theta, e_phi of unit vectors n (3, m); phi = 0 at an exact pole."""
    x, y, z = n
    rho = np.hypot(x, y)
    safe = np.where(rho > 0, rho, 1.0)
    cph = np.where(rho > 0, x / safe, 1.0)
    sph = np.where(rho > 0, y / safe, 0.0)
    et = np.stack([z * cph, z * sph, -rho])
    ep = np.stack([-sph, cph, np.zeros_like(rho)])
    return et, ep


def step(n, v):
    """Geodesic step from n (3, m) along the tangent vectors v (3, m): the
    new points and the parallel transport T (m, 2, 2) in the e_theta, e_phi
    bases of both ends."""
    t = np.linalg.norm(v, axis=0)
    moving = t > 0
    u = np.where(moving, v / np.where(moving, t, 1.0), 0.0)
    n2 = n * np.cos(t) + u * np.sin(t)
    # transported frame: u -> u cos t - n sin t, n x u unchanged
    b = np.cross(n.T, u.T).T
    u2 = u * np.cos(t) - n * np.sin(t)
    et, ep = basis(n)
    et2, ep2 = basis(n2)
    T = np.zeros((n.shape[1], 2, 2))
    for j, e in enumerate((et, ep)):
        a = np.sum(e * u, axis=0)
        c = np.sum(e * b, axis=0)
        pe = np.where(moving, a * u2 + c * b, e)  # transported basis vector
        T[:, 0, j] = np.sum(et2 * pe, axis=0)
        T[:, 1, j] = np.sum(ep2 * pe, axis=0)
    return n2, T


def trace(shells, weights, rays, with_distortion=True):
    """shells: list of (src (3, N_i), q (N_i,)); weights: w_i; rays: (3, m)
    initial unit vectors.  Returns the final rays (3, m) and A (4, m)."""
    n = np.array(rays, dtype=np.float64, copy=True)
    m = n.shape[1]
    A = np.tile(np.eye(2), (m, 1, 1))
    for (src, q), w in zip(shells, weights):
        _, alpha = direct(src, q, n)
        if with_distortion:
            h = hessian(src, q, n)
            H = np.stack([np.stack([h[0], h[1]], -1), np.stack([h[1], h[2]], -1)], -2)
            A = np.einsum("mij,mjk->mik", np.eye(2)[None] - w * H, A)
        n2, T = step(n, -w * alpha)
        if with_distortion:
            A = np.einsum("mij,mjk->mik", T, A)
        n = n2
    Aout = np.stack([A[:, 0, 0], A[:, 0, 1], A[:, 1, 0], A[:, 1, 1]])
    return n, Aout
