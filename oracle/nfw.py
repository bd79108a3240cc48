"""NFW test halo of Sec. 4.3 (TEST INFRASTRUCTURE ONLY: only tests/ use it):
the analytic
convergence of Eq. NFW and the shear of a radially symmetric profile, as
reference values for the sampling-noise experiment.

Eq. NFW gives kappa(x) = kappa_s f(x), x = r / R_s, with
  f(x) = 4/(x^2 - 1) [1 - 2/sqrt(1 - x^2) artanh sqrt((1 - x)/(1 + x))]  (x < 1)
       = 4/3                                                             (x = 1)
       = 4/(x^2 - 1) [1 - 2/sqrt(x^2 - 1) arctan sqrt((x - 1)/(x + 1))]   (x > 1),
and the paper's shear of any radially symmetric profile,
  gamma(r) = (1/r^2) int_0^r r' kappa(r') dr' - kappa(r)/2.
The enclosed integral of f has the closed form (derived here, checked in
the pins by quadrature): int_0^x x' f(x') dx' = 4 [log(x/2) + h(x)],
  h(x) = artanh sqrt(1 - x^2) / sqrt(1 - x^2)  (x < 1),  1 (x = 1),
  h(x) = arctan sqrt(x^2 - 1) / sqrt(x^2 - 1)   (x > 1).
"""
import numpy as np


def f_nfw(x):
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lo, hi, one = x < 1 - 1e-12, x > 1 + 1e-12, np.abs(x - 1) <= 1e-12
    xl = x[lo]
    out[lo] = 4 / (xl * xl - 1) * (1 - 2 / np.sqrt(1 - xl * xl) * np.arctanh(np.sqrt((1 - xl) / (1 + xl))))
    xh = x[hi]
    out[hi] = 4 / (xh * xh - 1) * (1 - 2 / np.sqrt(xh * xh - 1) * np.arctan(np.sqrt((xh - 1) / (xh + 1))))
    out[one] = 4.0 / 3.0
    return out


def enclosed(x):
    """int_0^x x' f(x') dx' (closed form)."""
    x = np.asarray(x, dtype=np.float64)
    h = np.empty_like(x)
    lo, hi, one = x < 1 - 1e-12, x > 1 + 1e-12, np.abs(x - 1) <= 1e-12
    s = np.sqrt(1 - x[lo] ** 2)
    h[lo] = np.arctanh(s) / s
    s = np.sqrt(x[hi] ** 2 - 1)
    h[hi] = np.arctan(s) / s
    h[one] = 1.0
    return 4 * (np.log(x / 2) + h)


def gamma_nfw(x):
    """Shear in units of kappa_s: (1/x^2) int_0^x x' f dx' - f(x)/2."""
    x = np.asarray(x, dtype=np.float64)
    return enclosed(x) / (x * x) - f_nfw(x) / 2


# ---- the halo on the unit sphere
# The projected profile is laid on the sphere around a centre by the
# equal-area radius r = 2 sin(theta/2) (the chord to the centre): the
# sphere's area element is 2 pi sin(theta) d theta = 2 pi r dr exactly, so
# the flat profile's mass in every ring is kept.  Truncated at r_vir =
# c r_s (the sampled halo has no mass beyond it).

def kappa_sphere(theta, kappa_s, r_s, c):
    r = 2 * np.sin(np.asarray(theta) / 2)
    x = r / r_s
    return np.where(x <= c, kappa_s * f_nfw(np.minimum(x, c)), 0.0)


def halo_mass(kappa_s, r_s, c):
    """Total mass (sphere integral of kappa) of the truncated halo."""
    return 2 * np.pi * kappa_s * r_s * r_s * float(enclosed(np.array([c]))[0])


def radial_deflection(theta, m_enclosed, q_total):
    """d psi / d theta of an azimuthally symmetric mass layout at angle
    theta from its centre, by Gauss's law on the cap (Eq. POI_EQU with the
    background kbar = Q/(4 pi)): the flux 2 pi sin(theta) dpsi/dtheta equals
    the enclosed mass minus kbar times the cap's area pi r^2, r = 2
    sin(theta/2)."""
    theta = np.asarray(theta, dtype=np.float64)
    r = 2 * np.sin(theta / 2)
    return (m_enclosed - q_total / (4 * np.pi) * np.pi * r * r) / (2 * np.pi * np.sin(theta))


def shear_sphere(theta, kappa_s, r_s, c):
    """Shear magnitude of the halo at angle theta from its centre, exact on
    the sphere for the mass layout above: H_rr = d^2 psi/d theta^2 and H_tt =
    cot(theta) dpsi/dtheta (Sec. 2.2), their sum kappa - kbar, so the
    trace-free part is gamma = cot(theta) dpsi/dtheta - (kappa - kbar)/2 in
    magnitude (the paper's flat formula for small theta)."""
    theta = np.asarray(theta, dtype=np.float64)
    r = 2 * np.sin(theta / 2)
    x = np.minimum(r / r_s, c)
    Q = halo_mass(kappa_s, r_s, c)
    M = 2 * np.pi * kappa_s * r_s * r_s * enclosed(x)
    kap = kappa_sphere(theta, kappa_s, r_s, c)
    return np.cos(theta) / np.sin(theta) * radial_deflection(theta, M, Q) - (kap - Q / (4 * np.pi)) / 2
