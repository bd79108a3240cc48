"""Pins of the NFW reference of Sec. 4.3 (oracle/nfw.py): the closed form of
the enclosed profile against quadrature of Eq. NFW, the value 4/3 at x = 1
and continuity there, the paper's flat shear formula as the small-angle
limit of the spherical one, and the spherical shear against the oracle's
Hessian direct sum over a ring decomposition of the halo."""
import numpy as np
import pytest
from scipy.integrate import quad

import oracle
from oracle import nfw


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def test_enclosed_closed_form_and_unit_point():
    for x in (1e-3, 0.2, 0.9, 1.0, 1.1, 3.0, 8.0):
        pts = [1.0] if x > 1 else None
        q, _ = quad(lambda t: t * nfw.f_nfw(np.array([t]))[0], 0, x, limit=400, points=pts, epsabs=1e-13)
        assert abs(q - nfw.enclosed(np.array([x]))[0]) <= 1e-9 * max(1.0, q), x
    assert nfw.f_nfw(np.array([1.0]))[0] == 4.0 / 3.0
    e = 1e-3
    lo, hi = nfw.f_nfw(np.array([1 - e, 1 + e]))
    assert lo > 4 / 3 > hi and abs(lo - 4 / 3) < 2e-3 and abs(hi - 4 / 3) < 2e-3


def test_flat_limit_of_the_spherical_shear():
    """For a small halo the spherical shear is the paper's
    (1/r^2) int_0^r r' kappa dr' - kappa/2."""
    ks, rs, c = 0.3, 1e-4, 5.0
    th = np.array([0.2, 0.5, 1.0, 2.0, 4.0]) * rs
    flat = ks * nfw.gamma_nfw(2 * np.sin(th / 2) / rs)
    sph = nfw.shear_sphere(th, ks, rs, c)
    assert np.allclose(sph, flat, rtol=1e-6)


def test_spherical_gauss_law_against_the_oracle_on_rings():
    """The halo as 2 x 60 Gauss-Legendre rings in x (on [0, 1] and [1, c]),
    4000 points each, every ring carrying its share of the profile's mass:
    at targets between the rings the oracle's direct-sum deflection (radial,
    e_theta at phi = 0) equals radial_deflection with the rings' own
    enclosed mass, and the trace-free part of its Hessian equals
    cot(theta) dpsi/dtheta - (0 - kbar)/2 (no density between rings)."""
    ks, rs, c = 0.3, 0.3, 5.0
    xg, wg = np.polynomial.legendre.leggauss(60)
    src, q, xr_all = [], [], []
    for lo, hi in ((0.0, 1.0), (1.0, c)):
        xr = lo + (hi - lo) * (xg + 1) / 2
        wr = wg * (hi - lo) / 2
        for x, w in zip(xr, wr):
            mass = 2 * np.pi * ks * rs * rs * x * nfw.f_nfw(np.array([x]))[0] * w
            th = 2 * np.arcsin(x * rs / 2)
            ph = np.linspace(0, 2 * np.pi, 4000, endpoint=False)
            src.append(np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.full(4000, np.cos(th))]))
            q.append(np.full(4000, mass / 4000))
            xr_all.append(np.full(4000, x))
    src = np.concatenate(src, axis=1)
    q = np.concatenate(q)
    xr_all = np.concatenate(xr_all)
    Q = q.sum()
    assert abs(Q - nfw.halo_mass(ks, rs, c)) <= 1e-6 * Q      # the quadrature of the profile's mass
    rings = np.unique(xr_all)
    xt = 0.5 * (rings[[20, 45, 70, 90, 110]] + rings[[21, 46, 71, 91, 111]])   # midway between rings
    tht = 2 * np.arcsin(xt * rs / 2)
    tgt = np.stack([np.sin(tht) * np.cos(1e-3), np.sin(tht) * np.sin(1e-3), np.cos(tht)])  # between ring points
    _, a = oracle.direct(src, q, tgt)
    h = oracle.hessian(src, q, tgt)
    m_in = np.array([q[xr_all < x].sum() for x in xt])
    dpsi = nfw.radial_deflection(tht, m_in, Q)
    et = np.stack([np.cos(tht) * np.cos(1e-3), np.cos(tht) * np.sin(1e-3), -np.sin(tht)])
    assert np.allclose(np.sum(a * et, axis=0), dpsi, rtol=1e-6)
    g = -(h[0] - h[2]) / 2
    assert np.allclose(g, np.cos(tht) / np.sin(tht) * dpsi + Q / (8 * np.pi), rtol=1e-6)
