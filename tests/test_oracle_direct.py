"""Pins of the oracle's direct sum (Eq. SUM, Eq. GRE_FUN, Eq. ALP_PSI and the
zero-mean gauge of Eq. STAND_CONDITION) against values the mathematics fixes
independently of the oracle's own formula:

* single point mass: closed form in the angular distance, with the deflection
  written as magnitude x geodesic direction (Sec. 2.1, App. A);
* a ring of equal masses: the exact product identity for the ring sum;
* a uniform cap: Gauss's-law closed forms, themselves pinned by the Legendre
  series of the Poisson equation (Eq. POI_EQU);
* invariants: zero mean over the sphere (Eq. STAND_CONDITION), rotation
  invariance, symmetry of G, alpha = grad psi by finite differences, the
  Laplacian Delta G = -1/(4 pi) away from sources (Eq. LAP_GRE);
* brute force at 50 digits with the kernel in its printed form
  log(1 - n.n') (not the oracle's |d|^2 form).
"""
import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2210_07021_amd import skies

FOUR_PI = 4.0 * np.pi


def _rot(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.sqrt((v * v).sum(axis=0))


def _geodesic_point(s, theta, az, rng=None):
    """Point at angular distance theta from s, azimuth az about s."""
    s = _unit(s)
    a = np.array([1.0, 0.0, 0.0]) if abs(s[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = _unit(np.cross(a, s))
    e2 = np.cross(s, e1)
    return _unit(np.cos(theta) * s + np.sin(theta) * (np.cos(az) * e1 + np.sin(az) * e2))


def test_single_point_mass_closed_form(oracle_lib):
    """psi = (q/4pi)[log((1 - cos T)/2) + 1] and |alpha| = (q/4pi) cot(T/2),
    pointing along the geodesic away from the mass."""
    mp.mp.dps = 50
    rng = np.random.default_rng(11)
    s = _unit(rng.standard_normal(3))
    q = 1.7
    thetas = [1e-7, 1e-4, 0.01, 0.3, 1.0, 2.0, 3.0, np.pi - 1e-5]
    tg = np.stack([_geodesic_point(s, th, rng.uniform(0, 2 * np.pi)) for th in thetas], axis=1)
    psi, defl = oracle.direct(s.reshape(3, 1), np.array([q]), tg)
    def on_sphere(v):
        # FP64 inputs are unit vectors to ~1e-16; the closed form lives on
        # the sphere, so project there in 50 digits
        v = [mp.mpf(float(c)) for c in v]
        r = mp.sqrt(sum(c * c for c in v))
        return [c / r for c in v]

    for i in range(tg.shape[1]):
        n = on_sphere(tg[:, i])
        S = on_sphere(s)
        c = sum(a * b for a, b in zip(n, S))
        cross = [n[1] * S[2] - n[2] * S[1], n[2] * S[0] - n[0] * S[2], n[0] * S[1] - n[1] * S[0]]
        T = mp.atan2(mp.sqrt(sum(v * v for v in cross)), c)
        exp_psi = q / (4 * mp.pi) * (mp.log((1 - mp.cos(T)) / 2) + 1)
        mag = q / (4 * mp.pi) * mp.cot(T / 2)
        direc = [(n[k] * mp.cos(T) - S[k]) / mp.sin(T) for k in range(3)]
        assert abs(psi[i] - float(exp_psi)) <= 1e-15 * max(1.0, abs(float(exp_psi)))
        for k in range(3):
            # near the antipode the terms (q/2pi)(d/|d|^2 - n/2) cancel from ~q/4pi
            assert abs(defl[k, i] - float(mag * direc[k])) <= 2e-15 * float(mag) + 1e-16 * q


def test_ring_product_identity(oracle_lib):
    """K equal masses at colatitude t0 (azimuths p0 + 2 pi j/K): sum_j
    log((1 - n.n_j)/2) = K log(b^2/((1+a^2)(1+a0^2))) + log(1 - 2 r^K cos K(p-p0)
    + r^{2K}), a = tan(t/2), a0 = tan(t0/2), b = max, r = min/max."""
    mp.mp.dps = 40
    K, t0, p0, q = 37, 0.9, 0.3, 0.8
    R = _rot(np.random.default_rng(5))
    src = np.stack([[np.sin(t0) * np.cos(p0 + 2 * np.pi * j / K),
                     np.sin(t0) * np.sin(p0 + 2 * np.pi * j / K), np.cos(t0)] for j in range(K)], axis=1)
    pts_tp = [(0.2, 1.0), (0.85, 0.4), (0.95, 2.0), (1.5, 5.0), (2.9, 0.1), (0.5, 3.3)]

    def closed(t, p):
        a, a0 = mp.tan(t / 2), mp.tan(mp.mpf(t0) / 2)
        b, r = max(a, a0), min(a, a0) / max(a, a0)
        raw = K * mp.log(b * b / ((1 + a * a) * (1 + a0 * a0))) + mp.log(
            1 - 2 * r ** K * mp.cos(K * (p - p0)) + r ** (2 * K))
        return q / (4 * mp.pi) * (raw + K)      # zero-mean gauge: + K q / (4 pi)

    tg = np.stack([[np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)] for t, p in pts_tp], axis=1)
    psi, defl = oracle.direct(R @ _unit(src), np.full(K, q), R @ _unit(tg))
    for i, (t, p) in enumerate(pts_tp):
        t, p = mp.mpf(t), mp.mpf(p)
        assert abs(psi[i] - float(closed(t, p))) < 1e-14 * max(1, abs(float(closed(t, p))))
        # alpha = d psi/dt e_t + (1/sin t) d psi/dp e_p, from the closed form
        dt = mp.diff(lambda x: closed(x, p), t)
        dp = mp.diff(lambda x: closed(t, x), p) / mp.sin(t)
        e_t = np.array([np.cos(float(t)) * np.cos(float(p)), np.cos(float(t)) * np.sin(float(p)), -np.sin(float(t))])
        e_p = np.array([-np.sin(float(p)), np.cos(float(p)), 0.0])
        exp = R @ (float(dt) * e_t + float(dp) * e_p)
        assert np.abs(defl[:, i] - exp).max() < 1e-13 * max(1.0, np.abs(exp).max())


def _cap_closed(theta, theta_c, Q):
    """Uniform cap of mass Q, radius theta_c, in the zero-mean gauge.
    Outside (Gauss's law): (Q/4pi)[log sin^2(t/2) - u_c log u_c/(1-u_c)],
    u_c = cos^2(theta_c/2); inside: psi(theta_c) + (Q/pi) k [log cos(theta_c/2)
    - log cos(t/2)], k = 1/(1 - cos theta_c) - 1/2."""
    uc = mp.cos(theta_c / 2) ** 2
    out = lambda t: Q / (4 * mp.pi) * (mp.log(mp.sin(t / 2) ** 2) - uc * mp.log(uc) / (1 - uc))
    if theta >= theta_c:
        return out(theta)
    k = 1 / (1 - mp.cos(theta_c)) - mp.mpf(1) / 2
    return out(theta_c) + Q / mp.pi * k * (mp.log(mp.cos(theta_c / 2)) - mp.log(mp.cos(theta / 2)))


def test_cap_closed_form_matches_legendre_series():
    """Pins the cap closed forms (and the zero-mean constant) with the series
    psi_l = -kappa_l/(l(l+1)), kappa_l = Q (P_{l-1}(x_c) - P_{l+1}(x_c))/(4pi(1-x_c)),
    which solves Delta psi = kappa - kappa_bar (Eq. POI_EQU) with no l = 0 term."""
    from scipy.special import eval_legendre
    theta_c, Q, L = 0.5, 1.0, 6000
    xc = np.cos(theta_c)
    ls = np.arange(1, L + 1)
    kap = Q * (eval_legendre(ls - 1, xc) - eval_legendre(ls + 1, xc)) / (4 * np.pi * (1 - xc))
    coef = -kap / (ls * (ls + 1.0))
    mp.mp.dps = 30
    for t in [0.1, 0.3, 0.7, 1.2, 2.0, 3.0]:
        series = float((coef * eval_legendre(ls, np.cos(t))).sum())
        assert abs(series - float(_cap_closed(mp.mpf(t), mp.mpf(theta_c), Q))) < 2e-9


def test_uniform_cap_direct_sum(oracle_lib):
    """A cap sampled on Gauss-Legendre rings in cos(theta') (K points each)
    reproduces the exterior closed form; alpha there is (Q/4pi) cot(t/2) e_t."""
    theta_c, Q, nr, K = 0.5, 1.0, 40, 240
    xc = np.cos(theta_c)
    x, w = np.polynomial.legendre.leggauss(nr)
    xr = 0.5 * (1 - xc) * x + 0.5 * (1 + xc)
    wr = 0.5 * (1 - xc) * w
    pts, qs = [], []
    for i in range(nr):
        ph = 2 * np.pi * (np.arange(K) + 0.37 * i) / K
        s = np.sqrt(1 - xr[i] ** 2)
        pts.append(np.stack([s * np.cos(ph), s * np.sin(ph), np.full(K, xr[i])]))
        qs.append(np.full(K, Q * wr[i] / ((1 - xc) * K)))
    src = _unit(np.concatenate(pts, axis=1))
    q = np.concatenate(qs)
    R = _rot(np.random.default_rng(3))
    ts = np.array([0.8, 1.0, 1.5, 2.2, 3.0])
    ps = np.array([0.1, 1.9, 3.0, 4.4, 6.0])
    tg = _unit(np.stack([np.sin(ts) * np.cos(ps), np.sin(ts) * np.sin(ps), np.cos(ts)]))
    psi, defl = oracle.direct(R @ src, q, R @ tg)
    mp.mp.dps = 30
    for i, t in enumerate(ts):
        assert abs(psi[i] - float(_cap_closed(mp.mpf(t), mp.mpf(theta_c), Q))) < 2e-14
        e_t = np.array([np.cos(t) * np.cos(ps[i]), np.cos(t) * np.sin(ps[i]), -np.sin(t)])
        exp = R @ (Q / (4 * np.pi) / np.tan(t / 2) * e_t)
        assert np.abs(defl[:, i] - exp).max() < 1e-14


def test_zero_mean_gauge(oracle_lib):
    """The sphere integral of psi vanishes in the zero-mean gauge and is -q for
    Eq. SUM as printed (the integral of G is -1).  One source at the pole:
    2 pi times a 1-D tanh-sinh quadrature over z of the oracle's own psi."""
    mp.mp.dps = 20
    src = np.array([[0.0], [0.0], [1.0]])
    q = np.array([1.3])

    def f(gauge):
        def g(z):
            z = float(z)
            s = np.sqrt(max(0.0, (1 - z) * (1 + z)))
            p, _ = oracle.direct(src, q, np.array([[s], [0.0], [z]]), gauge=gauge, nthreads=1)
            return p[0]
        return float(2 * mp.pi * mp.quad(g, [-1, 0, 0.9, 1]))

    assert abs(f(oracle.GAUGE_ZERO_MEAN)) < 1e-11
    assert abs(f(oracle.GAUGE_RAW) + 1.3) < 1e-11


def test_rotation_invariance_and_linearity(oracle_lib):
    rng = skies.rng_for(900)
    src = skies.uniform(500, rng)
    tgt = skies.uniform(50, rng)
    q = skies.masses_lognormal(500, rng)
    R = _rot(rng)
    psi, defl = oracle.direct(src, q, tgt)
    psi_r, defl_r = oracle.direct(R @ src, q, R @ tgt)
    scale = np.abs(psi).max()
    assert np.abs(psi_r - psi).max() < 1e-13 * scale
    assert np.abs(defl_r - R @ defl).max() < 1e-13 * np.abs(defl).max()
    psi2, defl2 = oracle.direct(src, 2.5 * q, tgt)
    assert np.abs(psi2 - 2.5 * psi).max() < 1e-14 * scale
    # G is symmetric: a unit mass at a seen from b equals b seen from a
    a, b = src[:, :1], tgt[:, :1]
    pa, _ = oracle.direct(a, np.ones(1), b)
    pb, _ = oracle.direct(b, np.ones(1), a)
    assert pa[0] == pb[0]


def test_deflection_is_tangent_gradient(oracle_lib):
    """n.alpha = 0 and alpha = grad psi by central differences along geodesics."""
    rng = skies.rng_for(901)
    src = skies.uniform(300, rng)
    q = skies.masses_lognormal(300, rng)
    tgt = skies.uniform(20, rng)
    psi, defl = oracle.direct(src, q, tgt)
    assert np.abs((defl * tgt).sum(axis=0)).max() < 1e-13 * np.abs(defl).max()
    h = 1e-5
    for i in range(tgt.shape[1]):
        n = tgt[:, i]
        e1 = _unit(np.cross(n, [0.3, 0.1, 1.0]))
        e2 = np.cross(n, e1)
        for e in (e1, e2):
            pp = _unit(np.cos(h) * n + np.sin(h) * e)
            pm = _unit(np.cos(h) * n - np.sin(h) * e)
            fd = (oracle.direct(src, q, pp.reshape(3, 1))[0][0]
                  - oracle.direct(src, q, pm.reshape(3, 1))[0][0]) / (2 * h)
            assert abs(fd - defl[:, i] @ e) < 1e-6 * (1 + abs(fd))


def test_laplacian_off_source(oracle_lib):
    """Delta psi = -Q_tot/(4pi) away from the sources (Eq. LAP_GRE), by the
    five-point geodesic stencil."""
    rng = skies.rng_for(902)
    src = skies.uniform(40, rng)
    q = skies.masses_lognormal(40, rng)
    tgt = skies.uniform(8, rng)
    h = 2e-3
    for i in range(tgt.shape[1]):
        n = tgt[:, i]
        e1 = _unit(np.cross(n, [0.3, 0.1, 1.0]))
        e2 = np.cross(n, e1)
        pts = [n] + [_unit(np.cos(h) * n + np.sin(h) * s * e) for e in (e1, e2) for s in (1, -1)]
        p, _ = oracle.direct(src, q, np.stack(pts, axis=1))
        lap = (p[1:].sum() - 4 * p[0]) / h ** 2
        assert abs(lap + q.sum() / FOUR_PI) < 1e-3 * q.sum() / FOUR_PI


def test_brute_force_50_digits(oracle_lib):
    """psi and alpha at 50 digits with G in its printed form
    (1/4pi)[log(1 - n.n') - log 2] and alpha the tangent part of its ambient
    gradient -(q/4pi) n'/(1 - n.n')."""
    mp.mp.dps = 50
    rng = skies.rng_for(903)
    n_src, n_tgt = 40, 12
    src = skies.uniform(n_src, rng)
    q = skies.masses_lognormal(n_src, rng)
    tgt = skies.uniform(n_tgt, rng)
    psi, defl = oracle.direct(src, q, tgt)
    def on_sphere(v):
        # the FP64 inputs are unit vectors only to ~1e-16; the printed and the
        # |d|^2 forms of G agree exactly on the sphere, so project there
        v = [mp.mpf(float(c)) for c in v]
        r = mp.sqrt(sum(c * c for c in v))
        return [c / r for c in v]

    S = [on_sphere(src[:, j]) for j in range(n_src)]
    Qt = sum(mp.mpf(float(v)) for v in q)
    for i in range(n_tgt):
        n = on_sphere(tgt[:, i])
        acc = mp.mpf(0)
        g = [mp.mpf(0)] * 3
        for j in range(n_src):
            dot = sum(a * b for a, b in zip(n, S[j]))
            qj = mp.mpf(float(q[j]))
            acc += qj / (4 * mp.pi) * (mp.log(1 - dot) - mp.log(2))
            for k in range(3):
                g[k] += -qj / (4 * mp.pi) * S[j][k] / (1 - dot)
        gn = sum(g[k] * n[k] for k in range(3))
        exp_a = [g[k] - gn * n[k] for k in range(3)]
        exp_p = acc + Qt / (4 * mp.pi)
        # input off-sphere error ~1e-16 enters each term as 1e-16/|d|^2
        assert abs(psi[i] - float(exp_p)) < 1e-13 * max(1.0, abs(float(exp_p)))
        for k in range(3):
            assert abs(defl[k, i] - float(exp_a[k])) < 1e-12 * max(1.0, abs(float(exp_a[k])))


def test_coincident_source_excluded(oracle_lib):
    """A source at exactly the target contributes no log term; its share
    q/(4pi) of the zero-mean constant stays."""
    rng = skies.rng_for(904)
    src = skies.uniform(100, rng)
    q = skies.masses_lognormal(100, rng)
    tgt = src[:, 7:8].copy()
    psi, defl = oracle.direct(src, q, tgt)
    keep = np.arange(100) != 7
    p2, d2 = oracle.direct(src[:, keep], q[keep], tgt)
    assert abs(psi[0] - (p2[0] + q[7] / FOUR_PI)) < 1e-14
    assert np.abs(defl - d2).max() < 1e-15
    assert np.isfinite(psi).all() and np.isfinite(defl).all()
