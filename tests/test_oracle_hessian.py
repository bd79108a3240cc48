"""Pins of the oracle's Hessian of psi (Sec. 2.2, the matrix H of Eq.
GAM_DEF): the point-mass closed form in the paper's spherical derivatives,
the trace fixed by Eq. LAP_GRE (tr H = kappa - kappa_bar = -Q_tot/(4 pi) off
the sources), the covariant derivative of the oracle's own (pinned)
deflection by finite differences along great circles, and the exact pole."""
import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _basis(n):
    x, y, z = n
    rho = np.hypot(x, y)
    cph, sph = (x / rho, y / rho) if rho > 0 else (1.0, 0.0)
    return np.array([z * cph, z * sph, -rho]), np.array([-sph, cph, 0.0])


def _unit(v):
    return v / np.linalg.norm(v)


def test_point_mass_closed_form():
    """A mass q at the north pole: psi = (q/4pi) log((1 - cos theta)/2), so
    d^2psi/dtheta^2 = -q/(8 pi sin^2(theta/2)), the mixed term vanishes and
    cot(theta) dpsi/dtheta = (q/4pi) cot(theta) cot(theta/2).  A mass
    anywhere: the same two values on the tangent direction away from the
    mass and the one across it."""
    rng = np.random.default_rng(1)
    q = 1.7
    for th in (1e-4, 0.01, 0.3, 1.0, 2.0, 3.1):
        ph = rng.uniform(0, 2 * np.pi)
        n = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
        h = oracle.hessian(np.array([[0.0], [0.0], [1.0]]), np.array([q]), n[:, None])[:, 0]
        s2 = np.sin(th / 2) ** 2
        want = (-q / (8 * np.pi * s2), 0.0, q / (4 * np.pi) / np.tan(th) / np.tan(th / 2))
        scale = q / (8 * np.pi * s2)
        assert np.allclose(h, want, rtol=0, atol=1e-12 * scale), (th, h, want)
    for _ in range(50):
        s = _unit(rng.normal(size=3))
        n = _unit(rng.normal(size=3))
        h = oracle.hessian(s[:, None], np.array([q]), n[:, None])[:, 0]
        theta = np.arccos(np.clip(s @ n, -1, 1))
        s2 = np.sin(theta / 2) ** 2
        huu = -q / (8 * np.pi * s2)
        htt = q / (8 * np.pi * s2) - q / (4 * np.pi)
        u = _unit((n - s) - n * (n @ (n - s)))          # away from the mass
        t = np.cross(n, u)
        et, ep = _basis(n)
        H = huu * np.outer(u, u) + htt * np.outer(t, t)
        want = (et @ H @ et, et @ H @ ep, ep @ H @ ep)
        assert np.allclose(h, want, rtol=0, atol=1e-11 * abs(huu))


def test_trace_is_minus_mean_density():
    """tr H = Laplacian of psi = -Q_tot/(4 pi) away from the sources."""
    rng = np.random.default_rng(2)
    src = np.array([_unit(v) for v in rng.normal(size=(300, 3))]).T
    q = rng.lognormal(0, 0.3, 300)
    tgt = np.array([_unit(v) for v in rng.normal(size=(200, 3))]).T
    h = oracle.hessian(src, q, tgt)
    tr = h[0] + h[2]
    scale = np.abs(h).max()
    assert np.allclose(tr, -q.sum() / (4 * np.pi), rtol=0, atol=1e-10 * scale)
    kk, g1, g2, mu = oracle.lensing(h)
    assert np.allclose(kk, tr) and np.allclose(g1, 0.5 * (h[0] - h[2])) and np.array_equal(g2, h[1])
    assert np.allclose(mu, 1.0 / ((1 - kk / 2) ** 2 - g1 ** 2 - g2 ** 2))


def test_hessian_is_derivative_of_deflection():
    """H_ab = e_b . d alpha / dt along the great circle through n in
    direction e_a (the covariant derivative of the tangent field alpha),
    central differences of the oracle's deflection; both orders of a, b."""
    rng = np.random.default_rng(3)
    src = np.array([_unit(v) for v in rng.normal(size=(40, 3))]).T
    q = rng.lognormal(0, 0.3, 40)
    hstep = 1e-5
    for _ in range(20):
        n = _unit(rng.normal(size=3))
        while np.min(np.linalg.norm(src - n[:, None], axis=0)) < 0.05:  # FD error grows like h^2/|d|^4
            n = _unit(rng.normal(size=3))
        et, ep = _basis(n)
        h = oracle.hessian(src, q, n[:, None])[:, 0]
        H = np.array([[h[0], h[1]], [h[1], h[2]]])
        E = (et, ep)
        fd = np.zeros((2, 2))
        for a in range(2):
            pts = np.stack([n * np.cos(hstep) + E[a] * np.sin(hstep), n * np.cos(hstep) - E[a] * np.sin(hstep)], 1)
            _, al = oracle.direct(src, q, pts)
            d = (al[:, 0] - al[:, 1]) / (2 * hstep)
            for b in range(2):
                fd[a, b] = E[b] @ d
        assert np.allclose(fd, H, rtol=0, atol=1e-6 * np.abs(H).max()), (fd, H)


def test_exact_pole_uses_phi_zero():
    """At an exact pole the basis is the limit at phi = 0:
    e_theta = (cos theta, 0, 0), e_phi = (0, 1, 0)."""
    s = _unit(np.array([0.3, -0.4, 0.5]))
    q = np.array([2.0])
    for z in (1.0, -1.0):
        n = np.array([0.0, 0.0, z])
        h = oracle.hessian(s[:, None], q, n[:, None])[:, 0]
        et, ep = np.array([z, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
        theta = np.arccos(s @ n)
        s2 = np.sin(theta / 2) ** 2
        u = _unit((n - s) - n * (n @ (n - s)))
        t = np.cross(n, u)
        H = -q[0] / (8 * np.pi * s2) * np.outer(u, u) + (q[0] / (8 * np.pi * s2) - q[0] / (4 * np.pi)) * np.outer(t, t)
        assert np.allclose(h, (et @ H @ et, et @ H @ ep, ep @ H @ ep), rtol=0, atol=1e-13)
