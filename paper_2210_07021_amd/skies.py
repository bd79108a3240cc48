"""Seeded synthetic skies: point masses and target sets on the unit sphere.

Inputs only.  This module holds none of the sFMM's arithmetic; the GPU path and
the CPU oracle both take their inputs from here and from nowhere else.  Every
generator returns host numpy arrays: positions as float64 planes of shape
(3, n) holding unit vectors normalised in FP64, masses as float64 (n,).

Recipes (the paper tests on random positions with random masses, Sec. 4.1, and
on sampled NFW haloes, Sec. 4.3; no data set is used, so none is needed):

* ``uniform``    z ~ U[-1, 1], phi ~ U[0, 2pi)  (uniform on the sphere).
* ``grid``       HEALPix ring-scheme pixel centres for a given nside, the
                 equal-area target grid (12 nside^2 points).
* ``clustered``  70% of the points in 2000 clumps whose centres are uniform on
                 the sphere; clump weights drawn from dN/dM ~ M^-1.9 on
                 [1, 1e3]; particle counts multinomial in those weights; each
                 clump's angular profile the projected NFW convergence of
                 Eq. NFW (Sec. 4.3), truncated at x = 5, with scale radius
                 lognormal about 0.5 arcmin (sigma_ln = 0.5); the other 30%
                 uniform.  Masses exp(0.3 g), g ~ N(0, 1).
* ``nfw_halo``   one projected NFW halo (Eq. NFW) at the north pole, for the
                 sampling-noise experiment of Sec. 4.3.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 2210070210
ARCMIN = np.pi / (180.0 * 60.0)


def rng_for(k: int) -> np.random.Generator:
    """The generator of workload k: numpy PCG64 seeded BASE_SEED + k."""
    return np.random.Generator(np.random.PCG64(BASE_SEED + int(k)))


def _normalise(v: np.ndarray) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    return np.ascontiguousarray(v / np.sqrt((v * v).sum(axis=0)))


def uniform(n: int, rng: np.random.Generator) -> np.ndarray:
    z = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    s = np.sqrt((1.0 - z) * (1.0 + z))
    return _normalise(np.stack([s * np.cos(phi), s * np.sin(phi), z]))


def grid(nside: int) -> np.ndarray:
    """HEALPix pixel centres, ring by ring from the north pole (Gorski et al.
    2005): polar rings i < nside hold 4i pixels at z = 1 - i^2/(3 nside^2);
    equatorial rings hold 4 nside pixels at z = 4/3 - 2i/(3 nside), offset by
    half a pixel on alternate rings; the south mirrors the north."""
    ns = int(nside)
    zs, phis = [], []
    for i in range(1, 4 * ns):
        if i < ns:
            z = 1.0 - i * i / (3.0 * ns * ns)
            k = 4 * i
            phi = (np.pi / (2.0 * i)) * (np.arange(1, k + 1) - 0.5)
        elif i <= 3 * ns:
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * ns)
            k = 4 * ns
            shift = 0.5 * ((i - ns + 1) % 2)
            phi = (np.pi / (2.0 * ns)) * (np.arange(1, k + 1) - shift)
        else:
            j = 4 * ns - i
            z = -1.0 + j * j / (3.0 * ns * ns)
            k = 4 * j
            phi = (np.pi / (2.0 * j)) * (np.arange(1, k + 1) - 0.5)
        zs.append(np.full(k, z))
        phis.append(phi)
    z = np.concatenate(zs)
    phi = np.concatenate(phis)
    s = np.sqrt((1.0 - z) * (1.0 + z))
    return _normalise(np.stack([s * np.cos(phi), s * np.sin(phi), z]))


def _nfw_enclosed(x: np.ndarray) -> np.ndarray:
    """Projected NFW mass inside radius x (in units of the scale radius), up to
    a constant: the integral of 2 pi x' kappa(x') of Eq. NFW."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lo = x < 1.0
    hi = x > 1.0
    xl = x[lo]
    out[lo] = np.log(xl / 2.0) + 2.0 / np.sqrt(1.0 - xl * xl) * np.arctanh(np.sqrt((1.0 - xl) / (1.0 + xl)))
    xh = x[hi]
    out[hi] = np.log(xh / 2.0) + 2.0 / np.sqrt(xh * xh - 1.0) * np.arctan(np.sqrt((xh - 1.0) / (xh + 1.0)))
    out[~(lo | hi)] = 1.0 + np.log(0.5)
    return out


def _nfw_radii(k: int, rng: np.random.Generator, xmax: float = 5.0) -> np.ndarray:
    """k radii x in (0, xmax] by inverse CDF of the tabulated enclosed mass."""
    xs = np.concatenate([np.geomspace(1e-8, 0.999, 4000), np.linspace(1.001, xmax, 2000)])
    cdf = _nfw_enclosed(xs)
    cdf = (cdf - cdf[0]) / (cdf[-1] - cdf[0])
    return np.interp(rng.uniform(0.0, 1.0, k), cdf, xs)


def _tangent_basis(c: np.ndarray):
    """Two unit vectors orthogonal to each column of c (3, k)."""
    a = np.where(np.abs(c[2]) < 0.9, 0.0, 1.0)
    ref = np.stack([a, np.zeros_like(a), 1.0 - a])
    e1 = np.cross(ref.T, c.T).T
    e1 /= np.sqrt((e1 * e1).sum(axis=0))
    e2 = np.cross(c.T, e1.T).T
    return e1, e2


def clustered(n: int, rng: np.random.Generator, n_clumps: int = 2000,
              clumped_fraction: float = 0.7) -> np.ndarray:
    n = int(n)
    n_in = int(round(clumped_fraction * n))
    n_clumps = min(n_clumps, max(n_in, 1))
    centres = uniform(n_clumps, rng)
    # clump weights from dN/dM ~ M^-1.9 on [1, 1e3] (inverse CDF)
    a = 1.0 - 1.9
    u = rng.uniform(0.0, 1.0, n_clumps)
    w = (1.0 + u * (1e3 ** a - 1.0)) ** (1.0 / a)
    counts = rng.multinomial(n_in, w / w.sum())
    theta_s = 0.5 * ARCMIN * np.exp(0.5 * rng.standard_normal(n_clumps))
    owner = np.repeat(np.arange(n_clumps), counts)
    r = _nfw_radii(n_in, rng) * theta_s[owner]
    az = rng.uniform(0.0, 2.0 * np.pi, n_in)
    c = centres[:, owner]
    e1, e2 = _tangent_basis(c)
    pts_in = np.cos(r) * c + np.sin(r) * (np.cos(az) * e1 + np.sin(az) * e2)
    pts = np.concatenate([_normalise(pts_in), uniform(n - n_in, rng)], axis=1)
    return _normalise(pts[:, rng.permutation(n)])


def nfw_halo(n: int, rng: np.random.Generator, kappa_s: float = 0.338, r_s: float = 0.3, c: float = 5.05):
    """A test halo of Sec. 4.3 at the north pole: n equal masses whose
    density follows the projected NFW profile of Eq. NFW (amplitude kappa_s,
    scale r_s, truncated at x = c), laid on the sphere by the equal-area
    radius r = 2 sin(theta / 2) (the sphere's area element is 2 pi r dr, so
    the flat profile's mass in every ring is kept).  Radii by inverse CDF of
    the enclosed profile, azimuths uniform.  Returns (src (3, n), q (n,)),
    the masses summing to the halo's 2 pi kappa_s r_s^2 int_0^c x f(x) dx."""
    n = int(n)
    x = _nfw_radii(n, rng, xmax=c)
    theta = 2.0 * np.arcsin(np.minimum(1.0, 0.5 * x * r_s))
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    st = np.sin(theta)
    src = _normalise(np.stack([st * np.cos(phi), st * np.sin(phi), np.cos(theta)]))
    # _nfw_enclosed(x) = (1/4) int_0^x x' f(x') dx' (it vanishes at x = 0)
    total = 2.0 * np.pi * kappa_s * r_s * r_s * 4.0 * float(_nfw_enclosed(np.array([c]))[0])
    return src, np.full(n, total / n)


def masses_lognormal(n: int, rng: np.random.Generator, sigma: float = 0.3) -> np.ndarray:
    return np.exp(sigma * rng.standard_normal(int(n)))


def workload(name: str, scale: float = 1.0):
    """Named workloads: returns (src, q, tgt).

    'uniform-1e4'       N = 1e4 equal masses uniform; targets = the sources
                        themselves plus 1e4 uniform points (M = 2e4).
    'clustered-1e6'     N = 1e6 clustered, lognormal masses; M = HEALPix
                        nside 256 grid (786,432).
    'clustered-1e7'     N = 1e7 clustered, lognormal masses; M = nside 512
                        grid (3,145,728).
    'clustered-1e8'     N = 1e8 clustered, lognormal masses; M = nside 1024
                        grid (12,582,912).
    ``scale`` shrinks N (not the target grid) for quick runs."""
    if name == "uniform-1e4":
        rng = rng_for(0)
        n = int(round(1e4 * scale))
        src = uniform(n, rng)
        q = np.ones(n)
        tgt = np.ascontiguousarray(np.concatenate([src, uniform(n, rng)], axis=1))
        return src, q, tgt
    if name == "clustered-1e6":
        rng = rng_for(1)
        n = int(round(1e6 * scale))
        return clustered(n, rng), masses_lognormal(n, rng), grid(256)
    if name == "clustered-1e7":
        rng = rng_for(2)
        n = int(round(1e7 * scale))
        return clustered(n, rng), masses_lognormal(n, rng), grid(512)
    if name == "clustered-1e8":
        rng = rng_for(4)
        n = int(round(1e8 * scale))
        return clustered(n, rng), masses_lognormal(n, rng), grid(1024)
    raise ValueError(f"unknown workload {name!r}")


def shells(n_shell: int = 40, n_min: float = 1e5, n_max: float = 5e6, nside: int = 256, scale: float = 1.0,
           base: int = 3):
    """Lensing shells of one light cone: shell s has N_s = round(exp U(ln n_min,
    ln n_max)) particles (times scale) on the clustered recipe, seeded with
    generator base + 100 s; every shell has the same HEALPix grid of targets.
    Returns lists (src, q, tgt) per shell."""
    out = []
    tgt = grid(nside)
    for s_ in range(n_shell):
        rng = rng_for(base + 100 * s_)
        n = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max))) * scale))
        src = clustered(n, rng)
        q = masses_lognormal(n, rng)
        out.append((src, q, tgt))
    return out

