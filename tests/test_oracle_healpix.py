"""Pins of the oracle's HEALPix geometry (sphere division of Sec. 3.1, box
radius of Sec. 3.5) against facts fixed by the published HEALPix definition
and by geometry:

* the 12 base pixel centres (faces 0-3 at z = 2/3, 4-7 on the equator, 8-11
  at z = -2/3);
* the ring-scheme pixel centres of an independent generator map one-to-one
  onto the nested indices;
* equal area: uniform points fall evenly into the pixels;
* nesting: the order-29 key truncated to order L is the order-L key;
* every point of a pixel, boundary included, lies within its radius;
* the paper's scale for the maximum depth (Sec. 3.1).
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2210_07021_amd import skies

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def test_base_face_centres(oracle_lib):
    for f in range(12):
        c = oracle.pix_point(0, f)
        if f < 4:
            z, phi = 2.0 / 3.0, np.pi / 4 + f * np.pi / 2
        elif f < 8:
            z, phi = 0.0, (f - 4) * np.pi / 2
        else:
            z, phi = -2.0 / 3.0, np.pi / 4 + (f - 8) * np.pi / 2
        s = np.sqrt(1 - z * z)
        assert np.allclose(c, [s * np.cos(phi), s * np.sin(phi), z], atol=1e-15)


@pytest.mark.parametrize("nside", [1, 2, 16, 64])
def test_ring_grid_bijection(oracle_lib, nside):
    order = int(np.log2(nside))
    g = skies.grid(nside)
    k = oracle.keys(g, order)
    assert sorted(k.tolist()) == list(range(12 * nside * nside))


def test_centre_round_trip(oracle_lib):
    rng = np.random.default_rng(7)
    for order in [0, 1, 3, 8, 15, 22, 29]:
        npix = 12 * 4 ** order
        for pix in rng.integers(0, npix, 50):
            c = oracle.pix_point(order, int(pix))
            assert oracle.key(*c, order=order) == pix


def test_equal_area(oracle_lib):
    pts = skies.uniform(120000, skies.rng_for(910))
    k = oracle.keys(pts, 2)
    counts = np.bincount(k, minlength=192)
    exp = 120000 / 192
    chi2 = ((counts - exp) ** 2 / exp).sum()
    # 191 degrees of freedom: mean 191, sd ~19.5
    assert chi2 < 191 + 6 * 19.5


def test_nesting_of_keys(oracle_lib):
    pts = skies.uniform(3000, skies.rng_for(911))
    k29 = oracle.keys(pts, 29)
    for order in [0, 4, 10, 17, 25]:
        kl = oracle.keys(pts, order)
        assert np.array_equal(k29 >> (2 * (29 - order)), kl)


@pytest.mark.parametrize("order", [0, 1, 2, 5, 12, 20, 29])
def test_pixel_within_radius(oracle_lib, order):
    """Boundary sampled densely and interior points: all within R of the
    centre, R = largest centre-vertex distance (the covering-circle reading)."""
    rng = np.random.default_rng(order)
    npix = 12 * 4 ** order
    pixels = range(npix) if npix <= 48 else rng.integers(0, npix, 40)
    t = np.linspace(0.0, 1.0, 101)
    for pix in pixels:
        c = oracle.pix_point(order, int(pix))
        R = oracle.box_radius(order, int(pix))
        fx = np.concatenate([t, t, np.zeros_like(t), np.ones_like(t), rng.random(100)])
        fy = np.concatenate([np.zeros_like(t), np.ones_like(t), t, t, rng.random(100)])
        for a, b in zip(fx, fy):
            p = oracle.pix_point(order, int(pix), a, b)
            assert oracle.angdist(c, p) <= R * (1 + 1e-12) + 1e-15


def test_points_inside_their_pixel(oracle_lib):
    pts = skies.uniform(400, skies.rng_for(912))
    k29 = oracle.keys(pts, 29)
    for order in [0, 3, 9, 16, 23, 29]:
        for i in range(pts.shape[1]):
            pix = int(k29[i]) >> (2 * (29 - order))
            c = oracle.pix_point(order, pix)
            assert oracle.angdist(c, pts[:, i]) <= oracle.box_radius(order, pix) * (1 + 1e-9)


def test_max_depth_scale_matches_paper(oracle_lib):
    """Sec. 3.1: maximum depth 29 ~ box radius 4e-4 arcsec."""
    ref = json.load(open(GOLDEN))["max_depth_box_radius_arcsec"]
    arcsec = np.pi / (180 * 3600)
    rng = np.random.default_rng(3)
    radii = [oracle.box_radius(29, int(p)) / arcsec for p in rng.integers(0, 12 * 4 ** 29, 20)]
    assert ref["max_level"] == 29
    assert 0.5 * ref["value"] < np.median(radii) < 1.5 * ref["value"]
