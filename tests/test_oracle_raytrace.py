"""Pins of the oracle's multi-plane backtracking (Sec. 2.1, Eq. DIS_PRO):
a point-mass layer moves each ray toward the mass by w (q/4pi) cot(Theta/2)
along the great circle; empty layers leave rays and distortion unchanged;
the parallel transport along a meridian is the identity in (e_theta,
e_phi); the distortion matrix is the derivative of the traced positions
(central differences); weak layers add up to the Born sum."""
import numpy as np
import pytest

import oracle
from oracle import raytrace as rt


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _unit(v):
    return v / np.linalg.norm(v, axis=0)


def test_point_mass_layer_closed_form():
    rng = np.random.default_rng(1)
    s = _unit(rng.normal(size=(3, 1)))
    q, w = np.array([0.01]), 0.7
    rays = _unit(rng.normal(size=(3, 200)))
    out, _ = rt.trace([(s, q)], [w], rays, with_distortion=False)
    theta = np.arccos(np.clip(s[:, 0] @ rays, -1, 1))
    shift = w * q[0] / (4 * np.pi) / np.tan(theta / 2)       # toward the mass
    theta_out = np.arccos(np.clip(s[:, 0] @ out, -1, 1))
    assert np.allclose(theta_out, theta - shift, rtol=0, atol=1e-12)
    # the ray stays on the great circle through the mass and its start
    nrm = np.cross(s[:, 0], rays.T)
    assert np.allclose(np.sum(nrm * out.T, axis=1), 0, atol=1e-13)
    assert np.allclose(np.linalg.norm(out, axis=0), 1, atol=1e-14)


def test_empty_layers_are_the_identity():
    rays = _unit(np.random.default_rng(2).normal(size=(3, 50)))
    empty = (np.zeros((3, 0)), np.zeros(0))
    out, A = rt.trace([empty, empty], [0.5, 0.3], rays)
    assert np.array_equal(out, rays)
    assert np.allclose(A, np.array([1, 0, 0, 1.0])[:, None])


def test_transport_along_a_meridian_is_the_identity():
    rng = np.random.default_rng(3)
    n = _unit(rng.normal(size=(3, 20)))
    et, _ = rt.basis(n)
    n2, T = rt.step(n, 0.1 * et)
    assert np.allclose(T, np.eye(2)[None], atol=1e-13)
    _, ep = rt.basis(n)
    n3, T3 = rt.step(n, 0.05 * ep)   # along a great circle that is not a meridian: a rotation
    assert np.allclose(np.einsum("mij,mkj->mik", T3, T3), np.eye(2)[None], atol=1e-13)
    assert np.allclose(np.linalg.det(T3), 1.0, atol=1e-13)


def test_distortion_is_derivative_of_traced_positions():
    rng = np.random.default_rng(4)
    shells = []
    for _ in range(3):
        src = _unit(rng.normal(size=(3, 30)))
        shells.append((src, rng.uniform(0.5, 1.5, 30) * 1e-4))
    w = [0.9, 0.6, 0.3]
    rays = _unit(rng.normal(size=(3, 10)))
    out, A = rt.trace(shells, w, rays)
    et0, ep0 = rt.basis(rays)
    et1, ep1 = rt.basis(out)
    h = 1e-6
    for j, e in enumerate((et0, ep0)):
        p, _ = rt.trace(shells, w, rays * np.cos(h) + e * np.sin(h), with_distortion=False)
        m, _ = rt.trace(shells, w, rays * np.cos(h) - e * np.sin(h), with_distortion=False)
        d = (p - m) / (2 * h)
        fd = np.stack([np.sum(et1 * d, 0), np.sum(ep1 * d, 0)])
        got = np.stack([A[j], A[2 + j]])            # column j of A
        assert np.allclose(fd, got, rtol=0, atol=1e-6), (j, np.abs(fd - got).max())


def test_weak_layers_add_up_to_the_born_sum():
    rng = np.random.default_rng(5)
    shells = [(_unit(rng.normal(size=(3, 20))), np.full(20, 1e-6)) for _ in range(4)]
    w = [0.8, 0.6, 0.4, 0.2]
    rays = _unit(rng.normal(size=(3, 30)))
    out, _ = rt.trace(shells, w, rays, with_distortion=False)
    born = rays.copy()
    for (s, q), wi in zip(shells, w):
        born -= wi * oracle.direct(s, q, rays)[1]
    shift = np.linalg.norm(out - rays, axis=0)
    assert np.all(np.linalg.norm(out - born, axis=0) <= 1e-3 * shift + 1e-15)
