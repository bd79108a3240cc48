"""Global-basis helpers of the C ABI (Sec. 3.6: the deflection's components in
the global frame by a change of coordinates).  Host functions of libsfmm.so,
checked on the CPU against the closed forms of the spherical basis and
against finite differences of the oracle's psi, which fixes the orientation
and normalisation of (alpha_theta, alpha_phi) independently of the library."""
import numpy as np
import pytest

import oracle
from paper_2210_07021_amd import skies


@pytest.fixture(scope="module")
def sf():
    import os
    import paper_2210_07021_amd as sf
    if not os.path.exists(sf.LIB_PATH):
        from paper_2210_07021_amd import build
        build.build()
    sf.load_library()
    return sf


def test_thetaphi_to_xyz_closed_form(sf):
    rng = np.random.default_rng(5)
    t = np.concatenate([[0.0, np.pi, np.pi / 2], np.arccos(rng.uniform(-1, 1, 200))])
    f = np.concatenate([[0.3, 1.0, -2.0], rng.uniform(-np.pi, 3 * np.pi, 200)])
    x = sf.thetaphi_to_xyz(t, f)
    assert x.shape == (3, t.size)
    np.testing.assert_allclose(np.linalg.norm(x, axis=0), 1.0, atol=1e-15)
    np.testing.assert_allclose(np.arccos(np.clip(x[2], -1, 1)), t, atol=2e-7)  # arccos loses digits near 0, pi
    far = (t > 0.1) & (t < np.pi - 0.1)
    np.testing.assert_allclose(np.mod(np.arctan2(x[1], x[0])[far] - f[far], 2 * np.pi) % (2 * np.pi), 0.0,
                               atol=1e-12)
    np.testing.assert_array_equal(x[:, 0], [0.0, 0.0, 1.0])
    assert abs(x[2, 1] + 1.0) == 0.0 and abs(x[0, 1]) < 1e-15


def test_defl_components_are_the_angular_derivatives_of_psi(sf):
    """alpha_theta = d psi / d theta, alpha_phi = (1/sin theta) d psi / d phi
    (Eq. ALP_PSI in spherical coordinates), by central differences of the
    oracle's psi; a swapped or sign-flipped basis vector fails."""
    rng = skies.rng_for(77)
    src = skies.uniform(300, rng)
    q = skies.masses_lognormal(300, rng)
    t = np.arccos(rng.uniform(-0.95, 0.95, 40))
    f = rng.uniform(0, 2 * np.pi, 40)
    xyz = sf.thetaphi_to_xyz(t, f)
    _, a = oracle.direct(src, q, xyz)
    comp = sf.defl_to_thetaphi(xyz, a)
    h = 1e-5
    pt = oracle.direct(src, q, sf.thetaphi_to_xyz(t + h, f))[0] - oracle.direct(src, q, sf.thetaphi_to_xyz(t - h, f))[0]
    pf = oracle.direct(src, q, sf.thetaphi_to_xyz(t, f + h))[0] - oracle.direct(src, q, sf.thetaphi_to_xyz(t, f - h))[0]
    d_t = pt / (2 * h)
    d_f = pf / (2 * h) / np.sin(t)
    scale = np.sqrt(np.mean(comp ** 2))
    # central differences: O(h^2) truncation, ~1e-6 relative next to a source
    np.testing.assert_allclose(comp[0], d_t, atol=1e-5 * scale)
    np.testing.assert_allclose(comp[1], d_f, atol=1e-5 * scale)
    # the tangent vector is recovered from its two components
    st, ct = np.sin(t), np.cos(t)
    e_t = np.array([ct * np.cos(f), ct * np.sin(f), -st])
    e_f = np.array([-np.sin(f), np.cos(f), np.zeros_like(f)])
    np.testing.assert_allclose(comp[0] * e_t + comp[1] * e_f, a, atol=1e-13 * scale)


@pytest.mark.parametrize("pole", [1.0, -1.0])
def test_pole_basis_is_the_limit_along_phi(sf, pole):
    """At an exact pole the components follow the meridian phi: alpha_theta
    is the one-sided derivative of psi along it (theta measured from the
    north pole, so at the south pole psi grows with -theta)."""
    rng = skies.rng_for(78)
    src = skies.uniform(200, rng)
    q = skies.masses_lognormal(200, rng)
    xyz = np.array([[0.0], [0.0], [pole]])
    _, a = oracle.direct(src, q, xyz)
    h = 1e-5
    tn = h if pole > 0 else np.pi - h  # one step off the pole along a meridian
    for phi in (0.0, 0.7, 2.5):
        comp = sf.defl_to_thetaphi(xyz, a, phi=np.array([phi]))
        on_phi = oracle.direct(src, q, sf.thetaphi_to_xyz([tn], [phi]))[0][0]
        opposite = oracle.direct(src, q, sf.thetaphi_to_xyz([tn], [phi + np.pi]))[0][0]
        # near the north pole, meridian phi leaves along +e_theta(phi); near
        # the south pole it arrives along +e_theta(phi), i.e. leaves the pole
        # along -e_theta(phi)
        d = (on_phi - opposite) / (2 * h) * (1.0 if pole > 0 else -1.0)
        assert abs(comp[0, 0] - d) < 1e-6 * np.linalg.norm(a)
        # alpha_phi: the derivative across the meridian, along e_phi(phi)
        side = oracle.direct(src, q, sf.thetaphi_to_xyz([tn], [phi + np.pi / 2]))[0][0]
        other = oracle.direct(src, q, sf.thetaphi_to_xyz([tn], [phi - np.pi / 2]))[0][0]
        d_f = (side - other) / (2 * h)  # e_phi(phi) is the same at both poles
        assert abs(comp[1, 0] - d_f) < 1e-6 * np.linalg.norm(a)
    # without phi the limit at phi = 0 is taken
    np.testing.assert_array_equal(sf.defl_to_thetaphi(xyz, a), sf.defl_to_thetaphi(xyz, a, phi=np.array([0.0])))


def test_helpers_reject_bad_arguments(sf):
    with pytest.raises(ValueError):
        sf.defl_to_thetaphi(np.zeros((3, 2)), np.zeros((3, 3)))
    lib = sf.load_library()
    assert lib.sfmm_thetaphi_to_xyz(None, None, -1, None) == sf.SFMM_ERR_INVALID_ARG
    assert lib.sfmm_defl_to_thetaphi(None, None, None, 3, None) == sf.SFMM_ERR_INVALID_ARG
    assert lib.sfmm_thetaphi_to_xyz(None, None, 0, None) == 0
