"""Pins of the seeded input generator (CPU only): closed forms for low
degrees, orthonormality under the grid's own Gauss quadrature, and
finite-difference checks of the analytic gradient."""
import numpy as np
import pytest

import oracle
import synthetic as sy


def _single(lmax, l, m, sin=False):
    c = np.zeros((1, lmax + 1, lmax + 1))
    s = np.zeros_like(c)
    (s if sin else c)[0, l, m] = 1.0
    return sy.SHCoeffs(c, s)


def test_closed_forms_low_degree():
    rng = np.random.default_rng(0)
    lon = rng.uniform(0, 2 * np.pi, 50)
    lat = rng.uniform(-1.5, 1.5, 50)
    val = lambda l, m, s=False: sy.synthesize(lon, lat, _single(2, l, m, s))[0]
    np.testing.assert_allclose(val(0, 0), 1.0, atol=1e-15)
    np.testing.assert_allclose(val(1, 0), np.sqrt(3) * np.sin(lat), atol=1e-14)
    np.testing.assert_allclose(val(1, 1), np.sqrt(3) * np.cos(lat) * np.cos(lon), atol=1e-14)
    np.testing.assert_allclose(val(1, 1, True), np.sqrt(3) * np.cos(lat) * np.sin(lon), atol=1e-14)
    np.testing.assert_allclose(val(2, 0), np.sqrt(5) * 0.5 * (3 * np.sin(lat) ** 2 - 1), atol=1e-14)
    np.testing.assert_allclose(val(2, 2), np.sqrt(15) / 2 * np.cos(lat) ** 2 * np.cos(2 * lon),
                               atol=1e-14)


@pytest.mark.parametrize("N,lmax", [(8, 6), (16, 8)])
def test_orthonormal_under_gauss_quadrature(N, lmax):
    m = oracle.Mesh(N)
    _, w = np.polynomial.legendre.leggauss(2 * N)
    wn = np.repeat(w[::-1] * 2 * np.pi / m.nx, m.nx)
    B = []
    for l in range(lmax + 1):
        for mm in range(l + 1):
            B.append(sy.synthesize(m.lon, m.lat, _single(lmax, l, mm))[0])
            if mm:
                B.append(sy.synthesize(m.lon, m.lat, _single(lmax, l, mm, True))[0])
    B = np.array(B)
    G = (B * wn) @ B.T / (4 * np.pi)
    np.testing.assert_allclose(G, np.eye(len(B)), atol=1e-13)


def test_gradient_matches_finite_differences():
    co = sy.random_coeffs(6, [sy.seed_rng(1, 2, 3), sy.seed_rng(1, 2, 4)])
    rng = np.random.default_rng(1)
    lon = rng.uniform(0, 2 * np.pi, 20)
    lat = rng.uniform(-1.4, 1.4, 20)
    g = sy.synthesize_gradient(lon, lat, co, R=2.0)
    h = 1e-6
    fx = (sy.synthesize(lon + h, lat, co) - sy.synthesize(lon - h, lat, co)) / (2 * h)
    fy = (sy.synthesize(lon, lat + h, co) - sy.synthesize(lon, lat - h, co)) / (2 * h)
    np.testing.assert_allclose(g[..., 0], fx / (2.0 * np.cos(lat)), rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(g[..., 1], fy / 2.0, rtol=1e-6, atol=1e-7)


def test_ring_fft_equals_direct_evaluation():
    m = oracle.Mesh(4)
    co = sy.random_coeffs(30, [sy.seed_rng(2, 0, 0)])  # degrees above nx/2: aliasing folds
    ring = sy.synthesize(m.lon, m.lat, co)
    perm = np.random.default_rng(0).permutation(m.V)   # breaks the ring layout
    direct = np.empty_like(ring)
    direct[:, perm] = sy.synthesize(m.lon[perm], m.lat[perm], co)
    np.testing.assert_allclose(ring, direct, atol=1e-11)


def test_seeds_reproducible_and_amplitude():
    m = oracle.Mesh(32)
    a = sy.level_field_stack(m.lon, m.lat, 3, 8, 2, 0, noise_eps=1e-3)
    b = sy.level_field_stack(m.lon, m.lat, 3, 8, 2, 0, noise_eps=1e-3)
    np.testing.assert_array_equal(a, b)
    f = sy.config_field(m.lon, m.lat, 16, 9, 0, amplitude=100.0)
    _, w = np.polynomial.legendre.leggauss(64)
    wn = np.repeat(w[::-1] * 2 * np.pi / m.nx, m.nx)
    rms = np.sqrt((wn * f ** 2).sum() / (4 * np.pi))
    assert 60 < rms < 140
