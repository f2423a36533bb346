"""Pins of the oracle's nabla operators (CPU only).

Section 4.7 / Figure 33 names gradient, divergence, curl and Laplacian of an
edge-based finite-volume method; Listing 12 fixes the gradient's output as
the two horizontal components.  The paper prints no operator values, so the
pins are mathematical: exactness of the median-dual Green-Gauss scheme for
linear data, conservation (fluxes telescope), the Galerkin identity checked
by brute force on every triangle, closed-form spherical harmonics, and
level independence (Section 4.3: the vertical is an extrusion of
independent levels).
"""
import numpy as np
import pytest

import oracle
import synthetic as sy

EPS = np.finfo(np.float64).eps


def _polar(m):
    p = np.zeros(m.V, bool)
    p[:20] = True
    p[-20:] = True
    return p


def _seam(m):
    """Nodes with an edge crossing lon = 0 (phi = lon jumps there)."""
    bad = np.zeros(m.V, bool)
    jump = np.abs(m.lon[m.edge[:, 0]] - m.lon[m.edge[:, 1]]) > np.pi
    bad[m.edge[jump, 0]] = True
    bad[m.edge[jump, 1]] = True
    return bad


def _flux_scale(m):
    """sum over a node's faces of |S| (cancellation bound of the sums)."""
    s = np.zeros(m.V)
    np.add.at(s, m.edge[:, 0], np.abs(m.S).sum(1))
    np.add.at(s, m.edge[:, 1], np.abs(m.S).sum(1))
    return s + 2 * np.pi / 20 * _polar(m)


@pytest.mark.parametrize("N,R", [(1, 1.0), (16, 1.0), (48, 6.371229e6)])
def test_gradient_of_constant_vanishes(N, R):
    m = oracle.Mesh(N, R)
    c = 3.5
    g = m.gradient(np.full(m.V, c))[:, 0, :]
    cos = np.cos(m.lat)
    # rounding of the sums plus the closure residual of the geometry, whose
    # normals are differences of coordinates of size ~pi
    bound = 8 * EPS * c * (_flux_scale(m) + np.pi) / (R * m.A)
    assert np.all(np.abs(g[:, 0]) <= bound / cos)
    assert np.all(np.abs(g[:, 1]) <= bound)


@pytest.mark.parametrize("N,R", [(2, 1.0), (16, 1.0), (64, 6.371229e6)])
def test_gradient_exact_for_linear_data(N, R):
    m = oracle.Mesh(N, R)
    inner = ~_polar(m)
    g = m.gradient(m.lat.copy())[:, 0, :]
    np.testing.assert_allclose(g[inner, 0], 0.0, atol=1e-12 / R)
    np.testing.assert_allclose(g[inner, 1], 1.0 / R, rtol=1e-12)
    ok = inner & ~_seam(m)
    g = m.gradient(m.lon.copy())[:, 0, :]
    np.testing.assert_allclose(g[ok, 0], 1.0 / (R * np.cos(m.lat[ok])), rtol=1e-12)
    np.testing.assert_allclose(g[ok, 1], 0.0, atol=1e-11 / R)
    # the polar nodes are NOT exact (the pole face carries (phi_i+phi_p)/2)
    g = m.gradient(m.lat.copy())[:, 0, :]
    assert np.abs(g[_polar(m), 1] - 1.0 / R).min() > 1e-3 / R


@pytest.mark.parametrize("N", [2, 16, 64])
def test_divergence_and_curl_exact_cases(N):
    m = oracle.Mesh(N)
    cos = np.cos(m.lat)
    inner = ~_polar(m)
    ok = inner & ~_seam(m)
    uv = np.zeros((m.V, 1, 2))
    uv[:, 0, 1] = m.lat / cos                  # v cos(lat) = lat
    np.testing.assert_allclose(m.divergence(uv)[inner, 0], 1 / cos[inner], rtol=1e-12)
    uv = np.zeros((m.V, 1, 2))
    uv[:, 0, 0] = m.lon                        # d u / d lon = 1
    np.testing.assert_allclose(m.divergence(uv)[ok, 0], 1 / cos[ok], rtol=1e-12)
    uv = np.zeros((m.V, 1, 2))
    uv[:, 0, 0] = m.lat / cos                  # -d(u cos)/d lat = -1
    np.testing.assert_allclose(m.curl(uv)[inner, 0], -1 / cos[inner], rtol=1e-12)
    uv = np.zeros((m.V, 1, 2))
    uv[:, 0, 1] = m.lon                        # d v / d lon = 1
    np.testing.assert_allclose(m.curl(uv)[ok, 0], 1 / cos[ok], rtol=1e-12)
    # the components are not interchangeable: swapping them breaks both
    uv = np.zeros((m.V, 1, 2))
    uv[:, 0, 0] = m.lat / cos
    assert np.abs(m.divergence(uv)[ok, 0] - 1 / cos[ok]).max() > 0.1


@pytest.mark.parametrize("N", [1, 16, 80])
def test_fluxes_telescope(N):
    m = oracle.Mesh(N)
    rng = np.random.default_rng(5)
    uv = rng.standard_normal((m.V, 3, 2))
    scale = (_flux_scale(m)[:, None] * np.abs(uv).max(2)).sum()
    for op in (m.divergence, m.curl):
        tot = (m.vol[:, None] * op(uv, 3)).sum(0)
        assert np.all(np.abs(tot) <= 8 * EPS * scale)
    # pole edges must not enter div/curl: with them the sum would not vanish
    tot_pole = sum(abs(m.pole_normal[k]) * np.abs(uv[m.pole_edge[k], :, 1]).sum()
                   for k in range(m.npole))
    assert tot_pole > 1e3 * 8 * EPS * scale


@pytest.mark.parametrize("N", [1, 4, 8])
def test_galerkin_identity_bruteforce(N):
    """At every non-polar node and for ANY nodal values, the edge sum equals
    sum over the node's triangles of |T|/3 times the gradient of the linear
    interpolant on T (computed here from each triangle by a 2x2 solve)."""
    m = oracle.Mesh(N)
    rng = np.random.default_rng(11)
    f = rng.standard_normal(m.V)
    P = m.tri
    x = m.lon[P].copy()
    y = m.lat[P].copy()
    for c in (1, 2):
        x[:, c] = x[:, 0] + (x[:, c] - x[:, 0] + np.pi) % (2 * np.pi) - np.pi
    acc = np.zeros((m.V, 2))
    for t in range(m.F):
        M = np.array([[x[t, 1] - x[t, 0], y[t, 1] - y[t, 0]],
                      [x[t, 2] - x[t, 0], y[t, 2] - y[t, 0]]])
        rhs = np.array([f[P[t, 1]] - f[P[t, 0]], f[P[t, 2]] - f[P[t, 0]]])
        grad = np.linalg.solve(M, rhs)
        area = 0.5 * np.linalg.det(M)
        for c in range(3):
            acc[P[t, c]] += area / 3 * grad
    g = m.gradient(f)[:, 0, :]
    G = np.stack([g[:, 0] * np.cos(m.lat) * m.A, g[:, 1] * m.A], axis=1)  # R = 1
    inner = ~_polar(m)
    np.testing.assert_allclose(G[inner], acc[inner], rtol=0,
                               atol=1e-13 * np.abs(f).max())


def test_levels_are_independent():
    m = oracle.Mesh(16)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((m.V, 5))
    uv = rng.standard_normal((m.V, 5, 2))
    G, D, C, L = m.gradient(f, 5), m.divergence(uv, 5), m.curl(uv, 5), m.laplacian(f, 5)
    for k in range(5):
        np.testing.assert_array_equal(G[:, k], m.gradient(f[:, k].copy())[:, 0])
        np.testing.assert_array_equal(D[:, k], m.divergence(uv[:, k].copy())[:, 0])
        np.testing.assert_array_equal(C[:, k], m.curl(uv[:, k].copy())[:, 0])
        np.testing.assert_array_equal(L[:, k], m.laplacian(f[:, k].copy())[:, 0])


def test_laplacian_is_div_of_grad():
    m = oracle.Mesh(16)
    f = np.random.default_rng(4).standard_normal((m.V, 2))
    np.testing.assert_array_equal(m.laplacian(f, 2), m.divergence(m.gradient(f, 2), 2))


@pytest.mark.parametrize("N", [8, 16])
def test_sampled_evaluators_bitwise_equal_dense(N):
    m = oracle.Mesh(N)
    rng = np.random.default_rng(6)
    f = rng.standard_normal((m.V, 3))
    uv = rng.standard_normal((m.V, 3, 2))
    nodes = np.concatenate([np.arange(25), rng.integers(0, m.V, 40), np.arange(m.V - 25, m.V)])
    np.testing.assert_array_equal(m.gradient_at(f, 3, nodes), m.gradient(f, 3)[nodes])
    np.testing.assert_array_equal(m.divergence_at(uv, 3, nodes), m.divergence(uv, 3)[nodes])
    np.testing.assert_array_equal(m.curl_at(uv, 3, nodes), m.curl(uv, 3)[nodes])
    np.testing.assert_array_equal(m.laplacian_at(f, 3, nodes), m.laplacian(f, 3)[nodes])


def _seam_distance(m):
    """Cells from the nearest octahedral seam: the quarter meridians
    (lon = 0, 90, 180, 270 deg) and the equator strip."""
    ring = np.repeat(np.arange(m.nrings), m.nx)
    idx = np.arange(m.V) - m.ring_off[ring]
    q = m.nx[ring] // 4
    dm = np.minimum(idx % q, q - idx % q)
    de = np.minimum(np.abs(ring - (m.N - 1)), np.abs(ring - m.N))
    return np.minimum(dm, de)


@pytest.mark.slow
def test_second_order_convergence_away_from_seams():
    """Random harmonic fields of degree <= 4: area-weighted RMS errors over
    |lat| <= 60 deg, at least 3 cells from the octahedron's seam lines,
    fall at second order: observed orders 1.89-1.95 for the operators and
    1.74-1.87 for the identities div(k x grad) = curl(grad) = 0, rising
    towards 2 with resolution."""
    errs = []
    for N in (64, 128, 256):
        m = oracle.Mesh(N)
        co = sy.random_coeffs(4, [sy.seed_rng(7, 0, 0)])
        f = sy.synthesize(m.lon, m.lat, co)[0]
        g = sy.synthesize_gradient(m.lon, m.lat, co)[0]
        lap = sy.synthesize(m.lon, m.lat, sy.laplacian_coeffs(co))[0]
        band = (np.abs(m.lat) <= np.radians(60)) & (_seam_distance(m) > 2)
        w = m.vol[band]

        def rms(e):
            return np.sqrt((w * e[band] ** 2).sum() / w.sum())

        rg = sy.rotated_gradient(g)
        errs.append([
            rms(np.hypot(*(m.gradient(f)[:, 0, :] - g).T)),
            rms(m.divergence(g[:, None, :].copy())[:, 0] - lap),
            rms(m.curl(rg[:, None, :].copy())[:, 0] - lap),
            rms(m.laplacian(f)[:, 0] - lap),
            rms(m.divergence(rg[:, None, :].copy())[:, 0]),   # div(k x grad) = 0
            rms(m.curl(g[:, None, :].copy())[:, 0]),          # curl(grad) = 0
        ])
    errs = np.array(errs)
    order = np.log2(errs[:-1] / errs[1:])
    assert np.all(order[:, :4] >= 1.85), order
    assert np.all(order[:, 4:] >= 1.7), order
    assert np.all(order[-1] >= 1.85), order
    # on the seams themselves the scheme is only first order (reported)


@pytest.mark.parametrize("N", [8, 24])
def test_computational_derivatives(N):
    """d/dlon and d/dlat (the computational-plane derivatives the first
    configuration compares): exact on lat and lon at interior nodes (off
    the seam for lon), and equal to (R cos(lat) grad_lon, R grad_lat) of the
    physical gradient for any field."""
    R = 3.0
    m = oracle.Mesh(N, R=R)
    ins = np.ones(m.V, bool)
    ins[:m.nx[0]] = False
    ins[m.V - m.nx[-1]:] = False
    d = m.gradient_lonlat(m.lat.copy(), 1)[:, 0, :]
    assert np.abs(d[ins, 0]).max() <= 1e-12 and np.abs(d[ins, 1] - 1.0).max() <= 1e-12
    seam = np.zeros(m.V, bool)
    jump = np.abs(m.lon[m.edge[:, 0]] - m.lon[m.edge[:, 1]]) > np.pi
    seam[m.edge[jump, 0]] = seam[m.edge[jump, 1]] = True
    ok = ins & ~seam
    d = m.gradient_lonlat(m.lon.copy(), 1)[:, 0, :]
    assert np.abs(d[ok, 0] - 1.0).max() <= 1e-12 and np.abs(d[ok, 1]).max() <= 1e-12
    f = np.random.default_rng(N).standard_normal((m.V, 3))
    g = m.gradient(f, 3)
    c = m.gradient_lonlat(f, 3)
    want = np.stack([R * np.cos(m.lat)[:, None] * g[..., 0], R * g[..., 1]], axis=-1)
    assert np.abs(c - want).max() <= 1e-12 * np.abs(want).max()
