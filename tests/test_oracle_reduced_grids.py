"""Pins of the oracle on reduced Gaussian grids other than O<N> (CPU only):
the regular Gaussian grid F<N> (Section 4.2.3.6: nx = 4N on all 2N
parallels) and a hand-made reduced grid (Section 4.2.3.7: any points per
parallel).  The same mathematical pins as for O<N>: Euler counts and
orientation, edge multiplicity, dual cells tiling the (lon, lat) rectangle
and closing, every dual cell rebuilt as polygons by brute force, exact
operators on linear data, telescoping fluxes, the Galerkin identity."""
import numpy as np
import pytest

import oracle

EPS = np.finfo(np.float64).eps

GRIDS = {
    "F1": oracle.regular_gaussian_nx(1),
    "F2": oracle.regular_gaussian_nx(2),
    "F4": oracle.regular_gaussian_nx(4),
    "F16": oracle.regular_gaussian_nx(16),
    "R3": np.array([6, 9, 13, 13, 10, 8], np.int32),   # odd interior parallels
}


def _mesh(name, R=1.0):
    return oracle.Mesh(nx=GRIDS[name], R=R)


def _polar(m):
    p = np.zeros(m.V, bool)
    p[:m.nx[0]] = True
    p[m.V - m.nx[-1]:] = True
    return p


def _seam(m):
    bad = np.zeros(m.V, bool)
    jump = np.abs(m.lon[m.edge[:, 0]] - m.lon[m.edge[:, 1]]) > np.pi
    bad[m.edge[jump, 0]] = True
    bad[m.edge[jump, 1]] = True
    return bad


def _tri_coords(m):
    x = m.lon[m.tri].copy()
    y = m.lat[m.tri].copy()
    for c in (1, 2):
        x[:, c] = x[:, 0] + (x[:, c] - x[:, 0] + np.pi) % (2 * np.pi) - np.pi
    return x, y


def test_invalid_grids_are_refused():
    for nx in ([5, 8, 8, 6], [6, 8, 8], [6, 3, 8, 6]):   # odd polar, odd count, < 4
        with pytest.raises(ValueError):
            oracle.Mesh(nx=np.array(nx, np.int32))


@pytest.mark.parametrize("name", sorted(GRIDS))
def test_counts_orientation_and_edges(name):
    m = _mesh(name)
    np.testing.assert_array_equal(m.nx, GRIDS[name])
    V, cap = int(GRIDS[name].sum()), int(GRIDS[name][0] + GRIDS[name][-1])
    assert (m.V, m.F, m.E, m.npole) == (V, 2 * V - cap, 3 * V - cap, cap // 2)
    x, y = _tri_coords(m)
    area = 0.5 * ((x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0])
                  - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0]))
    assert area.min() > 0
    band = 2 * np.pi * (m.lat[0] - m.lat[-1])
    assert abs(area.sum() - band) < 1e-12 * band
    keys = np.sort(m.tri[:, [0, 1, 1, 2, 2, 0]].reshape(-1, 2), axis=1)
    uniq, cnt = np.unique(keys[:, 0].astype(np.int64) * m.V + keys[:, 1], return_counts=True)
    np.testing.assert_array_equal(uniq, m.edge[:, 0].astype(np.int64) * m.V + m.edge[:, 1])
    # edges along the two polar parallels border one triangle, all others two
    n0, nl = m.nx[0], m.nx[-1]
    e0, e1 = m.edge[:, 0], m.edge[:, 1]
    north = (e0 < n0) & (e1 < n0)
    south = (e0 >= m.V - nl) & (e1 >= m.V - nl)
    assert north.sum() == n0 and south.sum() == nl
    np.testing.assert_array_equal(cnt[north | south], 1)
    np.testing.assert_array_equal(cnt[~(north | south)], 2)


@pytest.mark.parametrize("name", sorted(GRIDS))
def test_dual_cells_tile_and_close(name):
    m = _mesh(name)
    assert abs(m.A.sum() - 2 * np.pi ** 2) < 1e-12
    acc = np.zeros((m.V, 2))
    np.add.at(acc, m.edge[:, 0], m.S)
    np.add.at(acc, m.edge[:, 1], -m.S)
    for k in range(m.npole):
        for n in m.pole_edge[k]:
            acc[n, 1] += m.pole_normal[k]
    assert np.abs(acc).max() <= 8 * EPS * np.pi
    # pole edges pair each polar node with the node half-way round, normals
    # +-(2 pi / nx of the polar parallel)
    n0, nl = m.nx[0], m.nx[-1]
    pe = m.pole_edge
    np.testing.assert_array_equal(pe[:n0 // 2, 1] - pe[:n0 // 2, 0], n0 // 2)
    np.testing.assert_array_equal(pe[n0 // 2:, 1] - pe[n0 // 2:, 0], nl // 2)
    np.testing.assert_allclose(m.pole_normal[:n0 // 2], 2 * np.pi / n0, rtol=1e-15)
    np.testing.assert_allclose(m.pole_normal[n0 // 2:], -2 * np.pi / nl, rtol=1e-15)


@pytest.mark.parametrize("name", ["F1", "F2", "F4", "R3"])
def test_bruteforce_dual_polygons(name):
    """Each dual cell as explicit polygons: one median sub-quad per triangle
    corner plus the polar rectangle of width 2 pi / nx up to the pole line."""
    m = _mesh(name)
    x, y = _tri_coords(m)
    area = np.zeros(m.V)
    normal = {}

    def add(key, vec):
        normal[key] = normal.get(key, np.zeros(2)) + vec

    def shoelace(px, py):
        return 0.5 * np.sum(px * np.roll(py, -1) - np.roll(px, -1) * py)

    for t in range(m.F):
        cx, cy = x[t].mean(), y[t].mean()
        for c in range(3):
            i, jn, jp = c, (c + 1) % 3, (c + 2) % 3
            mnx, mny = 0.5 * (x[t, i] + x[t, jn]), 0.5 * (y[t, i] + y[t, jn])
            mpx, mpy = 0.5 * (x[t, i] + x[t, jp]), 0.5 * (y[t, i] + y[t, jp])
            a = shoelace(np.array([x[t, i], mnx, cx, mpx]), np.array([y[t, i], mny, cy, mpy]))
            assert a > 0
            area[m.tri[t, i]] += a
            add((m.tri[t, i], m.tri[t, jn]), np.array([cy - mny, -(cx - mnx)]))
            add((m.tri[t, i], m.tri[t, jp]), np.array([mpy - cy, -(mpx - cx)]))
    for side, j in ((1.0, 0), (-1.0, m.nrings - 1)):
        o, n = m.ring_off[j], m.nx[j]
        th, pole = m.lat[o], side * np.pi / 2
        for i in range(n):
            lam = 2 * np.pi * i / n
            w, e = lam - np.pi / n, lam + np.pi / n
            area[o + i] += (e - w) * abs(pole - th)
            # east face (towards i+1) and west face (towards i-1), outward
            h = abs(pole - th)
            add((o + i, o + (i + 1) % n), np.array([h, 0.0]))
            add((o + i, o + (i - 1) % n), np.array([-h, 0.0]))
            add((o + i, "pole"), np.array([0.0, side * (e - w)]))
    np.testing.assert_allclose(area, m.A, rtol=1e-13, atol=0)
    for e, (a, b) in enumerate(m.edge):
        np.testing.assert_allclose(normal[(a, b)], m.S[e], rtol=0, atol=1e-14)
        np.testing.assert_allclose(normal[(b, a)], -m.S[e], rtol=0, atol=1e-14)
    for k, (a, b) in enumerate(m.pole_edge):
        for n in (a, b):
            np.testing.assert_allclose(normal[(n, "pole")], [0.0, m.pole_normal[k]],
                                       rtol=0, atol=1e-14)


@pytest.mark.parametrize("name", ["F4", "F16", "R3"])
def test_operators_exact_for_linear_data(name):
    m = _mesh(name)
    cos = np.cos(m.lat)
    inner = ~_polar(m)
    ok = inner & ~_seam(m)
    g = m.gradient(m.lat.copy())[:, 0, :]
    np.testing.assert_allclose(g[inner, 0], 0.0, atol=1e-12)
    np.testing.assert_allclose(g[inner, 1], 1.0, rtol=1e-12)
    g = m.gradient(m.lon.copy())[:, 0, :]
    np.testing.assert_allclose(g[ok, 0], 1.0 / cos[ok], rtol=1e-12)
    uv = np.zeros((m.V, 1, 2))
    uv[:, 0, 1] = m.lat / cos
    np.testing.assert_allclose(m.divergence(uv)[inner, 0], 1 / cos[inner], rtol=1e-12)
    uv = np.zeros((m.V, 1, 2))
    uv[:, 0, 0] = m.lat / cos
    np.testing.assert_allclose(m.curl(uv)[inner, 0], -1 / cos[inner], rtol=1e-12)
    # the polar nodes are not exact (their pole faces carry the pole value)
    g = m.gradient(m.lat.copy())[:, 0, :]
    assert np.abs(g[_polar(m), 1] - 1.0).min() > 1e-3


@pytest.mark.parametrize("name", ["F4", "F16", "R3"])
def test_fluxes_telescope(name):
    m = _mesh(name)
    rng = np.random.default_rng(9)
    uv = rng.standard_normal((m.V, 3, 2))
    s = np.zeros(m.V)
    np.add.at(s, m.edge[:, 0], np.abs(m.S).sum(1))
    np.add.at(s, m.edge[:, 1], np.abs(m.S).sum(1))
    scale = (s[:, None] * np.abs(uv).max(2)).sum()
    for op in (m.divergence, m.curl):
        tot = (m.vol[:, None] * op(uv, 3)).sum(0)
        assert np.all(np.abs(tot) <= 8 * EPS * scale)


@pytest.mark.parametrize("name", ["F2", "R3"])
def test_galerkin_identity_bruteforce(name):
    m = _mesh(name)
    rng = np.random.default_rng(12)
    f = rng.standard_normal(m.V)
    x, y = _tri_coords(m)
    acc = np.zeros((m.V, 2))
    for t in range(m.F):
        M = np.array([[x[t, 1] - x[t, 0], y[t, 1] - y[t, 0]],
                      [x[t, 2] - x[t, 0], y[t, 2] - y[t, 0]]])
        rhs = np.array([f[m.tri[t, 1]] - f[m.tri[t, 0]], f[m.tri[t, 2]] - f[m.tri[t, 0]]])
        grad = np.linalg.solve(M, rhs)
        for c in range(3):
            acc[m.tri[t, c]] += 0.5 * np.linalg.det(M) / 3 * grad
    g = m.gradient(f)[:, 0, :]
    G = np.stack([g[:, 0] * np.cos(m.lat) * m.A, g[:, 1] * m.A], axis=1)
    inner = ~_polar(m)
    np.testing.assert_allclose(G[inner], acc[inner], rtol=0, atol=1e-13 * np.abs(f).max())
