"""Pins of the oracle on meshes with quadrilateral elements and on the
regular longitude-latitude grids (CPU only).

Section 4.3: for regular grids the mesh elements are a blocked arrangement
of quadrilaterals, and a mesh can hold several element types, stored one
block per type (Figure 27).  Section 4.2.3.8: the regular longitude-latitude
grids; the variants without points on the poles (latitude-shifted SLAT and
shifted S) carry the same polar closure as the Gaussian grids.  The oracle
meshes every strip between parallels of equal counts with quadrilaterals
when asked (all strips of a regular grid, the equator strip of O<N>) and
builds their median-dual cells about the element centres.

Pins: Euler counts, element orientation, edge multiplicity, dual cells
tiling the (lon, lat) rectangle and closing, every dual cell rebuilt by
brute force as polygons (element corners, polar rectangles, longitudes of
the nodes themselves so shifted grids are covered), exact gradient and
divergence on linear data at interior nodes, telescoping fluxes, and
second-order convergence to the analytic derivatives away from the poles."""
import numpy as np
import pytest

import oracle
import synthetic as sy

EPS = np.finfo(np.float64).eps


def _lonlat(nlon, nlat, shift=False, R=1.0):
    nx, lat = oracle.shifted_lonlat(nlon, nlat)
    return oracle.Mesh(nx=nx, lat=lat, shift=shift, quads=True, R=R)


MESHES = {
    "SLAT8x4": lambda: _lonlat(8, 4),
    "SLAT16x8": lambda: _lonlat(16, 8),
    "S16x8": lambda: _lonlat(16, 8, shift=True),
    "S12x7": lambda: _lonlat(12, 7, shift=True),            # odd count of parallels
    "O4q": lambda: oracle.Mesh(4, quads=True),               # triangles + one quad strip
    "F3q": lambda: oracle.Mesh(nx=oracle.regular_gaussian_nx(3), quads=True),
}


def _unwrapped(m, elems):
    x = m.lon[elems].copy()
    y = m.lat[elems].copy()
    for c in range(1, elems.shape[1]):
        x[:, c] = x[:, 0] + (x[:, c] - x[:, 0] + np.pi) % (2 * np.pi) - np.pi
    return x, y


def _shoelace(px, py):
    return 0.5 * np.sum(px * np.roll(py, -1, axis=-1) - np.roll(px, -1, axis=-1) * py, axis=-1)


@pytest.mark.parametrize("name", sorted(MESHES))
def test_counts_orientation_and_edges(name):
    m = MESHES[name]()
    nx = m.nx
    eq = nx[:-1] == nx[1:]
    assert m.Q == int(nx[:-1][eq].sum())
    assert m.F == int((nx[:-1] + nx[1:])[~eq].sum())
    assert m.V == int(nx.sum())
    # Euler for the sphere with the two polar caps removed: V - E + F = 0
    assert m.V - m.E + m.F + m.Q == 0
    for el in (m.tri, m.quad):
        if len(el):
            x, y = _unwrapped(m, el)
            assert np.all(_shoelace(x, y) > 0)
    # every edge lies in two elements, except the sides along the polar
    # parallels (one element each)
    count = {}
    for el in (m.tri, m.quad):
        k = el.shape[1] if len(el) else 0
        for c in range(k):
            a, b = el[:, c], el[:, (c + 1) % k]
            for p, q in zip(np.minimum(a, b), np.maximum(a, b)):
                count[(p, q)] = count.get((p, q), 0) + 1
    edges = {tuple(e) for e in m.edge}
    assert edges == set(count)
    polar = set(range(m.nx[0])) | set(range(m.V - m.nx[-1], m.V))
    for (p, q), c in count.items():
        on_polar_parallel = (p in polar and q in polar and
                             (p < m.nx[0]) == (q < m.nx[0]))
        assert c == (1 if on_polar_parallel else 2), (p, q, c)


@pytest.mark.parametrize("name", sorted(MESHES))
def test_dual_cells_tile_the_rectangle_and_close(name):
    m = MESHES[name]()
    assert abs(m.A.sum() - 2 * np.pi ** 2) <= 64 * EPS * 2 * np.pi ** 2
    acc = np.zeros((m.V, 2))
    for e, (a, b) in enumerate(m.edge):
        acc[a] += m.S[e]
        acc[b] -= m.S[e]
    for k, (a, b) in enumerate(m.pole_edge):
        acc[a, 1] += m.pole_normal[k]
        acc[b, 1] += m.pole_normal[k]
    assert np.abs(acc).max() <= 16 * EPS * np.pi


@pytest.mark.parametrize("name", sorted(MESHES))
def test_bruteforce_dual_polygons(name):
    """Every dual cell as explicit counter-clockwise polygons: one per
    element corner (corner, midpoint of the next side, element centre,
    midpoint of the previous side; centre = mean of the corners) and the
    polar rectangle; shoelace areas and outward face normals against the
    oracle."""
    m = MESHES[name]()
    area = np.zeros(m.V)
    normal = {}

    def add(key, vec):
        normal[key] = normal.get(key, np.zeros(2)) + vec

    for el in (m.tri, m.quad):
        if not len(el):
            continue
        k = el.shape[1]
        x, y = _unwrapped(m, el)
        cx, cy = x.mean(axis=1), y.mean(axis=1)
        for t in range(len(el)):
            for c in range(k):
                cn, cp = (c + 1) % k, (c - 1) % k
                mnx, mny = 0.5 * (x[t, c] + x[t, cn]), 0.5 * (y[t, c] + y[t, cn])
                mpx, mpy = 0.5 * (x[t, c] + x[t, cp]), 0.5 * (y[t, c] + y[t, cp])
                a = _shoelace(np.array([x[t, c], mnx, cx[t], mpx]),
                              np.array([y[t, c], mny, cy[t], mpy]))
                assert a > 0
                area[el[t, c]] += a
                d1 = np.array([cx[t] - mnx, cy[t] - mny])
                d2 = np.array([mpx - cx[t], mpy - cy[t]])
                add((el[t, c], el[t, cn]), np.array([d1[1], -d1[0]]))
                add((el[t, c], el[t, cp]), np.array([d2[1], -d2[0]]))
    for side, j in ((1.0, 0), (-1.0, m.nrings - 1)):
        o, n = m.ring_off[j], m.nx[j]
        th = m.lat[o]
        pole = side * np.pi / 2
        for i in range(n):
            lam = m.lon[o + i]
            mw, me = lam - np.pi / n, lam + np.pi / n
            if side > 0:
                px, py = np.array([mw, me, me, mw]), np.array([th, th, pole, pole])
            else:
                px, py = np.array([me, mw, mw, me]), np.array([th, th, pole, pole])
            area[o + i] += _shoelace(px, py)
            for s in range(4):
                d = np.array([px[(s + 1) % 4] - px[s], py[(s + 1) % 4] - py[s]])
                nv = np.array([d[1], -d[0]])
                if abs(py[s] - th) < 1e-15 and abs(py[(s + 1) % 4] - th) < 1e-15:
                    continue
                if abs(py[s] - pole) < 1e-15 and abs(py[(s + 1) % 4] - pole) < 1e-15:
                    add((o + i, "pole"), nv)
                else:
                    east = max(px[s], px[(s + 1) % 4]) > lam
                    nb = o + ((i + 1) % n if east else (i - 1) % n)
                    add((o + i, nb), nv)
    np.testing.assert_allclose(area, m.A, rtol=1e-13, atol=0)
    for e, (a, b) in enumerate(m.edge):
        np.testing.assert_allclose(normal[(a, b)], m.S[e], rtol=0, atol=1e-14)
        np.testing.assert_allclose(normal[(b, a)], -m.S[e], rtol=0, atol=1e-14)
    for k, (a, b) in enumerate(m.pole_edge):
        for n in (a, b):
            np.testing.assert_allclose(normal[(n, "pole")], [0.0, m.pole_normal[k]],
                                       rtol=0, atol=1e-14)


def _interior(m):
    ok = np.ones(m.V, bool)
    ok[:m.nx[0]] = False
    ok[m.V - m.nx[-1]:] = False
    return ok


def _off_seam(m):
    ok = np.ones(m.V, bool)
    jump = np.abs(m.lon[m.edge[:, 0]] - m.lon[m.edge[:, 1]]) > np.pi
    ok[m.edge[jump, 0]] = False
    ok[m.edge[jump, 1]] = False
    return ok


@pytest.mark.parametrize("name", sorted(MESHES))
def test_exact_on_linear_data(name):
    """lat and lon are linear in the computational plane: at interior
    nodes (off the lon 0 / 2 pi seam for lon) the gradient is exactly
    (0, 1/R) and (1/(R cos lat), 0), and the divergence of (0, lat/cos lat)
    is 1/(R cos lat), to rounding."""
    R = 2.5
    m = MESHES[name]()
    m = oracle.Mesh(nx=m.nx, lat=m.lat[m.ring_off[:-1]], shift=bool(m.lon[0] != 0.0),
                    quads=True, R=R)
    ins = _interior(m)
    g = m.gradient(m.lat.copy(), 1)[:, 0, :]
    assert np.abs(g[ins, 0]).max() <= 1e-12
    assert np.abs(g[ins, 1] - 1.0 / R).max() <= 1e-12
    ok = ins & _off_seam(m)
    g = m.gradient(m.lon.copy(), 1)[:, 0, :]
    assert np.abs(g[ok, 0] * R * np.cos(m.lat[ok]) - 1.0).max() <= 1e-12
    assert np.abs(g[ok, 1]).max() <= 1e-12
    uv = np.zeros((m.V, 1, 2))
    uv[:, 0, 1] = m.lat / np.cos(m.lat)
    d = m.divergence(uv, 1)[:, 0]
    assert np.abs(d[ins] * R * np.cos(m.lat[ins]) - 1.0).max() <= 1e-12


@pytest.mark.parametrize("name", sorted(MESHES))
def test_divergence_and_curl_telescope(name):
    m = MESHES[name]()
    rng = np.random.default_rng(3)
    uv = rng.standard_normal((m.V, 3, 2))
    for fn in (m.divergence, m.curl):
        out = fn(uv, 3)
        tot = (m.vol[:, None] * out).sum(axis=0)
        scale = (m.vol[:, None] * np.abs(out)).sum(axis=0)
        assert np.all(np.abs(tot) <= 1e-13 * scale)


def _errors(m, co):
    band = np.abs(m.lat) <= np.pi / 3
    w = m.vol[band]
    f = sy.synthesize(m.lon, m.lat, co)[0]
    g = m.gradient(f, 1)[:, 0, :]
    ga = sy.synthesize_gradient(m.lon, m.lat, co)[0]
    lap = m.laplacian(f, 1)[:, 0]
    la = sy.synthesize(m.lon, m.lat, sy.laplacian_coeffs(co))[0]
    eg = np.sqrt((w[:, None] * (g[band] - ga[band]) ** 2).sum() / w.sum())
    el = np.sqrt((w * (lap[band] - la[band]) ** 2).sum() / w.sum())
    return eg, el


@pytest.mark.parametrize("shift", [False, True])
def test_second_order_on_lonlat_quads(shift):
    """Random harmonics of degree <= 4 on SLAT / S grids of 32x16 .. 256x128:
    gradient and Laplacian RMS errors against the analytic derivatives over
    |lat| <= 60 deg fall at second order."""
    co = sy.random_coeffs(4, [sy.seed_rng(77, 0, 0)])
    errs = [_errors(_lonlat(4 * n, 2 * n, shift=shift), co) for n in (8, 16, 32, 64)]
    eg = np.array([e[0] for e in errs])
    el = np.array([e[1] for e in errs])
    og = np.log2(eg[:-1] / eg[1:])
    ol = np.log2(el[:-1] / el[1:])
    assert og[-1] >= 1.8, og
    assert ol[-1] >= 1.8, ol


def test_remap_refuses_quadrilateral_meshes():
    m = _lonlat(16, 8)
    with pytest.raises(ValueError):
        m.remap_weights(np.array([0.1]), np.array([0.1]))
