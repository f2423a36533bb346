"""Pins of the oracle's remap (CPU only).

Section 1 lists remapping or interpolation of fields between different
grids among the library's mathematical operations and gives no method.  The
reading implemented: the piecewise-linear (P1) interpolant of the nodal
values on the source mesh's triangles, in the (lon, lat) plane; targets
poleward of a polar parallel take the linear interpolant along that
parallel.  The pins: brute-force point location over every triangle on tiny
meshes, exact reproduction of the nodal values (identity), of constants and
of fields linear in (lon, lat), the closed form at edge midpoints, the polar
rule, second-order convergence on smooth fields, and level independence.
"""
import numpy as np
import pytest

import oracle
import synthetic as sy

EPS = np.finfo(np.float64).eps


def _random_points(n, seed, lat_max=np.pi / 2):
    rng = np.random.default_rng(seed)
    lon = rng.uniform(0.0, 2 * np.pi, n)
    lat = np.arcsin(rng.uniform(-np.sin(lat_max), np.sin(lat_max), n))
    return lon, lat


def _band(m, lat):
    return (lat <= m.lat[0]) & (lat >= m.lat[-1])


@pytest.mark.parametrize("N", [1, 2, 4, 16, 48])
def test_identity_on_own_nodes(N):
    m = oracle.Mesh(N)
    idx, w = m.remap_weights(m.lon, m.lat)
    k = np.argmax(w, axis=1)
    assert np.all(idx[np.arange(m.V), k] == np.arange(m.V))
    assert np.all(w[np.arange(m.V), k] == 1.0)
    assert np.all(np.sort(w, axis=1)[:, :2] == 0.0)
    x = np.random.default_rng(N).standard_normal((m.V, 3))
    assert np.array_equal(m.remap(x, 3, m.lon, m.lat), x)


def _brute_force(m, lon, lat):
    """Every triangle of the mesh that contains (lon, lat), with its
    barycentric weights: the triangle is unwrapped whole (its vertices
    within pi of its first vertex, shifted by 2 pi so that the first is
    within pi of the target), weights from the areas of the sub-triangles."""
    P = np.stack([m.lon[m.tri], m.lat[m.tri]], axis=-1)           # [F, 3, 2]
    x0 = P[:, 0, 0]
    for k in (1, 2):
        d = P[:, k, 0] - x0
        P[:, k, 0] -= 2 * np.pi * np.round(d / (2 * np.pi))
    shift = 2 * np.pi * np.round((lon - x0) / (2 * np.pi))
    P[:, :, 0] += shift[:, None]

    def area(a, b, c):
        return (b[..., 0] - a[..., 0]) * (c[..., 1] - a[..., 1]) - \
               (b[..., 1] - a[..., 1]) * (c[..., 0] - a[..., 0])
    t = np.broadcast_to(np.array([lon, lat]), P[:, 0].shape)
    whole = area(P[:, 0], P[:, 1], P[:, 2])
    w = np.stack([area(t, P[:, 1], P[:, 2]), area(P[:, 0], t, P[:, 2]),
                  area(P[:, 0], P[:, 1], t)], axis=1) / whole[:, None]
    inside = np.where(w.min(axis=1) >= -1e-12)[0]
    return [(m.tri[f], w[f]) for f in inside]


@pytest.mark.parametrize("N", [1, 2, 4])
def test_location_and_weights_match_brute_force(N):
    m = oracle.Mesh(N)
    lon, lat = _random_points(400, 10 + N)
    inband = _band(m, lat)
    idx, w = m.remap_weights(lon, lat)
    x = np.random.default_rng(N).standard_normal(m.V)
    got = m.remap(x, 1, lon, lat)[:, 0]
    checked = 0
    for t in np.where(inband)[0]:
        cands = _brute_force(m, lon[t], lat[t])
        assert cands, "a point of the band lies in no triangle"
        ok = False
        for verts, wb in cands:
            if set(verts.tolist()) == set(idx[t].tolist()):
                order = [list(verts).index(v) for v in idx[t]]
                assert np.allclose(w[t], wb[order], rtol=0, atol=1e-14)
                ok = True
        assert ok, (t, idx[t], [c[0] for c in cands])
        ref = float(np.dot(cands[0][1], x[cands[0][0]]))
        assert abs(got[t] - ref) <= 1e-14 * np.abs(x).max()
        checked += 1
    assert checked > 100


@pytest.mark.parametrize("N", [2, 16, 80])
def test_constants_and_weight_sums(N):
    m = oracle.Mesh(N)
    lon, lat = _random_points(5000, N)
    idx, w = m.remap_weights(lon, lat)
    assert np.all(np.abs(w.sum(axis=1) - 1.0) <= 8 * EPS)
    assert np.all(w >= -8 * EPS)
    out = m.remap(np.full((m.V, 2), 7.25), 2, lon, lat)
    assert np.all(np.abs(out - 7.25) <= 16 * EPS * 7.25)


@pytest.mark.parametrize("N", [4, 16, 64])
def test_linear_fields_reproduced(N):
    """f = a + b lon + c lat is reproduced at every target of the band whose
    triangle does not straddle lon = 0 (the nodal lon jumps there); in the
    polar caps f = a + c lat takes the value at the polar parallel."""
    m = oracle.Mesh(N)
    lon, lat = _random_points(20000, 3 * N)
    margin = 2 * np.pi / 20 + 1e-9  # one polar-ring cell, the widest
    f = 1.5 + 0.75 * m.lon - 2.0 * m.lat
    got = m.remap(f, 1, lon, lat)[:, 0]
    inb = _band(m, lat) & (lon > margin) & (lon < 2 * np.pi - margin)
    want = 1.5 + 0.75 * lon - 2.0 * lat
    assert np.all(np.abs(got - want)[inb] <= 64 * EPS * (1.5 + 0.75 * 2 * np.pi + 2 * np.pi))
    g = 1.5 - 2.0 * m.lat
    got = m.remap(g, 1, lon, lat)[:, 0]
    north, south = lat > m.lat[0], lat < m.lat[-1]
    assert np.all(np.abs(got[north] - (1.5 - 2.0 * m.lat[0])) <= 16 * EPS * 5)
    assert np.all(np.abs(got[south] - (1.5 - 2.0 * m.lat[-1])) <= 16 * EPS * 5)
    inb = _band(m, lat)
    assert np.all(np.abs(got[inb] - (1.5 - 2.0 * lat[inb])) <= 64 * EPS * 5)


@pytest.mark.parametrize("N", [2, 8])
def test_edge_midpoints_average_the_endpoints(N):
    m = oracle.Mesh(N)
    a, b = m.edge[:, 0], m.edge[:, 1]
    lb = m.lon[b] - 2 * np.pi * np.round((m.lon[b] - m.lon[a]) / (2 * np.pi))
    lon = np.mod(0.5 * (m.lon[a] + lb), 2 * np.pi)
    lat = 0.5 * (m.lat[a] + m.lat[b])
    x = np.random.default_rng(1).standard_normal(m.V)
    got = m.remap(x, 1, lon, lat)[:, 0]
    want = 0.5 * (x[a] + x[b])
    assert np.all(np.abs(got - want) <= 32 * EPS * np.abs(x).max())


def test_polar_caps_interpolate_along_the_polar_parallel():
    m = oracle.Mesh(8)
    nx0 = m.nx[0]
    i = np.arange(nx0)
    for lat in (m.lat[0] + 1e-3, 0.5 * np.pi, m.lat[-1] - 1e-3, -0.5 * np.pi):
        off = 0 if lat > 0 else m.ring_off[-2]
        lon_nodes = 2 * np.pi * i / nx0
        idx, w = m.remap_weights(lon_nodes, np.full(nx0, lat))
        k = np.argmax(w, axis=1)
        assert np.all(w[i, k] == 1.0) and np.all(idx[i, k] == off + i)
        mid = 2 * np.pi * (i + 0.25) / nx0
        x = np.random.default_rng(2).standard_normal(m.V)
        got = m.remap(x, 1, mid, np.full(nx0, lat))[:, 0]
        want = 0.75 * x[off + i] + 0.25 * x[off + (i + 1) % nx0]
        assert np.all(np.abs(got - want) <= 8 * EPS * np.abs(x).max())


def test_second_order_convergence_on_smooth_fields():
    """Interpolation error of a degree-4 harmonic field at random points
    with |lat| <= 60 degrees falls by ~4x per halving of the mesh spacing."""
    co = sy.random_coeffs(4, [sy.seed_rng(77, 0, 0)])
    lon, lat = _random_points(4000, 5, lat_max=np.pi / 3)
    exact = sy.synthesize(lon, lat, co)[0]
    errs = []
    for N in (16, 32, 64, 128):
        m = oracle.Mesh(N)
        f = sy.synthesize(m.lon, m.lat, co)[0]
        got = m.remap(f, 1, lon, lat)[:, 0]
        errs.append(np.sqrt(np.mean((got - exact) ** 2)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.8), (errs, orders)


def test_levels_are_independent_and_ordered():
    m = oracle.Mesh(8)
    lon, lat = _random_points(300, 9)
    x = np.random.default_rng(3).standard_normal((m.V, 5, 2))
    full = m.remap(x, 10, lon, lat).reshape(-1, 5, 2)
    for k in range(5):
        for c in range(2):
            one = m.remap(np.ascontiguousarray(x[:, k, c]), 1, lon, lat)[:, 0]
            assert np.array_equal(full[:, k, c], one)


def test_rejects_latitudes_off_the_sphere():
    m = oracle.Mesh(2)
    with pytest.raises(ValueError):
        m.remap_weights([0.0], [2.0])
    with pytest.raises(ValueError):
        m.remap_weights([np.nan], [0.0])
