"""Pins of the oracle's triangulation and median-dual geometry (CPU only).

The mesh (Section 4.3, Eq. 1) triangulates the band between the first and
last parallel; the geometry is the median dual in the (lon, lat) plane with
cells of the polar parallels closed up to the pole line.  The brute-force
test below rebuilds every dual cell as a polygon, independently of the
oracle's edge loop, and compares areas and face normals.
"""
import numpy as np
import pytest

import oracle


def _unwrap(x, ref):
    return ref + (x - ref + np.pi) % (2 * np.pi) - np.pi


def _tri_coords(m):
    P = m.tri
    x = m.lon[P].copy()
    y = m.lat[P].copy()
    x[:, 1] = _unwrap(x[:, 1], x[:, 0])
    x[:, 2] = _unwrap(x[:, 2], x[:, 0])
    return x, y


@pytest.mark.parametrize("N", [1, 2, 3, 8, 16, 48])
def test_euler_counts_and_orientation(N):
    m = oracle.Mesh(N)
    V = 4 * N * N + 36 * N
    assert (m.V, m.F, m.E) == (V, 2 * V - 40, 3 * V - 40)
    assert m.V - m.E + m.F == 0  # sphere minus two polar caps
    x, y = _tri_coords(m)
    area = 0.5 * ((x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0])
                  - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0]))
    assert area.min() > 0, "every triangle counter-clockwise, non-degenerate"
    band = 2 * np.pi * (m.lat[0] - m.lat[-1])
    assert abs(area.sum() - band) < 1e-12 * band


@pytest.mark.parametrize("N", [1, 2, 8, 16])
def test_edge_multiplicity(N):
    m = oracle.Mesh(N)
    keys = np.sort(m.tri[:, [0, 1, 1, 2, 2, 0]].reshape(-1, 2), axis=1)
    uniq, cnt = np.unique(keys[:, 0].astype(np.int64) * m.V + keys[:, 1], return_counts=True)
    ek = m.edge[:, 0].astype(np.int64) * m.V + m.edge[:, 1]
    np.testing.assert_array_equal(uniq, ek)  # sorted, unique, a < b
    assert np.all(m.edge[:, 0] < m.edge[:, 1])
    polar = np.zeros(m.V, bool)
    polar[:20] = True
    polar[-20:] = True
    ring_edge = polar[m.edge[:, 0]] & polar[m.edge[:, 1]] & (
        (m.edge[:, 0] < 20) == (m.edge[:, 1] < 20))
    assert ring_edge.sum() == 40
    np.testing.assert_array_equal(cnt[ring_edge], 1)
    np.testing.assert_array_equal(cnt[~ring_edge], 2)
    # every node connects to its two neighbours on its own parallel
    for j in range(m.nrings):
        o, n = m.ring_off[j], m.nx[j]
        for i in range(n):
            a, b = sorted((o + i, o + (i + 1) % n))
            assert np.any((m.edge[:, 0] == a) & (m.edge[:, 1] == b))


@pytest.mark.parametrize("N", [1, 2, 16, 160])
def test_dual_area_sum_and_closure(N):
    m = oracle.Mesh(N)
    # the dual cells tile the whole (lon, lat) rectangle [0, 2pi] x [-pi/2, pi/2]
    assert abs(m.A.sum() - 2 * np.pi ** 2) < 1e-12
    assert m.A.min() > 0
    # every cell is closed: sum of its outward face normals is zero
    acc = np.zeros((m.V, 2))
    np.add.at(acc, m.edge[:, 0], m.S)
    np.add.at(acc, m.edge[:, 1], -m.S)
    for k in range(m.npole):
        for n in m.pole_edge[k]:
            acc[n, 1] += m.pole_normal[k]
    # the normals are differences of coordinates of size ~pi, so their
    # rounding is absolute: a few ulps of pi
    assert np.abs(acc).max() <= 8 * np.finfo(np.float64).eps * np.pi


@pytest.mark.parametrize("N", [1, 2, 4, 8])
def test_bruteforce_dual_polygons(N):
    """Rebuild every median-dual cell as explicit counter-clockwise
    polygons (one sub-quad per triangle corner plus the polar rectangle)
    and compare shoelace areas and outward face normals with the oracle."""
    m = oracle.Mesh(N)
    x, y = _tri_coords(m)
    area = np.zeros(m.V)
    normal = {}  # (node, neighbour or 'pole') -> outward normal of that face

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
            qx = np.array([x[t, i], mnx, cx, mpx])
            qy = np.array([y[t, i], mny, cy, mpy])
            a = shoelace(qx, qy)
            assert a > 0
            area[m.tri[t, i]] += a
            # travelling counter-clockwise, the outward normal of a segment
            # d is (d_y, -d_x)
            d1 = np.array([cx - mnx, cy - mny])
            d2 = np.array([mpx - cx, mpy - cy])
            add((m.tri[t, i], m.tri[t, jn]), np.array([d1[1], -d1[0]]))
            add((m.tri[t, i], m.tri[t, jp]), np.array([d2[1], -d2[0]]))
    for side, j in ((1.0, 0), (-1.0, m.nrings - 1)):
        o, n = m.ring_off[j], m.nx[j]
        th = m.lat[o]
        pole = side * np.pi / 2
        for i in range(n):
            lam = 2 * np.pi * i / n
            mw, me = lam - np.pi / n, lam + np.pi / n
            if side > 0:
                px = np.array([mw, me, me, mw]); py = np.array([th, th, pole, pole])
            else:
                px = np.array([me, mw, mw, me]); py = np.array([th, th, pole, pole])
            a = shoelace(px, py)
            assert a > 0
            area[o + i] += a
            for s in range(4):
                d = np.array([px[(s + 1) % 4] - px[s], py[(s + 1) % 4] - py[s]])
                nv = np.array([d[1], -d[0]])
                if abs(py[s] - th) < 1e-15 and abs(py[(s + 1) % 4] - th) < 1e-15:
                    continue  # along the parallel: inside the node's own cell
                if abs(py[s] - pole) < 1e-15 and abs(py[(s + 1) % 4] - pole) < 1e-15:
                    add((o + i, "pole"), nv)
                else:  # vertical side: east side faces i+1, west side i-1
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
    # pole edges pair each polar node with the node half-way round
    pe = m.pole_edge
    assert pe.shape == (20, 2)
    np.testing.assert_array_equal(pe[:10, 1] - pe[:10, 0], 10)
    np.testing.assert_array_equal(pe[10:, 1] - pe[10:, 0], 10)
    np.testing.assert_allclose(m.pole_normal[:10], 2 * np.pi / 20)
    np.testing.assert_allclose(m.pole_normal[10:], -2 * np.pi / 20)


@pytest.mark.parametrize("N", [16, 320])
def test_volumes_converge_to_sphere_area(N):
    m = oracle.Mesh(N)
    total = m.vol.sum()
    assert abs(total - 4 * np.pi) < 40.0 / N ** 2
