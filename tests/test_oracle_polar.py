"""Pins of the oracle's gradient at the nodes of the two polar parallels.

The dual cells of the first and last parallel reach the pole line, and the
face they have there is the only part of the gradient that the interior
pins (Galerkin identity, exactness for linear data) do not reach.  The
reading of Section 4.7 taken for that face: its value is the pole value
estimated by linear interpolation, along the meridian through the pole,
between the node and the node half-way round its parallel.  Both sit at
the same distance from the pole, so the estimate is the mean of the two.

What pins it here, without restating it:
  * the polar cells are rebuilt by brute force (sub-quads of the incident
    triangles plus the rectangle up to the pole line; their face normals
    are pinned against the oracle's in test_oracle_mesh), the face sum of
    the mesh edges is formed from those polygons, and the pole-face value
    the oracle used is recovered from its output as
        P_i = (G_lat,i R A_i - face sum_i) / (normal of the pole face);
  * P_i must equal the analytic pole value exactly (to rounding) for every
    field of harmonics of odd order m, which vanish at the pole and change
    sign half-way round a parallel;
  * P_i must equal the node value for fields of even order only;
  * for general fields P_i must converge to the analytic pole value at
    second order in the polar distance (the one-sided node value, the
    other natural choice, converges at first order, and the test checks
    that it would fail);
  * the zonal component of a polar node carries no pole-face term.
"""
import numpy as np
import pytest

import oracle
import synthetic as sy


def _unwrap(x, ref):
    return ref + (x - ref + np.pi) % (2 * np.pi) - np.pi


def _polar_face_normals(m):
    """Outward face normals of the dual cells of the polar nodes, keyed by
    (node, neighbour), built from the triangles touching a polar parallel
    and the rectangle between the parallel and the pole line."""
    o_s = m.ring_off[m.nrings - 1]
    polar = np.zeros(m.V, bool)
    polar[:m.nx[0]] = True
    polar[o_s:] = True
    touch = polar[m.tri].any(axis=1)
    normal = {}

    def add(key, vec):
        normal[key] = normal.get(key, np.zeros(2)) + vec

    for t in np.nonzero(touch)[0]:
        ids = m.tri[t]
        x = m.lon[ids].copy()
        y = m.lat[ids].copy()
        x[1] = _unwrap(x[1], x[0])
        x[2] = _unwrap(x[2], x[0])
        cx, cy = x.mean(), y.mean()
        for c in range(3):
            if not polar[ids[c]]:
                continue
            jn, jp = (c + 1) % 3, (c + 2) % 3
            mn = np.array([0.5 * (x[c] + x[jn]), 0.5 * (y[c] + y[jn])])
            mp = np.array([0.5 * (x[c] + x[jp]), 0.5 * (y[c] + y[jp])])
            d1 = np.array([cx, cy]) - mn       # counter-clockwise: mn -> c -> mp
            d2 = mp - np.array([cx, cy])
            add((ids[c], ids[jn]), np.array([d1[1], -d1[0]]))
            add((ids[c], ids[jp]), np.array([d2[1], -d2[0]]))
    for side, j in ((1.0, 0), (-1.0, m.nrings - 1)):
        o, n = m.ring_off[j], m.nx[j]
        ext = np.pi / 2 - abs(m.lat[o])
        for i in range(n):
            # vertical sides of the rectangle [lon -/+ pi/n] x [lat0, pole]:
            # the east side faces i+1, the west side i-1
            add((o + i, o + (i + 1) % n), np.array([ext, 0.0]))
            add((o + i, o + (i - 1) % n), np.array([-ext, 0.0]))
            add((o + i, "pole"), np.array([0.0, side * 2 * np.pi / n]))
    return normal, polar


def _recover(m, f):
    """Face sums over the mesh edges, and the pole-face value the oracle
    used, at every polar node."""
    normal, polar = _polar_face_normals(m)
    nodes = np.nonzero(polar)[0]
    g = m.gradient_at(f, 1, nodes)[:, 0, :]
    out = []
    for s, i in enumerate(nodes):
        face = np.zeros(2)
        for key, nv in normal.items():
            if key[0] == i and key[1] != "pole":
                face += nv * 0.5 * (f[i] + f[key[1]])
        cell = np.array([g[s, 0] * m.R * np.cos(m.lat[i]) * m.A[i], g[s, 1] * m.R * m.A[i]])
        pole_n = normal[(i, "pole")][1]
        out.append((i, cell, face, (cell[1] - face[1]) / pole_n))
    return out


def _partner(m):
    p = np.full(m.V, -1)
    for a, b in m.pole_edge:
        p[a], p[b] = b, a
    return p


def _coeffs_by_order(lmax, seed, parity):
    co = sy.random_coeffs(lmax, [sy.seed_rng(30, seed, 0)])
    mm = np.arange(lmax + 1)
    keep = (mm % 2 == 1) if parity == "odd" else (mm % 2 == 0)
    return sy.SHCoeffs(co.c * keep[None, None, :], co.s * keep[None, None, :])


@pytest.mark.parametrize("N,R", [(1, 1.0), (2, 1.0), (8, 2.5), (16, 1.0)])
def test_zonal_component_has_no_pole_term(N, R):
    m = oracle.Mesh(N, R)
    f = np.random.default_rng(40 + N).standard_normal(m.V)
    for i, cell, face, _ in _recover(m, f):
        scale = np.abs(f).max() * 8 * np.pi
        assert abs(cell[0] - face[0]) <= 1e-14 * scale, i


@pytest.mark.parametrize("N", [2, 8, 16, 48])
def test_pole_face_exact_for_fields_vanishing_at_the_pole(N):
    """Harmonics of odd order m vanish at the pole and change sign half-way
    round a parallel: the pole face must carry exactly zero."""
    m = oracle.Mesh(N)
    co = _coeffs_by_order(6, N, "odd")
    f = sy.synthesize(m.lon, m.lat, co)[0]
    scale = np.abs(f).max()
    at_pole = sy.synthesize(np.zeros(2), np.array([np.pi / 2, -np.pi / 2]), co)[0]
    assert np.abs(at_pole).max() <= 1e-14 * scale
    P = np.array([r[3] for r in _recover(m, f)])
    assert np.abs(P).max() <= 1e-12 * scale, np.abs(P).max()


@pytest.mark.parametrize("N", [2, 8, 16])
def test_pole_face_equals_node_value_for_even_orders(N):
    """Even orders repeat half-way round a parallel, so the node and its
    partner agree and the pole face carries the node's own value (neither
    zero nor its negative: the face is present, with the right sign)."""
    m = oracle.Mesh(N)
    co = _coeffs_by_order(6, 100 + N, "even")
    f = sy.synthesize(m.lon, m.lat, co)[0]
    scale = np.abs(f).max()
    for i, _, _, P in _recover(m, f):
        assert abs(P - f[i]) <= 1e-12 * scale, (i, P, f[i])
    assert max(abs(f[i]) for i, *_ in _recover(m, f)) > 0.1 * scale


def test_pole_face_converges_to_the_pole_value_at_second_order():
    """General fields (degree <= 8, all orders): the recovered pole-face
    value tends to the field's value at the pole at second order in the
    polar distance; the node's own value, the one-sided alternative, only
    at first order."""
    co = sy.random_coeffs(8, [sy.seed_rng(31, 0, 0)])
    at_pole = sy.synthesize(np.zeros(2), np.array([np.pi / 2, -np.pi / 2]), co)[0]
    rows = []
    for N in (16, 32, 64, 128):
        m = oracle.Mesh(N)
        f = sy.synthesize(m.lon, m.lat, co)[0]
        rec = _recover(m, f)
        e_face = max(abs(P - (at_pole[0] if i < m.nx[0] else at_pole[1]))
                     for i, _, _, P in rec)
        e_node = max(abs(f[i] - (at_pole[0] if i < m.nx[0] else at_pole[1]))
                     for i, *_ in rec)
        rows.append((np.pi / 2 - m.lat[0], e_face, e_node))
    rows = np.array(rows)
    order = np.log(rows[:-1, 1:] / rows[1:, 1:]) / np.log(rows[:-1, :1] / rows[1:, :1])
    assert np.all(order[:, 0] >= 1.9), order
    assert np.all(order[:, 1] <= 1.2), order  # the one-sided value would fail


@pytest.mark.parametrize("N", [4, 16])
def test_partner_is_half_way_round(N):
    m = oracle.Mesh(N)
    p = _partner(m)
    for j in (0, m.nrings - 1):
        o, n = m.ring_off[j], m.nx[j]
        idx = np.arange(o, o + n)
        np.testing.assert_array_equal(p[idx], o + (idx - o + n // 2) % n)
        np.testing.assert_allclose(m.lat[p[idx]], m.lat[idx])
        dl = (m.lon[p[idx]] - m.lon[idx]) % (2 * np.pi)
        np.testing.assert_allclose(dl, np.pi, rtol=0, atol=1e-14)
