"""Pins of the oracle's grid (CPU only).

Section 4.2.3.5: Gaussian latitudes are the roots of a Legendre polynomial,
an even number of parallels, the first point of each parallel at x = 0.
Section 4.2.3.7, Listing 6: nx[j] = 20 + 4j up to the equator, mirrored.
Section 4.4, Figure 28: O32 has 5248 nodes; O1280 about 6.6 million.
"""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_grid_sizes.txt")


@pytest.mark.parametrize("N", [1, 2, 3, 8, 16, 48, 160, 320])
def test_gauss_mu_matches_leggauss(N):
    mu = oracle.gauss_mu(N)
    x, _ = np.polynomial.legendre.leggauss(2 * N)
    assert np.all(np.diff(mu) < 0), "latitudes must run north to south"
    np.testing.assert_allclose(mu, x[::-1], rtol=0, atol=1e-14)


@pytest.mark.parametrize("N", [1, 16, 1280])
def test_gauss_mu_symmetric_roots(N):
    mu = oracle.gauss_mu(N)
    assert mu.size == 2 * N
    np.testing.assert_array_equal(mu, -mu[::-1])
    # the roots annihilate P_2N (checked with numpy's Legendre series)
    c = np.zeros(2 * N + 1)
    c[-1] = 1.0
    if N <= 160:
        vals = np.polynomial.legendre.legval(mu, c)
        assert np.abs(vals).max() < 1e-12


def test_paper_node_counts():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert rows
    for name, N, nodes, tol in rows:
        N, nodes, tol = int(N), int(nodes), int(tol)
        assert name == f"O{N}"
        count = 4 * N * N + 36 * N
        assert abs(count - nodes) <= tol, (name, count, nodes)
        if N <= 320:
            assert oracle.Mesh(N).V == count


@pytest.mark.parametrize("N", [1, 2, 16, 33])
def test_nx_listing6_and_longitudes(N):
    m = oracle.Mesh(N)
    expect = np.empty(2 * N, np.int64)
    for j in range(N):
        expect[j] = 20 + 4 * j
        expect[2 * N - 1 - j] = expect[j]
    np.testing.assert_array_equal(m.nx, expect)
    np.testing.assert_array_equal(m.ring_off, np.concatenate([[0], np.cumsum(expect)]))
    mu = oracle.gauss_mu(N)
    for j in range(2 * N):
        sl = slice(m.ring_off[j], m.ring_off[j + 1])
        n = m.nx[j]
        np.testing.assert_allclose(m.lon[sl], 2 * np.pi * np.arange(n) / n, rtol=0, atol=0)
        assert m.lon[sl][0] == 0.0
        np.testing.assert_allclose(np.sin(m.lat[sl]), mu[j], rtol=0, atol=2e-16)


def test_workload_sizes():
    # sizes quoted for the workloads: O16 1,600; O320 421,120 nodes and
    # about 1.26 M edges; O1280 6,599,680 nodes, about 19.8 M edges
    assert oracle.Mesh(16).V == 1600
    m = oracle.Mesh(320)
    assert m.V == 421120 and abs(m.E - 1.26e6) < 0.01e6
    N = 1280
    assert 4 * N * N + 36 * N == 6599680
    assert abs(3 * (4 * N * N + 36 * N) - 40 - 19.8e6) < 0.01e6


def _mp_legendre_roots(n, count, dps=40):
    """The `count` largest roots of P_n to `dps` digits (mpmath Newton on the
    three-term recurrence from the asymptotic guess), each rounded to the
    nearest double."""
    import mpmath
    mpmath.mp.dps = dps
    out = []
    for j in range(count):
        x = mpmath.cos(mpmath.pi * (j + mpmath.mpf(3) / 4) / (n + mpmath.mpf(1) / 2))
        for _ in range(60):
            p0, p1 = mpmath.mpf(1), x
            for k in range(2, n + 1):
                p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
            dx = p1 / (n * (x * p1 - p0) / (x * x - 1))
            x -= dx
            if abs(dx) < mpmath.mpf(10) ** (-dps + 5):
                break
        out.append(float(x))  # mpf -> float rounds to nearest
    return np.array(out)


@pytest.mark.parametrize("N,count", [(1, 1), (2, 2), (16, 16), (48, 48), (1280, 8)])
def test_gauss_mu_correctly_rounded(N, count):
    """Each latitude is the double nearest the true Legendre root (Sec. 4.2.3.5):
    compared bit for bit with 40-digit roots for whole small grids and for the
    polar rings of O1280, where an ulp of latitude is a 2e-13 relative change
    of cos(lat)."""
    mu = oracle.gauss_mu(N)
    ref = _mp_legendre_roots(2 * N, count)
    np.testing.assert_array_equal(mu[:count], ref)
