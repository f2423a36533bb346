"""Real spherical-harmonic field synthesis on the nodes of a reduced grid.

Conventions
-----------
* Real, 4-pi normalised harmonics without the Condon-Shortley phase:
  Y_lm = Pbar_l^|m|(sin lat) * cos(m lon)   (m >= 0)
  Y_lm = Pbar_l^|m|(sin lat) * sin(|m| lon) (m < 0)
  with the surface mean of Y_lm^2 equal to one.
* A random field of degree <= L has (L+1)^2 i.i.d. N(0, 1) coefficients;
  "amplitude A" scales it by A / sqrt((L+1)^2) so its RMS is about A.
* Seeds: ``numpy.random.default_rng([20170331, config, field, level])``.

Nodes are grouped by latitude; a group whose longitudes are 2 pi i / n
(i = 0..n-1, the layout of every parallel of a reduced Gaussian grid) is
synthesised with one inverse FFT, any other group by direct evaluation.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

BASE_SEED = 20170331


def seed_rng(*key: int) -> np.random.Generator:
    return np.random.default_rng([BASE_SEED, *[int(k) for k in key]])


@dataclass
class SHCoeffs:
    """Coefficients of real harmonics up to degree lmax for nf fields.
    c[f, l, m] multiplies Pbar_l^m cos(m lon); s[f, l, m] multiplies
    Pbar_l^m sin(m lon) (s[:, :, 0] is unused and zero)."""
    c: np.ndarray
    s: np.ndarray

    @property
    def lmax(self) -> int:
        return self.c.shape[1] - 1

    @property
    def nf(self) -> int:
        return self.c.shape[0]

    def scaled(self, factor) -> "SHCoeffs":
        factor = np.asarray(factor, dtype=np.float64)
        return SHCoeffs(self.c * factor, self.s * factor)


def random_coeffs(lmax: int, rngs, amplitude: float | None = None) -> SHCoeffs:
    """One field per generator in ``rngs``: N(0,1) coefficients for every
    (l, m) with m <= l (cosine) and 1 <= m <= l (sine), drawn in the order
    l, then m, cosine before sine.  With ``amplitude`` the field is scaled
    by amplitude / (lmax+1) so that its RMS over the sphere is about
    ``amplitude``."""
    rngs = list(rngs)
    nf = len(rngs)
    c = np.zeros((nf, lmax + 1, lmax + 1))
    s = np.zeros((nf, lmax + 1, lmax + 1))
    nterm = (lmax + 1) ** 2
    for f, rng in enumerate(rngs):
        draws = rng.standard_normal(nterm)
        k = 0
        for l in range(lmax + 1):
            c[f, l, 0] = draws[k]
            k += 1
            for m in range(1, l + 1):
                c[f, l, m] = draws[k]
                s[f, l, m] = draws[k + 1]
                k += 2
        if amplitude is not None:
            c[f] *= amplitude / np.sqrt(nterm)
            s[f] *= amplitude / np.sqrt(nterm)
    return SHCoeffs(c, s)


def laplacian_coeffs(co: SHCoeffs, R: float = 1.0) -> SHCoeffs:
    """Coefficients of the surface Laplacian: Y_lm -> -l(l+1)/R^2 Y_lm."""
    l = np.arange(co.lmax + 1, dtype=np.float64)
    fac = (-l * (l + 1.0) / (R * R))[None, :, None]
    return SHCoeffs(co.c * fac, co.s * fac)


def _fourier_tables(mu: np.ndarray, co: SHCoeffs, want_dlat: bool):
    """For every latitude mu = sin(lat) return the Fourier coefficients
    Ac[f, r, m] = sum_l c[f,l,m] Pbar_l^m(mu_r) (and As, and their lat
    derivatives when ``want_dlat``)."""
    L = co.lmax
    nr = mu.size
    cosl = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    Ac = np.zeros((co.nf, nr, L + 1))
    As = np.zeros((co.nf, nr, L + 1))
    dAc = np.zeros_like(Ac) if want_dlat else None
    dAs = np.zeros_like(As) if want_dlat else None
    pmm = np.ones(nr)
    for m in range(L + 1):
        if m == 1:
            pmm = np.sqrt(3.0) * cosl
        elif m >= 2:
            pmm = np.sqrt((2.0 * m + 1.0) / (2.0 * m)) * cosl * pmm
        p_lm1 = np.zeros(nr)   # Pbar_{l-1}^m
        p_l = pmm.copy()       # Pbar_l^m, l = m
        for l in range(m, L + 1):
            if l == m + 1:
                p_lm1, p_l = p_l, np.sqrt(2.0 * m + 3.0) * mu * p_l
            elif l >= m + 2:
                a = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
                b = np.sqrt((2.0 * l + 1.0) * (l - m - 1.0) * (l + m - 1.0)
                            / ((2.0 * l - 3.0) * (l * l - m * m)))
                p_lm1, p_l = p_l, a * mu * p_l - b * p_lm1
            cl = co.c[:, l, m][:, None]
            sl = co.s[:, l, m][:, None]
            Ac[:, :, m] += cl * p_l[None, :]
            As[:, :, m] += sl * p_l[None, :]
            if want_dlat:
                # d Pbar_l^m / d lat = (-l mu Pbar_l^m
                #     + sqrt((2l+1)(l^2-m^2)/(2l-1)) Pbar_{l-1}^m) / cos(lat)
                k = np.sqrt((2.0 * l + 1.0) * (l * l - m * m) / (2.0 * l - 1.0)) if l > 0 else 0.0
                dp = (-l * mu * p_l + k * p_lm1) / cosl
                dAc[:, :, m] += cl * dp[None, :]
                dAs[:, :, m] += sl * dp[None, :]
    return Ac, As, dAc, dAs


def _ring_groups(lon: np.ndarray, lat: np.ndarray):
    ulat, inv = np.unique(lat, return_inverse=True)
    order = np.argsort(inv, kind="stable")
    bounds = np.searchsorted(inv[order], np.arange(ulat.size + 1))
    return ulat, order, bounds


def _fourier_eval(lon, idx, Ac_r, As_r):
    """Evaluate sum_m Ac_r[f,m] cos(m lon) + As_r[f,m] sin(m lon) at the
    nodes idx (one latitude group).  Returns [nf, len(idx)]."""
    n = idx.size
    lam = lon[idx]
    M = Ac_r.shape[1] - 1
    expected = 2.0 * np.pi * np.arange(n) / n
    if np.array_equal(lam, expected):
        C = np.zeros((Ac_r.shape[0], n), dtype=np.complex128)
        q = np.arange(M + 1) % n
        np.add.at(C, (slice(None), q), Ac_r - 1j * As_r)
        return np.real(np.fft.ifft(C, axis=1)) * n
    mm = np.arange(M + 1)[:, None] * lam[None, :]
    return Ac_r @ np.cos(mm) + As_r @ np.sin(mm)


def synthesize(lon: np.ndarray, lat: np.ndarray, co: SHCoeffs) -> np.ndarray:
    """Field values [nf, V] at nodes (lon, lat) in radians."""
    lon = np.asarray(lon, np.float64)
    lat = np.asarray(lat, np.float64)
    ulat, order, bounds = _ring_groups(lon, lat)
    Ac, As, _, _ = _fourier_tables(np.sin(ulat), co, want_dlat=False)
    out = np.empty((co.nf, lon.size))
    for r in range(ulat.size):
        idx = order[bounds[r]:bounds[r + 1]]
        out[:, idx] = _fourier_eval(lon, idx, Ac[:, r, :], As[:, r, :])
    return out


def synthesize_gradient(lon, lat, co: SHCoeffs, R: float = 1.0) -> np.ndarray:
    """Closed-form physical gradient [nf, V, 2] = (1/(R cos lat) d/dlon,
    1/R d/dlat) of the harmonic field."""
    lon = np.asarray(lon, np.float64)
    lat = np.asarray(lat, np.float64)
    ulat, order, bounds = _ring_groups(lon, lat)
    Ac, As, dAc, dAs = _fourier_tables(np.sin(ulat), co, want_dlat=True)
    m = np.arange(co.lmax + 1, dtype=np.float64)[None, :]
    out = np.empty((co.nf, lon.size, 2))
    for r in range(ulat.size):
        idx = order[bounds[r]:bounds[r + 1]]
        # d/dlon of (Ac cos + As sin) = (m As) cos + (-m Ac) sin
        dlon = _fourier_eval(lon, idx, m * As[:, r, :], -m * Ac[:, r, :])
        dlat = _fourier_eval(lon, idx, dAc[:, r, :], dAs[:, r, :])
        out[:, idx, 0] = dlon / (R * np.cos(ulat[r]))
        out[:, idx, 1] = dlat / R
    return out


def rotated_gradient(grad: np.ndarray) -> np.ndarray:
    """k x grad: (gx, gy) -> (-gy, gx).  Its divergence is zero and its
    radial curl is the Laplacian of the potential."""
    out = np.empty_like(grad)
    out[..., 0] = -grad[..., 1]
    out[..., 1] = grad[..., 0]
    return out


def noise(rng: np.random.Generator, shape, eps: float) -> np.ndarray:
    """eps * U(-1, 1)."""
    return eps * (2.0 * rng.random(shape) - 1.0)


def config_field(lon, lat, lmax: int, config: int, field: int,
                 amplitude: float | None = None, noise_eps: float = 0.0,
                 R: float = 1.0, with_gradient: bool = False):
    """One seeded single-level field (and optionally its analytic gradient):
    coefficients from seed (config, field, 0), noise from (config, field, 1)."""
    co = random_coeffs(lmax, [seed_rng(config, field, 0)], amplitude)
    f = synthesize(lon, lat, co)[0]
    if noise_eps:
        f = f + noise(seed_rng(config, field, 1), f.shape, noise_eps)
    if with_gradient:
        return f, synthesize_gradient(lon, lat, co, R)[0]
    return f


def level_field_stack(lon, lat, nlev: int, lmax: int, config: int, field: int,
                      nharm: int | None = None, amplitude: float | None = None,
                      noise_eps: float = 0.0, level_scale: str = "index",
                      dtype=np.float64) -> np.ndarray:
    """A [V][nlev] scalar field.

    nharm=None: level k is an independent harmonic field (seed (config,
    field, k)) times (k+1) ("scaled by level index").
    nharm=h: h harmonic fields H_0..H_{h-1} (seeds (config, field, j)) are
    cycled over the levels: level k = H_{k mod h} * (1 + k/nlev), so the
    levels stay distinct at a bounded synthesis cost.
    noise_eps adds eps*U(-1,1) per node and level (seed (config, field,
    10**6))."""
    V = np.asarray(lon).size
    out = np.empty((V, nlev), dtype=dtype)
    if nharm is None:
        co = random_coeffs(lmax, [seed_rng(config, field, k) for k in range(nlev)],
                           amplitude)
        H = synthesize(lon, lat, co)  # [nlev, V]
        for k in range(nlev):
            out[:, k] = H[k] * (k + 1.0)
    else:
        co = random_coeffs(lmax, [seed_rng(config, field, j) for j in range(nharm)],
                           amplitude)
        H = synthesize(lon, lat, co)  # [nharm, V]
        for k in range(nlev):
            out[:, k] = H[k % nharm] * (1.0 + k / nlev)
    if noise_eps:
        rng = seed_rng(config, field, 10 ** 6)
        chunk = max(1, (1 << 24) // max(1, nlev))
        for i0 in range(0, V, chunk):
            i1 = min(V, i0 + chunk)
            out[i0:i1] += noise(rng, (i1 - i0, nlev), noise_eps).astype(dtype)
    return out
