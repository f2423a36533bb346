"""Helpers shared by the GPU tests: seeded inputs and normwise comparison."""
from __future__ import annotations

import numpy as np

import synthetic as sy

OPS = ("grad", "div", "curl", "lapl")
TOL = {"f64": 1e-12, "f32": 1e-5}


def make_inputs(om, nlev, lmax=8, config=90, amplitude=None, noise_eps=1e-3):
    """Scalar field [V][nlev] (independent harmonics per level, scaled by
    level index, plus noise) and a vector field [V][nlev][2] whose levels are
    the analytic gradient of a second field (Sec. 4.7 operators need smooth
    but not trivial data)."""
    f = sy.level_field_stack(om.lon, om.lat, nlev, lmax, config, 0,
                             amplitude=amplitude, noise_eps=noise_eps)
    co = sy.random_coeffs(lmax, [sy.seed_rng(config, 1, k) for k in range(min(nlev, 4))])
    g = sy.synthesize_gradient(om.lon, om.lat, co, R=om.R)  # [nh, V, 2]
    uv = np.empty((om.V, nlev, 2))
    for k in range(nlev):
        uv[:, k, :] = g[k % g.shape[0]] * (1.0 + k / nlev)
    uv += sy.noise(sy.seed_rng(config, 2, 0), uv.shape, noise_eps)
    return f, uv


def oracle_apply(om, op, x, nlev):
    if op == "grad":
        return om.gradient(x, nlev)
    if op == "div":
        return om.divergence(x, nlev)
    if op == "curl":
        return om.curl(x, nlev)
    return om.laplacian(x, nlev)


def oracle_apply_at(om, op, x, nlev, nodes):
    if op == "grad":
        return om.gradient_at(x, nlev, nodes)
    if op == "div":
        return om.divergence_at(x, nlev, nodes)
    if op == "curl":
        return om.curl_at(x, nlev, nodes)
    return om.laplacian_at(x, nlev, nodes)


def normwise_error(got, ref):
    """max |got - ref| / max |ref| per output component (last axis for the
    gradient), and the RMS error relative to the RMS of ref."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    if ref.ndim == 3:
        comps = [(got[..., c], ref[..., c]) for c in range(ref.shape[-1])]
    else:
        comps = [(got, ref)]
    rel_max, rel_rms = [], []
    for g, r in comps:
        scale = np.abs(r).max()
        d = np.abs(g - r)
        rel_max.append(d.max() / scale if scale > 0 else d.max())
        rms = np.sqrt((r ** 2).mean())
        rel_rms.append(np.sqrt((d ** 2).mean()) / rms if rms > 0 else 0.0)
    return max(rel_max), max(rel_rms)
