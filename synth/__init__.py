"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module draws inputs only; it holds none of the gridding method's
arithmetic (no kernels, tables, FFTs or corrections). It simulates:

* uniform random (u, v) with Gaussian complex values (the small case);
* an east-west/north-south Gaussian array of 64 antennas (sigma = 1 km)
  tracked over +-3 h of hour angle at declination 45 deg, baselines i < j, in
  time-major order (all baselines at one time, then the next), which is the
  usual measurement-set order. w is dropped (the paper's small-field form).
  This stands in for the paper's VLA A-array simulation, whose antenna
  positions are not reproduced here.
* skies of point sources on pixel centres, observed through the measurement
  equation V = sum_s F_s exp(-i 2 pi (u p_s + v q_s) / N).

All draws use ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

LATITUDE_DEG = 34.08
DECLINATION_DEG = 45.0


def uniform_case(seed: int = 1, nvis: int = 2000, N: int = 128, half_width: float = 32.0):
    """u, v ~ U[-half_width, half_width) cells; Re V, Im V ~ N(0, 1); unit weights."""
    rng = np.random.default_rng(seed)
    uv = rng.uniform(-half_width, half_width, size=(nvis, 2))
    vis = rng.standard_normal(nvis) + 1j * rng.standard_normal(nvis)
    w = np.ones(nvis)
    return uv, vis, w


def antenna_positions(seed: int, n_ant: int = 64, sigma_m: float = 1000.0):
    """East and north offsets ~ N(0, sigma^2), up = 0; converted to the equatorial X, Y, Z frame."""
    rng = np.random.default_rng(seed)
    east = rng.normal(0.0, sigma_m, n_ant)
    north = rng.normal(0.0, sigma_m, n_ant)
    lat = math.radians(LATITUDE_DEG)
    return -north * math.sin(lat), east, north * math.cos(lat)


def array_tracks(seed: int, n_time: int, wavelength: float = 0.21, n_ant: int = 64,
                 ha_hours=(-3.0, 3.0), dec_deg: float = DECLINATION_DEG) -> np.ndarray:
    """(n_time * n_baselines, 2) uv in wavelengths, time-major, hour angles at sample midpoints."""
    X, Y, Z = antenna_positions(seed, n_ant)
    i, j = np.triu_indices(n_ant, k=1)
    bx, by, bz = X[j] - X[i], Y[j] - Y[i], Z[j] - Z[i]
    ha = (ha_hours[0] + (np.arange(n_time) + 0.5) * (ha_hours[1] - ha_hours[0]) / n_time) * (math.pi / 12.0)
    dec = math.radians(dec_deg)
    sh, ch = np.sin(ha)[:, None], np.cos(ha)[:, None]
    u = (bx[None, :] * sh + by[None, :] * ch) / wavelength
    v = (-bx[None, :] * math.sin(dec) * ch + by[None, :] * math.sin(dec) * sh + bz[None, :] * math.cos(dec)) / wavelength
    return np.stack([u.ravel(), v.ravel()], axis=1)


def cell_scale(uv_lambda: np.ndarray, N: int, W: int) -> float:
    """Cells per wavelength such that max(|u|, |v|) = N/4 - W (data inside the central half)."""
    return (N / 4.0 - W) / float(np.max(np.abs(uv_lambda)))


def point_sky(seed: int, n_src: int, N: int, x0: float):
    """n_src sources at integer pixels uniform in [-x0 N, x0 N)^2, fluxes U(0.1, 1) Jy."""
    rng = np.random.default_rng(seed + 1000)
    half = int(round(x0 * N))
    pos = rng.integers(-half, half, size=(n_src, 2))
    flux = rng.uniform(0.1, 1.0, n_src)
    return pos, flux


def sky_visibilities(uv_cells, N: int, pos, flux, device: str = "cpu", chunk: int = 1 << 21):
    """V_k = sum_s F_s exp(-i 2 pi (u_k p_s + v_k q_s) / N) in FP64 (the measurement equation).

    Evaluated with torch (threaded on the host, or on ``device``) purely for
    speed; returns a numpy complex128 array.
    """
    import torch
    uvt = torch.as_tensor(np.ascontiguousarray(uv_cells), dtype=torch.float64)
    out = np.empty(len(uvt), dtype=np.complex128)
    for s in range(0, len(uvt), chunk):
        part = uvt[s:s + chunk].to(device)
        acc = torch.zeros(len(part), dtype=torch.complex128, device=device)
        for (p, q), f in zip(np.asarray(pos), np.asarray(flux, dtype=np.float64)):
            ph = (part[:, 0] * float(p) + part[:, 1] * float(q)) * (-2.0 * math.pi / N)
            acc += float(f) * torch.polar(torch.ones_like(ph), ph)
        out[s:s + chunk] = acc.cpu().numpy()
    return out


@dataclass
class Case:
    """One synthetic workload: uv in cells, visibilities, weights and the imaging parameters."""
    name: str
    N: int
    W: int
    x0: float
    table_size: int
    degree: int
    uv: np.ndarray
    vis: np.ndarray
    weights: np.ndarray
    extra: dict = field(default_factory=dict)


def small_case(seed: int = 1, W: int = 7, degree: int = 3) -> Case:
    """2,000 visibilities uniform in the central half of a 128^2 grid, N(0,1) values, unit weights."""
    uv, vis, w = uniform_case(seed)
    rng = np.random.default_rng(seed + 500)
    model = rng.standard_normal((64, 64)) + 1j * rng.standard_normal((64, 64))
    return Case("uniform-2000-128", 128, W, 0.25, 300, degree, uv, vis, w, {"model_image": model})


def array_case(seed: int, n_time: int, N: int, W: int = 7, n_src: int = 50, x0: float = 0.25,
               degree: int = 3, with_vis: bool = True, device: str = "cpu") -> Case:
    """Synthetic array observation: 2,016 baselines x n_time samples, 50-source sky."""
    uvl = array_tracks(seed, n_time)
    uv = uvl * cell_scale(uvl, N, W)
    pos, flux = point_sky(seed, n_src, N, x0)
    vis = sky_visibilities(uv, N, pos, flux, device) if with_vis else None
    return Case(f"array-{len(uv)}-{N}", N, W, x0, 300, degree, uv, vis, np.ones(len(uv)),
                {"src_pos": pos, "src_flux": flux})


def array_1m_case(W: int = 7, with_vis: bool = True, device: str = "cpu") -> Case:
    """1,008,000 visibilities (2,016 baselines x 500 times), lambda = 0.21 m, 2048^2 grid."""
    return array_case(2, 500, 2048, W, with_vis=with_vis, device=device)


def array_16m_case(W: int = 7, with_vis: bool = True, device: str = "cpu") -> Case:
    """16,777,152 visibilities (2,016 baselines x 8,322 times) on a 4096^2 grid."""
    return array_case(3, 8322, 4096, W, with_vis=with_vis, device=device)


def differentiation_case(W: int = 7, with_vis: bool = True, device: str = "cpu") -> Case:
    """The 16,777,152-visibility tracks on an 8192^2 grid: with x0 = 1/4 the image is 4096^2."""
    return array_case(3, 8322, 8192, W, with_vis=with_vis, device=device)


def channel_counts(seed: int = 5, nchan: int = 256, lo: float = 1e4, hi: float = 2e5) -> np.ndarray:
    """Per-channel visibility counts, log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), nchan))).astype(np.int64)


def multichannel_case(seed: int = 5, nchan: int = 256, N: int = 1024, W: int = 5):
    """256 channels, lambda = 0.21 (0.8 + 0.4 c / 255) m, uneven counts; one cell scale set by the shortest lambda.

    Returns (uv (total, 2) cells, offsets (nchan + 1,), wavelengths).
    """
    counts = channel_counts(seed, nchan)
    lams = 0.21 * (0.8 + 0.4 * np.arange(nchan) / (nchan - 1))
    nbl = 64 * 63 // 2
    parts = []
    for c in range(nchan):
        nt = -(-int(counts[c]) // nbl)
        parts.append(array_tracks(seed, nt, wavelength=float(lams[c]))[: counts[c]])
    allv = np.concatenate(parts)
    scale = cell_scale(allv, N, W)        # the largest |u|, |v| come from the shortest wavelength
    offsets = np.concatenate([[0], np.cumsum(counts)])
    return allv * scale, offsets, lams


def multichannel_vis(n: int, seed: int = 55) -> np.ndarray:
    """Complex N(0, 1) visibilities for the multi-channel case, rounded to complex64."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
