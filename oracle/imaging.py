"""Gridding, FFT imaging, prediction and degridding, FP64 (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Paper: Ye, Gull, Tan & Nikolic (2019). Sec. 2.1 Eqs. (3)-(8) for imaging and
the misfit bound, Eq. (2) and Sec. 5 for prediction/degridding (degridding
is the transpose of gridding, Sec. 1). 2D forms use separability (Sec. 1,
condition (i)): C(u, v) = C(u) C(v) and h(x, y) = h(x) h(y).

Array conventions (shared with the library only as a documented layout,
never as code):

* ``uv`` is (n, 2) float64 in grid cells, column 0 = u, column 1 = v.
* The N x N grid is stored centred: ``G[m + N/2, n + N/2]`` holds G_{m,n}
  for m, n in [-N/2, N/2); rows follow v, columns follow u. Taps outside
  [-N/2, N/2) wrap modulo N (exact at the pixel samples x = p/N).
* Images keep pixels p, q in [-x0 N, x0 N) (x_p = p/N, y_q = q/N), stored as
  ``I[q + x0 N, p + x0 N]``.
"""
from __future__ import annotations

import numpy as np

from .lmtable import Table, tap_reference


# ----------------------------------------------------------------- taps --
def tap_geometry(coord: np.ndarray, W: int):
    """n_first = ceil(u - W/2) (the first cell of S_k, Eq. 6) and delta = u - (n_first + ref)."""
    coord = np.asarray(coord, dtype=np.float64)
    n_first = np.ceil(coord - W / 2.0)
    delta = coord - (n_first + tap_reference(W))
    return n_first.astype(np.int64), delta


def _axis_weights(coord: np.ndarray, table: Table, N: int):
    n_first, delta = tap_geometry(coord, table.W)
    wts = table.weights(delta)                                  # (n, W)
    cells = (n_first[:, None] + np.arange(table.W)[None, :] + N // 2) % N
    return cells, wts


# -------------------------------------------------------------- gridding --
def grid(uv: np.ndarray, vis: np.ndarray, weights, N: int, table: Table) -> np.ndarray:
    """G_{m,n} = sum_k w_k V_k C(m - v_k) C(n - u_k)  (Eq. 5 in 2D), FP64, centred storage."""
    uv = np.asarray(uv, dtype=np.float64)
    vis = np.asarray(vis, dtype=np.complex128)
    wv = vis if weights is None else vis * np.asarray(weights, dtype=np.float64)
    G = np.zeros(N * N, dtype=np.complex128)
    W = table.W
    for s in range(0, len(uv), 1 << 16):
        cu, wu = _axis_weights(uv[s:s + (1 << 16), 0], table, N)
        cv, wgtv = _axis_weights(uv[s:s + (1 << 16), 1], table, N)
        idx = (cv[:, :, None] * N + cu[:, None, :]).ravel()
        val = (wv[s:s + (1 << 16), None, None] * wgtv[:, :, None] * wu[:, None, :]).ravel()
        G += np.bincount(idx, weights=val.real, minlength=N * N) + 1j * np.bincount(idx, weights=val.imag, minlength=N * N)
        del idx, val
    return G.reshape(N, N)


def grid_cells(uv: np.ndarray, vis: np.ndarray, weights, N: int, table: Table, cells) -> np.ndarray:
    """Selected grid values G[row, col] (storage indices) by the definition of Eq. (5), summing only the
    visibilities whose W x W footprint contains the cell. For checking large grids at sample points."""
    uv = np.asarray(uv, dtype=np.float64)
    vis = np.asarray(vis, dtype=np.complex128)
    w = np.ones(len(uv)) if weights is None else np.asarray(weights, dtype=np.float64)
    W = table.W
    nu, _ = tap_geometry(uv[:, 0], W)
    nv, _ = tap_geometry(uv[:, 1], W)
    cu0 = (nu + N // 2) % N
    cv0 = (nv + N // 2) % N
    out = np.zeros(len(cells), dtype=np.complex128)
    for i, (r, c) in enumerate(cells):
        jv = (r - cv0) % N
        ju = (c - cu0) % N
        sel = np.nonzero((jv < W) & (ju < W))[0]
        if len(sel) == 0:
            continue
        wu = table.weights(tap_geometry(uv[sel, 0], W)[1])[np.arange(len(sel)), ju[sel]]
        wv = table.weights(tap_geometry(uv[sel, 1], W)[1])[np.arange(len(sel)), jv[sel]]
        out[i] = np.sum(w[sel] * vis[sel] * wv * wu)
    return out


def degrid(uv: np.ndarray, G: np.ndarray, table: Table) -> np.ndarray:
    """V_k = sum_{m,n} C(m - v_k) C(n - u_k) G_{m,n}: the transpose of :func:`grid` (Sec. 1, Sec. 5)."""
    uv = np.asarray(uv, dtype=np.float64)
    G = np.asarray(G, dtype=np.complex128)
    N = G.shape[0]
    out = np.empty(len(uv), dtype=np.complex128)
    for s in range(0, len(uv), 1 << 16):
        cu, wu = _axis_weights(uv[s:s + (1 << 16), 0], table, N)
        cv, wgtv = _axis_weights(uv[s:s + (1 << 16), 1], table, N)
        patch = G[cv[:, :, None], cu[:, None, :]]             # (n, W, W)
        out[s:s + (1 << 16)] = np.einsum("ki,kj,kij->k", wgtv, wu, patch)
    return out


# ------------------------------------------------------------------- FFT --
def _bit_reverse(n: int) -> np.ndarray:
    bits = n.bit_length() - 1
    idx = np.arange(n)
    rev = np.zeros(n, dtype=np.int64)
    for b in range(bits):
        rev |= ((idx >> b) & 1) << (bits - 1 - b)
    return rev


def fft_radix2(a: np.ndarray, sign: int) -> np.ndarray:
    """X[r] = sum_s a[s] exp(sign i 2 pi s r / n) along the last axis; iterative radix-2 Cooley-Tukey."""
    a = np.asarray(a, dtype=np.complex128)
    n = a.shape[-1]
    if n & (n - 1):
        raise ValueError("length must be a power of two")
    lead = a.shape[:-1]
    y = a[..., _bit_reverse(n)].copy()
    size = 2
    while size <= n:
        half = size // 2
        tw = np.exp(sign * 2j * np.pi * np.arange(half) / size)
        y = y.reshape(lead + (n // size, size))
        even = y[..., :half].copy()
        odd = y[..., half:] * tw
        y[..., :half] = even + odd
        y[..., half:] = even - odd
        y = y.reshape(lead + (n,))
        size *= 2
    return y


def centred_fft2(G: np.ndarray, sign: int) -> np.ndarray:
    """F_{q,p} = sum_{m,n} G_{m,n} exp(sign i 2 pi (n p + m q) / N), all indices centred in [-N/2, N/2).

    The kernel exp(i 2 pi n p / N) is N-periodic in n and p, so the centred
    sum equals an ordinary DFT of the array rolled to start at index 0.
    """
    N = G.shape[0]
    a = np.roll(np.asarray(G, dtype=np.complex128), (-(N // 2), -(N // 2)), axis=(0, 1))
    a = fft_radix2(a, sign)                    # over n (columns)
    a = fft_radix2(a.T, sign).T                # over m (rows)
    return np.roll(a, (N // 2, N // 2), axis=(0, 1))


def crop_size(N: int, x0: float) -> int:
    m = 2.0 * x0 * N
    if abs(m - round(m)) > 1e-9:
        raise ValueError("2 x0 N must be an integer")
    return int(round(m))


def dirty_from_grid(G: np.ndarray, hpix: np.ndarray, x0: float) -> np.ndarray:
    """I(x_p, y_q) = h(x_p) h(y_q) sum_{m,n} G_{m,n} e^{i 2 pi (n x_p + m y_q)} on |x|, |y| <= x0 (Eq. 4)."""
    N = G.shape[0]
    M = crop_size(N, x0)
    F = centred_fft2(G, +1)
    sl = slice(N // 2 - M // 2, N // 2 + M // 2)
    hc = np.asarray(hpix, dtype=np.float64)[sl]
    return F[sl, sl] * hc[:, None] * hc[None, :]


def grid_from_image(image: np.ndarray, hpix: np.ndarray, N: int, x0: float) -> np.ndarray:
    """Prediction grid: G_{m,n} = sum_{p,q} h(x_p) h(y_q) I_{q,p} e^{-i 2 pi (n x_p + m y_q)} (Eq. 2, Sec. 5)."""
    M = crop_size(N, x0)
    sl = slice(N // 2 - M // 2, N // 2 + M // 2)
    hc = np.asarray(hpix, dtype=np.float64)[sl]
    pad = np.zeros((N, N), dtype=np.complex128)
    pad[sl, sl] = np.asarray(image, dtype=np.complex128) * hc[:, None] * hc[None, :]
    return centred_fft2(pad, -1)


def make_dirty_image(uv, vis, weights, N: int, x0: float, table: Table, hpix) -> np.ndarray:
    """Grid, inverse FFT, correct and crop."""
    return dirty_from_grid(grid(uv, vis, weights, N, table), hpix, x0)


def predict_visibilities(uv, image, N: int, x0: float, table: Table, hpix) -> np.ndarray:
    """Correct, zero-pad, forward FFT and degrid."""
    return degrid(uv, grid_from_image(image, hpix, N, x0), table)


# ----------------------------------------------------------- ground truth --
def _pixels(N: int, x0: float) -> np.ndarray:
    M = crop_size(N, x0)
    return np.arange(M) - M // 2


def dft_dirty_image(uv, vis, weights, N: int, x0: float, pixels_x=None, pixels_y=None, chunk: int = 4096) -> np.ndarray:
    """I_D(x_p, y_q) = sum_k w_k V_k exp(i 2 pi (u_k x_p + v_k y_q))  (Eq. 3 in 2D), x_p = p/N.

    Computed as a chunked complex GEMM  E_y^T diag(w V) E_x ; returns [q, p].
    """
    uv = np.asarray(uv, dtype=np.float64)
    wv = np.asarray(vis, dtype=np.complex128)
    if weights is not None:
        wv = wv * np.asarray(weights, dtype=np.float64)
    px = _pixels(N, x0) if pixels_x is None else np.asarray(pixels_x)
    py = _pixels(N, x0) if pixels_y is None else np.asarray(pixels_y)
    out = np.zeros((len(py), len(px)), dtype=np.complex128)
    for s in range(0, len(uv), chunk):
        ex = np.exp(2j * np.pi * np.outer(uv[s:s + chunk, 0], px) / N)
        ey = np.exp(2j * np.pi * np.outer(uv[s:s + chunk, 1], py) / N)
        out += (ey * wv[s:s + chunk, None]).T @ ex
    return out


def direct_predict(uv, image, N: int, x0: float, chunk: int = 4096) -> np.ndarray:
    """V_k = sum_{p,q} I_{q,p} exp(-i 2 pi (u_k x_p + v_k y_q))  (Eq. 2 on the pixel lattice)."""
    uv = np.asarray(uv, dtype=np.float64)
    image = np.asarray(image, dtype=np.complex128)
    px = _pixels(N, x0)
    out = np.empty(len(uv), dtype=np.complex128)
    for s in range(0, len(uv), chunk):
        ex = np.exp(-2j * np.pi * np.outer(uv[s:s + chunk, 0], px) / N)     # (k, p)
        ey = np.exp(-2j * np.pi * np.outer(uv[s:s + chunk, 1], px) / N)     # (k, q)
        out[s:s + chunk] = np.einsum("kq,kq->k", ey, ex @ image.T)
    return out


def point_source_predict(uv, N: int, positions, fluxes) -> np.ndarray:
    """Direct prediction of a sky of point sources on pixel centres (Eq. 2 with delta functions)."""
    uv = np.asarray(uv, dtype=np.float64)
    out = np.zeros(len(uv), dtype=np.complex128)
    for (p, q), f in zip(np.asarray(positions), np.asarray(fluxes, dtype=np.float64)):
        out += f * np.exp(-2j * np.pi * (uv[:, 0] * p + uv[:, 1] * q) / N)
    return out


# ----------------------------------------------------------- misfit bound --
def _axis_phase_sum(coord, table: Table, N: int, xs: np.ndarray) -> np.ndarray:
    """sum_j C(n_j - u) exp(i 2 pi (n_j - u) x) for each visibility and each x, (n, len(xs))."""
    n_first, delta = tap_geometry(coord, table.W)
    wts = table.weights(delta)
    off = (n_first[:, None] + np.arange(table.W)[None, :]) - np.asarray(coord)[:, None]
    return np.einsum("kj,kjx->kx", wts, np.exp(2j * np.pi * off[:, :, None] * xs[None, None, :]))


def image_misfit_bound(uv, vis, weights, N: int, table: Table, hpix, pixels) -> np.ndarray:
    """Cauchy-Schwarz bound on |I_D - I_FFT|^2 at the given (p, q) pixels (Eqs. 7-8).

    bound = (sum_k w_k |V_k|^2) (sum_k w_k |b_k|^2),
    b_k = 1 - h(x) h(y) sum_{n,m} C(n-u_k) C(m-v_k) e^{i 2 pi ((n-u_k) x + (m-v_k) y)}.
    """
    uv = np.asarray(uv, dtype=np.float64)
    w = np.ones(len(uv)) if weights is None else np.asarray(weights, dtype=np.float64)
    pix = np.asarray(pixels)
    hp = np.asarray(hpix, dtype=np.float64)
    xs = pix[:, 0] / N
    ys = pix[:, 1] / N
    su = _axis_phase_sum(uv[:, 0], table, N, xs)
    sv = _axis_phase_sum(uv[:, 1], table, N, ys)
    hh = hp[pix[:, 0] + N // 2] * hp[pix[:, 1] + N // 2]
    b = 1.0 - hh[None, :] * su * sv
    return float(np.sum(w * np.abs(np.asarray(vis)) ** 2)) * (w @ (np.abs(b) ** 2))
