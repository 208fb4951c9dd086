"""Pins for the oracle's gridding / FFT / prediction path (CPU only)."""
import os

import numpy as np
import pytest

import synth
from oracle import imaging as im
from oracle import lmtable as lt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def w7():
    tab, h = lt.make_table(7, 0.25, 300, 3)
    return tab, h


# ------------------------------------------------------------------ FFT ---
@pytest.mark.parametrize("n", [2, 8, 64])
def test_fft_matches_dft_matrix(n):
    rng = np.random.default_rng(n)
    a = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    for sign in (+1, -1):
        M = np.exp(sign * 2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
        np.testing.assert_allclose(im.fft_radix2(a, sign), a @ M.T, atol=1e-12 * n)


def test_fft_matches_library():
    rng = np.random.default_rng(7)
    a = rng.standard_normal((4, 4096)) + 1j * rng.standard_normal((4, 4096))
    np.testing.assert_allclose(im.fft_radix2(a, -1), np.fft.fft(a), rtol=0, atol=1e-10)
    np.testing.assert_allclose(im.fft_radix2(a, +1), np.fft.ifft(a) * 4096, rtol=0, atol=1e-10)


def test_centred_fft2_brute_force():
    N = 16
    rng = np.random.default_rng(3)
    G = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    idx = np.arange(N) - N // 2
    E = np.exp(2j * np.pi * np.outer(idx, idx) / N)        # E[p, n]
    F = E @ G.T @ E.T                                        # F[p, q]... rows follow q after transpose
    np.testing.assert_allclose(im.centred_fft2(G, +1), F.T, atol=1e-11)


# ------------------------------------------------------------- gridding ---
def test_single_visibility_on_grid_point_reproduces_table(w7):
    """Eq. (5): V = 1 at integer (u, v) spreads exactly the node values C(j - 3) C(i - 3) (bitwise)."""
    tab, _ = w7
    N = 32
    G = im.grid(np.array([[3.0, -5.0]]), np.array([1.0 + 0j]), None, N, tab)
    c = tab.nodes[:, tab.Ms // 2]
    block = G[N // 2 - 5 - 3: N // 2 - 5 + 4, N // 2 + 3 - 3: N // 2 + 3 + 4]
    np.testing.assert_array_equal(block.real, np.outer(c, c))
    assert np.count_nonzero(G) == 49


def test_grid_wraps_modulo_N(w7):
    """Taps beyond the grid edge wrap (periodicity of the pixel-sampled transform)."""
    tab, _ = w7
    N = 32
    a = im.grid(np.array([[15.7, 0.2]]), np.array([1.0 + 2j]), None, N, tab)
    b = im.grid(np.array([[15.7 - N, 0.2]]), np.array([1.0 + 2j]), None, N, tab)
    np.testing.assert_allclose(a, b, atol=1e-15)
    assert np.count_nonzero(a[:, :3]) > 0


def test_adjoint_identity(w7):
    """Degridding is the transpose of gridding (Sec. 1): <grid(V), G> = <V, degrid(G)>."""
    tab, _ = w7
    N = 64
    rng = np.random.default_rng(11)
    uv = rng.uniform(-30, 30, (300, 2))
    V = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    G = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    lhs = np.vdot(im.grid(uv, V, None, N, tab), G)
    rhs = np.vdot(V, im.degrid(uv, G, tab))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_hermitian_completion_gives_real_image():
    """C real and even (Sec. 1) => visibilities with their conjugates at -uv give a real dirty image.

    Holds exactly for a mirror-symmetric lookup (linear interpolation). The
    forward Newton stencil of degree 3 (App. F) is not mirror-symmetric, so
    the cubic table leaves an imaginary part at its interpolation-error level.
    """
    h = lt.optimal_h(7, 0.25)
    N = 64
    rng = np.random.default_rng(5)
    uv = rng.uniform(-15, 15, (200, 2))
    V = rng.standard_normal(200) + 1j * rng.standard_normal(200)
    uv2 = np.concatenate([uv, -uv])
    V2 = np.concatenate([V, V.conj()])
    hp = lt.correction(h, 7, 0.25, N)
    lin = lt.Table(7, 0.25, 42, 1, lt.table_nodes(h, 7, 0.25, 42, 1))
    I = im.make_dirty_image(uv2, V2, None, N, 0.25, lin, hp)
    assert np.max(np.abs(I.imag)) < 1e-13 * np.max(np.abs(I.real))
    cub = lt.Table(7, 0.25, 42, 3, lt.table_nodes(h, 7, 0.25, 42, 3))
    I3 = im.make_dirty_image(uv2, V2, None, N, 0.25, cub, hp)
    assert 1e-13 < np.max(np.abs(I3.imag)) / np.max(np.abs(I3.real)) < 1e-6


# ----------------------------------------------------------- DFT truth ---
def test_dft_gemm_matches_loops():
    rng = np.random.default_rng(2)
    uv = rng.uniform(-8, 8, (13, 2))
    V = rng.standard_normal(13) + 1j * rng.standard_normal(13)
    w = rng.uniform(0.5, 2, 13)
    N, x0 = 16, 0.25
    I = im.dft_dirty_image(uv, V, w, N, x0, chunk=5)
    ref = np.zeros((8, 8), complex)
    for qi, q in enumerate(range(-4, 4)):
        for pi_, p in enumerate(range(-4, 4)):
            for k in range(13):
                ref[qi, pi_] += w[k] * V[k] * np.exp(2j * np.pi * (uv[k, 0] * p + uv[k, 1] * q) / N)
    np.testing.assert_allclose(I, ref, atol=1e-12)
    img = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    pred = im.direct_predict(uv, img, N, x0, chunk=4)
    refp = [sum(img[qi, pi_] * np.exp(-2j * np.pi * (uv[k, 0] * p + uv[k, 1] * q) / N)
                for qi, q in enumerate(range(-4, 4)) for pi_, p in enumerate(range(-4, 4))) for k in range(13)]
    np.testing.assert_allclose(pred, refp, atol=1e-12)


@pytest.fixture(scope="module")
def small_images(w7):
    tab, h = w7
    case = synth.small_case()
    hp = lt.correction(h, 7, 0.25, case.N)
    fft_img = im.make_dirty_image(case.uv, case.vis, case.weights, case.N, case.x0, tab, hp)
    dft_img = im.dft_dirty_image(case.uv, case.vis, case.weights, case.N, case.x0)
    return case, hp, fft_img, dft_img


def test_dft_fft_misfit_bound_every_pixel(w7, small_images):
    """Eqs. (7)-(8): |I_D - I_FFT|^2 <= (sum w |V|^2)(sum w |b_k|^2) at every retained pixel."""
    tab, _ = w7
    case, hp, fft_img, dft_img = small_images
    pq = np.stack(np.meshgrid(np.arange(-32, 32), np.arange(-32, 32), indexing="xy"), -1).reshape(-1, 2)
    bound = im.image_misfit_bound(case.uv, case.vis, case.weights, case.N, tab, hp, pq)
    err2 = np.abs(dft_img - fft_img).reshape(-1) ** 2
    assert np.all(err2 <= bound * (1 + 1e-9) + 1e-26)
    # the misfit is small: near the W = 7 single-precision level relative to the peak
    assert np.max(np.abs(dft_img - fft_img)) < 1e-5 * np.max(np.abs(dft_img))


def _map_error_2d(tab, hp, N, pix):
    """l_2D(x_p, y_q) of the separable kernel (Eq. 11 in 2D) for the table and correction used: averaging
    |1 - h(x) h(y) S_u(x) S_v(y)|^2 over both offsets gives 1 - 2 h_x h_y c_x c_y + h_x^2 h_y^2 D_x D_y with the
    1D c (Eq. 13) and D (Eq. 14). The nu integral over the piecewise-polynomial table uses a composite rule."""
    lo = lt.delta_low(tab.W)
    quad = lt.composite_midpoint(lo, lo + 1.0, tab.Ms * 16)
    _, hx, c, D = lt.map_error(lambda d: tab.weights(d).T, tab.W, pix / N, h_of_x=hp[pix + N // 2], quad=quad)
    return 1 - 2 * np.outer(hx * c, hx * c) + np.outer(hx * hx * D, hx * hx * D)      # [q, p]


def test_misfit_level_and_bound_from_the_map_error(w7, small_images):
    """The misfit bound of Eqs. (7)-(8) pinned from both sides by the map error (Eq. 11, Sec. 2.1).

    With independent visibilities at offsets spread evenly over the cell, the expected |I_D - I_FFT|^2 at a
    pixel is sum_k w_k^2 |V_k|^2 |b_k|^2 and the mean of |b_k|^2 over the visibilities is l_2D, so the RMS
    misfit is close to sqrt(mean l_2D * sum w^2 |V|^2); and the Cauchy-Schwarz bound, (sum w |V|^2)
    (sum w |b_k|^2), is close to (sum w |V|^2)(sum w) l_2D at every pixel. Both within 3x. A bound with a
    factor dropped (h, or one of the sums) fails the second check."""
    tab, _ = w7
    case, hp, fft_img, dft_img = small_images
    N = case.N
    p = np.arange(-32, 32)
    l2 = _map_error_2d(tab, hp, N, p)
    w = np.ones(len(case.uv)) if case.weights is None else np.asarray(case.weights, dtype=np.float64)
    v2 = np.abs(case.vis) ** 2
    rms = np.sqrt(np.mean(np.abs(fft_img - dft_img) ** 2))
    pred = np.sqrt(l2.mean() * np.sum(w * w * v2))
    assert pred / 3 < rms < 3 * pred
    pq = np.stack(np.meshgrid(p, p, indexing="xy"), -1).reshape(-1, 2)
    bound = im.image_misfit_bound(case.uv, case.vis, case.weights, N, tab, hp, pq)
    ratio = bound / (np.sum(w * v2) * np.sum(w) * l2.reshape(-1))
    assert np.all(ratio > 1 / 3) and np.all(ratio < 3)


def test_point_sources_predict_as_a_delta_image(w7):
    """Eq. (2): a sky of point sources on pixel centres is the image with those pixels set to the fluxes, so
    the per-source sum equals the direct prediction of that image (a different evaluation of the same sum)."""
    N, x0 = 64, 0.25
    rng = np.random.default_rng(21)
    uv = rng.uniform(-16, 16, (300, 2))
    pos = rng.integers(-16, 16, (9, 2))
    flux = rng.uniform(0.1, 1.0, 9)
    img = np.zeros((32, 32), complex)
    for (px, qy), f in zip(pos, flux):
        img[qy + 16, px + 16] += f
    np.testing.assert_allclose(im.point_source_predict(uv, N, pos, flux), im.direct_predict(uv, img, N, x0),
                               rtol=0, atol=1e-12)
    # and a single unit source at the origin has V = 1 everywhere
    np.testing.assert_allclose(im.point_source_predict(uv, N, [(0, 0)], [1.0]), np.ones(300), atol=0)


def test_misfit_larger_for_smaller_width(small_images):
    """Sec. 2.2/4.1: the image misfit falls steeply with W (W = 3 far worse than W = 7)."""
    case, _, fft7, dft = small_images
    tab3, h3 = lt.make_table(3, 0.25, 300, 3)
    fft3 = im.make_dirty_image(case.uv, case.vis, case.weights, case.N, case.x0, tab3, lt.correction(h3, 3, 0.25, case.N))
    e7 = np.linalg.norm(fft7 - dft)
    e3 = np.linalg.norm(fft3 - dft)
    assert e3 > 100 * e7


def test_single_visibility_at_origin_misfit(w7):
    """Eq. (4) with one visibility at u = v = 0: misfit = 1 - h(x) c0(x) h(y) c0(y), c0(x) = sum_j C_j(0) cos 2 pi j x."""
    tab, h = w7
    N = 64
    hp = lt.correction(h, 7, 0.25, N)
    I = im.make_dirty_image(np.zeros((1, 2)), np.ones(1, complex), None, N, 0.25, tab, hp)
    x = (np.arange(32) - 16) / N
    c = tab.nodes[:, tab.Ms // 2]
    c0 = (c[None, :] * np.cos(2 * np.pi * np.outer(x, np.arange(7) - 3))).sum(1)
    hx = hp[16:48]
    expect = 1 - np.outer(hx * c0, hx * c0)
    np.testing.assert_allclose(1 - I.real, expect, atol=1e-14)
    assert np.max(np.abs(1 - I)) < 1e-6


def test_prediction_bound_and_accuracy(w7):
    """Sec. 5: FFT + degrid prediction obeys |V - V_hat|^2 <= (sum |I|^2)(sum |b_k|^2) for each visibility."""
    tab, h = w7
    case = synth.small_case()
    img = case.extra["model_image"]
    hp = lt.correction(h, 7, 0.25, case.N)
    vh = im.predict_visibilities(case.uv, img, case.N, 0.25, tab, hp)
    vd = im.direct_predict(case.uv, img, case.N, 0.25)
    p = np.arange(-32, 32)
    su = im._axis_phase_sum(case.uv[:, 0], tab, case.N, p / case.N)     # (k, p)
    sv = im._axis_phase_sum(case.uv[:, 1], tab, case.N, p / case.N)     # (k, q)
    hh = hp[32:96]
    # b_k(x_p, y_q) for the prediction: conjugate phases (forward transform); modulus is the same
    b2 = np.abs(1 - (hh[None, None, :] * su[:, None, :]) * (hh[None, :, None] * sv[:, :, None])) ** 2
    bound = np.sum(np.abs(img) ** 2) * b2.reshape(len(vh), -1).sum(1)
    assert np.all(np.abs(vh - vd) ** 2 <= bound * (1 + 1e-9))
    assert np.linalg.norm(vh - vd) / np.linalg.norm(vd) < 1e-5


def test_table_rate_trend_nearest_neighbour():
    """Sec. 6.1 table: nearest-neighbour visibility misfit falls about tenfold per decade of M_s.

    Sky: the paper's 34-source test card (App. D). The uv coverage is a
    synthetic array (the VLA configuration is not reproduced), so only the
    trend is pinned, not the printed values.
    """
    card = np.loadtxt(os.path.join(GOLDEN, "testcard_34_sources.txt"))
    paper = {}
    for line in open(os.path.join(GOLDEN, "nn_visibility_misfit.txt")):
        if not line.startswith("#") and line.split()[0].isdigit():
            paper[int(line.split()[0])] = float(line.split()[1])
    N, x0, W = 2048, 0.25, 7
    uvl = synth.array_tracks(9, 4)
    uv = uvl * synth.cell_scale(uvl, N, W)
    pos = card[:, 1:3].astype(int)
    flux = card[:, 3]
    truth = im.point_source_predict(uv, N, pos, flux)
    h = lt.optimal_h(W, x0)
    hp = lt.correction(h, W, x0, N)
    img = np.zeros((1024, 1024), complex)
    img[pos[:, 1] + 512, pos[:, 0] + 512] = flux
    Ghat = im.grid_from_image(img, hp, N, x0)
    rms = {}
    for Ms in (100, 1000, 10000):
        tab = lt.Table(W, x0, Ms, 0, lt.table_nodes(h, W, x0, Ms, 0))
        rms[Ms] = np.sqrt(np.mean(np.abs(im.degrid(uv, Ghat, tab) - truth) ** 2)) / np.sqrt(np.mean(np.abs(truth) ** 2))
    for a, b in ((100, 1000), (1000, 10000)):
        ours = rms[a] / rms[b]
        theirs = paper[a] / paper[b]
        assert 0.5 * theirs < ours < 2.0 * theirs


def test_grid_cells_equals_full_grid(w7):
    """The sampled-cell form of Eq. (5) used for large-grid checks equals the full scatter."""
    tab, _ = w7
    N = 64
    rng = np.random.default_rng(12)
    uv = rng.uniform(-34, 34, (500, 2))
    V = rng.standard_normal(500) + 1j * rng.standard_normal(500)
    w = rng.uniform(0.1, 2.0, 500)
    G = im.grid(uv, V, w, N, tab)
    cells = [(0, 0), (1, 63), (32, 32), (40, 17), (63, 2)]
    np.testing.assert_allclose(im.grid_cells(uv, V, w, N, tab, cells), [G[r, c] for r, c in cells], rtol=1e-13, atol=1e-13)


def test_exact_kernel_gridding_matches_a_fine_table():
    """Direct calculation (Sec. 6): gridding and degridding with the exact kernel at every offset agree with a
    cubic table so fine (M_s = 20,000) that its interpolation error is below 1e-14, through the table's own
    lookup code (App. F); an independent path for the weights."""
    W, x0, N = 7, 0.25, 64
    h = lt.optimal_h(W, x0)
    ek = lt.ExactKernel(W, x0, h)
    fine, _ = lt.make_table(W, x0, W * 20000, 3, h)
    rng = np.random.default_rng(6)
    uv = rng.uniform(-12, 12, (300, 2))
    vis = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    a, b = im.grid(uv, vis, None, N, ek), im.grid(uv, vis, None, N, fine)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-12
    G = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    va, vb = im.degrid(uv, G, ek), im.degrid(uv, G, fine)
    assert np.linalg.norm(va - vb) / np.linalg.norm(vb) < 1e-12
