"""Pins for the oracle's least-misfit table machinery (CPU only).

Each test checks the oracle against something the paper or mathematics fixes,
not against a retyped copy of the same formula.
"""
import os

import numpy as np
import pytest

from oracle import lmtable as lt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def paper_value(key):
    for line in open(os.path.join(GOLDEN, "paper_values.txt")):
        if line.startswith(key + " "):
            return float(line.split()[1])
    raise KeyError(key)


def true_ell(W, x0, xs, h=None):
    """l(x) of Eq. (11) with the exact kernel and the optimal correction, accurate nu quadrature."""
    hc = lt.optimal_h(W, x0) if h is None else h
    ell, hx, c, D = lt.map_error(lambda d: lt.kernel_from_h(hc, W, x0, d), W, xs)
    return ell, hx, c, D


# ------------------------------------------------------ closed forms ---
def test_box_kernel_closed_form():
    """C1 (nearest neighbour box): h = sinc x, l = 1 - sinc^2 x (from Eqs. 12-15; Sec. 2.2 list item 1)."""
    x = np.linspace(0.0, 0.5, 41)
    ell, h, c, D = lt.map_error(lambda d: np.ones((1, len(d))), 1, x)
    s = np.sinc(x)
    np.testing.assert_allclose(c, s, atol=1e-13)
    np.testing.assert_allclose(D, 1.0, atol=1e-13)            # sum_n sinc^2(x - n) = 1 (Eq. 14)
    np.testing.assert_allclose(h, s, atol=1e-13)
    np.testing.assert_allclose(ell, 1.0 - s * s, atol=1e-13)


def test_triangle_kernel_closed_form():
    """C2 (linear interpolation), W = 2: c = sinc^2, D = 2/3 + cos(2 pi x)/3 (Eq. 14), h = c / D."""
    x = np.linspace(0.0, 0.5, 41)
    taps = lambda d: np.vstack([1.0 - d, d])      # C(0 - d) = 1 - d, C(1 - d) = d for d in (0, 1]
    ell, h, c, D = lt.map_error(taps, 2, x)
    s2 = np.sinc(x) ** 2
    den = 2.0 / 3.0 + np.cos(2 * np.pi * x) / 3.0
    np.testing.assert_allclose(c, s2, atol=1e-13)
    np.testing.assert_allclose(D, den, atol=1e-13)
    np.testing.assert_allclose(h, s2 / den, atol=1e-13)
    np.testing.assert_allclose(ell, 1.0 - s2 * s2 / den, atol=1e-13)


def test_aliased_sum_identity_least_misfit():
    """Eq. (14): the nu-integral denominator equals sum_n c(x - n)^2, with c the Fourier transform (Eq. 13)."""
    W, x0 = 5, 0.25
    h = lt.optimal_h(W, x0)
    taps = lambda d: lt.kernel_from_h(h, W, x0, d)
    x = np.linspace(0.0, 0.45, 4)
    _, _, _, D = lt.map_error(taps, W, x)
    n = np.arange(-150, 151)
    _, _, cshift, _ = lt.map_error(taps, W, (x[:, None] - n[None, :]).ravel(), nquad=1024)
    alias = (cshift.reshape(len(x), len(n)) ** 2).sum(axis=1)
    np.testing.assert_allclose(alias, D, rtol=0, atol=1e-7)
    assert np.all(alias > cshift.reshape(len(x), len(n))[:, 150] ** 2)   # the aliased copies add


def test_map_error_identity_at_optimum():
    """Sec. 3, Eq. (20): with the optimal h, l(x) = 1 - h(x) c(x)."""
    W, x0 = 7, 0.25
    x = np.linspace(0.0, 0.5, 51)
    ell, h, c, D = true_ell(W, x0, x)
    np.testing.assert_allclose(ell, 1.0 - h * c, atol=2e-15)


# ------------------------------------------------ least-misfit optimum ---
def test_w7_reaches_single_precision_level():
    """Secs. 2.2 and 3: at W = 7, x0 = 0.25 the map error over |x| <= x0 is of order 1e-14.

    Reading: the optimiser minimises E, the mean of l over the field (Eq. 16),
    and that minimum is 1.46-1.49e-14 under every fair reading of App. A tried
    (N_g = 32 or 64, M_g = 16 or 32); since max l >= mean l, no reading puts l
    below 1e-14 over the whole field, so the printed "less than 1e-14" is an
    order of magnitude (the same paragraph says l "at" 1e-14). Pinned here to
    the level the optimum reaches, tightly enough that an optimiser stopping at
    twice the minimal E fails: E and the mean of l within [1, 2] x 1e-14, the
    median below 1.5e-14, the edge value l(x0) (the maximum, 1.83e-13) below
    2.5e-13.
    """
    level = paper_value("ell_level_W7_x0_0.25")
    x = np.linspace(0.0, 0.25, 501)
    ell, _, _, _ = true_ell(7, 0.25, x)
    E = lt.integrated_misfit_coarse(lt.optimal_h(7, 0.25), 7, 0.25)
    assert level < E < 2 * level
    assert level < ell.mean() < 2 * level
    assert level / 10 < np.median(ell) < 1.5 * level
    assert ell.max() == ell[-1] and ell.max() < 2.5e-13
    # W = 6 does not reach that level; W = 8 goes well below it (Sec. 2.2: W = 7 is the smallest choice)
    ell6, _, _, _ = true_ell(6, 0.25, x)
    assert np.median(ell6) > 10 * level


def test_w7_optimum_is_a_local_minimum_of_E():
    """App. A: h minimises E. At the optimiser's h, moving the 32 free samples by a relative 1e-8 along random
    directions raises E by the same amount in both senses (no first-order term: the gradient vanishes). An h
    with twice the minimal E has a gradient whose first-order change (~2.6e-2 E here) would swamp the
    second-order rise (~1.7e-4 E) and lower E on one side."""
    W, x0 = 7, 0.25
    h = lt.optimal_h(W, x0)
    E0 = lt.integrated_misfit_coarse(h, W, x0)
    rng = np.random.default_rng(17)
    eps = 1e-8
    for _ in range(6):
        d = rng.standard_normal(32)
        d /= np.linalg.norm(d)
        up, dn = h.copy(), h.copy()
        up[1:] *= 1 + eps * d
        dn[1:] *= 1 - eps * d
        rp = lt.integrated_misfit_coarse(up, W, x0) / E0 - 1
        rm = lt.integrated_misfit_coarse(dn, W, x0) / E0 - 1
        assert rp > 1e-6 and rm > 1e-6
        assert abs(rp - rm) < 0.05 * (rp + rm)


def test_misfit_falls_with_width_and_with_x0():
    """Sec. 2.2: E falls as W rises and as x0 falls (more of the image is discarded)."""
    E = [lt.integrated_misfit_coarse(lt.optimal_h(W, 0.25), W, 0.25) for W in range(1, 8)]
    assert all(a > 10 * b for a, b in zip(E[:-1], E[1:]))
    Ex = [lt.integrated_misfit_coarse(lt.optimal_h(6, x0), 6, x0) for x0 in (0.2, 0.25, 0.3)]
    assert Ex[0] < Ex[1] < Ex[2]


@pytest.mark.parametrize("W", [3, 5, 7])
def test_correction_fixed_point(W):
    """Envelope theorem at the optimum of App. A: h_i = c(x_i) / D(x_i) with the M_g-point nu sums (Eq. 12)."""
    x0 = 0.25
    h = lt.optimal_h(W, x0)
    x, _ = lt.coarse_x(x0)
    nu = lt.nu_grid()
    C = lt.kernel_from_h(h, W, x0, nu)
    t = lt.tap_offsets(W)
    S = np.einsum("jm,jmi->mi", C, np.exp(2j * np.pi * (t[:, None, None] - nu[None, :, None]) * x[None, None, :]))
    c = S.real.mean(axis=0)
    D = (np.abs(S) ** 2).mean(axis=0)
    np.testing.assert_allclose(h, c / D, rtol=5e-9)


def test_qr_optimum_keeps_falling_past_w11():
    """App. B: with the kernel solved by QR from W = 12, the optimised misfit keeps falling with W (Sec. 2.2),
    to sqrt(E) ~ 1e-14 at W = 14, FP64's limit; the normal-equation solve departs from QR there by
    cond(A) eps (5e-10 at W = 12), enough to stall the optimiser."""
    E = {W: lt.integrated_misfit_coarse(lt.optimal_h(W, 0.25), W, 0.25) for W in (11, 12, 13, 14)}
    assert E[11] > 10 * E[12] > 100 * E[13] > 1000 * E[14]
    assert np.sqrt(E[14]) < 1e-13
    h = lt.optimal_h(12, 0.25)
    d = np.linspace(-0.5, 0.5, 9)
    diff = np.max(np.abs(lt.kernel_from_h(h, 12, 0.25, d) - lt.kernel(h, 12, 0.25, d)))
    assert 1e-12 < diff < 1e-15 * np.linalg.cond(lt.normal_matrix(h, 12, 0.25)) * 100


@pytest.mark.parametrize("W", [2, 3, 5, 7, 9])
def test_correction_shape(W):
    """h(0) = 1 and h increases on [0, x0] for W >= 2 (App. A; Sec. 3)."""
    h = lt.optimal_h(W, 0.25)
    assert h[0] == 1.0
    assert np.all(np.diff(h) > 0)


@pytest.mark.parametrize("W", [3, 5, 7, 9, 11])
def test_normal_equations_match_qr(W):
    """App. B: the QR least-squares solution equals the A-matrix solution (rounding scaled by cond A)."""
    x0 = 0.25
    h = lt.optimal_h(W, x0) if W <= 7 else np.linspace(1.0, 2.0 + 0.3 * W, 33)
    d = np.linspace(-0.5, 0.5, 11)
    ca = lt.kernel_from_h(h, W, x0, d)
    cq = lt.kernel_qr(h, W, x0, d)
    cond = np.linalg.cond(lt.normal_matrix(h, W, x0))
    assert np.max(np.abs(ca - cq)) < 1e-15 * cond * 100


def test_kernel_symmetry():
    """C is real and even (Sec. 1, condition (ii)): C(t_j - d) = C(t_{W-1-j} + d)."""
    for W in (3, 4, 7):
        h = lt.optimal_h(W, 0.25)
        d = np.linspace(-0.5, 0.5, 9) if W % 2 else np.linspace(0.0, 1.0, 9)
        c = lt.kernel_from_h(h, W, 0.25, d)
        if W % 2:
            c_m = lt.kernel_from_h(h, W, 0.25, -d)
            np.testing.assert_allclose(c, c_m[::-1, :], atol=1e-13)
        else:   # even W: offsets (0, 1]; reflection maps d -> 1 - d and tap j -> W-1-j... within the branch
            c_m = lt.kernel_from_h(h, W, 0.25, 1.0 - d)
            np.testing.assert_allclose(c, c_m[::-1, :], atol=1e-13)


def test_small_width_shapes():
    """App. C: W=1 is ~1 on |u|<1/2 and larger at the grid point than midway; W=2 is close to, but not,
    1-|u|; W=3 has visible jumps at |u| = 1/2 and 3/2; for W >= 4 the edge values are very small."""
    h1 = lt.optimal_h(1, 0.25)
    c1 = lt.kernel_from_h(h1, 1, 0.25, np.array([0.0, 0.49]))[0]
    assert abs(c1[0] - 1) < 0.1 and c1[0] > c1[1]
    h2 = lt.optimal_h(2, 0.25)
    d = np.linspace(0.01, 0.99, 50)
    c2 = lt.kernel_from_h(h2, 2, 0.25, d)       # tap 0 is C(-d), tap 1 is C(1-d)
    dev = np.max(np.abs(c2[0] - (1 - d)))
    assert 1e-3 < dev < 0.2
    h3 = lt.optimal_h(3, 0.25)
    top = lt.kernel_from_h(h3, 3, 0.25, np.array([0.5]))[:, 0]     # u just below a half-integer
    bot = lt.kernel_from_h(h3, 3, 0.25, np.array([-0.5]))[:, 0]    # the same u from the other tap set
    # tap j at delta=+1/2 and tap j+1 at delta=-1/2 sit at the same distance from the visibility
    jumps = np.abs(top[:-1] - bot[1:])
    assert jumps.max() > 1e-3
    for W in (4, 5, 7):
        hW = lt.optimal_h(W, 0.25)
        edge = lt.kernel_from_h(hW, W, 0.25, np.array([0.5 if W % 2 else 1.0]))[:, 0]
        centre = lt.kernel_from_h(hW, W, 0.25, np.array([0.0 if W % 2 else 0.5]))[:, 0]
        assert abs(edge[0]) < 0.05 * np.max(np.abs(centre))      # tap 0 at the top offset sits at u = -W/2


# ---------------------------------------------------------- look-up table ---
def test_interpolation_exact_on_polynomials():
    """Newton forward interpolation of degree d reproduces polynomials of degree d (App. F)."""
    W, Ms = 3, 10
    deltas = -0.5 + np.arange(Ms + 4) / Ms
    rng = np.random.default_rng(0)
    q = rng.standard_normal((W, 4))
    poly = lambda d: np.array([np.polyval(q[j], d) for j in range(W)])
    nodes = poly(deltas)
    d = rng.uniform(-0.5, 0.5, 200)
    np.testing.assert_allclose(lt.interpolate(nodes, W, Ms, 3, d), poly(d), atol=1e-12)
    lin = np.array([np.polyval(q[j, 2:], deltas) for j in range(W)])
    np.testing.assert_allclose(lt.interpolate(lin, W, Ms, 1, d), np.array([np.polyval(q[j, 2:], d) for j in range(W)]), atol=1e-13)


def test_nearest_neighbour_rule():
    """Degree 0 returns the closest node, ties to the upper node (App. F)."""
    W, Ms = 1, 4
    nodes = np.arange(Ms + 1, dtype=float)[None, :]   # node i has value i at delta = -1/2 + i/4
    d = np.array([-0.5, -0.38, -0.375, -0.3, 0.124, 0.125, 0.5])
    np.testing.assert_array_equal(lt.interpolate(nodes, W, Ms, 0, d)[0], [0, 0, 1, 1, 2, 3, 4])


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
def test_interpolation_error_order(degree):
    """App. F: table error is O(M_s^-(d+1)) (nearest neighbour: O(1/M_s))."""
    W, x0 = 7, 0.25
    h = lt.optimal_h(W, x0)
    d = np.random.default_rng(1).uniform(-0.5, 0.5, 400)
    exact = lt.kernel_from_h(h, W, x0, d)
    errs = []
    for Ms in (40, 80):
        nodes = lt.table_nodes(h, W, x0, Ms, degree)
        errs.append(np.max(np.abs(lt.interpolate(nodes, W, Ms, degree, d) - exact)))
    ratio = errs[0] / errs[1]
    assert 2 ** (degree + 1) * 0.6 < ratio < 2 ** (degree + 1) * 1.6


def test_rms_bound_rates_with_table():
    """App. F: sqrt(E) with a tabulated kernel approaches the exact floor as M_s^-(d+1);
    nearest neighbour needs M_s ~ 1e6 and linear ~ 1e3 to reach the W = 7 floor."""
    W, x0 = 7, 0.25
    h = lt.optimal_h(W, x0)
    x = np.linspace(0.0, x0, 201)
    hopt = lt.correction(h, W, x0, 400)[200:301]          # x_p = p/400 for p = 0..100
    floor = np.sqrt(np.mean(true_ell(W, x0, x)[0]))

    def rms(Ms, degree):
        nodes = lt.table_nodes(h, W, x0, Ms, degree)
        ell, _, _, _ = lt.map_error(lambda d: lt.interpolate(nodes, W, Ms, degree, d), W, x[::2],
                                    h_of_x=hopt, nquad=4096 if degree == 0 else 512)
        return np.sqrt(np.mean(ell))

    lin = [rms(m, 1) - floor for m in (100, 200)]
    assert 3.0 < lin[0] / lin[1] < 5.5                     # ~ M_s^-2
    assert rms(int(paper_value("linear_rate_single_precision_W7")) * 4, 1) < 3 * floor
    def rms_nn(Ms):
        nodes = lt.table_nodes(h, W, x0, Ms, 0)
        ell, _, _, _ = lt.map_error(lambda d: lt.interpolate(nodes, W, Ms, 0, d), W, x[::4], h_of_x=hopt[::2],
                                    quad=lt.composite_midpoint(-0.5, 0.5, 8 * Ms))
        return np.sqrt(np.mean(ell))

    nn = [rms_nn(m) for m in (1000, 10000)]
    assert 5 < nn[0] / nn[1] < 20                          # ~ M_s^-1
    assert rms_nn(10000) > 10 * floor                      # nearest neighbour far from the floor at 1e4


def test_table_node_lattice_and_tie_values():
    """App. E lattice: W=7, T=300 gives M_s = 42; node M_s/2 of each tap is the exact kernel at delta = 0."""
    tab, h = lt.make_table(7, 0.25, 300, 3)
    assert tab.Ms == 42 and tab.nodes.shape == (7, 46)
    np.testing.assert_allclose(tab.nodes[:, 21], lt.kernel_from_h(h, 7, 0.25, np.array([0.0]))[:, 0], atol=0)
    np.testing.assert_allclose(tab.nodes[:, ::-1][::-1, 3:], tab.nodes[:, :43], atol=1e-13)   # even kernel
