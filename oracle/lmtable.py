"""Least-misfit gridding and correcting functions, FP64 (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Paper: Ye, Gull, Tan & Nikolic (2019), Sec. 2.1 and Appendices A, B, E, F.
Numbering of equations follows the paper's main text: (10) map error as a sum
over visibilities, (11) its integral form over the fractional offset nu,
(12)-(15) optimal correction, (16) integrated misfit E, (17)-(19) normal
equations A C(nu) = B(nu).

Conventions used here (readings where the paper leaves a choice):

* A visibility at coordinate u (in grid cells) is spread onto the W cells
  n_first .. n_first+W-1 with n_first = ceil(u - W/2); this is exactly the set
  S_k of Sec. 2.1, Eq. (6).
* The offset of the visibility from the reference tap is
  ``delta = u - (n_first + ref)`` with ref = (W-1)/2 (odd W) or W/2-1 (even W).
  It lies in (-1/2, 1/2] for odd W and in (0, 1] for even W. Tap j then sits
  at ``t_j - delta`` from the visibility, with t_j = j - ref. In the paper's
  notation (Eq. 9) this is r - nu with r = t_j (nu <= 1/2) or r = t_j + 1
  (nu > 1/2); the two descriptions give the same C values because C is even
  and A depends only on r' - r.
* h is represented on N_g+1 equally spaced points of [0, x0] (App. A) with
  h(0) = 1 fixed (E is unchanged by h -> a h, C -> C / a).
"""
from __future__ import annotations

import functools
from dataclasses import dataclass

import numpy as np
from scipy import linalg, optimize

NG_DEFAULT = 32   # N_g, App. A
MG_DEFAULT = 16   # M_g, App. A


# ---------------------------------------------------------------- geometry --
def tap_reference(W: int) -> float:
    """Offset of the reference tap from n_first: (W-1)/2 (odd W), W/2-1 (even W)."""
    return (W - 1) / 2.0 if W % 2 else W / 2.0 - 1.0


def tap_offsets(W: int) -> np.ndarray:
    """t_j = j - ref for j = 0..W-1 (the r-set of Sec. 2.1, Eq. 9, for nu <= 1/2)."""
    return np.arange(W, dtype=np.float64) - tap_reference(W)


def delta_low(W: int) -> float:
    """Lower end of the offset interval: -1/2 (odd W) or 0 (even W)."""
    return -0.5 if W % 2 else 0.0


def coarse_x(x0: float, Ng: int = NG_DEFAULT):
    """x_i = i x0 / N_g, i = 0..N_g, with trapezoid weights on [0, x0] (App. A, steps 1, 2, 4)."""
    x = np.arange(Ng + 1, dtype=np.float64) * (x0 / Ng)
    tau = np.full(Ng + 1, x0 / Ng)
    tau[0] *= 0.5
    tau[-1] *= 0.5
    return x, tau


def nu_grid(Mg: int = MG_DEFAULT) -> np.ndarray:
    """M_g equally spaced points inside (0, 1/2) (App. A): the cell midpoints (m - 1/2)/(2 M_g)."""
    return (np.arange(1, Mg + 1, dtype=np.float64) - 0.5) / (2.0 * Mg)


# ------------------------------------------------------- normal equations --
def normal_matrix(h: np.ndarray, W: int, x0: float, Ng: int = NG_DEFAULT) -> np.ndarray:
    """A_{r'r} = int_{-x0}^{x0} h(x)^2 cos(2 pi (r'-r) x) dx  (Eq. 19), trapezoid rule.

    h is even, so the symmetric integral is twice the [0, x0] trapezoid sum.
    """
    x, tau = coarse_x(x0, Ng)
    t = tap_offsets(W)
    diff = t[:, None] - t[None, :]
    return 2.0 * np.einsum("i,abi->ab", tau * h * h, np.cos(2 * np.pi * diff[:, :, None] * x))


def normal_rhs(h: np.ndarray, W: int, x0: float, delta, Ng: int = NG_DEFAULT) -> np.ndarray:
    """B_{r'}(nu) = int_{-x0}^{x0} h(x) cos(2 pi (r' - nu) x) dx  (Eq. 18), as a W x n array over delta."""
    x, tau = coarse_x(x0, Ng)
    t = tap_offsets(W)
    d = np.atleast_1d(np.asarray(delta, dtype=np.float64))
    arg = (t[:, None] - d[None, :])[:, :, None] * x
    return 2.0 * np.einsum("i,jdi->jd", tau * h, np.cos(2 * np.pi * arg))


def kernel_from_h(h: np.ndarray, W: int, x0: float, delta, Ng: int = NG_DEFAULT) -> np.ndarray:
    """Exact least-misfit kernel: C(t_j - delta) = [A^{-1} B(delta)]_j  (Eq. 18), W x n.

    A is symmetric positive definite; solved by Cholesky. The same formula
    continues analytically past the ends of the offset interval.
    """
    A = normal_matrix(h, W, x0, Ng)
    B = normal_rhs(h, W, x0, delta, Ng)
    return linalg.cho_solve(linalg.cho_factor(A), B)


def kernel_qr(h: np.ndarray, W: int, x0: float, delta, Ng: int = NG_DEFAULT) -> np.ndarray:
    """The same kernel from the least-squares form of App. B: min ||d - B c|| per offset.

    The rows are the cos and sin parts at the 2 N_g + 1 symmetric samples of
    [-x0, x0], each scaled by the square root of its trapezoid weight so that
    the normal equations of this problem are exactly Eq. (18). Solved by QR
    (numpy's lstsq), never forming A.
    """
    xh, tauh = coarse_x(x0, Ng)
    hs = np.concatenate([h[:0:-1], h])
    xs = np.concatenate([-xh[:0:-1], xh])
    taus = np.concatenate([tauh[:0:-1], tauh])
    taus[Ng] = 2.0 * tauh[0]
    sw = np.sqrt(taus)
    t = tap_offsets(W)
    out = []
    for d in np.atleast_1d(np.asarray(delta, dtype=np.float64)):
        ph = 2 * np.pi * (t[None, :] - d) * xs[:, None]
        Bm = np.vstack([(sw * hs)[:, None] * np.cos(ph), (sw * hs)[:, None] * np.sin(ph)])
        dv = np.concatenate([sw, np.zeros_like(sw)])
        out.append(np.linalg.lstsq(Bm, dv, rcond=None)[0])
    return np.array(out).T


QR_MIN_W = 12   # App. B: from here the normal equations lose the kernel's accuracy (cond(A) ~ 7e7 at W = 12)


def kernel(h: np.ndarray, W: int, x0: float, delta, Ng: int = NG_DEFAULT) -> np.ndarray:
    """The least-misfit kernel, W x n: Eq. (18) by Cholesky below W = 12, App. B's QR form from W = 12."""
    if W >= QR_MIN_W:
        return kernel_qr(h, W, x0, delta, Ng)
    return kernel_from_h(h, W, x0, delta, Ng)


# --------------------------------------------------------- misfit and LM --
def _phase_sum(C: np.ndarray, W: int, nu: np.ndarray, x: np.ndarray) -> np.ndarray:
    """S(nu, x) = sum_r C_r(nu) exp(i 2 pi (r - nu) x), shape (n_nu, n_x)."""
    t = tap_offsets(W)
    return np.einsum("jm,jmi->mi", C, np.exp(2j * np.pi * (t[:, None, None] - nu[None, :, None]) * x[None, None, :]))


def misfit_residuals(hfree: np.ndarray, W: int, x0: float, Ng: int = NG_DEFAULT, Mg: int = MG_DEFAULT) -> np.ndarray:
    """Residual vector whose sum of squares is E  (App. A steps 1-4).

    rho_{i,m} = sqrt(tau_i / (x0 M_g)) (1 - h_i S(nu_m, x_i)), real and imaginary
    parts, so sum rho^2 = (1/x0) sum_i tau_i l(x_i) with l from Eq. (11) and the
    nu integral replaced by the mean over the M_g points (the (1/2, 1) half
    of the nu interval gives the complex conjugate and the same modulus).
    """
    h = np.concatenate([[1.0], hfree])
    x, tau = coarse_x(x0, Ng)
    nu = nu_grid(Mg)
    C = kernel(h, W, x0, nu, Ng)
    r = (1.0 - h[None, :] * _phase_sum(C, W, nu, x)) * np.sqrt(tau / (x0 * Mg))[None, :]
    return np.concatenate([r.real.ravel(), r.imag.ravel()])


def integrated_misfit_coarse(h: np.ndarray, W: int, x0: float, Ng: int = NG_DEFAULT, Mg: int = MG_DEFAULT) -> float:
    """E of Eq. (16) as the optimiser sees it (trapezoid in x, M_g-point mean in nu)."""
    r = misfit_residuals(h[1:] / h[0], W, x0, Ng, Mg)
    return float(r @ r)


def optimise_h(W: int, x0: float, h_init: np.ndarray, Ng: int = NG_DEFAULT, Mg: int = MG_DEFAULT) -> np.ndarray:
    """Levenberg-Marquardt minimisation of E over h_1..h_Ng (App. A; scipy's MINPACK LM)."""
    res = optimize.least_squares(
        misfit_residuals, np.asarray(h_init[1:], dtype=np.float64) / h_init[0], method="lm",
        args=(W, x0, Ng, Mg), xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=4000 * Ng)
    return np.concatenate([[1.0], res.x])


@functools.lru_cache(maxsize=None)
def _optimal_h_cached(W: int, x0: float, Ng: int, Mg: int) -> tuple:
    if W <= 4:
        init = np.ones(Ng + 1)                       # h_W = 1 for W <= 4 (App. A)
    else:
        h1 = np.array(_optimal_h_cached(W - 1, x0, Ng, Mg))
        h2 = np.array(_optimal_h_cached(W - 2, x0, Ng, Mg))
        init = h1 * h1 / h2                          # h_W = h_{W-1}^2 / h_{W-2} (App. A)
    return tuple(optimise_h(W, x0, init, Ng, Mg))


def optimal_h(W: int, x0: float, Ng: int = NG_DEFAULT, Mg: int = MG_DEFAULT) -> np.ndarray:
    """Least-misfit correcting function on the coarse grid, with App. A's initial-guess chain."""
    if W < 1:
        raise ValueError("W must be >= 1")
    return np.array(_optimal_h_cached(int(W), float(x0), int(Ng), int(Mg)))


# ------------------------------------------------- map error, correction --
def _gauss_legendre(a: float, b: float, n: int):
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * t + 0.5 * (b + a), 0.5 * (b - a) * w


def map_error(taps_at, W: int, x: np.ndarray, h_of_x=None, nquad: int = 64, delta_lo: float | None = None,
              quad=None):
    """Map error l(x) (Eq. 11), c(x) (Eq. 13), the aliased sum D(x) (Eq. 14) and h(x) (Eq. 12).

    ``taps_at(delta)`` returns the W x n array C(t_j - delta) for offsets in
    one unit interval [delta_lo, delta_lo + 1] (the integral over nu in
    (0, 1) of Eq. 11 is the integral over delta in that interval). The
    integrand is smooth inside the interval, so Gauss-Legendre with ``nquad``
    nodes is used unless explicit ``quad = (nodes, weights)`` are given (a
    piecewise-constant table needs a composite rule instead).
    If ``h_of_x`` is None the optimal h = c / D is used (Eq. 12); otherwise
    the given correction values at x (App. F uses h_opt with a tabulated C).
    Returns (ell, h, c, D).
    """
    lo = delta_low(W) if delta_lo is None else delta_lo
    d, wd = _gauss_legendre(lo, lo + 1.0, nquad) if quad is None else quad
    C = taps_at(d)
    x = np.asarray(x, dtype=np.float64)
    t = tap_offsets(W)
    S = np.zeros((len(d), len(x)), dtype=np.complex128)
    for j in range(W):
        S += C[j][:, None] * np.exp(2j * np.pi * np.outer(t[j] - d, x))
    c = wd @ S.real
    D = wd @ (np.abs(S) ** 2)
    h = c / D if h_of_x is None else np.asarray(h_of_x, dtype=np.float64)
    ell = wd @ (np.abs(1.0 - h[None, :] * S) ** 2)
    return ell, h, c, D


def composite_midpoint(lo: float, hi: float, n: int):
    """n-point midpoint rule on [lo, hi] (exact for piecewise constants on a finer lattice)."""
    d = lo + (np.arange(n) + 0.5) * (hi - lo) / n
    return d, np.full(n, (hi - lo) / n)


def correction(h_coarse: np.ndarray, W: int, x0: float, N: int, Ng: int = NG_DEFAULT, nquad: int = 64) -> np.ndarray:
    """Optimal correction h(x_p) at x_p = p/N, p = -N/2 .. N/2-1 (Eq. 12 with the exact kernel)."""
    xp = (np.arange(N, dtype=np.float64) - N // 2) / N
    _, h, _, _ = map_error(lambda d: kernel(h_coarse, W, x0, d, Ng), W, xp, nquad=nquad)
    return h


# ------------------------------------------------------- look-up tables --
def samples_per_cell(W: int, table_size: int) -> int:
    """M_s from the total entry count T = W M_s (a 300-entry W=3 table has M_s = 100, Sec. 7)."""
    return table_size // W


def table_nodes(h_coarse: np.ndarray, W: int, x0: float, Ms: int, degree: int, Ng: int = NG_DEFAULT) -> np.ndarray:
    """Tabulated kernel (App. E): for each tap j, C(t_j - delta_i) at delta_i = delta_lo + i/M_s.

    i runs over 0..M_s+degree: the nodes past the top of the interval are the
    analytic continuation of A^{-1}B, so that the forward Newton stencils of
    App. F never leave one tap's smooth branch. Shape W x (M_s + 1 + degree).
    """
    deltas = delta_low(W) + np.arange(Ms + 1 + degree, dtype=np.float64) / Ms
    return kernel(h_coarse, W, x0, deltas, Ng)


@dataclass(frozen=True)
class Table:
    """An oracle look-up table: kernel nodes plus the interpolation degree."""
    W: int
    x0: float
    Ms: int
    degree: int
    nodes: np.ndarray   # W x (Ms + 1 + degree)

    def weights(self, delta) -> np.ndarray:
        """Interpolated C(t_j - delta) for all taps, shape (n, W)."""
        return interpolate(self.nodes, self.W, self.Ms, self.degree, delta).T


@dataclass(frozen=True)
class ExactKernel:
    """Direct calculation of the weights (Sec. 6): the exact kernel at every offset, no table.

    Same interface as :class:`Table`; each call solves Eq. (18) at the given
    offsets with :func:`kernel` (Cholesky, or QR from W = 12).
    """
    W: int
    x0: float
    h: np.ndarray

    def weights(self, delta) -> np.ndarray:
        return kernel(self.h, self.W, self.x0, delta).T


def interpolate(nodes: np.ndarray, W: int, Ms: int, degree: int, delta) -> np.ndarray:
    """Kernel values from the table (App. F), W x n.

    degree 0: the nearest node, ties rounded up. degree d >= 1: the polynomial
    through nodes k..k+d with delta_k <= delta < delta_{k+1}, in Newton's
    forward-difference form f_k + t D f_k + t(t-1)/2! D^2 f_k + ... (the
    Gregory-Newton formula the paper cites from Abramowitz & Stegun).
    """
    d = np.atleast_1d(np.asarray(delta, dtype=np.float64))
    p = (d - delta_low(W)) * Ms
    if degree == 0:
        k = np.floor(p + 0.5).astype(np.int64)
        return nodes[:, k]
    k = np.floor(p).astype(np.int64)
    t = p - k
    out = nodes[:, k].copy()
    diffs = [nodes[:, k + s] for s in range(degree + 1)]
    coef = np.ones_like(t)
    for s in range(1, degree + 1):
        diffs = [diffs[i + 1] - diffs[i] for i in range(len(diffs) - 1)]   # s-th forward differences
        coef = coef * (t - (s - 1)) / s
        out = out + coef[None, :] * diffs[0]
    return out


def make_table(W: int, x0: float, table_size: int, degree: int, h_coarse: np.ndarray | None = None) -> tuple:
    """(Table, h_coarse) for the least-misfit kernel with a T-entry table."""
    h = optimal_h(W, x0) if h_coarse is None else np.asarray(h_coarse, dtype=np.float64)
    Ms = samples_per_cell(W, table_size)
    return Table(W, float(x0), Ms, int(degree), table_nodes(h, W, x0, Ms, degree)), h
