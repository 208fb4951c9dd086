"""Prolate spheroidal gridding function (alpha = 1), FP64 (oracle): the comparison system of the paper.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``). Nothing in the
library uses this kernel; it is the conventional gridding function the paper
measures the least-misfit functions against (Sec. 1, where the spheroidal
family with weighting exponent alpha is introduced; Sec. 2.2, map error for
W = 6 .. 14; Sec. 4, alias suppression).

Definition used (readings where the paper leaves a choice):

* For support W (cells) the gridding function is C(u) = (1 - eta^2) psi(eta)
  with eta = 2 u / W for |u| < W/2 and zero outside, where psi is the
  alpha = 1 spheroidal function of concentration c = pi W / 2: the solution
  of the weighted finite Fourier transform eigenproblem
  int_{-1}^{1} exp(i c x eta) (1 - eta^2) psi(eta) d eta = lambda psi(x).
* psi = S_11(c, eta) / sqrt(1 - eta^2), with S_11 the prolate spheroidal
  angular function of the first kind of order 1 and degree 1 (scipy's
  ``pro_ang1``); so C(u) = sqrt(1 - eta^2) S_11(c, eta). The overall scale of
  C is irrelevant: the correction (Eq. 12) divides it out.
* The correction is the optimal one of Eq. 12 (as for the least-misfit
  kernels), evaluated with ``lmtable.map_error``.
"""
from __future__ import annotations

import numpy as np
from scipy import special

from . import lmtable as lt


def concentration(W: int) -> float:
    """c = pi W / 2: support W cells, the whole map |x| < 1/2 as the concentration interval."""
    return np.pi * W / 2.0


def psi(W: int, eta) -> np.ndarray:
    """The alpha = 1 spheroidal function psi(eta) = S_11(c, eta) / sqrt(1 - eta^2), |eta| < 1."""
    eta = np.atleast_1d(np.asarray(eta, dtype=np.float64))
    c = concentration(W)
    s = np.array([special.pro_ang1(1, 1, c, e)[0] for e in eta])
    return s / np.sqrt(1.0 - eta * eta)


def kernel(W: int, u) -> np.ndarray:
    """C(u) = (1 - eta^2) psi(eta), eta = 2 u / W, zero for |u| >= W / 2."""
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    eta = 2.0 * u / W
    out = np.zeros_like(u)
    inside = np.abs(eta) < 1.0
    out[inside] = (1.0 - eta[inside] ** 2) * psi(W, eta[inside])
    return out


def taps(W: int, delta) -> np.ndarray:
    """C(t_j - delta) for the W taps (same tap set and offset convention as ``lmtable``), W x n."""
    t = lt.tap_offsets(W)
    d = np.atleast_1d(np.asarray(delta, dtype=np.float64))
    return kernel(W, (t[:, None] - d[None, :]).ravel()).reshape(W, len(d))


def map_error(W: int, x, nquad: int = 128):
    """l(x), h(x), c(x), D(x) of the spheroidal kernel with its optimal correction (Eqs. 11-14)."""
    return lt.map_error(lambda d: taps(W, d), W, np.asarray(x, dtype=np.float64), nquad=nquad)


def table(W: int, Ms: int, degree: int) -> lt.Table:
    """An oracle look-up table of the spheroidal kernel on the same node lattice as ``lmtable.table_nodes``
    (nodes past the interval's top continue the kernel, zero beyond the support)."""
    deltas = lt.delta_low(W) + np.arange(Ms + 1 + degree, dtype=np.float64) / Ms
    return lt.Table(W, 0.5, Ms, degree, taps(W, deltas))


def correction(W: int, N: int) -> np.ndarray:
    """Optimal correction h(x_p) of the spheroidal kernel at x_p = p / N, p = -N/2 .. N/2 - 1 (Eq. 12)."""
    xp = (np.arange(N, dtype=np.float64) - N // 2) / N
    _, h, _, _ = map_error(W, xp)
    return h
