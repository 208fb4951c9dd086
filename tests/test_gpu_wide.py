"""Wide kernels (W = 12 .. 16, 16 being the widest support the library takes): tables whose kernel is
App. B's QR least-squares solution.

The library optimises h (Levenberg-Marquardt over QR-solved kernels); the
oracle builds its table from that h with its own QR solve, and the library
takes the oracle's nodes (the parity protocol of the other tests). Gridding,
degridding and the dirty image are compared at 1e-12 (FP64) and 1e-5 (FP32)
relative RMS.
"""
import numpy as np
import pytest

import synth
from oracle import imaging as im
from oracle import lmtable as lt

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1906_07102_amd as lmg  # noqa: E402

TOL = {lmg.F32: 1e-5, lmg.F32_KAHAN: 1e-5, lmg.F64: 1e-12}
DEV = "cuda:0"
_T = {}


def rel_rms(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def cdt(prec):
    return torch.complex128 if prec == lmg.F64 else torch.complex64


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device=DEV, dtype=dtype)


def wide_tables(W):
    if W not in _T:
        h, _ = lmg.Table.create(W, 0.25, 300, 3).export()
        otab, _ = lt.make_table(W, 0.25, 300, 3, h_coarse=h)
        _T[W] = (otab, lmg.Table.from_nodes(W, 0.25, 300, 3, h, otab.nodes), h)
    return _T[W]


@pytest.mark.parametrize("prec", [lmg.F32, lmg.F32_KAHAN, lmg.F64])
@pytest.mark.parametrize("W", [12, 14, 15, 16])
def test_wide_grid_degrid(prec, W):
    print(f"wide grid/degrid W={W} prec={prec}", flush=True)
    otab, gtab, _ = wide_tables(W)
    c = synth.small_case()
    plan = lmg.Plan(gtab, c.N, dev(c.uv, torch.float64), prec)
    g = plan.grid(dev(c.vis, cdt(prec))).cpu().numpy()
    assert rel_rms(g, im.grid(c.uv, c.vis, None, c.N, otab)) < TOL[prec]
    rng = np.random.default_rng(2)
    G = rng.standard_normal((c.N, c.N)) + 1j * rng.standard_normal((c.N, c.N))
    v = plan.degrid(dev(G, cdt(prec))).cpu().numpy()
    assert rel_rms(v, im.degrid(c.uv, G, otab)) < TOL[prec]


@pytest.mark.parametrize("W", [12, 14, 16])
def test_wide_dirty_image(W):
    print(f"wide dirty image W={W}", flush=True)
    otab, gtab, h = wide_tables(W)
    c = synth.small_case()
    plan = lmg.Plan(gtab, c.N, dev(c.uv, torch.float64), lmg.F64)
    img = plan.make_dirty_image(dev(c.vis, torch.complex128)).cpu().numpy()
    ref = im.make_dirty_image(c.uv, c.vis, None, c.N, 0.25, otab, lt.correction(h, W, 0.25, c.N))
    assert rel_rms(img, ref) < 1e-12
