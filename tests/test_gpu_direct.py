"""Direct calculation of the weights (Sec. 6): the library evaluates the exact kernel per visibility.

The library table comes from lmg_table_create_direct on a table built from
the oracle's h; the oracle grids with :class:`oracle.lmtable.ExactKernel`
(Eq. 18 solved at every offset). Tolerances are those of the table path:
relative RMS 1e-12 in FP64 and 1e-5 in FP32. The device evaluates the
kernel from the 33-term expansion of A^{-1} B in FP64; its rounding relative
to the oracle's Cholesky solve is about cond(A) eps (cond(A) is 1e4 at W = 7),
a few 1e-13 at worst on single weights and well below the FP64 tolerance in
the RMS over a grid.
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
PRECS = [lmg.F32, lmg.F32_KAHAN, lmg.F64]
DEV = "cuda:0"
_T = {}


def rel_rms(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def cdt(prec):
    return torch.complex128 if prec == lmg.F64 else torch.complex64


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device=DEV, dtype=dtype)


def direct_tables(W, x0=0.25):
    """(oracle exact kernel, library direct table, library tabulated table, oracle table, h)."""
    if (W, x0) not in _T:
        otab, h = lt.make_table(W, x0, 300, 3)
        tab = lmg.Table.from_nodes(W, x0, 300, 3, h, otab.nodes)
        _T[(W, x0)] = (lt.ExactKernel(W, x0, h), tab.direct_calculation(), tab, otab, h)
    return _T[(W, x0)]


def mid_case(seed, nvis, N, W):
    """Uniform uv over the central half, a count that leaves ragged tiles and items."""
    rng = np.random.default_rng(seed)
    uv = rng.uniform(-N / 4 + W, N / 4 - W, (nvis, 2))
    vis = rng.standard_normal(nvis) + 1j * rng.standard_normal(nvis)
    w = rng.uniform(0.5, 2.0, nvis).astype(np.float32)
    return uv, vis, w


def test_direct_table_reports_itself():
    _, dtab, tab, _, _ = direct_tables(7)
    assert dtab.direct and not tab.direct
    assert (dtab.W, dtab.x0) == (tab.W, tab.x0)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("W", [7, 5, 4, 3])
def test_direct_grid_degrid_small(prec, W):
    print(f"direct grid/degrid prec={prec} W={W}", flush=True)
    ek, dtab, _, _, _ = direct_tables(W)
    c = synth.small_case()
    N = c.N
    plan = lmg.Plan(dtab, N, dev(c.uv, torch.float64), prec)
    g = plan.grid(dev(c.vis, cdt(prec)), dev(c.weights, torch.float32) if c.weights is not None else None)
    ref = im.grid(c.uv, c.vis, c.weights, N, ek)
    assert rel_rms(g.cpu().numpy(), ref) < TOL[prec]
    rng = np.random.default_rng(4)
    G = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    v = plan.degrid(dev(G, cdt(prec))).cpu().numpy()
    assert rel_rms(v, im.degrid(c.uv, G, ek)) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_direct_ragged_tiles_and_items(prec):
    """30,011 visibilities on 256^2 with W = 7 and items capped at 97 visibilities: many tiles, split items,
    ragged tails."""
    import os
    print(f"direct ragged prec={prec}", flush=True)
    ek, dtab, _, _, _ = direct_tables(7)
    uv, vis, w = mid_case(12, 30011, 256, 7)
    old = os.environ.get("LMG_CAP")
    os.environ["LMG_CAP"] = "97"
    try:
        plan = lmg.Plan(dtab, 256, dev(uv, torch.float64), prec)
    finally:
        if old is None:
            os.environ.pop("LMG_CAP", None)
        else:
            os.environ["LMG_CAP"] = old
    g = plan.grid(dev(vis, cdt(prec)), dev(w, torch.float32)).cpu().numpy()
    assert rel_rms(g, im.grid(uv, vis, w.astype(np.float64), 256, ek)) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_direct_dirty_image_and_prediction(prec):
    print(f"direct image/predict prec={prec}", flush=True)
    ek, dtab, _, _, h = direct_tables(7)
    c = synth.small_case()
    hp = lt.correction(h, 7, 0.25, c.N)
    plan = lmg.Plan(dtab, c.N, dev(c.uv, torch.float64), prec)
    img = plan.make_dirty_image(dev(c.vis, cdt(prec))).cpu().numpy()
    assert rel_rms(img, im.make_dirty_image(c.uv, c.vis, None, c.N, 0.25, ek, hp)) < TOL[prec]
    model = c.extra["model_image"]
    out = plan.predict_visibilities(dev(model, cdt(prec))).cpu().numpy()
    assert rel_rms(out, im.predict_visibilities(c.uv, model, c.N, 0.25, ek, hp)) < TOL[prec]


def test_direct_no_worse_than_table_against_dft():
    """Against the direct DFT (Eq. 3) the exact kernel leaves the method's misfit alone: in FP64 its error
    is at most the tabulated kernel's (which adds the table's interpolation error), up to rounding."""
    ek, dtab, tab, _, _ = direct_tables(7)
    c = synth.small_case()
    dft = im.dft_dirty_image(c.uv, c.vis, None, c.N, 0.25)
    errs = {}
    for name, t in (("direct", dtab), ("table", tab)):
        plan = lmg.Plan(t, c.N, dev(c.uv, torch.float64), lmg.F64)
        errs[name] = rel_rms(plan.make_dirty_image(dev(c.vis, torch.complex128)).cpu().numpy(), dft)
    print(f"dirty image vs DFT: direct {errs['direct']:.4e}  table {errs['table']:.4e}", flush=True)
    assert errs["direct"] <= errs["table"] * (1 + 1e-6) + 1e-14


def test_direct_full_size_sampled():
    """16.8M array visibilities on 4096^2, FP32 accumulation: sampled cells and visibilities vs the oracle."""
    print("direct full size", flush=True)
    c = synth.array_16m_case(with_vis=False)
    ek, dtab, _, _, _ = direct_tables(7)
    rng = np.random.default_rng(8)
    vis = (rng.standard_normal(len(c.uv)) + 1j * rng.standard_normal(len(c.uv))).astype(np.complex64)
    plan = lmg.Plan(dtab, c.N, dev(c.uv, torch.float64), lmg.F32)
    g = plan.grid(dev(vis, torch.complex64))
    k = rng.integers(0, len(c.uv), 16)
    nf = np.ceil(c.uv[k] - 3.5).astype(np.int64) + rng.integers(0, 7, (16, 2))
    cells = [((int(b) + c.N // 2) % c.N, (int(a) + c.N // 2) % c.N) for a, b in nf]
    got = np.array([g[r, cc].item() for r, cc in cells])
    ref = im.grid_cells(c.uv, vis.astype(np.complex128), None, c.N, ek, cells)
    assert rel_rms(got, ref) < 1e-5
    G = np.zeros((c.N, c.N), np.complex64)
    band = slice(c.N // 4 - 8, 3 * c.N // 4 + 8)
    G[band, band] = rng.standard_normal(G[band, band].shape) + 1j * rng.standard_normal(G[band, band].shape)
    out = plan.degrid(dev(G, torch.complex64))
    sel = rng.integers(0, len(c.uv), 1000)
    assert rel_rms(out[sel].cpu().numpy(), im.degrid(c.uv[sel], G.astype(np.complex128), ek)) < 1e-5


def test_direct_batched_channels():
    """A direct table in a batched plan: each of 5 uneven channels against the oracle's exact kernel (FP64)."""
    ek, dtab, _, _, _ = direct_tables(5)
    rng = np.random.default_rng(17)
    counts = np.array([700, 0, 1, 2500, 333])
    off = np.concatenate([[0], np.cumsum(counts)])
    N = 128
    uv = rng.uniform(-N / 4, N / 4, (int(off[-1]), 2))
    vis = rng.standard_normal(len(uv)) + 1j * rng.standard_normal(len(uv))
    plan = lmg.BatchPlan(dtab, N, dev(uv, torch.float64), off, lmg.F64, 16)
    G = plan.grid(dev(vis, torch.complex128)).cpu().numpy()
    for c in range(len(counts)):
        a, b = off[c], off[c + 1]
        if a == b:
            assert np.all(G[c] == 0)
            continue
        assert rel_rms(G[c], im.grid(uv[a:b], vis[a:b], None, N, ek)) < 1e-12, c
