"""The gridder in use: alias suppression (Sec. 4) and the major cycle of iterative imaging (Sec. 5).

Alias suppression: a unit point source outside the image, at x = 1/2 + d
(d = 1/4, 3/8, 1/2; the grid's periodicity folds it into |x| <= x0), must
leave the retained field of the dirty image as the direct DFT (Eq. 3) has it:
the gridded image's departure from the DFT, in units of the source's dirty
peak (sum of weights), is the alias the kernel lets through, about 1e-7 at
W = 7 by the paper's estimate; each pixel also obeys the misfit bound of
Eqs. (7)-(8).

Major cycle: with the true sky as the model (50 point sources on pixel
centres, 1,008,000 array visibilities, 2048^2 grid), predict -> subtract ->
grid residuals through one plan; the residual visibilities and the residual
dirty image must sit at the method's error level (relative RMS ~1e-7 at
W = 7 in FP64), far below the data.
"""
import numpy as np
import pytest

import synth
from oracle import imaging as im
from oracle import lmtable as lt

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1906_07102_amd as lmg  # noqa: E402

DEV = "cuda:0"
_T = {}


def tables(W=7):
    if W not in _T:
        otab, h = lt.make_table(W, 0.25, 300, 3)
        _T[W] = (otab, lmg.Table.from_nodes(W, 0.25, 300, 3, h, otab.nodes), h)
    return _T[W]


@pytest.mark.parametrize("d", [0.25, 0.375, 0.5])
def test_alias_of_a_source_outside_the_field(d):
    otab, gtab, h = tables(7)
    c = synth.small_case()
    N, x0 = c.N, 0.25
    xs = 0.5 + d                                              # image coordinate of the source (x = p / N)
    vis = np.exp(-2j * np.pi * (c.uv[:, 0] * xs + c.uv[:, 1] * 0.1))
    plan = lmg.Plan(gtab, N, torch.as_tensor(c.uv, device=DEV), lmg.F64)
    img = plan.make_dirty_image(torch.as_tensor(vis, device=DEV)).cpu().numpy()
    dft = im.dft_dirty_image(c.uv, vis, None, N, x0)
    alias = np.abs(img - dft) / len(vis)                      # in units of the source's dirty peak
    print(f"d = {d}: largest alias {alias.max():.2e}, RMS {np.sqrt(np.mean(alias ** 2)):.2e} of the flux", flush=True)
    assert alias.max() < 1e-6
    M = 2 * int(x0 * N)
    pq = np.stack(np.meshgrid(np.arange(-M // 2, M // 2), np.arange(-M // 2, M // 2), indexing="xy"), -1).reshape(-1, 2)
    bound = im.image_misfit_bound(c.uv, vis, None, N, otab, lt.correction(h, 7, x0, N), pq)
    assert np.all(np.abs(dft - img).ravel() ** 2 <= bound * (1 + 1e-9))


@pytest.mark.parametrize("prec", [lmg.F64, lmg.F32])
def test_major_cycle_with_the_true_model(prec):
    print(f"major cycle prec={prec}", flush=True)
    _, gtab, _ = tables(7)
    c = synth.array_1m_case(with_vis=True, device="cuda")
    cdt = torch.complex128 if prec == lmg.F64 else torch.complex64
    plan = lmg.Plan(gtab, c.N, torch.as_tensor(c.uv, device=DEV), prec)
    M = plan.M
    model = torch.zeros((M, M), dtype=cdt, device=DEV)
    pos, flux = c.extra["src_pos"], c.extra["src_flux"]
    for (p, q), f in zip(pos, flux):
        model[q + M // 2, p + M // 2] += float(f)
    V = torch.as_tensor(c.vis, device=DEV).to(cdt)
    for cycle in range(2):                                    # the plan serves every cycle
        resid = V - plan.predict_visibilities(model)
        rimg = plan.make_dirty_image(resid)
    dimg = plan.make_dirty_image(V)
    rv = (torch.linalg.vector_norm(resid) / torch.linalg.vector_norm(V)).item()
    ri = (rimg.abs().max() / dimg.abs().max()).item()
    print(f"residual visibilities {rv:.2e} (relative RMS), residual image peak {ri:.2e} of the dirty peak",
          flush=True)
    assert rv < (1e-6 if prec == lmg.F64 else 2e-5)
    assert ri < (1e-6 if prec == lmg.F64 else 2e-5)


@pytest.mark.parametrize("prec", [lmg.F64, lmg.F32])
def test_spheroidal_table_through_the_library(prec):
    """A table of the comparison system (the alpha = 1 spheroidal function, oracle-side) taken as data by
    lmg_table_create_from_nodes: the kernels grid and degrid with it as with any table (the correction is
    not involved)."""
    from oracle import spheroidal as sp
    stab = sp.table(7, 42, 3)
    gtab = lmg.Table.from_nodes(7, 0.25, 300, 3, np.ones(33), stab.nodes)
    c = synth.small_case()
    cdt = torch.complex128 if prec == lmg.F64 else torch.complex64
    plan = lmg.Plan(gtab, c.N, torch.as_tensor(c.uv, device=DEV), prec)
    g = plan.grid(torch.as_tensor(c.vis, device=DEV).to(cdt)).cpu().numpy()
    ref = im.grid(c.uv, c.vis, None, c.N, stab)
    tol = 1e-12 if prec == lmg.F64 else 1e-5
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < tol
    rng = np.random.default_rng(43)
    G = rng.standard_normal((c.N, c.N)) + 1j * rng.standard_normal((c.N, c.N))
    out = plan.degrid(torch.as_tensor(G, device=DEV).to(cdt)).cpu().numpy()
    ref_v = im.degrid(c.uv, G, stab)
    assert np.linalg.norm(out - ref_v) / np.linalg.norm(ref_v) < tol
