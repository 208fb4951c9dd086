"""GPU checks of the call semantics through the C ABI: accumulation into a grid, run-to-run reproducibility,
device-side data errors, tile edges at the support width, and degree-2 tables.

Expected values come from the FP64 oracle on the same seeded inputs (the oracle's table handed to the library
with lmg_table_create_from_nodes); tolerances are relative RMS 1e-12 in FP64 and 1e-5 in FP32.
"""
import os

import numpy as np
import pytest

import synth
from oracle import imaging as im
from oracle import lmtable as lt

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1906_07102_amd as lmg  # noqa: E402

DEV = "cuda:0"
TOL = {lmg.F32: 1e-5, lmg.F32_KAHAN: 1e-5, lmg.F64: 1e-12}
PRECS = [lmg.F32, lmg.F32_KAHAN, lmg.F64]
_TABLES = {}


def tables(W, degree=3, table_size=300, x0=0.25):
    key = (W, degree, table_size, x0)
    if key not in _TABLES:
        otab, h = lt.make_table(W, x0, table_size, degree)
        _TABLES[key] = (otab, lmg.Table.from_nodes(W, x0, table_size, degree, h, otab.nodes))
    return _TABLES[key]


def rel_rms(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def cdt(prec):
    return torch.complex128 if prec == lmg.F64 else torch.complex64


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device=DEV, dtype=dtype)


@pytest.fixture(autouse=True)
def _reset_env():
    old = os.environ.get("LMG_TILE")
    yield
    if old is None:
        os.environ.pop("LMG_TILE", None)
    else:
        os.environ["LMG_TILE"] = old


# ---------------------------------------------------------- accumulation ---
@pytest.mark.parametrize("prec", PRECS)
def test_chunks_accumulate_into_one_grid(prec):
    """Eq. (5) is a sum over visibilities: gridding two chunks into one grid (the second call adding) gives the
    grid of the whole set, through planned calls and through the accumulating one-shot lmg_grid."""
    print(f"accumulate chunks prec={prec}", flush=True)
    otab, gtab = tables(7)
    c = synth.small_case()
    rng = np.random.default_rng(31)
    w = rng.uniform(0.5, 2.0, len(c.uv)).astype(np.float32)
    ref = im.grid(c.uv, c.vis, w.astype(np.float64), c.N, otab)
    cut = 1234
    uvd, vd, wd = dev(c.uv, torch.float64), dev(c.vis, cdt(prec)), dev(w, torch.float32)
    p1 = lmg.Plan(gtab, c.N, uvd[:cut].contiguous(), prec)
    p2 = lmg.Plan(gtab, c.N, uvd[cut:].contiguous(), prec)
    g = p1.grid(vd[:cut].contiguous(), wd[:cut].contiguous())
    p2.grid(vd[cut:].contiguous(), wd[cut:].contiguous(), out=g, accumulate=True)
    assert rel_rms(g.cpu().numpy(), ref) < TOL[prec]
    kahan = prec == lmg.F32_KAHAN
    g1 = lmg.grid(gtab, c.N, uvd[:cut].contiguous(), vd[:cut].contiguous(), wd[:cut].contiguous(), kahan=kahan)
    lmg.grid(gtab, c.N, uvd[cut:].contiguous(), vd[cut:].contiguous(), wd[cut:].contiguous(), kahan=kahan, out=g1)
    assert rel_rms(g1.cpu().numpy(), ref) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_accumulate_adds_and_leaves_other_cells_alone(prec):
    """Accumulating adds G to the grid's values; tiles no footprint reaches are neither read nor written (their
    cells keep their bits), and the cells that are reached equal G0 + G."""
    print(f"accumulate into a filled grid prec={prec}", flush=True)
    otab, gtab = tables(7)
    N = 256
    rng = np.random.default_rng(32)
    uv = rng.uniform(-20, 20, (3000, 2))           # footprints stay inside the central tiles of a 256^2 grid
    vis = rng.standard_normal(3000) + 1j * rng.standard_normal(3000)
    G0 = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    plan = lmg.Plan(gtab, N, dev(uv, torch.float64), prec)
    g = dev(G0, cdt(prec))
    before = g.clone()
    plan.grid(dev(vis, cdt(prec)), out=g, accumulate=True)
    got = g.cpu().numpy()
    G = im.grid(uv, vis, None, N, otab)
    ref = G0.astype(np.complex64 if prec != lmg.F64 else np.complex128) + G
    assert rel_rms(got - before.cpu().numpy(), G) < (1e-5 if prec != lmg.F64 else 1e-12)
    assert rel_rms(got, ref) < TOL[prec]
    tile = plan.info()["tile"]
    far = np.ones((N, N), bool)
    lo, hi = N // 2 - 24, N // 2 + 24
    far[(lo // tile) * tile: -(-hi // tile) * tile, (lo // tile) * tile: -(-hi // tile) * tile] = False
    np.testing.assert_array_equal(got[far], before.cpu().numpy()[far])
    with pytest.raises(ValueError):
        plan.grid(dev(vis, cdt(prec)), accumulate=True)          # nothing to add to


# ----------------------------------------------------------- reproducible ---
@pytest.mark.parametrize("prec", PRECS)
def test_plans_rebuilt_give_identical_bits(prec):
    """The plan's ranks are taken in a fixed order, so the summation order is a function of the coordinates:
    plans built again from the same uv (1,008,000 time-major array visibilities, many per cell) grid and
    degrid to identical bits, in every mode; repeated calls on one plan too."""
    print(f"bitwise reproducibility prec={prec}", flush=True)
    c = synth.array_1m_case(with_vis=False)
    _, gtab = tables(c.W)
    rng = np.random.default_rng(33)
    vis = dev((rng.standard_normal(len(c.uv)) + 1j * rng.standard_normal(len(c.uv))), cdt(prec))
    uvd = dev(c.uv, torch.float64)
    grids, outs = [], []
    for _ in range(3):
        plan = lmg.Plan(gtab, c.N, uvd, prec)
        g = plan.grid(vis)
        grids.append(g)
        outs.append(plan.degrid(g))
        del plan
    g_again = lmg.Plan(gtab, c.N, uvd, prec)
    grids.append(g_again.grid(vis))
    grids.append(g_again.grid(vis))
    for g in grids[1:]:
        assert torch.equal(g, grids[0])
    for o in outs[1:]:
        assert torch.equal(o, outs[0])


@pytest.mark.parametrize("prec", [lmg.F32, lmg.F32_KAHAN])
def test_batched_equals_single_channel_bitwise(prec):
    """A batched plan lays each channel out as the single-channel plan of that channel does (same tile, same
    blocks, same ranks), so each channel's grid is the same bits."""
    print(f"batched vs single bitwise prec={prec}", flush=True)
    uv, off, _ = synth.multichannel_case(nchan=24)
    rng = np.random.default_rng(34)
    vis = (rng.standard_normal(len(uv)) + 1j * rng.standard_normal(len(uv))).astype(np.complex64)
    _, gtab = tables(5)
    N = 1024
    uvd, vd = dev(uv, torch.float64), dev(vis, torch.complex64)
    plan = lmg.BatchPlan(gtab, N, uvd, off, prec)
    G = plan.grid(vd)
    for c in range(0, len(off) - 1, 5):
        a, b = int(off[c]), int(off[c + 1])
        single = lmg.Plan(gtab, N, uvd[a:b].contiguous(), prec)
        assert single.info()["tile"] == plan.info()["tile"]
        assert torch.equal(single.grid(vd[a:b].contiguous()), G[c]), c


# ---------------------------------------------------------- data errors ---
def test_sync_status_reports_non_finite_coordinates_once():
    """lmg_sync_status: LMG_EDATA after a plan met non-finite coordinates on the device, then LMG_OK."""
    _, gtab = tables(7)
    assert lmg.sync_status() in (0, -4)                          # clear anything earlier tests left
    assert lmg.sync_status() == 0
    uv = np.array([[1.0, 2.0], [np.nan, 0.0], [3.0, np.inf]])
    plan = lmg.Plan(gtab, 64, dev(uv, torch.float64), lmg.F32)
    assert lmg.sync_status() == -4
    assert lmg.sync_status() == 0
    assert plan.check() == -4                                    # the plan keeps its own record
    ok = lmg.Plan(gtab, 64, dev(uv[:1], torch.float64), lmg.F32)
    assert lmg.sync_status() == 0 and ok.check() == 0


# ------------------------------------------------------ tile at support ---
@pytest.mark.parametrize("W,tile", [(8, 8), (9, 16), (14, 16), (16, 16)])
@pytest.mark.parametrize("prec", [lmg.F32, lmg.F64])
def test_tile_at_the_support_width(W, tile, prec):
    """Footprints as wide as the tile (T = W) or nearly (W = 14, 16 at T = 16) reach the right, lower and
    lower-right tiles: grid and degrid against the oracle with the tile edge forced."""
    print(f"tile edge W={W} tile={tile} prec={prec}", flush=True)
    h = lt.optimal_h(7, 0.25)          # any h defines a kernel (Eq. 18); both sides take the same h and nodes
    otab = lt.Table(W, 0.25, 300 // W, 1, lt.table_nodes(h, W, 0.25, 300 // W, 1))
    gtab = lmg.Table.from_nodes(W, 0.25, 300, 1, h, otab.nodes)
    N = 128
    rng = np.random.default_rng(35 + W)
    uv = rng.uniform(-40, 40, (4000, 2))
    vis = rng.standard_normal(4000) + 1j * rng.standard_normal(4000)
    plan = lmg.BatchPlan(gtab, N, dev(uv, torch.float64), [0, len(uv)], prec, tile=tile)
    assert plan.info()["tile"] == tile
    g = plan.grid(dev(vis, cdt(prec))).cpu().numpy()          # one channel: an N x N grid
    assert rel_rms(g, im.grid(uv, vis, None, N, otab)) < TOL[prec]
    G = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    out = plan.degrid(dev(G, cdt(prec))).cpu().numpy()
    assert rel_rms(out, im.degrid(uv, G, otab)) < TOL[prec]


@pytest.mark.parametrize("tile", [64])
@pytest.mark.parametrize("prec", [lmg.F32, lmg.F32_KAHAN, lmg.F64])
def test_large_tiles(tile, prec):
    """Tiles of 64 cells: the item sort's per-wave cell counters would exceed its LDS budget, so its waves
    take turns on one set of counters (the sort's other layout path). Dense cells (full 32-entry pieces and
    tails) over several work items: grid and degrid against the oracle, and a second plan gives the same
    bits."""
    print(f"large tiles tile={tile} prec={prec}", flush=True)
    h = lt.optimal_h(7, 0.25)
    otab = lt.Table(7, 0.25, 42, 3, lt.table_nodes(h, 7, 0.25, 42, 3))
    gtab = lmg.Table.from_nodes(7, 0.25, 300, 3, h, otab.nodes)
    N = 256
    rng = np.random.default_rng(71 + tile)
    uv = np.clip(rng.normal(0.0, 12.0, (60000, 2)), -100, 100)
    vis = rng.standard_normal(len(uv)) + 1j * rng.standard_normal(len(uv))
    uvd, vd = dev(uv, torch.float64), dev(vis, cdt(prec))
    plan = lmg.BatchPlan(gtab, N, uvd, [0, len(uv)], prec, tile=tile)
    assert plan.info()["tile"] == tile
    g = plan.grid(vd)
    assert rel_rms(g.cpu().numpy(), im.grid(uv, vis, None, N, otab)) < TOL[prec]
    G = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    out = plan.degrid(dev(G, cdt(prec))).cpu().numpy()
    assert rel_rms(out, im.degrid(uv, G, otab)) < TOL[prec]
    again = lmg.BatchPlan(gtab, N, uvd, [0, len(uv)], prec, tile=tile)
    assert torch.equal(again.grid(vd), g)


def test_tile_whose_patch_exceeds_lds_is_refused():
    """A 128-cell tile at W = 7 needs a (128 + 6)^2-cell gridding patch, more LDS than a workgroup has: the
    plan is refused with LMG_ENOTSUP rather than built."""
    gtab = lmg.Table.create(7, 0.25, 300, 3)
    uv = dev(np.random.default_rng(72).uniform(-50, 50, (100, 2)), torch.float64)
    with pytest.raises(lmg.LmgError) as e:
        lmg.BatchPlan(gtab, 256, uv, [0, 100], lmg.F32, tile=128)
    assert e.value.status == -5


def test_tile_override_below_the_support_is_raised():
    """LMG_TILE below W is raised to the smallest power of two >= W, and the grid stays right."""
    os.environ["LMG_TILE"] = "8"
    h = lt.optimal_h(7, 0.25)          # any h defines a kernel (Eq. 18); both sides take the same h and nodes
    otab = lt.Table(12, 0.25, 25, 1, lt.table_nodes(h, 12, 0.25, 25, 1))
    gtab = lmg.Table.from_nodes(12, 0.25, 300, 1, h, otab.nodes)
    rng = np.random.default_rng(36)
    uv = rng.uniform(-30, 30, (2000, 2))
    vis = rng.standard_normal(2000) + 1j * rng.standard_normal(2000)
    plan = lmg.Plan(gtab, 128, dev(uv, torch.float64), lmg.F64)
    assert plan.info()["tile"] == 16
    assert rel_rms(plan.grid(dev(vis, torch.complex128)).cpu().numpy(), im.grid(uv, vis, None, 128, otab)) < 1e-12


# ------------------------------------------------------------ degree 2 ---
@pytest.mark.parametrize("prec", PRECS)
def test_degree_two_table(prec):
    """App. F quadratic interpolation (the degree the other tests skip): grid, degrid and the dirty image."""
    print(f"degree 2 prec={prec}", flush=True)
    otab, gtab = tables(7, degree=2)
    c = synth.small_case()
    plan = lmg.Plan(gtab, c.N, dev(c.uv, torch.float64), prec)
    g = plan.grid(dev(c.vis, cdt(prec))).cpu().numpy()
    assert rel_rms(g, im.grid(c.uv, c.vis, None, c.N, otab)) < TOL[prec]
    rng = np.random.default_rng(37)
    G = rng.standard_normal((c.N, c.N)) + 1j * rng.standard_normal((c.N, c.N))
    assert rel_rms(plan.degrid(dev(G, cdt(prec))).cpu().numpy(), im.degrid(c.uv, G, otab)) < TOL[prec]
    h = lt.optimal_h(7, 0.25)
    img = plan.make_dirty_image(dev(c.vis, cdt(prec))).cpu().numpy()
    ref = im.dirty_from_grid(im.grid(c.uv, c.vis, None, c.N, otab), lt.correction(h, 7, 0.25, c.N), 0.25)
    assert rel_rms(img, ref) < TOL[prec]


# ----------------------------------------------------------- plan order ---
@pytest.mark.parametrize("prec", PRECS)
def test_plan_order_calls_match_caller_order(prec):
    """Gridding and degridding on plan-ordered data give the caller-order calls' results bit for bit (the same
    kernels after the same reordering), and the round trip through plan order restores the caller's array
    (zero for a dropped visibility)."""
    print(f"plan order prec={prec}", flush=True)
    otab, gtab = tables(7)
    c = synth.small_case()
    uv = c.uv.copy()
    uv[17] = np.nan                                              # one dropped visibility
    rng = np.random.default_rng(39)
    w = rng.uniform(0.5, 2.0, len(uv)).astype(np.float32)
    plan = lmg.Plan(gtab, c.N, dev(uv, torch.float64), prec)
    vd, wd = dev(c.vis, cdt(prec)), dev(w, torch.float32)
    vp = plan.to_plan_order(vd, wd)
    assert vp.shape[0] == plan.plan_order_length() >= len(uv)
    g = plan.grid_ordered(vp)
    assert torch.equal(g, plan.grid(vd, wd))
    keep = np.arange(len(uv)) != 17
    assert rel_rms(g.cpu().numpy(), im.grid(uv[keep], c.vis[keep], w[keep].astype(np.float64), c.N, otab)) < TOL[prec]
    g2 = g.clone()
    plan.grid_ordered(vp, out=g2, accumulate=True)
    assert rel_rms(g2.cpu().numpy(), 2 * g.cpu().numpy()) < TOL[prec]
    G = dev(rng.standard_normal((c.N, c.N)) + 1j * rng.standard_normal((c.N, c.N)), cdt(prec))
    back = plan.from_plan_order(plan.degrid_ordered(G))
    assert torch.equal(back, plan.degrid(G))
    assert back[17].item() == 0
    unit = plan.from_plan_order(plan.to_plan_order(vd))
    ref = vd.clone()
    ref[17] = 0
    assert torch.equal(unit, ref)
