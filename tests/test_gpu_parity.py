"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Every case feeds both sides the same seeded inputs and the same table (the
oracle's h and nodes, handed to the library with lmg_table_create_from_nodes).
Tolerances are relative RMS over the compared outputs: 1e-12 in FP64 and 1e-5
in FP32 (compensated or not).
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

TOL = {lmg.F32: 1e-5, lmg.F32_KAHAN: 1e-5, lmg.F64: 1e-12}
PRECS = [lmg.F32, lmg.F32_KAHAN, lmg.F64]
DEV = "cuda:0"


def rel_rms(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def ctype(prec):
    return torch.complex128 if prec == lmg.F64 else torch.complex64


def to_dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device=DEV, dtype=dtype)


_TABLES = {}


def tables(W, degree, table_size=300, x0=0.25):
    key = (W, degree, table_size, x0)
    if key not in _TABLES:
        otab, h = lt.make_table(W, x0, table_size, degree)
        gtab = lmg.Table.from_nodes(W, x0, table_size, degree, h, otab.nodes)
        _TABLES[key] = (otab, gtab, h)
    return _TABLES[key]


def gpu_grid(gtab, N, uv, vis, w, prec):
    plan = lmg.Plan(gtab, N, to_dev(uv, torch.float64), prec)
    g = plan.grid(to_dev(vis, ctype(prec)), None if w is None else to_dev(w, torch.float32))
    torch.cuda.synchronize()
    return plan, g.cpu().numpy()


def small():
    c = synth.small_case()
    return c.uv, c.vis, c.weights, c.extra["model_image"]


@pytest.fixture(autouse=True)
def _reset_env():
    old = {k: os.environ.get(k) for k in ("LMG_CAP", "LMG_TILE")}
    yield
    for k, v in old.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v


# ------------------------------------------------------------- gridding ---
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("W,degree", [(7, 3), (5, 3), (3, 3), (7, 1), (7, 0)])
def test_grid_small(prec, W, degree):
    print(f"grid small prec={prec} W={W} d={degree}", flush=True)
    otab, gtab, h = tables(W, degree)
    uv, vis, w, _ = small()
    rng = np.random.default_rng(3)
    w = rng.uniform(0.2, 2.0, len(vis)).astype(np.float32).astype(np.float64)   # weights are FP32 in every mode
    _, g = gpu_grid(gtab, 128, uv, vis, w, prec)
    ref = im.grid(uv, vis, w, 128, otab)
    assert rel_rms(g, ref) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("cap,tile", [("97", None), ("1", None), ("50", "16")])
def test_grid_split_items_and_tiles(prec, cap, tile):
    """Dense tiles split into many work items (down to one visibility each) and other tile sizes."""
    print(f"grid split prec={prec} cap={cap} tile={tile}", flush=True)
    os.environ["LMG_CAP"] = cap
    if tile:
        os.environ["LMG_TILE"] = tile
    otab, gtab, _ = tables(7, 3)
    uv, vis, w, _ = small()
    plan, g = gpu_grid(gtab, 128, uv, vis, None, prec)
    assert plan.info()["items"] >= plan.info()["busy_tiles"]
    assert rel_rms(g, im.grid(uv, vis, None, 128, otab)) < TOL[prec]


def test_grid_single_visibility_exact():
    """One V = 1 at integer (u, v) reproduces the node products exactly in FP64 (Eq. 5)."""
    otab, gtab, _ = tables(7, 3)
    uv = np.array([[3.0, -5.0]])
    _, g = gpu_grid(gtab, 64, uv, np.array([1.0 + 0j]), None, lmg.F64)
    ref = im.grid(uv, np.array([1.0 + 0j]), None, 64, otab)
    np.testing.assert_array_equal(g, ref)


@pytest.mark.parametrize("prec", PRECS)
def test_grid_edges_wrap_and_ties(prec):
    """Footprints crossing the grid edge wrap; exact half-integer and integer coordinates."""
    otab, gtab, _ = tables(7, 3)
    N = 64
    uv = np.array([[31.9, 0.0], [-32.0, -31.7], [31.5, 31.5], [-2.5, 4.0], [0.5, -0.5], [12.0, 13.0],
                   [-31.999, 31.999], [20.25, -10.75]])
    rng = np.random.default_rng(4)
    vis = rng.standard_normal(len(uv)) + 1j * rng.standard_normal(len(uv))
    _, g = gpu_grid(gtab, N, uv, vis, None, prec)
    assert rel_rms(g, im.grid(uv, vis, None, N, otab)) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("degree", [0, 1, 3])
def test_offsets_on_table_nodes_and_midpoints(prec, degree):
    """Offsets exactly on table nodes and exactly halfway between two (App. F). With M_s = 32 (a 224-entry
    W = 7 table) both are binary fractions, so the device and the oracle see the same s = M_s x and take the
    same interval, and for degree 0 the same nearest node (halfway rounds up). delta runs over (-1/2, 1/2],
    x = delta + 1/2 over (0, 1]: nodes 1 .. 32 (32 is the interval's top end) and midpoints 0.5 .. 31.5."""
    print(f"table nodes and midpoints prec={prec} degree={degree}", flush=True)
    otab, gtab, _ = tables(7, degree, table_size=224)
    assert otab.Ms == 32
    N = 64
    f = np.concatenate([-0.5 + np.arange(1, 33) / 32.0, -0.5 + (np.arange(32) + 0.5) / 32.0])
    rng = np.random.default_rng(61)
    n = rng.integers(-24, 24, size=(len(f), 2))
    uv = np.stack([n[:, 0] + f, n[:, 1] + f[rng.permutation(len(f))]], axis=1)
    vis = rng.standard_normal(len(uv)) + 1j * rng.standard_normal(len(uv))
    plan, g = gpu_grid(gtab, N, uv, vis, None, prec)
    assert rel_rms(g, im.grid(uv, vis, None, N, otab)) < TOL[prec]
    G = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    out = plan.degrid(to_dev(G, ctype(prec))).cpu().numpy()
    assert rel_rms(out, im.degrid(uv, G, otab)) < TOL[prec]


@pytest.mark.parametrize("prec", [lmg.F32, lmg.F64])
def test_largest_grid(prec):
    """N = 8192, the largest grid the library takes (the plan's tiles are then 64 cells: at most 128 x 128
    tiles): 20,000 visibilities over the whole grid, wrapping at its edges. Grid cells sampled inside the
    data footprint against the oracle's sums by the definition (Eq. 5), and degridding of a random grid."""
    print(f"largest grid prec={prec}", flush=True)
    otab, gtab, _ = tables(7, 3)
    N = 8192
    rng = np.random.default_rng(81)
    uv = rng.uniform(-N / 2, N / 2, (20000, 2))
    vis = rng.standard_normal(len(uv)) + 1j * rng.standard_normal(len(uv))
    plan, g = gpu_grid(gtab, N, uv, vis, None, prec)
    assert plan.info()["tile"] == 64
    cu, cv = im.tap_geometry(uv[:, 0], 7)[0], im.tap_geometry(uv[:, 1], 7)[0]
    k = rng.integers(0, len(uv), 500)
    cells = np.stack([(cv[k] + N // 2 + rng.integers(0, 7, 500)) % N,
                      (cu[k] + N // 2 + rng.integers(0, 7, 500)) % N], axis=1)
    ref = im.grid_cells(uv, vis, None, N, otab, cells)
    assert rel_rms(g[cells[:, 0], cells[:, 1]], ref) < TOL[prec]
    G = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))).astype(np.complex64)
    out = plan.degrid(to_dev(G, ctype(prec))).cpu().numpy()
    assert rel_rms(out, im.degrid(uv, G.astype(np.complex128), otab)) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_empty_and_non_finite(prec):
    otab, gtab, _ = tables(7, 3)
    N = 64
    plan, g = gpu_grid(gtab, N, np.zeros((0, 2)), np.zeros(0, complex), None, prec)
    assert np.count_nonzero(g) == 0 and plan.check() == 0
    uv = np.array([[1.2, 3.4], [np.nan, 0.0], [5.5, np.inf], [-7.1, 2.2]])
    vis = np.array([1 + 1j, 2 + 0j, 3 + 0j, -1 + 0.5j])
    plan, g = gpu_grid(gtab, N, uv, vis, None, prec)
    assert plan.check() == -4 and plan.info()["valid"] == 2
    keep = [0, 3]
    assert rel_rms(g, im.grid(uv[keep], vis[keep], None, N, otab)) < TOL[prec]
    G = np.random.default_rng(5).standard_normal((N, N)) * (1 + 0j)
    out = plan.degrid(to_dev(G, ctype(prec))).cpu().numpy()
    assert out[1] == 0 and out[2] == 0
    assert rel_rms(out[keep], im.degrid(uv[keep], G, otab)) < TOL[prec]


# ----------------------------------------------------------- degridding ---
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("W,degree", [(7, 3), (3, 3), (7, 0)])
def test_degrid_small(prec, W, degree):
    print(f"degrid small prec={prec} W={W} d={degree}", flush=True)
    otab, gtab, _ = tables(W, degree)
    uv, _, _, _ = small()
    rng = np.random.default_rng(6)
    G = rng.standard_normal((128, 128)) + 1j * rng.standard_normal((128, 128))
    plan = lmg.Plan(gtab, 128, to_dev(uv, torch.float64), prec)
    out = plan.degrid(to_dev(G, ctype(prec))).cpu().numpy()
    assert rel_rms(out, im.degrid(uv, G, otab)) < TOL[prec]


def test_adjoint_identity_gpu():
    """<grid(V), G> = <V, degrid(G)> on the device in FP64 (Sec. 1: transpose operations)."""
    _, gtab, _ = tables(7, 3)
    uv, vis, _, _ = small()
    rng = np.random.default_rng(7)
    G = rng.standard_normal((128, 128)) + 1j * rng.standard_normal((128, 128))
    plan = lmg.Plan(gtab, 128, to_dev(uv, torch.float64), lmg.F64)
    g = plan.grid(to_dev(vis, torch.complex128)).cpu().numpy()
    d = plan.degrid(to_dev(G, torch.complex128)).cpu().numpy()
    lhs, rhs = np.vdot(g, G), np.vdot(vis, d)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


# ------------------------------------------------------- images and FFT ---
def sampled_centred_dft(G, n, N, sign, k1, k2):
    """Outputs (k1 x k2) of the centred 2D DFT of G, whose non-zero block is G[:n, :n]: the transform of
    ifftshift(G) read through fftshift, summed directly (phases reduced mod N in integers)."""
    m = np.arange(n) - N // 2
    e1 = np.exp(sign * 2j * np.pi * ((((k1 + N // 2) % N)[:, None] * m[None, :]) % N) / N)
    e2 = np.exp(sign * 2j * np.pi * ((((k2 + N // 2) % N)[:, None] * m[None, :]) % N) / N)
    return e1 @ G[:n, :n] @ e2.T


@pytest.mark.parametrize("prec", [lmg.F32, lmg.F64])
@pytest.mark.parametrize("N", [4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192])
def test_fft2_centred(prec, N):
    """Every supported N: log2 N a multiple of 3 (radix-8 stages only), or one more radix-2 or radix-4 stage;
    the smallest sizes run with unpadded rows and a few threads per workgroup. N = 8192 also covers, in FP64,
    the pass whose rows are unpadded and whose quarter-wave twiddle table fits LDS only unpadded; it is checked
    on 48 x 48 sampled outputs against a direct sum."""
    print(f"fft2 prec={prec} N={N}", flush=True)
    rng = np.random.default_rng(N)
    n = min(N, 512)
    G = np.zeros((N, N), complex)
    G[:n, :n] = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    k1, k2 = rng.integers(0, N, 48), rng.integers(0, N, 48)
    for sign in (+1, -1):
        d = to_dev(G, ctype(prec))
        lmg.fft2_centred(d, sign)
        if N > 4096:
            out = d[torch.as_tensor(k1, device=d.device)][:, torch.as_tensor(k2, device=d.device)].cpu().numpy()
            ref = sampled_centred_dft(G, n, N, sign, k1, k2)
            print(f"  sign {sign:+d}: sampled rel RMS {rel_rms(out, ref):.2e}", flush=True)
            assert rel_rms(out, ref) < (3e-6 if prec == lmg.F32 else 1e-13)
            continue
        out = d.cpu().numpy()
        ref = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(G))) if sign < 0 else \
            np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(G))) * N * N
        if N <= 128:
            ref2 = im.centred_fft2(G, sign)
            assert rel_rms(ref, ref2) < 1e-13
            assert rel_rms(sampled_centred_dft(G, n, N, sign, k1, k2), ref[np.ix_(k1, k2)]) < 1e-13
        assert rel_rms(out, ref) < (2e-6 if prec == lmg.F32 else 1e-13)


@pytest.mark.parametrize("prec", PRECS)
def test_dirty_image_small(prec):
    otab, gtab, h = tables(7, 3)
    uv, vis, w, _ = small()
    plan = lmg.Plan(gtab, 128, to_dev(uv, torch.float64), prec)
    img = plan.make_dirty_image(to_dev(vis, ctype(prec))).cpu().numpy()
    ref = im.dirty_from_grid(im.grid(uv, vis, None, 128, otab), lt.correction(h, 7, 0.25, 128), 0.25)
    assert rel_rms(img, ref) < TOL[prec]
    if prec == lmg.F64:      # and the DFT misfit bound of Eqs. (7)-(8) holds on the device result
        pq = np.stack(np.meshgrid(np.arange(-32, 32), np.arange(-32, 32), indexing="xy"), -1).reshape(-1, 2)
        bound = im.image_misfit_bound(uv, vis, None, 128, otab, lt.correction(h, 7, 0.25, 128), pq)
        dft = im.dft_dirty_image(uv, vis, None, 128, 0.25)
        assert np.all(np.abs(dft - img).ravel() ** 2 <= bound * (1 + 1e-9))


@pytest.mark.parametrize("prec", PRECS)
def test_predict_small(prec):
    otab, gtab, h = tables(7, 3)
    uv, _, _, model = small()
    plan = lmg.Plan(gtab, 128, to_dev(uv, torch.float64), prec)
    out = plan.predict_visibilities(to_dev(model, ctype(prec))).cpu().numpy()
    ref = im.predict_visibilities(uv, model, 128, 0.25, otab, lt.correction(h, 7, 0.25, 128))
    assert rel_rms(out, ref) < TOL[prec]
    truth = im.direct_predict(uv, model, 128, 0.25)
    assert rel_rms(out, truth) < (3e-5 if prec != lmg.F64 else 1e-6)


def test_one_shot_equals_planned():
    """One-shot calls build the same plan internally, and plans fix the summation order, so the results are
    the same bits (the one-shot gridding adds into a zeroed grid: 0 + x = x)."""
    _, gtab, _ = tables(7, 3)
    uv, vis, _, model = small()
    duv = to_dev(uv, torch.float64)
    dv = to_dev(vis, torch.complex128)
    plan = lmg.Plan(gtab, 128, duv, lmg.F64)
    np.testing.assert_array_equal(lmg.grid(gtab, 128, duv, dv).cpu().numpy(), plan.grid(dv).cpu().numpy())
    img = to_dev(model, torch.complex128)
    np.testing.assert_array_equal(lmg.predict_visibilities(gtab, 128, duv, img).cpu().numpy(),
                                  plan.predict_visibilities(img).cpu().numpy())
    np.testing.assert_array_equal(lmg.make_dirty_image(gtab, 128, duv, dv).cpu().numpy(),
                                  plan.make_dirty_image(dv).cpu().numpy())
    G = plan.grid(dv)
    np.testing.assert_array_equal(lmg.degrid(gtab, 128, duv, G).cpu().numpy(), plan.degrid(G).cpu().numpy())


# ---------------------------------------------------- full-size sampled ---
def sample_cells(uv, N, W, n, seed):
    """Cells inside the data footprint plus a few empty ones."""
    rng = np.random.default_rng(seed)
    k = rng.integers(0, len(uv), n)
    nf = np.ceil(uv[k] - W / 2.0).astype(np.int64) + rng.integers(0, W, (n, 2))
    cells = [((int(b) + N // 2) % N, (int(a) + N // 2) % N) for a, b in nf]
    return cells + [(0, 0), (N - 1, N // 2), (N // 2, 5)]


_FULL = {}


def full_case(which):
    if which not in _FULL:
        _FULL[which] = synth.array_1m_case(with_vis=False) if which == "1m" else synth.array_16m_case(with_vis=False)
    return _FULL[which]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("which", ["1m", "16m"])
def test_full_size_grid_degrid_sampled(which, prec):
    """Full-size array cases in every mode (FP32 is the benchmark configuration): grid cells sampled inside the
    data footprint (each summed by the oracle from the definition, Eq. 5) and 2,000 degridded visibilities."""
    c = full_case(which)
    print(f"full-size {c.name} prec={prec}", flush=True)
    otab, gtab, _ = tables(c.W, 3)
    rng = np.random.default_rng(8)
    vis = (rng.standard_normal(len(c.uv)) + 1j * rng.standard_normal(len(c.uv))).astype(np.complex64)
    duv = to_dev(c.uv, torch.float64)
    plan = lmg.Plan(gtab, c.N, duv, prec)
    g = plan.grid(to_dev(vis, ctype(prec)))
    cells = sample_cells(c.uv, c.N, c.W, 24, 9)
    got = np.array([g[r, cc].item() for r, cc in cells])
    ref = im.grid_cells(c.uv, vis.astype(np.complex128), None, c.N, otab, cells)
    assert rel_rms(got, ref) < TOL[prec]
    del g
    G = np.zeros((c.N, c.N), np.complex64)
    band = slice(c.N // 4 - 8, 3 * c.N // 4 + 8)
    G[band, band] = (rng.standard_normal(G[band, band].shape) + 1j * rng.standard_normal(G[band, band].shape))
    out = plan.degrid(to_dev(G, ctype(prec)))
    k = rng.integers(0, len(c.uv), 2000)
    assert rel_rms(out[k].cpu().numpy(), im.degrid(c.uv[k], G.astype(np.complex128), otab)) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_array_1m_dirty_image_and_prediction(prec):
    """1,008,000 array visibilities on 2048^2 (the 1M configuration): the whole 1024^2 dirty image and all
    predicted visibilities element by element against the oracle (grid, radix-2 FFT, correct, crop; pad, FFT,
    degrid), and the dirty image against the direct DFT (Eq. 3) on a 64 x 64 lattice of the retained field
    within the method's own error (the oracle's misfit on the same lattice, plus the FP32 floor)."""
    c = synth.array_1m_case(with_vis=True)
    print(f"1M images prec={prec}", flush=True)
    otab, gtab, h = tables(c.W, 3)
    hp = lt.correction(h, c.W, c.x0, c.N)
    vis = c.vis.astype(np.complex64).astype(np.complex128)
    plan = lmg.Plan(gtab, c.N, to_dev(c.uv, torch.float64), prec)
    img = plan.make_dirty_image(to_dev(vis, ctype(prec))).cpu().numpy()
    ref = im.make_dirty_image(c.uv, vis, None, c.N, c.x0, otab, hp)
    e_img = rel_rms(img, ref)
    print(f"  dirty image rel RMS vs oracle {e_img:.2e}", flush=True)
    assert e_img < TOL[prec]
    pix = np.arange(-512, 512, 16)
    dft = im.dft_dirty_image(c.uv, vis, None, c.N, c.x0, pix, pix)
    sel = pix + 512
    e_dft = rel_rms(img[np.ix_(sel, sel)], dft)
    e_or = rel_rms(ref[np.ix_(sel, sel)], dft)
    print(f"  vs DFT: device {e_dft:.3e}, oracle {e_or:.3e}", flush=True)
    assert e_dft < e_or * (1 + 1e-6) + (3e-7 if prec != lmg.F64 else 1e-12)
    rng = np.random.default_rng(38)
    model = rng.standard_normal((1024, 1024)) + 1j * rng.standard_normal((1024, 1024))
    vh = plan.predict_visibilities(to_dev(model, ctype(prec))).cpu().numpy()
    vref = im.predict_visibilities(c.uv, model, c.N, c.x0, otab, hp)
    e_vis = rel_rms(vh, vref)
    print(f"  prediction rel RMS vs oracle {e_vis:.2e}", flush=True)
    assert e_vis < TOL[prec]


def test_plan_used_from_another_stream():
    """Plan creation only enqueues work; a call on another stream waits for the plan on the device."""
    print("plan on one stream, calls on another", flush=True)
    uv, vis, w, _ = small()
    otab, gtab, _ = tables(7, 3)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    duv = to_dev(uv, torch.float64)
    dvis = to_dev(vis, torch.complex128)
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        plan = lmg.Plan(gtab, 128, duv, lmg.F64)
    with torch.cuda.stream(s2):
        g = plan.grid(dvis)
        v = plan.degrid(g)
    torch.cuda.synchronize()
    assert plan.info()["items"] > 0
    assert rel_rms(g.cpu().numpy(), im.grid(uv, vis, None, 128, otab)) < 1e-12
    assert rel_rms(v.cpu().numpy(), im.degrid(uv, g.cpu().numpy(), otab)) < 1e-12
