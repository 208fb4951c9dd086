"""Host-side checks of the C-ABI library (no GPU): symbols, table generator, error paths.

The library's C++ table generator is independent of the oracle's (its own LM,
Cholesky and Gauss-Legendre code); two optimisers agree only to their
tolerance, so the LM result is compared at the optimiser level and the
deterministic steps (normal-equation solve, correction) from a shared h.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1906_07102_amd as lmg
from oracle import lmtable as lt

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lmgrid.h")

pytestmark = pytest.mark.skipif(not os.path.exists(lmg.library_path()), reason="library not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lmg_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = lmg.load()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.parametrize("W", [3, 5, 7])
def test_table_optimiser_matches_oracle_at_optimiser_level(W):
    t = lmg.Table.create(W, 0.25, 300, 3)
    h_lib, _ = t.export()
    h_or = lt.optimal_h(W, 0.25)
    E_or = lt.integrated_misfit_coarse(h_or, W, 0.25)
    assert abs(t.integrated_misfit - E_or) <= 0.01 * E_or
    assert np.max(np.abs(h_lib / h_or - 1)) < 1e-4


@pytest.mark.parametrize("W", [12, 14])
def test_wide_tables_by_qr(W):
    """From W = 12 both sides solve App. B's least squares by QR (the library through one factorisation and
    rotated right-hand sides, the oracle by a least-squares solve per offset): the same h gives the same
    kernel and correction, and the library's optimiser reaches the oracle's misfit level."""
    t = lmg.Table.create(W, 0.25, 300, 3)
    h_lib, _ = t.export()
    E_or = lt.integrated_misfit_coarse(h_lib, W, 0.25)
    # the same E formula on the same h; E sums squares of residuals rho ~ sqrt(E / 1056) made of O(1) terms,
    # so rounding of ~4 eps in each rho moves E by ~8 eps / rho relative (about 1 % at W = 14)
    rho = np.sqrt(E_or / 1056)
    assert abs(t.integrated_misfit - E_or) <= max(1e-3, 4 * 8 * 2.2e-16 / rho) * E_or
    assert t.integrated_misfit < (5e-24 if W == 12 else 5e-28)      # below the Cholesky-limited optimum
    d = np.linspace(-0.5, 0.5, 13) if W % 2 else np.linspace(0.0, 1.0, 13)
    np.testing.assert_allclose(t.kernel(d).T, lt.kernel(h_lib, W, 0.25, d), rtol=0, atol=1e-11)
    _, nodes = t.export()
    np.testing.assert_allclose(nodes, lt.table_nodes(h_lib, W, 0.25, 300 // W, 3), rtol=0, atol=1e-11)
    np.testing.assert_allclose(t.correction(256), lt.correction(h_lib, W, 0.25, 256), rtol=1e-10)
    lib = lmg.load()
    out = ctypes.c_void_p()
    assert lib.lmg_table_create_direct(t.handle, ctypes.byref(out)) == -5       # LMG_ENOTSUP


def test_table_from_h_matches_oracle_nodes():
    h = lt.optimal_h(7, 0.25)
    t = lmg.Table.from_h(7, 0.25, 300, 3, h)
    _, nodes = t.export()
    ref = lt.table_nodes(h, 7, 0.25, 42, 3)
    cond = np.linalg.cond(lt.normal_matrix(h, 7, 0.25))
    assert np.max(np.abs(nodes - ref)) < 1e-15 * cond * 50
    d = np.linspace(-0.7, 0.7, 15)
    np.testing.assert_allclose(t.kernel(d).T, lt.kernel_from_h(h, 7, 0.25, d), atol=1e-15 * cond * 50)


@pytest.mark.parametrize("W,N", [(3, 128), (7, 256), (7, 4096)])
def test_correction_matches_oracle(W, N):
    h = lt.optimal_h(W, 0.25)
    t = lmg.Table.from_h(W, 0.25, 300, 3, h)
    a, b = t.correction(N), lt.correction(h, W, 0.25, N)
    keep = slice(N // 4, 3 * N // 4)          # the retained field |x| <= x0
    np.testing.assert_allclose(a[keep], b[keep], rtol=1e-13)
    # towards |x| = 1/2, c(x) is small and h picks up the rounding of the
    # ill-conditioned solve (cond(A) ~ 1e4 at W = 7) on each side
    np.testing.assert_allclose(a, b, rtol=1e-10)


def test_map_error_matches_oracle_and_paper_level():
    h = lt.optimal_h(7, 0.25)
    t = lmg.Table.from_h(7, 0.25, 300, 3, h)
    x = np.linspace(0, 0.25, 26)
    exact, tab = t.map_error(x)
    ref, _, _, _ = lt.map_error(lambda d: lt.kernel_from_h(h, 7, 0.25, d), 7, x)
    np.testing.assert_allclose(exact, ref, atol=1e-15)
    assert np.median(exact) < 3e-14          # the W = 7 level of Sec. 2.2
    assert np.all(tab >= exact * 0.999)      # a cubic 300-entry table adds error (App. F)
    assert np.median(tab) < 1e-12


def test_from_nodes_roundtrip():
    tab, h = lt.make_table(5, 0.25, 300, 1)
    t = lmg.Table.from_nodes(5, 0.25, 300, 1, h, tab.nodes)
    h2, n2 = t.export()
    np.testing.assert_array_equal(h2, h)
    np.testing.assert_array_equal(n2, tab.nodes)
    assert t.Ms == 60 and t.degree == 1 and t.W == 5


def test_direct_calculation_table():
    """lmg_table_create_direct: same W, x0 and h; no table error in the map error; NULL arguments rejected."""
    otab, h = lt.make_table(7, 0.25, 300, 3)
    t = lmg.Table.from_nodes(7, 0.25, 300, 3, h, otab.nodes)
    d = t.direct_calculation()
    assert d.direct and not t.direct
    assert (d.W, d.x0, d.Ms, d.degree) == (t.W, t.x0, t.Ms, t.degree)
    np.testing.assert_array_equal(d.export()[0], h)
    x = np.linspace(0.0, 0.25, 9)
    ell_exact, ell_direct = d.map_error(x)
    # the two columns integrate over nu with different rules (64 Gauss-Legendre points, 8 per table interval),
    # and l(x) ~ 1e-14 is the small difference of O(1) terms: they agree to about 1e-8
    np.testing.assert_allclose(ell_direct, ell_exact, rtol=1e-6, atol=1e-30)
    _, ell_table = t.map_error(x)
    assert np.max(ell_table) > np.max(ell_direct)        # the table adds its interpolation error
    lib = lmg.load()
    out = ctypes.c_void_p()
    assert lib.lmg_table_create_direct(None, ctypes.byref(out)) == -1
    assert lib.lmg_table_create_direct(t.handle, None) == -1
    flag = ctypes.c_int(7)
    assert lib.lmg_table_is_direct(None, ctypes.byref(flag)) == -1


@pytest.mark.parametrize("args", [(0, 0.25, 300, 3), (17, 0.25, 300, 3), (7, 0.0, 300, 3), (7, 0.6, 300, 3),
                                  (7, 0.25, 6, 3), (7, 0.25, 300, 4), (7, 0.25, 300, -1)])
def test_table_invalid_arguments(args):
    with pytest.raises(lmg.LmgError) as e:
        lmg.Table.create(*args)
    assert e.value.status == -1


def test_size_queries_and_invalid_grids():
    lib = lmg.load()
    n = ctypes.c_size_t()
    assert lib.lmg_workspace_size(4096, 7, 0.25, 16777152, lmg.F32, lmg.OP_DIRTY, ctypes.byref(n)) == 0
    assert n.value > 16777152 * 14
    for N in (100, 32, 16384):
        assert lib.lmg_workspace_size(N, 7, 0.25, 10, lmg.F32, lmg.OP_GRID, ctypes.byref(n)) == -1
    assert lib.lmg_workspace_size(128, 7, 0.2, 10, lmg.F32, lmg.OP_GRID, ctypes.byref(n)) == -1   # 2 x0 N not even int
    assert lib.lmg_workspace_size(128, 7, 0.25, -1, lmg.F32, lmg.OP_GRID, ctypes.byref(n)) == -1
    assert lib.lmg_workspace_size(128, 7, 0.25, 10, 3, lmg.OP_GRID, ctypes.byref(n)) == -1
    assert lib.lmg_plan_create(None, 128, 0, 0, None, None, 0, None, ctypes.byref(ctypes.c_void_p())) == -1
    assert lmg.load().lmg_status_string(-2).decode().startswith("workspace")


def test_batch_plan_rejects_bad_arguments_before_any_launch():
    """Argument errors of the batched plan are found on the host (nothing reaches a device)."""
    lib = lmg.load()
    import ctypes
    t = lmg.Table.create(5, 0.25, 300, 3)
    out = ctypes.c_void_p()
    I64 = ctypes.c_int64

    def create(offsets, tile=0, N=128, nchan=None):
        off = (I64 * len(offsets))(*offsets)
        nc = len(offsets) - 1 if nchan is None else nchan
        return lib.lmg_batch_plan_create(t.handle, N, lmg.F32, nc, off, None, tile, None, 0, None, ctypes.byref(out))

    assert create([1, 5]) == -1             # offsets[0] != 0
    assert create([0, 5, 3]) == -1          # decreasing
    assert create([0, 0], nchan=0) == -1    # no channel
    assert create([0, 0], tile=24) == -1    # not a power of two
    assert create([0, 0], tile=4) == -1     # below 8
    assert create([0, 0], tile=256) == -1   # above N
    assert create([0, 0], tile=8, N=2048) == -1   # more than 128 x 128 tiles
    assert create([0, 0]) == -2             # valid arguments, no workspace
    n = ctypes.c_size_t()
    assert lib.lmg_batch_workspace_size(1024, 5, 256, 16_000_000, lmg.F32, ctypes.byref(n)) == 0
    assert n.value > 0
    assert lib.lmg_batch_workspace_size(1024, 5, 0, 10, lmg.F32, ctypes.byref(n)) == -1
    assert lib.lmg_workspace_size_batched(1024, 5, 4, 100, lmg.F32, lmg.OP_DIRTY, ctypes.byref(n)) == -1


def test_tile_below_support_is_rejected():
    """A footprint (W cells, Eq. 6) must not reach two tiles away: an explicit tile edge below W is an argument
    error, found on the host before anything is enqueued (T = W is accepted: no workspace is the next error)."""
    lib = lmg.load()
    out = ctypes.c_void_p()
    off = (ctypes.c_int64 * 2)(0, 0)
    for W, tile, expect in ((12, 8, -1), (9, 8, -1), (16, 8, -1), (8, 8, -2), (12, 16, -2), (16, 16, -2)):
        t = lmg.Table.from_h(W, 0.25, 300, 1, np.ones(33))
        st = lib.lmg_batch_plan_create(t.handle, 128, lmg.F32, 1, off, None, tile, None, 0, None, ctypes.byref(out))
        assert st == expect, (W, tile, st)


def test_python_wrappers_check_arguments_on_the_host():
    """The one-shot wrappers check dtype, shape and contiguity before any pointer reaches the library (on host
    tensors these checks run first; a well-formed host tensor is then refused as not on the device)."""
    torch = pytest.importorskip("torch")
    t = lmg.Table.from_h(7, 0.25, 300, 3, lt.optimal_h(7, 0.25))
    uv = torch.zeros((10, 2), dtype=torch.float64)
    vis = torch.zeros(10, dtype=torch.complex64)
    w = torch.ones(10, dtype=torch.float32)
    with pytest.raises(ValueError):
        lmg.grid(t, 64, torch.zeros((10, 3), dtype=torch.float64), vis)           # uv not (nvis, 2)
    with pytest.raises(TypeError):
        lmg.grid(t, 64, uv.float(), vis)                                           # uv not float64
    with pytest.raises(ValueError):
        lmg.grid(t, 64, uv, torch.zeros(11, dtype=torch.complex64))               # vis longer than uv
    with pytest.raises(TypeError):
        lmg.grid(t, 64, uv, vis, w.double())                                       # weights not float32
    with pytest.raises(ValueError):
        lmg.grid(t, 64, uv, vis, torch.ones(9, dtype=torch.float32))              # weights too short
    with pytest.raises(ValueError):
        lmg.grid(t, 64, uv, vis, out=torch.zeros((64, 32), dtype=torch.complex64))   # grid too small
    with pytest.raises(ValueError):
        lmg.grid(t, 64, torch.zeros((2, 10), dtype=torch.float64).t(), vis)       # non-contiguous uv
    with pytest.raises(TypeError):
        lmg.grid(t, 64, uv, vis.real.contiguous())                                 # real visibilities
    with pytest.raises(ValueError):
        lmg.degrid(t, 64, uv, torch.zeros((32, 32), dtype=torch.complex64))       # grid not N x N
    with pytest.raises(ValueError):
        lmg.make_dirty_image(t, 64, uv, torch.zeros(9, dtype=torch.complex128))
    with pytest.raises(ValueError):
        lmg.predict_visibilities(t, 64, uv, torch.zeros((64, 64), dtype=torch.complex64))   # image not M x M
    with pytest.raises(ValueError):
        lmg.grid_batched(t, 64, uv, [0, 4, 9], vis)                               # offsets end before nvis
    with pytest.raises(ValueError):
        lmg.degrid_batched(t, 64, uv, [0, 6, 4, 10], torch.zeros((3, 64, 64), dtype=torch.complex64))
    with pytest.raises(ValueError):
        lmg.fft2_centred(torch.zeros((8, 16), dtype=torch.complex64), +1)
    with pytest.raises(TypeError):                                                  # well formed, but on the host
        lmg.grid(t, 64, uv, vis, w)
