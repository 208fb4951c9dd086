"""The allocation-free gridding entry point, lmg_grid_planned_noalloc, through the C ABI.

Its scratch is the library's fixed per-device array (which keeps the previous
call's contents), so the checks run two calls in a row, the second on a
smaller plan, and compare each with lmg_grid_planned on the same plan (the
plan fixes the summation order, so the bits must match) and with the FP64
oracle (relative RMS 1e-12 in FP64, 1e-5 in FP32).
"""
import ctypes

import numpy as np
import pytest

from oracle import imaging as im
from oracle import lmtable as lt

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1906_07102_amd as lmg  # noqa: E402

DEV = "cuda:0"
TOL = {lmg.F32: 1e-5, lmg.F32_KAHAN: 1e-5, lmg.F64: 1e-12}


def rel_rms(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("prec", [lmg.F32, lmg.F32_KAHAN, lmg.F64])
def test_noalloc_grid_equals_planned_on_two_calls(prec):
    lib = lmg.load()
    otab, h = lt.make_table(7, 0.25, 300, 3)
    gtab = lmg.Table.from_nodes(7, 0.25, 300, 3, h, otab.nodes)
    cdt = torch.complex128 if prec == lmg.F64 else torch.complex64
    N = 512
    rng = np.random.default_rng(40 + prec)
    for nvis, accumulate in ((200_000, 0), (30_000, 1)):       # the second call is smaller
        print(f"noalloc prec={prec} nvis={nvis} accumulate={accumulate}", flush=True)
        uv = rng.uniform(-N / 4, N / 4, (nvis, 2))
        vis = rng.standard_normal(nvis) + 1j * rng.standard_normal(nvis)
        w = rng.uniform(0.5, 2.0, nvis).astype(np.float32)
        plan = lmg.Plan(gtab, N, torch.from_numpy(uv).to(DEV), prec)
        vd = torch.from_numpy(vis).to(DEV, cdt)
        wd = torch.from_numpy(w).to(DEV)
        G0 = torch.from_numpy(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))).to(DEV, cdt)
        ref = plan.grid(vd, wd, out=G0.clone(), accumulate=bool(accumulate))
        got = G0.clone()
        st = lib.lmg_grid_planned_noalloc(plan.handle, _ptr(vd), _ptr(wd), _ptr(got), accumulate, _stream())
        assert st == 0, lmg.load().lmg_status_string(st)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        expect = im.grid(uv, vis, w.astype(np.float64), N, otab)
        if accumulate:
            expect = expect + G0.cpu().numpy()
        assert rel_rms(got.cpu().numpy(), expect) < TOL[prec]


def test_noalloc_rejects_plans_beyond_the_static_scratch():
    lib = lmg.load()
    otab, h = lt.make_table(7, 0.25, 300, 3)
    gtab = lmg.Table.from_nodes(7, 0.25, 300, 3, h, otab.nodes)
    nvis = 5_000_000                       # 80 MB of FP64 visibilities in entry order: above 64 MiB
    uv = torch.rand((nvis, 2), dtype=torch.float64, device=DEV) * 100 - 50
    plan = lmg.Plan(gtab, 512, uv, lmg.F64)
    need = ctypes.c_size_t()
    assert lib.lmg_plan_scratch_size(plan.handle, lmg.OP_GRID, ctypes.byref(need)) == 0
    assert need.value > (64 << 20)
    vis = torch.zeros(nvis, dtype=torch.complex128, device=DEV)
    g = torch.zeros((512, 512), dtype=torch.complex128, device=DEV)
    assert lib.lmg_grid_planned_noalloc(plan.handle, _ptr(vis), None, _ptr(g), 0, _stream()) == -5   # LMG_ENOTSUP
    assert lib.lmg_grid_planned_noalloc(None, _ptr(vis), None, _ptr(g), 0, _stream()) == -1
    assert lib.lmg_grid_planned_noalloc(plan.handle, _ptr(vis), None, _ptr(g), 2, _stream()) in (-1, -5)
