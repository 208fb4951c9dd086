"""Tables larger than the kernels' LDS budget (App. F's rates of 1e3 .. 1e6 samples per cell), read from a
device copy attached to the table, against the FP64 oracle (the oracle's h and nodes handed to the library).
Tolerances: relative RMS 1e-12 in FP64, 1e-5 in FP32."""
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


def rel_rms(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device=DEV, dtype=dtype)


@pytest.mark.parametrize("prec", [lmg.F32, lmg.F32_KAHAN, lmg.F64])
@pytest.mark.parametrize("W,Ms,degree", [(7, 1000, 3), (7, 20000, 0), (5, 4000, 1), (14, 2000, 1)])
def test_large_table_grid_degrid(prec, W, Ms, degree):
    print(f"large table W={W} Ms={Ms} d={degree} prec={prec}", flush=True)
    h = lt.optimal_h(7, 0.25)                   # any h defines a kernel (Eq. 18); both sides take the same
    otab = lt.Table(W, 0.25, Ms, degree, lt.table_nodes(h, W, 0.25, Ms, degree))
    gtab = lmg.Table.from_nodes(W, 0.25, W * Ms, degree, h, otab.nodes)
    assert gtab.device_bytes(prec) > 32768
    c = synth.small_case()
    uvd = dev(c.uv, torch.float64)
    with pytest.raises(lmg.LmgError) as e:      # too large for LDS and no device copy attached
        lmg.Plan(gtab, c.N, uvd, prec)
    assert e.value.status == -5
    gtab.attach_device(prec)
    plan = lmg.Plan(gtab, c.N, uvd, prec)
    cdt = torch.complex128 if prec == lmg.F64 else torch.complex64
    g = plan.grid(dev(c.vis, cdt)).cpu().numpy()
    assert rel_rms(g, im.grid(c.uv, c.vis, None, c.N, otab)) < TOL[prec]
    rng = np.random.default_rng(41)
    G = rng.standard_normal((c.N, c.N)) + 1j * rng.standard_normal((c.N, c.N))
    assert rel_rms(plan.degrid(dev(G, cdt)).cpu().numpy(), im.degrid(c.uv, G, otab)) < TOL[prec]


def test_small_tables_need_no_device_copy():
    t = lmg.Table.create(7, 0.25, 300, 3)
    assert t.device_bytes(lmg.F32) == 0 and t.device_bytes(lmg.F64) == 0
    assert t.attach_device(lmg.F64) is None


_LIMIT = {}


def _limit_table(table_size):
    """W = 1, degree-1 tables of 2^24 - 1 and 2^24 intervals from the oracle's h (built once each)."""
    if table_size not in _LIMIT:
        h = lt.optimal_h(1, 0.25)
        _LIMIT[table_size] = (lmg.Table.from_h(1, 0.25, table_size, 1, h), h)
    return _LIMIT[table_size]


@pytest.mark.parametrize("prec", [lmg.F32, lmg.F64])
def test_interval_count_limit_of_the_packed_offsets(prec):
    """A packed offset word holds the table interval in at most 24 bits (in an FP32 word at T = 32 that
    leaves 3 fraction bits, still finer in x than 2^-26). A degree-1 table of 2^24 - 1 intervals grids like
    the oracle's exact kernel (the table's own error, of order M_s^-2, is far below the tolerance); a table
    of 2^24 intervals is refused with LMG_ENOTSUP."""
    print(f"interval count limit prec={prec}", flush=True)
    c = synth.small_case()
    uvd = dev(c.uv, torch.float64)
    cdt = torch.complex128 if prec == lmg.F64 else torch.complex64
    tab, h = _limit_table((1 << 24) - 1)
    assert tab.Ms == (1 << 24) - 1
    tab.attach_device(prec)
    plan = lmg.Plan(tab, c.N, uvd, prec)
    g = plan.grid(dev(c.vis, cdt)).cpu().numpy()
    assert rel_rms(g, im.grid(c.uv, c.vis, None, c.N, lt.ExactKernel(1, 0.25, h))) < TOL[prec]
    big, _ = _limit_table(1 << 24)
    assert big.Ms == 1 << 24
    big.attach_device(prec)
    with pytest.raises(lmg.LmgError) as e:
        lmg.Plan(big, c.N, uvd, prec)
    assert e.value.status == -5
