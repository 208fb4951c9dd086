"""App. F on the device: the table's interpolation error falls as M_s^-(d+1).

For the 1,008,000-visibility array case on a 2048^2 grid (W = 7, x0 = 1/4,
FP64), each dirty image from a table of M_s samples per cell and degree d is
compared with the image from direct calculation of the weights (the exact
kernel, same plan geometry), so that the difference is the table's
contribution alone. Over M_s = 18 .. 144 the log-log slope must be -(d + 1)
within 0.15: the order of nearest-node (d = 0) and Newton forward
interpolation (App. F). The errors must also fall with d at every M_s >= 9.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1906_07102_amd as lmg  # noqa: E402

SIZES = (9, 18, 36, 72, 144)


def test_table_error_order_on_device():
    c = synth.array_1m_case(with_vis=True, device="cuda")
    uv = torch.from_numpy(c.uv).to("cuda:0")
    vis = torch.from_numpy(c.vis).to("cuda:0", torch.complex128)
    base = lmg.Table.create(7, 0.25, 300, 3)
    h, _ = base.export()
    ref = lmg.Plan(base.direct_calculation(), c.N, uv, lmg.F64).make_dirty_image(vis)
    nref = torch.linalg.vector_norm(ref).item()
    errs = {}
    for d in (0, 1, 2, 3):
        errs[d] = []
        for ms in SIZES:
            img = lmg.Plan(lmg.Table.from_h(7, 0.25, 7 * ms, d, h), c.N, uv, lmg.F64).make_dirty_image(vis)
            errs[d].append(torch.linalg.vector_norm(img - ref).item() / nref)
        slope = np.polyfit(np.log(SIZES[1:]), np.log(errs[d][1:]), 1)[0]
        print(f"degree {d}: slope {slope:.3f} errors {['%.2e' % e for e in errs[d]]}", flush=True)
        assert abs(slope + (d + 1)) < 0.15, (d, slope)
    for i in range(len(SIZES)):
        assert errs[0][i] > errs[1][i] > errs[2][i] > errs[3][i], i
